"""Projective-measurement sampling from the tree tensor network: the CPU
oracle.

TEST INFRASTRUCTURE.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import or call this module; it shares no
code with the device library.

The paper extracts the statistics of projective measurements of all atoms
directly from the TTN, one million shots for its 8x8 histograms (Sec. on
parallel quantum algorithms, Fig. setup c).  It gives no sampling algorithm;
the one here draws each shot exactly from |psi(s)|^2 using the isometric
(root-canonical) form of the network, top-down:

  * a node v receives a normalised pure state u on its parent link (the root
    receives u = 1); its two child links carry B[l, r] = sum_p Q_v[l, r, p] u_p;
  * because the states of the right subtree are orthonormal, the marginal of
    the left subtree's outcome is the mixture over columns r with weights
    ||B[:, r]||^2 of the pure states B[:, r] / ||B[:, r]||: one uniform picks a
    column (cumulative weights in index order), and the left subtree is
    sampled from that pure state;
  * with the left outcome fixed and its amplitude vector phi_L[l] = <s_L|l>,
    the right subtree's conditional state is v[r] = sum_l phi_L[l] B[l, r],
    normalised;
  * at a bottom node the two sites are drawn one after the other from
    sum_{s_r} |B[s_l, s_r]|^2 and then |B[s_l, s_r]|^2;
  * every node returns phi_v[p] = sum_{l, r} phi_L[l] phi_R[r] Q_v[l, r, p], so
    the root returns the amplitude psi(s) of the drawn configuration.

Random numbers: Philox4x32 with 10 rounds (Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC 2011), counter (shot low
word, shot high word, draw index, 0), key (seed low word, seed high word);
a uniform in [0, 1) takes the first output word as its high 32 bits and the
top 21 bits of the second word below them, times 2^-53.  Draw indices: node v
uses draw v; the bottom node with index j uses draws n_nodes + 2 j and
n_nodes + 2 j + 1.  The device library implements the same generator from
the same definition.

Pinned by tests/test_oracle_sampling.py (amplitudes equal the network's own
amplitudes of the drawn configurations; frequencies against exact |psi|^2
from the dense state; generator uniformity and bijectivity).
"""
from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np
import torch

from oracle.ttn_oracle import CDT, OracleTTN

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK32 = 0xFFFFFFFF


def philox4x32_10(ctr: np.ndarray, key: Tuple[int, int]) -> np.ndarray:
    """Philox4x32-10 of an (n, 4) array of 32-bit counters under one key."""
    c = [ctr[:, i].astype(np.uint64) for i in range(4)]
    k0, k1 = np.uint64(key[0] & MASK32), np.uint64(key[1] & MASK32)
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + np.uint64(W0)) & np.uint64(MASK32)
            k1 = (k1 + np.uint64(W1)) & np.uint64(MASK32)
        p0 = np.uint64(M0) * c[0]
        p1 = np.uint64(M1) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK32)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK32)
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack(c, axis=1)


def uniform(seed: int, shot: np.ndarray, draw: int) -> np.ndarray:
    """53-bit uniforms in [0, 1) for the given shots and draw index."""
    shot = np.asarray(shot, dtype=np.uint64)
    ctr = np.stack([shot & np.uint64(MASK32), shot >> np.uint64(32),
                    np.full_like(shot, draw), np.zeros_like(shot)], axis=1)
    out = philox4x32_10(ctr, (seed & MASK32, (seed >> 32) & MASK32))
    bits = (out[:, 0] << np.uint64(21)) | (out[:, 1] >> np.uint64(11))
    return bits.astype(np.float64) * (2.0 ** -53)


def _pick(weights: torch.Tensor, u: float) -> int:
    """Smallest k with u * sum(w) < w_0 + ... + w_k (cumulative in index order)."""
    target = u * float(weights.sum())
    acc = 0.0
    for k in range(weights.shape[0]):
        acc += float(weights[k])
        if target < acc:
            return k
    return weights.shape[0] - 1   # u * sum rounded up to the total


def sample(st: OracleTTN, n_shots: int, seed: int, shot0: int = 0):
    """Draws n_shots configurations (site-indexed, values 0..d-1) with their
    amplitudes psi(s).  The network must be canonical toward the root (as the
    TDVP sweep leaves it) and normalised."""
    tr = st.tree
    nn = tr.n_nodes
    N = tr.N
    configs = np.zeros((n_shots, N), dtype=np.uint8)
    amps = np.zeros(n_shots, dtype=np.complex128)
    for b in range(n_shots):
        shot = shot0 + b

        def u_at(draw):
            return float(uniform(seed, np.array([shot]), draw)[0])

        def visit(v, u_in: torch.Tensor) -> torch.Tensor:
            Q = st.T[v]
            B = torch.einsum("lrp,p->lr", Q, u_in)
            if tr.is_bottom(v):
                j = tr.idx[v]
                sa, sb = tr.child_sites(v, 0)[0], tr.child_sites(v, 1)[0]
                p2 = B.abs() ** 2
                s_l = _pick(p2.sum(dim=1), u_at(nn + 2 * j))
                s_r = _pick(p2[s_l], u_at(nn + 2 * j + 1))
                configs[b, sa] = s_l
                configs[b, sb] = s_r
                return Q[s_l, s_r, :]
            col = (B.abs() ** 2).sum(dim=0)
            r = _pick(col, u_at(v))
            uL = B[:, r] / torch.sqrt(col[r])
            phiL = visit(tr.children[v][0], uL)
            vR = torch.einsum("l,lr->r", phiL, B)
            uR = vR / torch.linalg.vector_norm(vR)
            phiR = visit(tr.children[v][1], uR)
            return torch.einsum("l,r,lrp->p", phiL, phiR, Q)

        phi = visit(tr.root, torch.ones(1, dtype=CDT))
        amps[b] = complex(phi[0])
    return configs, amps


def config_amplitude(st: OracleTTN, config) -> complex:
    """<s|psi> for one configuration, by the network's product-state overlap."""
    d = st.tree.d
    states = np.zeros((st.tree.N, d), dtype=np.complex128)
    for s, x in enumerate(config):
        states[s, int(x)] = 1.0
    return st.product_overlap(states)
