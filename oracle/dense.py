"""Dense state-vector reference: the plain definition of the evolution.

TEST INFRASTRUCTURE (same import rule as ttn_oracle).  For small lattices
the TDVP oracle is pinned against psi_{n+1} = exp(-i H(t_n + dt/2) dt) psi_n
with the full Hamiltonian of Eq. (eq:ham)/(eq:c6) (read as in ttn_oracle:
Omega/2 on |1><r| + h.c., -Delta |r><r|, optional leak coupling, positive
C6/d^6 over pairs i < j) built as a sparse matrix on the product basis
(site 0 the slowest index), and evolved with scipy's expm_multiply.  At
maximal bond dimension single-site TDVP reproduces this exactly (the
exactness of projector-splitting integrators, Lubich, Oseledets and
Vandereycken 2015).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _ops(d):
    X = np.zeros((d, d), complex)
    n = np.zeros((d, d), complex)
    Lk = np.zeros((d, d), complex)
    X[1, 2] = X[2, 1] = 1
    n[2, 2] = 1
    if d >= 4:
        Lk[3, 2] = Lk[2, 3] = 1
    return X, n, Lk


def _embed(op, site, N, d):
    out = sp.identity(1, dtype=complex, format="csr")
    for s in range(N):
        out = sp.kron(out, sp.csr_matrix(op) if s == site else sp.identity(d, dtype=complex),
                      format="csr")
    return out


def hamiltonian(pos, d, omega_t, delta_t, c6=1.0, r_cut=0.0, leak_ratio=0.0):
    N = len(pos)
    X, n, Lk = _ops(d)
    H = sp.csr_matrix((d ** N, d ** N), dtype=complex)
    nsite = [_embed(n, s, N, d) for s in range(N)]
    for s in range(N):
        hl = omega_t[s] / 2 * (X + leak_ratio * Lk) - delta_t[s] * n
        if np.any(hl != 0):
            H = H + _embed(hl, s, N, d)
    for i in range(N):
        for j in range(i + 1, N):
            dist = math.hypot(pos[i][0] - pos[j][0], pos[i][1] - pos[j][1])
            if r_cut > 0 and dist > r_cut:
                continue
            H = H + (c6 / dist ** 6) * (nsite[i] @ nsite[j])
    return H


def product_vector(states):
    v = np.ones(1, complex)
    for s in states:
        v = np.kron(v, np.asarray(s, complex))
    return v


def apply_local(psi, U, site, N, d):
    t = psi.reshape([d] * N)
    t = np.moveaxis(np.tensordot(U, t, axes=([1], [site])), 0, site)
    return t.reshape(-1)


def pulse_index(edges, t):
    for s in range(len(edges) - 1):
        if edges[s] <= t < edges[s + 1]:
            return s
    return -1


def run(w, psi0, n_steps=None, step0=0, apply_final_events=True):
    """Evolve psi0 (site 0 slowest) with the workload's program."""
    N, d = w.n_sites, w.d
    n_steps = w.n_steps if n_steps is None else n_steps
    psi = np.asarray(psi0, complex).copy()
    for n in range(step0, step0 + n_steps):
        for (k, s, U) in w.events:
            if k == n:
                psi = apply_local(psi, U, s, N, d)
        t = (n + 0.5) * w.dt
        sidx = pulse_index(w.seg_edges, t)
        om = w.omega[:, sidx] if sidx >= 0 else np.zeros(N)
        de = w.delta[:, sidx] if sidx >= 0 else np.zeros(N)
        H = hamiltonian(w.pos_xy, d, om, de, w.c6, w.r_cut, w.leak_ratio)
        psi = spla.expm_multiply(-1j * w.dt * H, psi)
    if apply_final_events:
        for (k, s, U) in w.events:
            if k == step0 + n_steps:
                psi = apply_local(psi, U, s, N, d)
    return psi
