"""Two-site (two-tensor) TDVP on the device (Sec. "Tensor network
simulations": TDVP with a two-tensor update, the bond dimension as the
convergence knob) against the dense evolution and the two-site oracle
(oracle/two_site.py), and its eigensolver against numpy.

* The Jacobi eigensolver of the split (ttn_herm_eig): eigenvalues of random
  Hermitian positive semi-definite matrices within 1e-13 of their largest
  against numpy.linalg.eigvalsh, residual |A v - lambda v| and orthonormality
  of the eigenvectors within 1e-12.
* Maximal chi (2x2, 2x4): every two-site space is the whole space, so the
  integrator is exact -- the device state after several steps equals the
  dense evolution from the same (dressed, full-rank) initial state to 1e-10.
* Truncated chi (4x4, d = 3, chi = 12, random drive; 8x8, d = 3, chi = 12,
  the bond dimension of the paper's runs, GHZ program): the device state
  against the two-site oracle's on the same inputs, 1e-10 in the state
  infidelity C
  (the node tensors differ by a gauge: the device spans the kept singular
  subspace with Jacobi eigenvectors and Cholesky-QR factors, the oracle with
  LAPACK's singular vectors), fidelity, norm, energy, and the largest
  discarded weight of each step.
"""
import ctypes as C
import sys

import numpy as np
import pytest
import torch

from oracle import dense as D
from oracle import ttn_oracle as O
from oracle import two_site as TS
from paper_2210_03763_amd import ttn as T
from paper_2210_03763_amd import workload as W
from test_gpu_parity import gpu_state_as_oracle

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("n", [1, 5, 16, 81, 144, 256])
def test_jacobi_eigensolver(n):
    L = T.lib()
    L.ttn_herm_eig.restype = C.c_int
    L.ttn_herm_eig.argtypes = [C.c_int32] + [C.c_void_p] * 5
    rng = np.random.default_rng(n)
    M = rng.standard_normal((n + 3, n)) + 1j * rng.standard_normal((n + 3, n))
    M[:, -1] *= 1e-3                   # a spread of singular values
    A = M.conj().T @ M
    planar = lambda z: torch.tensor(np.concatenate([z.real.ravel(order="F"), z.imag.ravel(order="F")]),
                                    dtype=torch.float64, device="cuda")
    dA = planar(A)
    dV = torch.zeros(2 * n * n, dtype=torch.float64, device="cuda")
    dw = torch.zeros(n, dtype=torch.float64, device="cuda")
    do = torch.zeros(n, dtype=torch.int32, device="cuda")
    rc = L.ttn_herm_eig(n, dA.data_ptr(), dV.data_ptr(), dw.data_ptr(), do.data_ptr(),
                        torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    w = dw.cpu().numpy()
    order = do.cpu().numpy()
    Vp = dV.cpu().numpy()
    V = (Vp[:n * n] + 1j * Vp[n * n:]).reshape(n, n, order="F")[:, order]
    ref = np.linalg.eigvalsh(A)[::-1]
    scale = ref[0]
    assert np.all(np.diff(w) <= 0)
    assert np.abs(w - ref).max() <= 1e-13 * scale, np.abs(w - ref).max() / scale
    assert np.abs(A @ V - V * w).max() <= 1e-12 * scale
    assert np.abs(V.conj().T @ V - np.eye(n)).max() <= 1e-12
    assert sorted(order.tolist()) == list(range(n))


@pytest.mark.parametrize("Lx,Ly,chi", [(2, 2, 9), (4, 2, 81)])
def test_maximal_chi_matches_dense(Lx, Ly, chi):
    w = W.make_random_drive(Lx, Ly, 3, chi, 6, 0.05, 3, seed=7, plus_sites=(0, 1, 2, 3), eps=0.1).copy(update=1)
    _say(f"[two-site] {Lx}x{Ly} chi={chi} vs dense")
    st = O.build(w)
    psi0 = st.dense_state().numpy()
    ref = D.run(w, psi0)
    g = T.TTN(w)
    stats = g.step(w.n_steps, stats=True)
    gs = gpu_state_as_oracle(g, st)
    err = float(np.abs(gs.dense_state().numpy() - ref).max())
    _say(f"[two-site] max |psi - psi_dense| = {err:.2e}, discarded {max(s['max_discarded'] for s in stats):.1e}")
    assert err < 1e-10
    assert max(s["max_discarded"] for s in stats) < 1e-20   # nothing of weight dropped at maximal chi
    g.close()


_TS_ORACLE = {}


def _truncated_case():
    return W.make_random_drive(4, 4, 3, 12, 2, 0.01, 2, seed=5, plus_sites=tuple(range(16)), eps=0.05).copy(update=1)


@pytest.mark.parametrize("case", ["4x4 d3 chi12 drive", "8x8 d3 chi12 ghz"])
def test_truncated_chi_vs_two_site_oracle(case):
    if case.startswith("4x4"):
        w = _truncated_case()
    else:
        # the paper's bond dimension on the 8x8 GHZ program, one step
        w = W.make_ghz_program(8, 8, 3, 12, 1, 0.005, 2210037632, eps=0.05).copy(update=1)
    _say(f"[two-site] {case}, {w.n_steps} steps: oracle")
    st = TS.build(w)
    st, recs = O.run(w, st=st)
    Fo, _ = st.ghz_fidelity(w.target_sites)
    splits = 2 * (st.tree.n_nodes - 1)
    disc_o = [max(st.discarded[i * splits:(i + 1) * splits]) for i in range(w.n_steps)]
    _say("[two-site] device")
    g = T.TTN(w)
    stats = g.step(w.n_steps, stats=True)
    Fg, _ = g.fidelity()
    gs = gpu_state_as_oracle(g, st)
    Cst = 1 - abs(O.ttn_overlap(st, gs)) ** 2
    disc_g = [s["max_discarded"] for s in stats]
    res = dict(C=Cst, dF=abs(Fg - Fo), dN=abs(stats[-1]["norm2"] - recs[-1]["norm2"]),
               dE=abs(stats[-1]["energy"] - recs[-1]["energy"]), disc_oracle=disc_o, disc_device=disc_g, F=Fo)
    _say(f"[two-site] {res}")
    assert Cst <= 1e-10 and res["dF"] <= 1e-10 and res["dN"] <= 1e-10 and res["dE"] <= 1e-10, res
    for a, b in zip(disc_g, disc_o):
        assert abs(a - b) <= 1e-6 * b + 1e-14, res
    assert max(disc_o) > 1e-14      # chi = 12 truncates here
    g.close()
