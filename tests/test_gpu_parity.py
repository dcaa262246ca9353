"""Parity of the HIP TDVP path (through the C ABI) with the CPU FP64 oracle.

Tolerances: the FP64 path must agree with the oracle within 1e-10 in
fidelity, energy (relative), norm and the state infidelity
C(psi_gpu, psi_oracle) = 1 - |<psi_gpu|psi_oracle>|^2 (Tab. conv8x8
definition).  The mixed path (contractions in complex FP32) must keep
C <= 1e-5 and |dF| <= 1e-5 against the oracle.
"""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import dense as D
from oracle import ttn_oracle as O
from paper_2210_03763_amd import ttn as T
from paper_2210_03763_amd import workload as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_state_as_oracle(g: T.TTN, st_like: O.OracleTTN) -> O.OracleTTN:
    """Load the exported device tensors into an oracle-shaped network (CPU)."""
    flat = g.export_state()
    other = O.OracleTTN.__new__(O.OracleTTN)
    other.tree = st_like.tree
    other.T = []
    off = 0
    for v in range(st_like.tree.n_nodes):
        DL, DR, DP = st_like.tree.dims[v]
        n = DL * DR * DP
        blk = torch.as_tensor(flat[off:off + n]).reshape(DP, DR, DL).permute(2, 1, 0).contiguous()
        other.T.append(blk)
        off += n
    return other


def compare(w, n_steps=None, tol=1e-10, tolC=None, check_energy=True):
    n_steps = w.n_steps if n_steps is None else n_steps
    _say(f"[parity] {w.name} N={w.n_sites} d={w.d} chi={w.chi} steps={n_steps} prec={w.precision}")
    st, recs = O.run(w, n_steps=n_steps)
    Fo, _ = st.ghz_fidelity(w.target_sites)
    g = T.TTN(w)
    stats = g.step(n_steps, stats=True)
    Fg, _ = g.fidelity()
    gs = gpu_state_as_oracle(g, st)
    ov = O.ttn_overlap(st, gs)
    Cst = 1 - abs(ov) ** 2
    n2g, Eg = stats[-1]["norm2"], stats[-1]["energy"]
    # smallest R_kk of the step's gauge moves (the QR conditioning monitor)
    rrel = max(abs(s["min_r_diag"] - r["min_r_diag"]) / r["min_r_diag"] for s, r in zip(stats, recs))
    res = dict(dF=abs(Fg - Fo), C=Cst, dN=abs(n2g - recs[-1]["norm2"]),
               dE=abs(Eg - recs[-1]["energy"]) / max(1.0, abs(recs[-1]["energy"])), F=Fo,
               min_r=min(s["min_r_diag"] for s in stats), min_r_rel=rrel)
    _say(f"[parity] {res}")
    tolC = tol if tolC is None else tolC
    assert res["dF"] <= tol, res
    assert res["C"] <= tolC, res
    assert res["dN"] <= tol, res
    if check_energy:
        assert res["dE"] <= tol, res
    if w.precision == T.PREC_FP64:
        assert rrel <= 1e-6, res
    g.close()
    return res


def test_c1_ent_fp64():
    compare(W.config("c1-ent"))


def test_c1_drive_dressed_fp64():
    # the 4x4 chi=16 drive with |+> on site 0, dressed so that every QR is full rank
    w = W.config("c1").copy(dress_eps=1e-2)
    w.dress_noise = W._complex_normal(np.random.Generator(np.random.PCG64(77)),
                                      W.noise_len(16, 3, 16))
    compare(w)


@pytest.mark.parametrize("d", [3, 4])
def test_maximal_chi_2x2_matches_dense(d):
    w = W.make_random_drive(2, 2, d, d * d, 8, 0.05, 3, seed=11 + d, plus_sites=(0, 1, 2, 3), eps=0.1)
    _say(f"[dense] 2x2 d={d}")
    st = O.build(w)
    psi0 = st.dense_state().numpy()
    ref = D.run(w, psi0)
    g = T.TTN(w)
    g.step(w.n_steps)
    gs = gpu_state_as_oracle(g, st)
    assert np.abs(gs.dense_state().numpy() - ref).max() < 1e-10
    g.close()


def test_gate_program_2x4_truncated_fp64():
    w = W.make_ghz_program(4, 2, 3, 5, 16, 0.02, seed=21, n_layers=4, seg_per_layer=2, eps=0.05)
    compare(w)


def test_gate_program_4x4_d4_fp64():
    w = W.make_ghz_program(4, 4, 4, 12, 10, 0.01, seed=23, n_layers=6, seg_per_layer=2, eps=0.02)
    compare(w)


def test_c1_ent_mixed_precision():
    w = W.config("c1-ent").copy(precision=T.PREC_FP32)
    res = compare(w, tol=1e-5, tolC=1e-5, check_energy=False)
    assert res["dE"] < 1e-4


def test_observables_and_local_expectation():
    w = W.config("c1-ent").copy(n_steps=5)
    _say("[obs] c1-ent 5 steps")
    st, recs = O.run(w, n_steps=5)
    g = T.TTN(w)
    g.step(5)
    n2, E = g.observables()
    assert abs(n2 - recs[-1]["norm2"]) < 1e-10
    assert abs(E - recs[-1]["energy"]) < 1e-10
    n_op = np.diag([0, 0, 1.0]).astype(complex)
    for s in (0, 5, 15):
        a = g.local_expectation(s, n_op)
        b = st.local_expectation(s, n_op)
        assert abs(a - b) < 1e-10
    g2 = T.TTN(w)
    ov = g.overlap(g2)        # evolved vs initial
    gs = gpu_state_as_oracle(g, st)
    g2s = gpu_state_as_oracle(g2, st)
    assert abs(ov - O.ttn_overlap(gs, g2s)) < 1e-10
    g.close()
    g2.close()


def test_undressed_rank_deficient_state_reports_enumeric():
    # an undressed product state is rank deficient above its Schmidt rank:
    # the CholeskyQR2 gauge move reports it instead of producing garbage
    w = W.config("c1")
    _say("[err] undressed c1")
    with pytest.raises(T.TTNError) as e:
        g = T.TTN(w)
        g.step(1)
    assert e.value.code == T.TTN_ENUMERIC


def test_interaction_cutoff_fp64():
    # interaction-range cut-off (Sec. "Tensor network simulations"): pairs
    # farther than r_cut = 1.2 dropped (only nearest neighbours kept), 4x4
    # chi=16 dressed drive, 20 steps
    w = W.config("c1-ent").copy(r_cut=1.2)
    compare(w)
    # the cut is effective: the all-pairs oracle run ends in another state
    # (C = 1.2e-7 between the two)
    st_cut, _ = O.run(w, record=False)
    st_all, _ = O.run(w.copy(r_cut=0.0), record=False)
    C = 1 - abs(O.ttn_overlap(st_cut, st_all)) ** 2
    assert C > 1e-8, C


def test_nonfinite_pulses_rejected_state_unchanged():
    # a NaN in the pulse table is rejected before any device work
    # (TTN_EINVAL), and the handle keeps its program and state
    w = W.config("c1-ent").copy(n_steps=2)
    g = T.TTN(w)
    g.step(1)
    before = g.export_state()
    om = np.array(w.omega, copy=True)
    om[3, 1] = np.nan
    with pytest.raises(T.TTNError) as e:
        g.set_pulses(w.seg_edges, om, w.delta, w.events)
    assert e.value.code == T.TTN_EINVAL
    assert np.array_equal(g.export_state(), before)
    g.step(1)
    st, _ = O.run(w, n_steps=2)
    Fo, _ = st.ghz_fidelity(w.target_sites)
    assert abs(g.fidelity()[0] - Fo) < 1e-10
    g.close()


def test_zero_hamiltonian_is_a_happy_breakdown():
    # every drive zero and C6 = 0: H = 0, so every Krylov recursion breaks
    # down after its first vector (beta_1 = 0) and each step is the identity
    # on the state (the gauge moves of the sweep re-gauge the node tensors,
    # so the state is compared, not the tensors; 2x2 at maximal chi, dressed
    # so that every gauge move is full rank)
    w = W.make_random_drive(2, 2, 3, 9, 4, 0.05, 2, seed=3, plus_sites=(0, 1, 2, 3), eps=0.1)
    w.omega[:] = 0.0
    w.delta[:] = 0.0
    w.c6 = 0.0
    g0 = T.TTN(w)
    g = T.TTN(w)
    F0, _ = g.fidelity()
    stats = g.step(4, stats=True)
    assert all(s["min_krylov"] == 1 for s in stats), stats
    ov = g.overlap(g0)
    assert abs(ov - 1) < 1e-12, ov
    assert abs(g.fidelity()[0] - F0) < 1e-13
    g.close()
    g0.close()
