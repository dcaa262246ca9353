"""Parity with the oracle on networks large enough to take the full-size
kernel paths of the 8x8, chi = 128 workload.

On 4 x 4 lattices at chi = 128 and 160 the node tensors are 81 x 81 x chi
(d = 3) or 128^3 (d = 4), so the contractions take the 128 x 128 FP32 MFMA
tiles with 32-wide k-tiles, the BF16x3 kernel (in that mode), split-K with
the vector reduction, and at chi = 160 the Cholesky of gauge moves wider
than 128 (global-memory panels).  The oracle (plain FP64 CPU) is run here on
the same seeded inputs (dressed product state, |+> on every site, random
piecewise drive; Sec. "Tensor network simulations" for the method, Tab.
conv8x8 for the state infidelity C).

Bars: FP64 path -- every entry of every exported node tensor within 1e-10
of the oracle's (the gauge is unique: thin QR with real positive R_kk),
|dF|, relative |dE| and |d norm^2| <= 1e-10, the smallest R_kk of each step
equal to the oracle's to 1e-6 relative; FP32 and BF16x3 paths -- C <= 1e-5
and |dF| <= 1e-5 against the oracle, with the kernel classes that ran
checked from a profiling window.
"""
import sys

import numpy as np
import pytest

from oracle import ttn_oracle as O
from paper_2210_03763_amd import ttn as T
from paper_2210_03763_amd import workload as W
from test_gpu_parity import gpu_state_as_oracle

pytestmark = pytest.mark.gpu

CASES = {
    # name: (d, chi, steps)
    "4x4 d3 chi128": (3, 128, 3),
    "4x4 d3 chi160": (3, 160, 3),
    "4x4 d4 chi128": (4, 128, 2),
}
_ORACLE = {}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _workload(name):
    d, chi, steps = CASES[name]
    return W.make_random_drive(4, 4, d, chi, steps, 0.01, min(3, steps), 2210037640 + chi + d,
                               plus_sites=tuple(range(16)), eps=1e-2, name=name)


def _oracle(name):
    if name not in _ORACLE:
        w = _workload(name)
        _say(f"[fullsize] oracle {name}: {w.n_steps} steps")
        st, recs = O.run(w)
        F, _ = st.ghz_fidelity(w.target_sites)
        _ORACLE[name] = (st, recs, F)
    return _ORACLE[name]


def _flat(st):
    return np.concatenate([t.numpy().transpose(2, 1, 0).reshape(-1) for t in st.T])


def _run_gpu(w, profile_last=True):
    g = T.TTN(w)
    stats = g.step(w.n_steps - 1, stats=True) if w.n_steps > 1 else []
    prof = launches = None
    if profile_last:
        g.profile_begin()
        stats += g.step(1, stats=True)
        prof = g.profile_end()
        launches = g.profile_launches()
    else:
        stats += g.step(1, stats=True)
    F, _ = g.fidelity()
    return g, stats, F, prof, launches


@pytest.mark.parametrize("name", list(CASES))
def test_fp64_elementwise_vs_oracle(name):
    w = _workload(name)
    st, recs, Fo = _oracle(name)
    _say(f"[fullsize] fp64 {name}")
    g, stats, Fg, prof, launches = _run_gpu(w)
    gs = gpu_state_as_oracle(g, st)
    a, b = _flat(gs), _flat(st)
    err = float(np.abs(a - b).max())
    dN = abs(stats[-1]["norm2"] - recs[-1]["norm2"])
    dE = abs(stats[-1]["energy"] - recs[-1]["energy"]) / max(1.0, abs(recs[-1]["energy"]))
    rmin = [(s["min_r_diag"], r["min_r_diag"]) for s, r in zip(stats, recs)]
    rrel = max(abs(x - y) / y for x, y in rmin)
    big = sum(1 for r in launches if r["kernel"] == 2 and r["splits"] > 1)
    res = dict(max_entry_err=err, dF=abs(Fg - Fo), dN=dN, dE=dE, min_r=rmin, min_r_rel=rrel,
               mfma_splitk_launches=big, F=Fo)
    _say(f"[fullsize] {res}")
    assert err <= 1e-10, res
    assert res["dF"] <= 1e-10 and dN <= 1e-10 and dE <= 1e-10, res
    assert rrel <= 1e-6, res
    assert big > 0, res
    g.close()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", [T.PREC_FP32, T.PREC_BF16X3])
def test_reduced_precision_vs_oracle(name, prec):
    w = _workload(name).copy(precision=prec)
    st, recs, Fo = _oracle(name)
    _say(f"[fullsize] prec={prec} {name}")
    g, stats, Fg, prof, launches = _run_gpu(w)
    gs = gpu_state_as_oracle(g, st)
    ov = O.ttn_overlap(st, gs)
    C = 1 - abs(ov) ** 2
    kinds = sorted({(r["kernel"], r["prec"]) for r in launches})
    res = dict(C=C, dF=abs(Fg - Fo), dN=abs(stats[-1]["norm2"] - recs[-1]["norm2"]),
               dE=abs(stats[-1]["energy"] - recs[-1]["energy"]), kinds=kinds,
               bf16_launches=prof.gemm_bf16x3.launches, F=Fo)
    _say(f"[fullsize] {res}")
    assert C <= 1e-5 and res["dF"] <= 1e-5, res
    assert (2, 1) in kinds, res                       # FP32 MFMA kernel ran
    if prec == T.PREC_BF16X3:
        assert prof.gemm_bf16x3.launches > 0, res     # and the BF16x3 kernel
    else:
        assert prof.gemm_bf16x3.launches == 0, res
    g.close()


def test_chi160_takes_the_wide_gauge_moves():
    # a link of width 160 (> 128, the largest Cholesky held in LDS) exists
    w = _workload("4x4 d3 chi160")
    dims = W.node_shapes(w.n_sites, w.d, w.chi)
    assert max(max(s) for s in dims) == 160
