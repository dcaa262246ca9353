"""Parity at the 8x8 sizes, in the launch configuration bench.py times.

* 8x8, d=3, chi=64 GHZ program (node tensors 64^3, every contraction on the
  MFMA path, split-K launches): two FP64 steps against the oracle, 1e-10 in
  fidelity, relative energy, norm and the state infidelity C.
* 8x8, d=4, chi=128 (the bench workload): the oracle needs minutes per step
  there, so the checks are properties that hold at any size plus the mixed
  path against the FP64 path: C(psi_mixed, psi_fp64) <= 1e-5 and
  |dF| <= 1e-5 after two steps; norm conserved to 1e-10 (FP64) and 1e-6
  (mixed); the |0> population of every site (conserved by H, every term
  annihilates |0>) within 1e-8 of its initial value on the FP64 path.
"""
import sys

import numpy as np
import pytest

from oracle import ttn_oracle as O
from paper_2210_03763_amd import ttn as T
from paper_2210_03763_amd import workload as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_8x8_d3_chi64_two_steps_fp64_vs_oracle():
    from test_gpu_parity import compare
    w = W.config("c2")
    compare(w, n_steps=2)


def _zero_pops(g, w):
    P0 = np.zeros((w.d, w.d), complex)
    P0[0, 0] = 1.0
    return np.array([g.local_expectation(s, P0).real for s in range(w.n_sites)])


def test_8x8_d4_chi128_mixed_vs_fp64_and_invariants():
    w = W.config("c3")
    n = 2
    _say("[large] c3 fp64 2 steps")
    g64 = T.TTN(w.copy(precision=T.PREC_FP64))
    p0 = _zero_pops(g64, w)
    s64 = g64.step(n, stats=True)
    F64, _ = g64.fidelity()
    p1 = _zero_pops(g64, w)
    _say("[large] c3 mixed 2 steps")
    gm = T.TTN(w)
    sm = gm.step(n, stats=True)
    Fm, _ = gm.fidelity()
    ov = gm.overlap(g64)
    C = 1 - abs(ov) ** 2
    res = dict(C=C, dF=abs(Fm - F64), n64=s64[-1]["norm2"], nm=sm[-1]["norm2"],
               dpop=float(np.abs(p1 - p0).max()), F=F64)
    _say(f"[large] {res}")
    assert C <= 1e-5, res
    assert abs(Fm - F64) <= 1e-5, res
    assert abs(s64[-1]["norm2"] - 1) <= 1e-10, res
    assert abs(sm[-1]["norm2"] - 1) <= 1e-6, res
    # populations change only through the gate events applied so far
    # (those at steps 0..n; the ones at step n close the call)
    gated = {s for (k, s, _) in w.events if k <= n}
    idle = [s for s in range(w.n_sites) if s not in gated]
    assert np.abs(p1[idle] - p0[idle]).max() <= 1e-8, res
    g64.close()
    gm.close()


def test_8x8_d4_chi256_repetition_code_mixed_vs_fp64():
    # the chi = 256 network (256^3 nodes, Cholesky of 256 x 256 Gram matrices
    # outside LDS): one step of the repetition-code program, mixed against FP64
    w = W.config("c5")
    n = 1
    _say("[large] c5 fp64 1 step")
    g64 = T.TTN(w.copy(precision=T.PREC_FP64))
    s64 = g64.step(n, stats=True)
    F64, _ = g64.fidelity()
    _say("[large] c5 mixed 1 step")
    gm = T.TTN(w)
    sm = gm.step(n, stats=True)
    Fm, _ = gm.fidelity()
    C = 1 - abs(gm.overlap(g64)) ** 2
    res = dict(C=C, dF=abs(Fm - F64), n64=s64[-1]["norm2"], nm=sm[-1]["norm2"], F=F64)
    _say(f"[large] {res}")
    assert C <= 1e-5 and abs(Fm - F64) <= 1e-5, res
    assert abs(s64[-1]["norm2"] - 1) <= 1e-10 and abs(sm[-1]["norm2"] - 1) <= 1e-6, res
    g64.close()
    gm.close()
