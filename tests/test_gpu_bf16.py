"""The BF16x3 precision mode (split bf16 products on the bf16 matrix cores,
FP32 accumulation) against FP64 references.

Per contraction: relative error of a 128^3 stage within 1e-4 of the operand
scale (the split keeps about 16 bits per operand).  Whole path: the 4x4
workload with |+> on every site against the oracle, and the 8x8, d = 4,
chi = 128 GHZ program against the FP64 path, both at the mixed bar (1e-5 in
the fidelity and in C).
"""
import ctypes as C
import sys

import numpy as np
import pytest
import torch

from oracle import ttn_oracle as O
from paper_2210_03763_amd import ttn as T
from paper_2210_03763_amd import workload as W
from test_gpu_parity import compare

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("leg,K,xpo,sm,shift", [(0, 17, 0, 0, 0), (1, 16, 0, 0, 0), (1, 17, 1, 1, 0), (2, 33, 1, 1, 0),
                                                (0, 17, 0, 0, 1), (2, 33, 1, 1, 1)])
def test_bf16x3_stage_accuracy(leg, K, xpo, sm, shift):
    """shift = 1 moves both operands one element off 16-byte alignment, which
    takes the k-fast operands off the vector-load path."""
    L = T.lib()
    L.ttn_leg_contract.restype = C.c_int
    L.ttn_leg_contract.argtypes = [C.c_int32] * 6 + [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32,
                                                     C.c_int32, C.c_void_p]
    chi = 128
    n = chi ** 3
    g = torch.Generator(device="cuda").manual_seed(11 + leg)
    ops = torch.randn(K, 2 * chi * chi, dtype=torch.float64, device="cuda", generator=g)
    x = torch.randn(K if xpo else 1, 2 * n, dtype=torch.float64, device="cuda", generator=g)
    outs = {}
    st = torch.cuda.current_stream().cuda_stream
    for prec, dt in ((T.PREC_FP64, torch.float64), (T.PREC_BF16X3, torch.float32), (T.PREC_FP32, torch.float32)):
        o = torch.zeros(ops.numel() + shift, dtype=dt, device="cuda")[shift:].view_as(ops)
        xx = torch.zeros(x.numel() + shift, dtype=dt, device="cuda")[shift:].view_as(x)
        o.copy_(ops)
        xx.copy_(x)
        y = torch.zeros(1 if sm else K, 2 * n, dtype=dt, device="cuda")
        rc = L.ttn_leg_contract(prec, leg, chi, chi, chi, K, o.data_ptr(), xx.data_ptr(), xpo, y.data_ptr(), sm, 0, st)
        torch.cuda.synchronize()
        assert rc == 0
        outs[prec] = y.double()
    ref = outs[T.PREC_FP64]
    scale = ref.abs().max().item()
    e16 = (outs[T.PREC_BF16X3] - ref).abs().max().item() / scale
    e32 = (outs[T.PREC_FP32] - ref).abs().max().item() / scale
    _say(f"[bf16] leg {leg} K {K} shift {shift}: relative max error bf16x3 {e16:.2e}, fp32 {e32:.2e}")
    assert e16 < 1e-4
    assert e16 > e32   # the split really ran


def test_bf16x3_c1_ent_vs_oracle():
    w = W.config("c1-ent").copy(precision=T.PREC_BF16X3)
    res = compare(w, tol=1e-5, tolC=1e-5, check_energy=False)
    assert res["dE"] < 1e-3


def test_bf16x3_8x8_chi128_vs_fp64():
    w = W.config("c3")
    n = 4
    gb = T.TTN(w.copy(precision=T.PREC_BF16X3))
    g64 = T.TTN(w.copy(precision=T.PREC_FP64))
    gb.step(n)
    g64.step(n)
    Fb, _ = gb.fidelity()
    F64, _ = g64.fidelity()
    C_ = 1 - abs(gb.overlap(g64)) ** 2
    _say(f"[bf16] 8x8 chi128 after {n} steps: |dF| {abs(Fb - F64):.2e}, C {C_:.2e}")
    assert abs(Fb - F64) < 1e-5 and C_ < 1e-5
    gb.close()
    g64.close()
