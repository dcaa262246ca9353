"""The contraction kernel (through the C ABI's ttn_leg_contract) against a
plain complex128 einsum of the same leg operation, at the node shapes of the
8x8, d=4, chi=128 network (128^3 nodes, 16x16x128 level-1 nodes, 4x4x16
bottom nodes), the d=3 shapes, and ragged sizes that leave partial tiles.

FP64: max |y - ref| <= 1e-12 max|ref|.  FP32 inputs rounded from the same
data: <= 1e-5 max|ref| (single-precision products, FP32 accumulation over
K <= 33*128 terms)."""
import ctypes as C
import sys

import numpy as np
import pytest
import torch

from paper_2210_03763_amd import ttn as T

pytestmark = pytest.mark.gpu


def _lib():
    L = T.lib()
    L.ttn_leg_contract.restype = C.c_int
    L.ttn_leg_contract.argtypes = [C.c_int32] * 6 + [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                                     C.c_int32, C.c_int32, C.c_void_p]
    return L


def _planar(z: torch.Tensor, dtype):
    # (..., n) complex -> (..., 2n) real planar per item
    return torch.cat([z.real, z.imag], dim=-1).to(dtype).contiguous()


def _unplanar(p: torch.Tensor, n: int):
    return torch.complex(p[..., :n].double(), p[..., n:].double())


def _ref(leg, ops, xs):
    # ops (K, D, D) [a, b]; xs (K or 1, DL, DR, DP) -> op_k applied on leg
    eq = {0: "kab,kbrp->karp", 1: "kab,klbp->klap", 2: "kab,klrb->klra"}[leg]
    return torch.einsum(eq, ops, xs.expand(ops.shape[0], *xs.shape[1:]))


CASES = [
    # (DL, DR, DP, leg, n_ops, x_per_op, sum)
    (128, 128, 128, 0, 17, 0, 0),     # stage A at a level-4 node
    (128, 128, 128, 1, 16, 0, 0),     # stage B
    (128, 128, 128, 1, 6, 1, 1),      # stage C (two-level contraction index)
    (128, 128, 128, 2, 5, 1, 1),      # stage D
    (128, 128, 128, 2, 1, 0, 0),
    (16, 16, 128, 0, 3, 0, 0),        # level-1 node, d=4
    (16, 16, 128, 2, 9, 1, 1),
    (4, 4, 16, 1, 2, 1, 1),           # bottom node, d=4
    (3, 3, 9, 0, 2, 0, 0),            # bottom node, d=3
    (64, 64, 64, 2, 33, 1, 1),        # 8x8 d=3 chi=64 level-4 node
    (81, 81, 81, 1, 4, 1, 0),         # ragged tiles
    (128, 1, 128, 0, 33, 0, 0),       # bond as a (D, 1, D) tensor
    (128, 1, 128, 2, 33, 1, 1),
]


@pytest.mark.parametrize("prec", [T.PREC_FP64, T.PREC_FP32])
@pytest.mark.parametrize("case", CASES)
def test_leg_contract_matches_einsum(case, prec):
    DL, DR, DP, leg, K, xpo, sm = case
    print(f"[kernel] {case} prec={prec}", flush=True)
    L = _lib()
    g = torch.Generator().manual_seed(hash(case) % 1000 + prec)
    D = (DL, DR, DP)[leg]
    ops = torch.complex(torch.randn(K, D, D, generator=g, dtype=torch.float64),
                        torch.randn(K, D, D, generator=g, dtype=torch.float64))
    nx = K if xpo else 1
    xs = torch.complex(torch.randn(nx, DL, DR, DP, generator=g, dtype=torch.float64),
                       torch.randn(nx, DL, DR, DP, generator=g, dtype=torch.float64))
    dt = torch.float32 if prec == T.PREC_FP32 else torch.float64
    if prec == T.PREC_FP32:   # reference on the rounded inputs
        ops = ops.to(torch.complex64).to(torch.complex128)
        xs = xs.to(torch.complex64).to(torch.complex128)
    n = DL * DR * DP
    # device layouts: op column-major [a + D b]; x with l fastest
    ops_flat = ops.transpose(1, 2).reshape(K, D * D)
    xs_flat = xs.permute(0, 3, 2, 1).reshape(nx, n)
    d_ops = _planar(ops_flat, dt).cuda()
    d_x = _planar(xs_flat, dt).cuda()
    ny = 1 if sm else K
    d_y = torch.zeros(ny, 2 * n, dtype=dt, device="cuda")
    rc = L.ttn_leg_contract(prec, leg, DL, DR, DP, K, d_ops.data_ptr(), d_x.data_ptr(), xpo, d_y.data_ptr(),
                            sm, 0, torch.cuda.current_stream().cuda_stream)
    assert rc == 0, L.ttn_last_error(None)
    ref = _ref(leg, ops, xs)
    if sm:
        ref = ref.sum(0, keepdim=True)
    ref_flat = ref.permute(0, 3, 2, 1).reshape(ny, n)
    got = _unplanar(d_y.cpu(), n)
    err = (got - ref_flat).abs().max().item()
    scale = ref_flat.abs().max().item()
    tol = 1e-12 if prec == T.PREC_FP64 else 1e-5
    print(f"[kernel] err/scale = {err / scale:.2e}", flush=True)
    assert err <= tol * scale


def test_leg_contract_accumulates():
    L = _lib()
    DL = DR = DP = 32
    g = torch.Generator().manual_seed(5)
    op = torch.complex(torch.randn(1, DL, DL, generator=g, dtype=torch.float64),
                       torch.randn(1, DL, DL, generator=g, dtype=torch.float64))
    x = torch.complex(torch.randn(1, DL, DR, DP, generator=g, dtype=torch.float64),
                      torch.randn(1, DL, DR, DP, generator=g, dtype=torch.float64))
    n = DL * DR * DP
    y0 = torch.complex(torch.randn(1, n, generator=g, dtype=torch.float64),
                       torch.randn(1, n, generator=g, dtype=torch.float64))
    d_y = _planar(y0, torch.float64).cuda()
    d_op = _planar(op.transpose(1, 2).reshape(1, -1), torch.float64).cuda()   # kept alive across the call
    d_x = _planar(x.permute(0, 3, 2, 1).reshape(1, n), torch.float64).cuda()
    rc = L.ttn_leg_contract(0, 0, DL, DR, DP, 1, d_op.data_ptr(), d_x.data_ptr(), 0,
                            d_y.data_ptr(), 0, 1, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert rc == 0
    ref = y0 + _ref(0, op, x).permute(0, 3, 2, 1).reshape(1, n)
    assert (_unplanar(d_y.cpu(), n) - ref).abs().max() < 1e-11


def test_leg_contract_rejects_bad_sizes():
    L = _lib()
    assert L.ttn_leg_contract(0, 3, 4, 4, 4, 1, 1, 1, 0, 1, 0, 0, None) == T.TTN_EINVAL
    assert L.ttn_leg_contract(5, 0, 4, 4, 4, 1, 1, 1, 0, 1, 0, 0, None) == T.TTN_EINVAL
    assert L.ttn_leg_contract(0, 0, 4, 4, 4, 1, 1, 1, 0, 1, 1, 0, None) == T.TTN_EINVAL   # sum needs x_per_op
