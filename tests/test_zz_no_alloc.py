"""ttn_leg_contract_noalloc (split-K scratch in a file-scope device array,
no device allocation) against ttn_leg_contract (allocates its scratch) on
the same inputs: the same kernels and split factors, so the outputs must be
bit-identical.  Two calls in a row, the second with a smaller input (the
array keeps the first call's partial sums, which must not leak into the
second), in FP64, FP32 and BF16x3, on shapes that take split-K (the parent-
leg sum of a 128^3 node) and on shapes that do not."""
import ctypes as C
import sys

import pytest
import torch

from paper_2210_03763_amd import ttn as T

pytestmark = pytest.mark.gpu

ARGS = [C.c_int32] * 6 + [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]


def _lib():
    L = T.lib()
    for name in ("ttn_leg_contract", "ttn_leg_contract_noalloc"):
        f = getattr(L, name)
        f.restype = C.c_int
        f.argtypes = ARGS
    return L


def _case(precision, leg, D, n_ops, x_per_op, sum_ops, accumulate, seed):
    dt = torch.float64 if precision == T.PREC_FP64 else torch.float32
    g = torch.Generator(device="cuda").manual_seed(seed)
    n = D ** 3
    ops = torch.randn(n_ops, 2 * D * D, dtype=dt, device="cuda", generator=g)
    x = torch.randn(n_ops if x_per_op else 1, 2 * n, dtype=dt, device="cuda", generator=g)
    y0 = torch.randn(1 if sum_ops else n_ops, 2 * n, dtype=dt, device="cuda", generator=g)
    return ops, x, y0


def _run(L, name, precision, leg, D, n_ops, x_per_op, sum_ops, accumulate, ops, x, y0):
    y = y0.clone()
    st = torch.cuda.current_stream().cuda_stream
    rc = getattr(L, name)(precision, leg, D, D, D, n_ops, ops.data_ptr(), x.data_ptr(), x_per_op, y.data_ptr(),
                          sum_ops, accumulate, st)
    torch.cuda.synchronize()
    assert rc == 0, (name, rc, T.lib().ttn_last_error(None))
    return y


@pytest.mark.parametrize("precision", [T.PREC_FP64, T.PREC_FP32, T.PREC_BF16X3])
def test_noalloc_matches_allocating_entry_point(precision):
    L = _lib()
    # first call: parent-leg sum over 33 operator/tensor pairs of a 128^3 node
    # (split-K), then a smaller one: the left-leg stack of a 64^3 node with
    # accumulation (16 operators on a shared tensor)
    calls = [(2, 128, 33, 1, 1, 0, 11), (0, 64, 16, 0, 0, 1, 12)]
    for leg, D, n_ops, xpo, sm, acc, seed in calls:
        print(f"[noalloc] prec={precision} leg={leg} D={D} ops={n_ops}", flush=True)
        sys.stdout.flush()
        ops, x, y0 = _case(precision, leg, D, n_ops, xpo, sm, acc, seed)
        ya = _run(L, "ttn_leg_contract", precision, leg, D, n_ops, xpo, sm, acc, ops, x, y0)
        yb = _run(L, "ttn_leg_contract_noalloc", precision, leg, D, n_ops, xpo, sm, acc, ops, x, y0)
        assert torch.isfinite(ya).all()
        assert torch.equal(ya, yb), float((ya - yb).abs().max())
        assert not torch.equal(ya, y0)


def test_noalloc_rejects_bad_arguments():
    L = _lib()
    st = torch.cuda.current_stream().cuda_stream
    buf = torch.zeros(16, dtype=torch.float64, device="cuda")
    rc = L.ttn_leg_contract_noalloc(T.PREC_FP64, 3, 2, 2, 2, 1, buf.data_ptr(), buf.data_ptr(), 0, buf.data_ptr(),
                                    0, 0, st)
    assert rc == T.TTN_EINVAL
    rc = L.ttn_leg_contract_noalloc(T.PREC_FP64, 0, 2, 2, 2, 1, buf.data_ptr(), buf.data_ptr(), 0, buf.data_ptr(),
                                    1, 0, st)
    assert rc == T.TTN_EINVAL      # sum_ops without x_per_op
