"""The C-ABI library loads and exports every symbol include/ttn.h declares;
host-side validation paths (no device work) behave as documented."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2210_03763_amd import ttn as T
from paper_2210_03763_amd import workload as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ttn.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|int64_t|const char\*)\s+(ttn_\w+)\s*\(", src, re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("ttn_init", "ttn_set_pulses", "ttn_tdvp_step", "ttn_fidelity", "ttn_backward",
              "ttn_adjoint_query", "ttn_record_begin"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(T.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n


def test_workspace_query_sizes():
    w = W.config("c1-ent")
    b = T.workspace_bytes(w)
    assert 1 << 20 < b < 1 << 31
    w3 = W.make_ghz_program(8, 8, 4, 128, 1, 0.005, seed=1, eps=0.0, precision=T.PREC_FP32)
    b3 = T.workspace_bytes(w3)
    # node tensors of the 8x8 d=4 chi=128 network alone are ~0.5 GB in FP64
    assert b3 > 5e8


@pytest.mark.parametrize("field,value", [("n_sites", 12), ("d", 5), ("chi", 0), ("krylov_dim", 17),
                                         ("precision", 7), ("gamma", -0.1), ("gamma", float("nan"))])
def test_invalid_config_rejected(field, value):
    w = W.config("c1-ent")
    keep = []
    cfg = T.make_config(w, keep)
    setattr(cfg, field, value)
    out = C.c_size_t(0)
    assert T.lib().ttn_workspace_query(C.byref(cfg), C.byref(out)) == T.TTN_EINVAL


def test_non_permutation_leaf_order_rejected():
    w = W.config("c1-ent")
    w = w.copy(leaf_order=np.zeros(16, np.int32))
    with pytest.raises(T.TTNError) as e:
        T.workspace_bytes(w)
    assert e.value.code == T.TTN_EINVAL


def test_null_handle_calls():
    L = T.lib()
    assert L.ttn_tdvp_step(None, 0.01, 1, None) == T.TTN_EINVAL
    assert L.ttn_destroy(None) == T.TTN_EINVAL
    assert L.ttn_backward(None, 0, None, 1.0, None, None) == T.TTN_EINVAL
    assert L.ttn_record_begin(None, 1, 1, None, 0) == T.TTN_EINVAL
    assert L.ttn_rydberg_population(None, None) == T.TTN_EINVAL
    assert L.ttn_set_qubit_pulses(None, None, None) == T.TTN_EINVAL


def _validate(w, n_steps=1):
    keep = []
    cfg = T.make_config(w, keep)
    msg = C.create_string_buffer(512)
    L = T.lib()
    L.ttn_validate_plan.restype = C.c_int
    L.ttn_validate_plan.argtypes = [C.POINTER(T.Config), C.c_int32, C.c_char_p, C.c_int32]
    rc = L.ttn_validate_plan(C.byref(cfg), n_steps, msg, 512)
    return rc, msg.value.decode()


@pytest.mark.parametrize("case", [
    ("2x1 d3 chi9", lambda: W.make_random_drive(2, 1, 3, 9, 1, 0.01, 1, seed=1)),
    ("2x2 d3 chi9", lambda: W.make_random_drive(2, 2, 3, 9, 1, 0.01, 1, seed=1)),
    ("2x2 d4 chi16", lambda: W.make_random_drive(2, 2, 4, 16, 1, 0.01, 1, seed=1)),
    ("2x4 d3 chi5", lambda: W.make_random_drive(4, 2, 3, 5, 1, 0.01, 1, seed=1)),
    ("2x4 d3 chi81", lambda: W.make_random_drive(4, 2, 3, 81, 1, 0.01, 1, seed=1)),
    ("4x4 d3 chi16", lambda: W.make_random_drive(4, 4, 3, 16, 1, 0.01, 1, seed=1)),
    ("4x4 d4 chi12 fp32", lambda: W.make_random_drive(4, 4, 4, 12, 1, 0.01, 1, seed=1, precision=1)),
    ("8x8 d3 chi64", lambda: W.make_ghz_program(8, 8, 3, 64, 1, 0.005, seed=1, eps=0.0)),
    ("8x8 d4 chi128 fp32", lambda: W.make_ghz_program(8, 8, 4, 128, 1, 0.005, seed=1, eps=0.0,
                                                     precision=1)),
    ("8x8 d4 chi128 fp64", lambda: W.make_ghz_program(8, 8, 4, 128, 1, 0.005, seed=1, eps=0.0)),
    ("2x1 d3 chi9 open", lambda: W.make_random_drive(2, 1, 3, 9, 1, 0.01, 1, seed=1).copy(gamma=0.1)),
    ("4x4 d4 chi12 fp32 open", lambda: W.make_random_drive(4, 4, 4, 12, 1, 0.01, 1, seed=1,
                                                           precision=1).copy(gamma=0.1)),
    ("2x4 hex d3 chi8 pulse gates", lambda: W.make_ghz_program(4, 2, 3, 8, 40, 0.02, 5, n_layers=4, seg_per_layer=2,
                                                               lattice="hex", gates="pulse")),
    ("8x8 d4 chi128 fp32 open", lambda: W.make_ghz_program(8, 8, 4, 128, 1, 0.005, seed=1, eps=0.0,
                                                          precision=1).copy(gamma=0.02)),
    ("2x2 d3 chi9 two-site", lambda: W.make_random_drive(2, 2, 3, 9, 1, 0.01, 1, seed=1).copy(update=1)),
    ("2x4 d3 chi81 two-site", lambda: W.make_random_drive(4, 2, 3, 81, 1, 0.01, 1, seed=1).copy(update=1)),
    ("4x4 d3 chi16 two-site", lambda: W.make_random_drive(4, 4, 3, 16, 1, 0.01, 1, seed=1).copy(update=1)),
    ("4x4 d4 chi16 two-site", lambda: W.make_random_drive(4, 4, 4, 16, 1, 0.01, 1, seed=1).copy(update=1)),
    ("8x8 d3 chi12 two-site", lambda: W.make_ghz_program(8, 8, 3, 12, 1, 0.005, seed=1, eps=0.0).copy(update=1)),
    ("8x8 d4 chi16 two-site", lambda: W.make_ghz_program(8, 8, 4, 16, 1, 0.005, seed=1, eps=0.0).copy(update=1)),
])
def test_launch_plan_stays_in_bounds(case):
    """Every GEMM operand and vector launch of init + steps + observables stays
    inside its workspace allocation (checked on the host, no device)."""
    name, mk = case
    rc, msg = _validate(mk(), 2)
    assert rc == T.TTN_OK, (name, msg)


def test_adjoint_query_sizes():
    from paper_2210_03763_amd import workload as W
    keep = []
    w = W.config("c1-ent")
    cfg = T.make_config(w, keep)
    import ctypes as C
    out = [C.c_size_t(0) for _ in range(3)]
    L = T.lib()
    assert L.ttn_adjoint_query(C.byref(cfg), 20, 10, C.byref(out[0])) == T.TTN_OK
    assert L.ttn_adjoint_query(C.byref(cfg), 20, 1, C.byref(out[1])) == T.TTN_OK
    assert L.ttn_adjoint_query(C.byref(cfg), 40, 10, C.byref(out[2])) == T.TTN_OK
    state = sum(16 * a * b * c for (a, b, c) in [(3, 3, 9)] * 8 + [(9, 9, 16)] * 4 + [(16, 16, 16)] * 2
                + [(16, 16, 1)])
    state = (state + 255) // 256 * 256     # every buffer is 256-byte aligned
    # 20 checkpoints + 1 slot vs 2 checkpoints + 10 slots: 9 states apart
    assert out[1].value - out[0].value == 9 * state
    assert out[2].value - out[0].value == 2 * state
    assert L.ttn_adjoint_query(C.byref(cfg), 20, 0, C.byref(out[0])) == T.TTN_EINVAL



@pytest.mark.parametrize("case,code", [
    ("two-site mixed precision", T.TTN_ENOTSUP),
    ("two-site open system", T.TTN_ENOTSUP),
    ("two-site split above 256", T.TTN_ENOTSUP),
    ("unknown update", T.TTN_EINVAL),
])
def test_two_site_limits(case, code):
    w = W.make_random_drive(4, 4, 3, 16, 1, 0.01, 1, seed=1).copy(update=1)
    if case == "two-site mixed precision":
        w = w.copy(precision=T.PREC_FP32)
    elif case == "two-site open system":
        w = w.copy(gamma=0.1)
    elif case == "two-site split above 256":
        w = W.make_random_drive(8, 8, 3, 32, 1, 0.01, 1, seed=1).copy(update=1)   # 32^2 x 32^2 splits
    else:
        w = w.copy(update=2)
    with pytest.raises(T.TTNError) as e:
        T.workspace_bytes(w)
    assert e.value.code == code, case
