"""The adjoint (reverse-mode) gradient of the GHZ fidelity with respect to
the pulse table, through the C ABI, against the oracle's gradient.

FP64 path: max |g_gpu - g_oracle| <= 1e-10 max(1, |g_oracle|_inf) on small
programs (truncated and maximal chi, d = 3 and 4, gate events inside and at
the end of the recording).  At the 8x8, d = 3, chi = 64 size the oracle
gradient is out of reach, so the gradient is checked against central
differences of the device forward map (relative 1e-6) on sampled entries.
"""
import sys

import numpy as np
import pytest

from oracle import dense as D
from oracle import ttn_oracle as O
from paper_2210_03763_amd import ttn as T
from paper_2210_03763_amd import workload as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _gpu_grad(w, ckpt_every=4):
    g = T.TTN(w)
    g.record(w.n_steps, ckpt_every)
    g.step(w.n_steps)
    F, _ = g.fidelity()
    go, gd = g.backward()
    F2, _ = g.fidelity()
    g.close()
    return F, F2, go, gd


def _compare(w, go, gd, ro, rd, tol=1e-10):
    scale = max(1.0, np.abs(ro).max(), np.abs(rd).max())
    err = max(np.abs(go - ro).max(), np.abs(gd - rd).max())
    _say(f"[adjoint] {w.name}: max|g| {max(np.abs(ro).max(), np.abs(rd).max()):.3e} err {err:.3e}")
    assert err <= tol * scale, err


def test_adjoint_matches_oracle_gradient_2x4_truncated():
    w = W.make_ghz_program(4, 2, 3, 6, 16, 0.1, seed=31, n_layers=4, seg_per_layer=2, eps=0.05)
    _say("[adjoint] 2x4 d3 chi6")
    F, F2, go, gd = _gpu_grad(w)
    Fo, ro, rd = O.fidelity_gradient(w)
    assert abs(F - Fo) < 1e-10 and F2 == F
    _compare(w, go, gd, ro, rd)


def test_adjoint_matches_dense_gradient_2x2_d4_maximal_chi():
    w = W.make_ghz_program(2, 2, 4, 16, 12, 0.1, seed=41, n_layers=3, seg_per_layer=2, eps=0.05)
    _say("[adjoint] 2x2 d4 chi16")
    F, _, go, gd = _gpu_grad(w, ckpt_every=5)
    psi0 = O.build(w).dense_state().numpy()
    Fd, ro, rd = D.fidelity_gradient(w, psi0)
    assert abs(F - Fd) < 1e-10
    _compare(w, go, gd, ro, rd)


def test_adjoint_matches_oracle_gradient_4x4():
    w = W.make_ghz_program(4, 4, 3, 12, 12, 0.1, seed=33, n_layers=6, seg_per_layer=2, eps=0.05)
    _say("[adjoint] 4x4 d3 chi12")
    F, _, go, gd = _gpu_grad(w, ckpt_every=3)
    Fo, ro, rd = O.fidelity_gradient(w)
    assert abs(F - Fo) < 1e-10
    _compare(w, go, gd, ro, rd)


def test_checkpoint_interval_does_not_change_the_gradient():
    w = W.make_ghz_program(4, 2, 3, 6, 10, 0.1, seed=35, n_layers=4, seg_per_layer=2, eps=0.05)
    res = [_gpu_grad(w, ckpt_every=k)[2:] for k in (1, 3, 10)]
    for go, gd in res[1:]:
        assert np.abs(go - res[0][0]).max() <= 1e-14 and np.abs(gd - res[0][1]).max() <= 1e-14


def test_backward_error_paths():
    w = W.make_ghz_program(4, 2, 3, 6, 6, 0.1, seed=35, n_layers=4, seg_per_layer=2, eps=0.05)
    g = T.TTN(w)
    with pytest.raises(T.TTNError) as e:
        g.backward()
    assert e.value.code == T.TTN_ESTATE
    import ctypes as C
    import torch
    buf = torch.empty(1024, dtype=torch.uint8, device="cuda")
    rc = T.lib().ttn_record_begin(g.h, 4, 2, C.c_void_p(buf.data_ptr()), 1024)
    assert rc == T.TTN_ENOMEM
    g.record(2, 1)
    g.step(3)                     # one step more than recorded
    with pytest.raises(T.TTNError) as e:
        g.backward()
    assert e.value.code == T.TTN_ESTATE
    g.close()


def test_adjoint_8x8_chi64_against_central_differences():
    # every site driven on 8 global segments (1024 pulse parameters); the
    # target is the GHZ state of the atoms made bright by the gates at step 0,
    # so that F is of order one (the gradient grows as the square of the time)
    w = W.config("c4").copy(n_steps=10)
    bright = sorted({s for (k, s, _) in w.events if k == 0})
    _say(f"[adjoint] 8x8 d3 chi64, 10 steps, target {bright}")
    g = T.TTN(w)
    g.record(w.n_steps, 4)
    g.step(w.n_steps)
    F, _ = g.fidelity(bright)
    go, gd = g.backward(bright)
    g.close()
    scale = max(np.abs(go).max(), np.abs(gd).max())
    _say(f"[adjoint] F {F:.6f} max|g| {scale:.3e}")
    assert scale > 1e-5
    seg = 0
    h = 1e-4
    for i in bright[:3]:
        for arr, grad in ((w.omega, go), (w.delta, gd)):
            base = arr[i, seg]
            Fs = []
            for x in (base + h, base - h):
                arr[i, seg] = x
                gg = T.TTN(w)
                gg.step(w.n_steps)
                Fs.append(gg.fidelity(bright)[0])
                gg.close()
            arr[i, seg] = base
            fd = (Fs[0] - Fs[1]) / (2 * h)
            _say(f"[adjoint] site {i}: adjoint {grad[i, seg]:.10e} fd {fd:.10e}")
            assert abs(fd - grad[i, seg]) <= 1e-6 * scale


def test_mixed_precision_adjoint_matches_oracle_4x4():
    # mixed mode: the taped re-run and the environment-adjoint contractions run
    # in complex FP32; the gradient must stay within the mixed tolerance
    w = W.make_ghz_program(4, 4, 3, 12, 12, 0.1, seed=33, n_layers=6, seg_per_layer=2, eps=0.05,
                           precision=T.PREC_FP32)
    _say("[adjoint] 4x4 d3 chi12 mixed")
    F, _, go, gd = _gpu_grad(w, ckpt_every=3)
    Fo, ro, rd = O.fidelity_gradient(w.copy(precision=T.PREC_FP64))
    assert abs(F - Fo) < 1e-5
    _compare(w, go, gd, ro, rd, tol=1e-5)


def test_mixed_precision_adjoint_matches_fp64_8x8_chi64():
    w = W.config("c4").copy(n_steps=4, precision=T.PREC_FP32)
    bright = sorted({s for (k, s, _) in w.events if k == 0})
    res = {}
    for prec in (T.PREC_FP32, T.PREC_FP64):
        g = T.TTN(w.copy(precision=prec))
        g.record(w.n_steps, 2)
        g.step(w.n_steps)
        F, _ = g.fidelity(bright)
        res[prec] = (F,) + g.backward(bright)
        g.close()
    (Fm, gom, gdm), (F64, go64, gd64) = res[T.PREC_FP32], res[T.PREC_FP64]
    scale = max(np.abs(go64).max(), np.abs(gd64).max())
    err = max(np.abs(gom - go64).max(), np.abs(gdm - gd64).max())
    _say(f"[adjoint] 8x8 chi64 mixed vs FP64: |dF| {abs(Fm - F64):.2e}, max|g| {scale:.3e}, err {err:.3e}")
    assert scale > 1e-6
    assert abs(Fm - F64) < 1e-5 and err <= 1e-5 * scale


def test_autograd_function_matches_oracle_gradient():
    # the torch.autograd.Function front end: F(Omega, Delta) on tensors, an
    # upstream factor of 2 through a loss, against the oracle's gradient
    import torch
    w = W.make_ghz_program(4, 2, 3, 6, 16, 0.1, seed=31, n_layers=4, seg_per_layer=2, eps=0.05)
    om = torch.tensor(w.omega, dtype=torch.float64, device="cuda", requires_grad=True)
    de = torch.tensor(w.delta, dtype=torch.float64, device="cuda", requires_grad=True)
    F = T.ttn_fidelity(om, de, w, ckpt_every=4)
    (2.0 * F).backward()
    Fo, ro, rd = O.fidelity_gradient(w)
    _say(f"[adjoint] autograd: F {float(F):.12f} vs {Fo:.12f}")
    assert abs(float(F) - Fo) < 1e-10
    _compare(w, om.grad.cpu().numpy(), de.grad.cpu().numpy(), 2 * ro, 2 * rd)


@pytest.mark.parametrize("precision", [T.PREC_FP64, T.PREC_FP32])
def test_backward_graph_replays_match_eager(precision):
    """The backward pass replays one captured graph for every recorded step
    after the first (the tape restarts at the same offsets each step); the
    gradient must equal that of the eagerly launched backward pass.  Twelve
    recorded steps with a checkpoint every three: the graph is replayed
    eleven times, with the pulse-gradient read-back, the gate events and the
    forward re-runs from the checkpoints in between."""
    w = W.make_ghz_program(4, 4, 3, 12, 12, 0.1, seed=33, n_layers=6, seg_per_layer=2, eps=0.05,
                           precision=precision)
    out = []
    for graphs in (True, False):
        g = T.TTN(w)
        g.set_graphs(graphs)
        g.record(w.n_steps, 3)
        g.step(w.n_steps)
        out.append(g.backward())
        g.close()
    (go1, gd1), (go0, gd0) = out
    scale = max(1.0, np.abs(go0).max(), np.abs(gd0).max())
    err = max(np.abs(go1 - go0).max(), np.abs(gd1 - gd0).max()) / scale
    _say(f"[adjoint] graph vs eager backward (precision {precision}): max|g| {scale:.3e}, err {err:.3e}")
    assert np.abs(go0).max() > 0
    assert err <= 1e-13
