"""Single-qubit drive channels (Omega^x sigma^x + Omega^z sigma^z of
Eq. (eq:ham)) and hexagonal lattices on the HIP path, against the oracle.

GHZ programs whose Hadamards are square sigma^x/sigma^z pulses through the
TDVP (no exact gate events), on the hexagonal arrangement: FP64 against the
dense evolution at maximal chi and against the oracle at truncated chi
(1e-10), mixed against the oracle (1e-5), and the 8x8, d = 4, chi = 128
program mixed against FP64 over its first steps (1e-5).  The adjoint
gradient with respect to Omega and Delta stays exact with the qubit channels
on (1e-10 against the oracle's gradient).
"""
import sys

import numpy as np
import pytest

from oracle import dense as D
from oracle import ttn_oracle as O
from paper_2210_03763_amd import ttn as T
from paper_2210_03763_amd import workload as W
from test_gpu_parity import compare, gpu_state_as_oracle

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _hex(Lx, Ly, d, chi, steps, dt, seed, n_layers, precision=T.PREC_FP64):
    return W.make_ghz_program(Lx, Ly, d, chi, steps, dt, seed, n_layers=n_layers, seg_per_layer=2, eps=0.05,
                              precision=precision, lattice="hex", gates="pulse", gate_steps=2,
                              name=f"{Lx}x{Ly} hex pulse-gate GHZ d{d} chi{chi}")


def test_hex_pulse_maximal_chi_matches_dense():
    w = _hex(2, 2, 3, 9, 24, 0.02, 17, 3)
    _say("[qubit] 2x2 hex pulse gates, max chi")
    st = O.build(w)
    psi0 = st.dense_state().numpy()
    ref = D.run(w, psi0)
    g = T.TTN(w)
    g.step(w.n_steps)
    gs = gpu_state_as_oracle(g, st)
    err = np.abs(gs.dense_state().numpy() - ref).max()
    _say(f"[qubit] |psi - dense| = {err:.2e}")
    assert err < 1e-10
    g.close()


def test_hex_pulse_2x4_truncated_fp64():
    compare(_hex(4, 2, 3, 6, 40, 0.02, 19, 4))


def test_hex_pulse_4x4_d4_fp64():
    compare(_hex(4, 4, 4, 12, 36, 0.01, 23, 6))


def test_hex_pulse_4x4_mixed():
    res = compare(_hex(4, 4, 3, 12, 36, 0.01, 29, 6, precision=T.PREC_FP32), tol=1e-5, tolC=1e-5,
                  check_energy=False)
    assert res["dE"] < 1e-4


def test_hex_pulse_8x8_chi128_mixed_vs_fp64():
    w = W.config("hex-pulse")
    n = 4
    _say(f"[qubit] {w.name}: {n} steps mixed and FP64")
    gm = T.TTN(w)
    g64 = T.TTN(w.copy(precision=T.PREC_FP64))
    gm.step(n)
    g64.step(n)
    Fm, _ = gm.fidelity()
    F64, _ = g64.fidelity()
    C = 1 - abs(gm.overlap(g64)) ** 2
    _say(f"[qubit] F {Fm:.10f} vs {F64:.10f}, C {C:.2e}")
    assert abs(Fm - F64) < 1e-5 and C < 1e-5
    gm.close()
    g64.close()


def test_adjoint_with_qubit_channels_matches_oracle():
    w = _hex(4, 2, 3, 6, 32, 0.05, 31, 4)
    _say("[qubit] adjoint, 2x4 hex pulse gates")
    g = T.TTN(w)
    g.record(w.n_steps, 4)
    g.step(w.n_steps)
    F, _ = g.fidelity()
    go, gd = g.backward()
    g.close()
    Fo, ro, rd = O.fidelity_gradient(w)
    scale = max(1.0, np.abs(ro).max(), np.abs(rd).max())
    err = max(np.abs(go - ro).max(), np.abs(gd - rd).max())
    _say(f"[qubit] F {F:.12f} vs {Fo:.12f}; max|g| {max(np.abs(ro).max(), np.abs(rd).max()):.3e} err {err:.3e}")
    assert abs(F - Fo) < 1e-10
    assert err <= 1e-10 * scale
