"""Open-system mode (Eq. (eq:hoqs): -i gamma |r><r| on every site) of the
HIP path against the CPU oracle, through the C ABI.

The state is not normalised: its squared norm is the no-decay probability.
Per step the device's norm, energy (real part) and total Rydberg population
sum_i <psi|n_i|psi> must match the oracle; the final state must match it in
the normalised infidelity C = 1 - |<a|b>|^2 / (<a|a><b|b>) and in norm.
FP64: 1e-10.  Mixed (complex FP32 contractions): 1e-5 in C, norm and the
GHZ fidelity, the tolerance of the closed system.
"""
import math
import sys

import numpy as np
import pytest

from oracle import dense as D
from oracle import ttn_oracle as O
from paper_2210_03763_amd import ttn as T
from paper_2210_03763_amd import workload as W
from test_gpu_parity import gpu_state_as_oracle

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _open(Lx, Ly, d, chi, steps, dt, gamma, seed, precision=T.PREC_FP64, eps=0.05):
    w = W.make_random_drive(Lx, Ly, d, chi, steps, dt, 4, seed, plus_sites=tuple(range(Lx * Ly)), eps=eps,
                            precision=precision)
    return w.copy(gamma=gamma)


def _compare(w, tol):
    _say(f"[open] N={w.n_sites} d={w.d} chi={w.chi} gamma={w.gamma} steps={w.n_steps} prec={w.precision}")
    st, recs = O.run(w)
    g = T.TTN(w)
    pops = []
    for n in range(w.n_steps):
        s = g.step(1, stats=True)[0]
        pops.append(g.rydberg_population())
        assert abs(s["norm2"] - recs[n]["norm2"]) < tol, (n, s["norm2"], recs[n]["norm2"])
        assert abs(s["energy"] - recs[n]["energy"]) < tol * max(1.0, abs(recs[n]["energy"]))
        assert abs(pops[-1] - recs[n]["rydberg_population"]) < tol
    gs = gpu_state_as_oracle(g, st)
    ab = O.ttn_overlap(st, gs)
    C = 1 - abs(ab) ** 2 / (st.norm2() * O.ttn_overlap(gs, gs).real)
    Fg, _ = g.fidelity()
    Fo, _ = st.ghz_fidelity(w.target_sites)
    _say(f"[open] norm {recs[-1]['norm2']:.6f} C {C:.2e} dF {abs(Fg - Fo):.2e}")
    assert recs[-1]["norm2"] < 0.999        # the decay is visible
    assert C < tol and abs(Fg - Fo) < tol
    g.close()
    return recs


def test_open_maximal_chi_fp64_equals_dense():
    w = _open(2, 2, 3, 9, 12, 0.05, 0.3, seed=41)
    psi0 = O.build(w).dense_state().numpy()
    ref = D.run(w, psi0)
    g = T.TTN(w)
    g.step(w.n_steps)
    gs = gpu_state_as_oracle(g, O.build(w))
    psi = gs.dense_state().numpy()
    _say(f"[open] 2x2 max chi: |psi - dense| = {np.abs(psi - ref).max():.2e}, norm {np.vdot(ref, ref).real:.6f}")
    assert np.abs(psi - ref).max() < 1e-10
    g.close()


def test_open_truncated_fp64_vs_oracle():
    _compare(_open(4, 2, 3, 6, 10, 0.04, 0.25, seed=43), 1e-10)


def test_open_truncated_d4_fp64_vs_oracle():
    _compare(_open(2, 2, 4, 7, 8, 0.05, 0.2, seed=44), 1e-10)


def test_open_truncated_mixed_vs_oracle():
    _compare(_open(4, 4, 3, 12, 6, 0.04, 0.25, seed=45, precision=T.PREC_FP32), 1e-5)


def test_open_8x8_chi128_mixed_vs_fp64():
    # the 8x8, d = 4, chi = 128 GHZ program with decay: the mixed bar (1e-5)
    w = W.config("c3").copy(gamma=0.05)
    gm = T.TTN(w)
    g64 = T.TTN(w.copy(precision=T.PREC_FP64))
    for n in range(4):
        sm = gm.step(1, stats=True)[0]
        s64 = g64.step(1, stats=True)[0]
        _say(f"[open] c3 step {n}: norm {sm['norm2']:.12f} (fp64 {s64['norm2']:.12f})")
        assert abs(sm["norm2"] - s64["norm2"]) < 1e-5
    ab = gm.overlap(g64)
    C = 1 - abs(ab) ** 2 / (sm["norm2"] * s64["norm2"])
    Fm, _ = gm.fidelity()
    F64, _ = g64.fidelity()
    pm, p64 = gm.rydberg_population(), g64.rydberg_population()
    _say(f"[open] c3 mixed vs fp64: C {C:.2e} dF {abs(Fm - F64):.2e} dP_R {abs(pm - p64):.2e}")
    assert C < 1e-5 and abs(Fm - F64) < 1e-5 and abs(pm - p64) < 1e-5 * max(1.0, p64)
    # the adjoint is for closed systems only
    with pytest.raises(T.TTNError) as e:
        gm.record(1, 1)
    assert e.value.code == T.TTN_EINVAL
    gm.close()
    g64.close()


@pytest.mark.parametrize("prec", [T.PREC_FP64, T.PREC_FP32])
def test_open_8x8_chi128_norm_law(prec):
    # every atom driven, starting from (|1> + |r>)/sqrt 2 on every site, so
    # that the decay is visible within a few steps: ||psi||^2 = 1 - 2 gamma T_R
    # (trapezoid T_R, second-order residual)
    w = W.make_random_drive(8, 8, 4, 128, 3, 0.005, 1, seed=46, plus_sites=(), eps=1e-2, precision=prec)
    r_plus = np.zeros(4, complex)
    r_plus[1] = r_plus[2] = 1 / math.sqrt(2)
    w = w.copy(gamma=0.05, init_product=np.tile(r_plus, (64, 1)))
    g = T.TTN(w)
    pops, norms = [g.rydberg_population()], [1.0]
    for n in range(3):
        s = g.step(1, stats=True)[0]
        pops.append(g.rydberg_population())
        norms.append(s["norm2"])
        _say(f"[open] 8x8 driven, prec {prec}, step {n}: norm {s['norm2']:.10f} pop {pops[-1]:.6f}")
        assert s["norm2"] < norms[-2] + 1e-12
    TR = w.dt * (sum(pops) - 0.5 * (pops[0] + pops[-1]))
    loss = 1 - norms[-1]
    _say(f"[open] loss {loss:.4e} vs 2 gamma T_R {2 * w.gamma * TR:.4e}")
    assert loss > 0 and abs(loss - 2 * w.gamma * TR) < 1e-2 * loss
    g.close()
