"""Projective-measurement sampling on the device (ttn_sample) against the
sampling oracle.

Both sides draw with the same Philox4x32-10 stream (counter = shot, draw
index), so the same seed must give the same configurations; the device's
amplitude of every drawn configuration must equal the network's amplitude
(1e-12), and frequencies must follow |psi|^2 (chi-square against the dense
state at maximal chi; binomial bounds on the dominant configurations of the
8x8, d=4, chi=128 network).
"""
import math
import sys

import numpy as np
import pytest

from oracle import dense as D
from oracle import sampling as S
from oracle import ttn_oracle as O
from paper_2210_03763_amd import ttn as T
from paper_2210_03763_amd import workload as W
from test_gpu_parity import gpu_state_as_oracle

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_shots_equal_the_oracle_sampler_2x4():
    w = W.make_ghz_program(4, 2, 3, 6, 6, 0.1, seed=31, n_layers=4, seg_per_layer=2, eps=0.05)
    g = T.TTN(w)
    g.step(6)
    st = gpu_state_as_oracle(g, O.build(w))
    n, seed = 300, 777
    cfg_g, amp_g = g.sample(n, seed)
    cfg_o, amp_o = S.sample(st, n, seed)
    same = (cfg_g == cfg_o).all(axis=1)
    _say(f"[sample] 2x4: {same.sum()} of {n} shots identical")
    assert same.mean() >= 0.99
    assert np.abs(amp_g[same] - amp_o[same]).max() < 1e-12
    for c, a in zip(cfg_g[:60], amp_g[:60]):
        assert abs(a - S.config_amplitude(st, c)) < 1e-12
    # a split run (shot0) continues the same stream
    cfg_2, _ = g.sample(100, seed, shot0=200)
    assert (cfg_2 == cfg_g[200:300]).all()
    g.close()


def test_frequencies_follow_the_dense_state_2x2():
    w = W.make_random_drive(2, 2, 3, 9, 8, 0.1, 3, seed=13, plus_sites=(0, 1, 2, 3), eps=0.1)
    psi0 = O.build(w).dense_state().numpy()
    psi = D.run(w, psi0)
    p = np.abs(psi) ** 2
    g = T.TTN(w)
    g.step(w.n_steps)
    n = 200000
    cfg, amp = g.sample(n, 4242)
    idx = np.zeros(n, dtype=np.int64)
    for s in range(4):
        idx = idx * 3 + cfg[:, s]
    counts = np.bincount(idx, minlength=81)
    keep = p * n > 5
    chi2 = ((counts[keep] - n * p[keep]) ** 2 / (n * p[keep])).sum()
    dof = int(keep.sum()) - 1
    _say(f"[sample] 2x2 chi2 {chi2:.1f} dof {dof}")
    assert chi2 < dof + 8 * math.sqrt(2 * dof)
    assert np.allclose(np.abs(amp) ** 2, p[idx], atol=1e-10)
    g.close()


def test_8x8_chi128_shots_and_frequencies():
    w = W.config("c3")
    g = T.TTN(w)
    g.step(2)
    n = 50000
    _say("[sample] 8x8 chi128: 50000 shots")
    cfg, amp = g.sample(n, 2210)
    st = gpu_state_as_oracle(g, O.build(w.copy(precision=T.PREC_FP64)))
    # the first shots bit for bit against the oracle sampler (same stream)
    cfg_o, amp_o = S.sample(st, 8, 2210)
    assert (cfg_o == cfg[:8]).all()
    assert np.abs(amp_o - amp[:8]).max() < 1e-10
    # amplitudes of drawn configurations are the network's amplitudes
    for c, a in zip(cfg[:16], amp[:16]):
        assert abs(a - S.config_amplitude(st, c)) < 1e-10
    # frequencies of the configurations expected at least 100 times, within 6 sigma
    keys, inv, counts = np.unique(cfg, axis=0, return_inverse=True, return_counts=True)
    checked = 0
    for t in np.argsort(-counts)[:8]:
        pt = abs(amp[np.flatnonzero(inv.reshape(-1) == t)[0]]) ** 2
        if n * pt < 100:
            continue
        sig = math.sqrt(n * pt * (1 - pt))
        _say(f"[sample] count {counts[t]} expected {n * pt:.1f}")
        assert abs(counts[t] - n * pt) <= 6 * sig
        checked += 1
    assert checked >= 2
    g.close()
