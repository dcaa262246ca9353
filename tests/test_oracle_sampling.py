"""Pins of the sampling oracle (oracle/sampling.py).

  * Every drawn configuration comes with the amplitude the sampler
    accumulated top-down; it must equal the network's own amplitude of that
    configuration (product-state overlap) -- pins the bookkeeping of the
    amplitude vectors and of the site assignment.
  * Frequencies of many shots against the exact |psi(s)|^2 of the dense state
    at maximal bond dimension (a chi-square statistic far below its failure
    threshold for the fixed seed) -- pins that the draws follow |psi|^2,
    i.e. the column mixture and the conditional states.
  * The generator: the published Philox4x32-10 known-answer vectors
    (tests/golden/philox4x32_10_kat.txt; a wrong multiplier, Weyl constant,
    round count or output permutation fails them), mean and bin counts of
    uniforms, and distinct outputs for distinct counters (Philox is a
    bijection of the counter for a fixed key).
"""
import os
import math

import numpy as np
import torch

from oracle import dense as D
from oracle import sampling as S
from oracle import ttn_oracle as O
from paper_2210_03763_amd import workload as W


def _evolved(w, n_steps):
    st, _ = O.run(w, n_steps=n_steps, record=False)
    return st


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_philox_known_answer_vectors():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(x, 16) for x in line.split()])
    assert len(rows) == 3
    for r in rows:
        out = S.philox4x32_10(np.array([r[:4]], dtype=np.uint64), (r[4], r[5]))
        assert [int(x) for x in out[0]] == r[6:], (r, out)


def test_generator_uniformity_and_bijectivity():
    u = S.uniform(12345, np.arange(200000), 7)
    assert abs(u.mean() - 0.5) < 0.003
    hist = np.histogram(u, bins=20, range=(0, 1))[0]
    chi2 = ((hist - 10000) ** 2 / 10000).sum()
    assert chi2 < 60          # 19 degrees of freedom
    ctr = np.stack([np.arange(100000, dtype=np.uint64), np.zeros(100000, np.uint64),
                    np.full(100000, 3, np.uint64), np.zeros(100000, np.uint64)], axis=1)
    out = S.philox4x32_10(ctr, (1, 2))
    assert len({tuple(r) for r in out.tolist()}) == 100000
    # different draw indices give different streams
    assert not np.allclose(S.uniform(5, np.arange(1000), 0), S.uniform(5, np.arange(1000), 1))


def test_amplitudes_are_the_network_amplitudes():
    w = W.make_ghz_program(4, 2, 3, 6, 6, 0.1, seed=31, n_layers=4, seg_per_layer=2, eps=0.05)
    st = _evolved(w, 6)
    configs, amps = S.sample(st, 40, seed=99)
    for c, a in zip(configs, amps):
        assert abs(a - S.config_amplitude(st, c)) < 1e-12


def test_frequencies_follow_the_dense_state():
    w = W.make_random_drive(2, 2, 3, 9, 8, 0.1, 3, seed=13, plus_sites=(0, 1, 2, 3), eps=0.1)
    st = _evolved(w, 8)
    psi = st.dense_state().numpy()          # site 0 slowest
    p = np.abs(psi) ** 2
    n = 20000
    configs, amps = S.sample(st, n, seed=2024)
    idx = np.zeros(n, dtype=np.int64)
    for s in range(4):
        idx = idx * 3 + configs[:, s]
    counts = np.bincount(idx, minlength=81)
    keep = p * n > 5
    chi2 = ((counts[keep] - n * p[keep]) ** 2 / (n * p[keep])).sum()
    dof = keep.sum() - 1
    # a failed sampler lands many standard deviations above dof
    assert chi2 < dof + 8 * math.sqrt(2 * dof), (chi2, dof)
    assert counts[~keep].sum() <= 5 * max(1, (~keep).sum())
    assert np.allclose(np.abs(amps) ** 2, p[idx], atol=1e-12)
