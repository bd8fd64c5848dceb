"""Pins of the simplification passes of the CPU reference (no GPU)."""
from __future__ import annotations

import itertools

import numpy as np


def _sequential_inclusion(w, k):
    """Exact inclusion probabilities of drawing k items one at a time without
    replacement, each draw with probability proportional to w among the rest."""
    n = len(w)
    p = np.zeros(n)
    for seq in itertools.permutations(range(n), k):
        prob, rest = 1.0, float(sum(w))
        for i in seq:
            prob *= w[i] / rest
            rest -= w[i]
        for i in seq:
            p[i] += prob
    return p


def test_race_sampling_matches_sequential_definition(oracle):
    rng = np.random.default_rng(0)
    w = np.array([1.0, 2.0, 3.0, 4.0, 0.5])
    k = 2
    exact = _sequential_inclusion(w, k)
    trials = 200_000
    u = 1.0 - rng.random((trials, w.size))  # (0, 1]
    e = -np.log(u) / w
    kept = np.argsort(e, axis=1, kind="stable")[:, :k]
    freq = np.bincount(kept.reshape(-1), minlength=w.size) / trials
    np.testing.assert_allclose(freq, exact, atol=4e-3)
    # the oracle's selection equals the k smallest race times per trial
    for t in range(20):
        m = oracle.sample_keep(w, u[t], k)
        assert set(np.nonzero(m)[0]) == set(kept[t].tolist())


def test_sample_keep_special_cases(oracle):
    rng = np.random.default_rng(1)
    u = 1.0 - rng.random(100)
    # equal scores: the kept set is the n_keep largest uniforms
    m = oracle.sample_keep(np.ones(100), u, 30)
    assert set(np.nonzero(m)[0]) == set(np.argsort(-u, kind="stable")[:30].tolist())
    # zero scores are drawn last, by index
    s = np.where(np.arange(100) < 10, 0.0, 1.0)
    m = oracle.sample_keep(s, u, 95)
    assert m[10:].all() and m[:5].all() and not m[5:10].any()
    assert oracle.sample_keep(s, u, 0).sum() == 0


def test_mass_keep_is_the_cumulative_cut(oracle):
    s = np.array([0.0, 5.0, 1.0, 3.0, 1.0])   # total 10, 99% = 9.9
    # order 5, 3, 1 (idx 2), 1 (idx 4): prefix sums 5, 8, 9, 10 -> four kept
    assert oracle.mass_keep(s, 0.99).tolist() == [False, True, True, True, True]
    assert oracle.mass_keep(s, 0.5).tolist() == [False, True, False, False, False]


def test_compact_keeps_order(oracle):
    a = np.arange(30, dtype=np.float32).reshape(3, 10)
    b = np.arange(10, dtype=np.uint8)
    keep = np.arange(10) % 3 == 1
    ca, cb = oracle.compact([a, b], keep)
    np.testing.assert_array_equal(ca, a[:, [1, 4, 7]])
    np.testing.assert_array_equal(cb, [1, 4, 7])
