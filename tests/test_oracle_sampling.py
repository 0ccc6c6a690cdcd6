"""Pins of the checker's probabilities (QMCUR_length / QMCUR_uniform,
Section 3.1) and of its index sampler."""
import itertools
import os

import numpy as np
import pytest
from scipy import stats

from oracle.quat import chi
from oracle.sampling import (probs_length, probs_uniform, draw, splitmix64_nth, weights,
                             uniform64)


def test_splitmix64_published_vector(golden_dir):
    with open(os.path.join(golden_dir, "splitmix64_seed1234567.txt")) as f:
        ref = [int(x) for x in f if x.strip() and not x.startswith("#")]
    assert [splitmix64_nth(1234567, i) for i in range(5)] == ref


def test_length_probs_brute_force_3x3():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((4, 3, 3))
    p, q, f2 = probs_length(A)
    tot = 0.0
    col = [0.0] * 3
    row = [0.0] * 3
    for i in range(3):
        for j in range(3):
            a2 = A[0, i, j] ** 2 + A[1, i, j] ** 2 + A[2, i, j] ** 2 + A[3, i, j] ** 2
            col[j] += a2
            row[i] += a2
            tot += a2
    assert f2 == pytest.approx(tot, rel=1e-15)
    assert p == pytest.approx(np.array(col) / tot, rel=1e-14)
    assert q == pytest.approx(np.array(row) / tot, rel=1e-14)


def test_length_probs_sum_to_one_and_match_complex_adjoint():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((4, 17, 11))
    p, q, _ = probs_length(A)
    assert p.sum() == pytest.approx(1.0, abs=1e-14)
    assert q.sum() == pytest.approx(1.0, abs=1e-14)
    M = chi(A)
    coln = np.linalg.norm(M[:17, :11], axis=0) ** 2 + np.linalg.norm(M[17:, :11], axis=0) ** 2
    assert p == pytest.approx(coln / (np.linalg.norm(M) ** 2 / 2), rel=1e-12)


def test_length_probs_zero_matrix_rejected():
    with pytest.raises(ValueError):
        probs_length(np.zeros((4, 3, 3)))


def test_uniform_probs_exact():
    p, q = probs_uniform(5, 7)
    assert (p == 1.0 / 7).all() and (q == 1.0 / 5).all()
    assert weights([1.0 / 256])[0] == 2 ** 52


def test_draw_deterministic_sorted_unique():
    rng = np.random.default_rng(3)
    p = rng.random(50)
    p /= p.sum()
    a = draw(p, 20, seed=9, set_id=0)
    b = draw(p, 20, seed=9, set_id=0)
    c = draw(p, 20, seed=9, set_id=1)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)
    assert (np.diff(a) > 0).all() and a.min() >= 0 and a.max() < 50


def test_draw_never_picks_zero_weight_and_can_take_all():
    p = np.array([0.25, 0.0, 0.25, 0.0, 0.5])
    assert draw(p, 3, 1, 0).tolist() == [0, 2, 4]
    with pytest.raises(ValueError):
        draw(p, 4, 1, 0)
    with pytest.raises(ValueError):
        draw(np.array([0.5, 1.5]), 1, 1, 0)


def test_with_replacement_frequencies_chi_square():
    p = np.array([0.05, 0.1, 0.15, 0.2, 0.25, 0.125, 0.075, 0.05])
    idx = draw(p, 40000, seed=123, set_id=0, with_replacement=True)
    counts = np.bincount(idx, minlength=8)
    chi2, pval = stats.chisquare(counts, 40000 * p)
    assert pval > 1e-4, (counts, pval)


def test_without_replacement_inclusion_probabilities():
    # exact inclusion probabilities of successive draws without replacement,
    # enumerated over all ordered pairs, against 6000 seeded draws of size 2
    p = np.array([0.1, 0.2, 0.3, 0.4])
    exact = np.zeros(4)
    for a, b in itertools.permutations(range(4), 2):
        pr = p[a] * p[b] / (1 - p[a])
        exact[a] += pr
        exact[b] += pr
    assert exact.sum() == pytest.approx(2.0)
    hits = np.zeros(4)
    N = 6000
    for s in range(N):
        for j in draw(p, 2, seed=s, set_id=0):
            hits[j] += 1
    freq = hits / N
    sd = np.sqrt(exact * (1 - exact) / N)
    assert (np.abs(freq - exact) < 5 * sd).all(), (freq, exact)


def test_uniform_draw_target_in_range():
    # tau = floor(u * T / 2^64) always lies in [0, T)
    for t in range(200):
        u = uniform64(77, 3, t)
        T = 2 ** 60 - 12345
        tau = (u * T) >> 64
        assert 0 <= tau < T


def test_golden_draws_reproduce(golden_dir):
    import json
    with open(os.path.join(golden_dir, "draws.json")) as f:
        cases = json.load(f)
    assert len(cases) >= 6
    for c in cases:
        p = np.array([float.fromhex(x) for x in c["p"]])
        idx = draw(p, c["count"], c["seed"], c["set_id"], c["with_replacement"])
        assert idx.tolist() == c["idx"], c["name"]
