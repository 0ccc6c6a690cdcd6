"""Pins of the checker's completion with index sets redrawn at every step
(Algorithm 2 with the sampling of Section 3.1 applied to each iterate) and of
the k log k sample size of Section 3.1."""
import math

import numpy as np
import pytest

from oracle.complete import complete_resampled, sample_size
from oracle.quat import qmul, fro2
from oracle.sampling import draw, probs_length, probs_uniform


def _lowrank(m=40, n=30, k=2, p_obs=0.7, seed=5):
    rng = np.random.default_rng(seed)
    A = qmul(rng.standard_normal((4, m, k)), rng.standard_normal((4, k, n)))
    mask = (rng.random((m, n)) < p_obs).astype(np.uint8)
    Y = np.where(mask[None] == 1, A, rng.standard_normal(A.shape))  # garbage where unobserved
    return A, Y, mask


def test_sample_size_closed_form():
    # ceil(k ln k): 20 ln 20 = 59.91, 10 ln 10 = 23.03, 3 ln 3 = 3.30, 50 ln 50 = 195.6
    assert sample_size(20, 1000) == 60
    assert sample_size(10, 1000) == 24
    assert sample_size(3, 1000) == 4
    assert sample_size(50, 1000) == 196
    assert sample_size(50, 100) == 100      # at most the available count
    assert sample_size(2, 1000) == 2        # 2 ln 2 = 1.39 < k
    assert sample_size(1, 7) == 1
    for k in range(2, 300):
        s = sample_size(k, 10 ** 6)
        assert s - 1 < k * math.log(k) <= s
    with pytest.raises(ValueError):
        sample_size(0, 5)


def test_fully_observed_is_a_fixed_point():
    # P_Omega(Y) = Y: the first step restores every entry, the change is 0
    A, Y, mask = _lowrank(p_obs=1.1)
    out = complete_resampled(A, np.ones(A.shape[1:], np.uint8), 6, 6, "length", seed=9, max_iter=50, tol=1e-4)
    assert out["iters"] == 1 and out["rel"] == 0.0
    assert np.array_equal(out["X"], A)


def test_first_step_draws_from_the_observed_entries():
    A, Y, mask = _lowrank()
    X0 = np.where(mask[None] == 1, Y, 0.0)
    for sampling in ("length", "uniform"):
        out = complete_resampled(Y, mask, 7, 5, sampling, seed=123, max_iter=1, tol=0.0)
        p, q = probs_length(X0)[:2] if sampling == "length" else probs_uniform(*X0.shape[1:])
        assert np.array_equal(out["J"], draw(p, 5, 123, 0))
        assert np.array_equal(out["I"], draw(q, 7, 123, 1))


def test_observed_entries_kept_and_steps_counted():
    A, Y, mask = _lowrank(p_obs=0.5)
    out = complete_resampled(Y, mask, 6, 6, "uniform", seed=1, max_iter=5, tol=0.0)
    keep = np.broadcast_to(mask[None] == 1, Y.shape)
    assert np.array_equal(out["X"][keep], Y[keep])
    assert out["iters"] == 5


@pytest.mark.parametrize("sampling", ["length", "uniform"])
def test_converges_to_the_low_rank_matrix(sampling):
    # a rank-2 matrix with 30% of its entries missing: every step keeps the
    # observed entries and replaces the rest by a rank <= 2 reconstruction;
    # the iterates approach A
    A, Y, mask = _lowrank()
    miss = np.broadcast_to(mask[None] == 0, A.shape)
    errs = []
    for steps in (20, 300):
        out = complete_resampled(Y, mask, 8, 8, sampling, seed=3, max_iter=steps, tol=0.0)
        errs.append(np.linalg.norm((out["X"] - A)[miss]) / np.linalg.norm(A[miss]))
    assert errs[1] < 1e-6 and errs[1] < errs[0]


def test_stopping_rule():
    A, Y, mask = _lowrank()
    out = complete_resampled(Y, mask, 8, 8, "length", seed=3, max_iter=200, tol=1e-2)
    assert out["rel"] <= 1e-2 and out["iters"] < 200
