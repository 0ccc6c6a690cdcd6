"""Pins of the checker's completion loop (Algorithm 2; Example 4.4)."""
import numpy as np

import workloads
from oracle.complete import complete
from oracle.quat import qmul, fro2


def _problem(m=60, n=50, k=3, p_obs=0.3, c=9, seed=11, full_cross=True):
    L, Rt, _ = workloads.lowrank_gaussian_factors(m, n, k, seed)
    A = qmul(L, Rt)
    rng = np.random.default_rng(seed)
    mask = (rng.random((m, n)) < p_obs).astype(np.uint8)
    I = np.sort(rng.choice(m, c, replace=False))
    J = np.sort(rng.choice(n, c, replace=False))
    if full_cross:
        mask[I, :] = 1
        mask[:, J] = 1
    Y = np.where(mask[None] == 1, A, rng.standard_normal(A.shape))  # garbage where unobserved
    return A, Y, mask, I, J


def test_exact_recovery_when_the_sampled_cross_is_observed():
    # With rows I and columns J fully observed and A of rank k = rank W,
    # A is a fixed point (C C^+ A R^+ R = A, Lemma 1) and the masked step
    # contracts onto it: the iterates converge to A itself.
    for p_obs, c in ((0.3, 9), (0.2, 4)):
        A, Y, mask, I, J = _problem(p_obs=p_obs, c=c)
        out = complete(Y, mask, I, J, max_iter=400, tol=1e-13)
        assert out["rel"] <= 1e-13
        assert np.sqrt(fro2(out["X"] - A) / fro2(A)) < 1e-10


def test_observed_entries_are_kept_exactly():
    A, Y, mask, I, J = _problem(full_cross=False, p_obs=0.5, c=6)
    out = complete(Y, mask, I, J, max_iter=7, tol=0.0)
    keep = mask[None] == 1
    assert np.array_equal(out["X"][np.broadcast_to(keep, Y.shape)], Y[np.broadcast_to(keep, Y.shape)])
    assert out["iters"] == 7


def test_stopping_rule():
    A, Y, mask, I, J = _problem(p_obs=0.3, c=9)
    out = complete(Y, mask, I, J, max_iter=200, tol=1e-4)
    assert out["iters"] < 200 and out["rel"] <= 1e-4
    # one step fewer has not reached the tolerance yet
    before = complete(Y, mask, I, J, max_iter=out["iters"] - 1, tol=0.0)
    assert before["rel"] > 1e-4


def test_fully_observed_matrix_stops_after_one_step():
    A, Y, mask, I, J = _problem()
    full = np.ones_like(mask)
    out = complete(A, full, I, J, max_iter=50, tol=1e-4)
    assert out["iters"] == 1 and out["rel"] == 0.0
    assert np.array_equal(out["X"], A)
