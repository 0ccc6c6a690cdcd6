"""Pins of the checker's Theorem 1 experiment (Section 3.2, Example 4.1):
polar factors and spectral norms through a second embedding (the real
representation instead of the complex adjoint), the singular values of the
constructed low-rank matrix, Theorem 1's bound, exact recovery without noise
and first-order linearity in the noise."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle.perturbation import lowrank_product, perturbation_errors, polar_factor
from oracle.pinv import singular_values
from oracle.quat import qH, qmul, real_rep, spectral_norm, unstack


def _polar_real_rep(G):
    # the real representation is a *-homomorphism too, so its polar factor
    # is the representation of the quaternion polar factor
    _, p, q = G.shape
    U, _, Vt = np.linalg.svd(real_rep(G), full_matrices=False)
    return unstack((U @ Vt)[:, :q])


def test_polar_factor_definition_and_second_embedding():
    rng = np.random.default_rng(5)
    G = rng.standard_normal((4, 23, 6))
    Q = polar_factor(G)
    assert np.abs(real_rep(qmul(qH(Q), Q)) - np.eye(24)).max() < 1e-13
    H = real_rep(qmul(qH(Q), G))  # Q^H G = (G^H G)^{1/2}: symmetric positive definite
    assert np.abs(H - H.T).max() < 1e-12
    assert np.linalg.eigvalsh(0.5 * (H + H.T)).min() > 0
    assert np.abs(Q - _polar_real_rep(G)).max() < 1e-12


def test_polar_factor_of_a_real_matrix_is_the_real_one():
    rng = np.random.default_rng(6)
    G = np.zeros((4, 9, 4))
    G[0] = rng.standard_normal((9, 4))
    U, _, Vt = np.linalg.svd(G[0], full_matrices=False)
    Q = polar_factor(G)
    assert np.abs(Q[0] - U @ Vt).max() < 1e-13 and np.abs(Q[1:]).max() < 1e-13


def test_spectral_norm_through_the_real_representation():
    rng = np.random.default_rng(7)
    for p, q in ((11, 7), (5, 13)):
        A = rng.standard_normal((4, p, q))
        assert spectral_norm(A) == pytest.approx(np.linalg.norm(real_rep(A), 2), rel=1e-13)


def test_lowrank_product_has_the_prescribed_singular_values():
    GW, GV, sig, _ = wl.perturbation_factors(30, 26, 5, seed=2)
    X = lowrank_product(polar_factor(GW), sig, polar_factor(GV))
    s = singular_values(X)
    assert np.allclose(s[:5], sig, rtol=1e-13, atol=0)
    assert s[5:].max() < 1e-13 * sig[0]


def _setup(m=40, n=36, k=4, seed=3):
    GW, GV, sig, E0 = wl.perturbation_factors(m, n, k, seed)
    W, V = polar_factor(GW), polar_factor(GV)
    X = lowrank_product(W, sig, V)
    c = r = max(k, math.ceil(k * math.log(k)))
    return X, W, V, E0, c, r


@pytest.mark.parametrize("sampling", ["length", "uniform"])
def test_theorem1_bound_holds(sampling):
    X, W, V, E0, c, r = _setup()
    for sigma in (1e-1, 1e-2, 1e-4, 1e-6):
        out = perturbation_errors(X, sigma * E0, W, V, c, r, sampling, seed=4)
        assert np.isfinite(out["bound"])
        assert out["err"] <= out["bound"]
        assert out["norm_E"] == pytest.approx(sigma * spectral_norm(E0), rel=1e-12)


def test_noiseless_matrix_is_recovered():
    X, W, V, E0, c, r = _setup()
    out = perturbation_errors(X, 0.0 * E0, W, V, c, r, "length", seed=4)
    assert out["norm_E"] == 0.0 and out["err"] < 1e-12 * spectral_norm(X)


def test_error_is_linear_in_the_noise_for_small_noise():
    # first-order perturbation: err = ||L(E)||_2 + O(||E||^2) for a linear L
    # fixed by the index sets, so err / ||E|| settles to a constant
    X, W, V, E0, c, r = _setup()
    a = perturbation_errors(X, 1e-4 * E0, W, V, c, r, "length", seed=4)
    b = perturbation_errors(X, 1e-6 * E0, W, V, c, r, "length", seed=4)
    assert np.array_equal(a["I"], b["I"]) and np.array_equal(a["J"], b["J"])
    assert a["err"] / a["norm_E"] == pytest.approx(b["err"] / b["norm_E"], rel=1e-3)
