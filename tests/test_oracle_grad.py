"""Pins of the checker's derivatives: central finite differences in FP64
(h = 1e-6), the pinv adjoint against a finite-difference of the pinv, and
the degenerate cases (empty mask, exact-rank point)."""
import numpy as np
import pytest

from oracle.quat import qmul, fro2, inner
from oracle.pinv import pinv
from oracle.grad import (cur_vjp, cur_of, masked_loss, masked_loss_grad, pinv_vjp,
                         central_difference)


def _problem(seed, m=12, n=10, k=2, noise=0.0):
    rng = np.random.default_rng(seed)
    A = qmul(rng.standard_normal((4, m, k)), rng.standard_normal((4, k, n)))
    A = A + noise * rng.standard_normal(A.shape)
    return A, rng


def test_pinv_adjoint_matches_finite_difference():
    rng = np.random.default_rng(31)
    W = rng.standard_normal((4, 5, 4))
    U, _ = pinv(W)
    gU = rng.standard_normal(U.shape)
    gW = pinv_vjp(W, U, gU)
    for _ in range(3):
        V = rng.standard_normal(W.shape)
        fd = central_difference(lambda X: inner(gU, pinv(X)[0]), W, V)
        assert inner(gW, V) == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_pinv_adjoint_rank_deficient_fixed_rank():
    # at an exactly rank-2 point the rank-2 truncated pinv is differentiable
    rng = np.random.default_rng(32)
    W = qmul(rng.standard_normal((4, 6, 2)), rng.standard_normal((4, 2, 5)))
    U, k = pinv(W, max_rank=2)
    assert k == 2
    gU = rng.standard_normal(U.shape)
    gW = pinv_vjp(W, U, gU)
    V = rng.standard_normal(W.shape)
    fd = central_difference(lambda X: inner(gU, pinv(X, max_rank=2)[0]), W, V)
    assert inner(gW, V) == pytest.approx(fd, rel=1e-5)


def test_cur_vjp_matches_finite_difference():
    A, rng = _problem(33, noise=0.1)
    I, J = [0, 3, 5, 9], [1, 4, 6, 8]
    gB = rng.standard_normal(A.shape)
    dA = cur_vjp(A, I, J, gB)
    for _ in range(3):
        V = rng.standard_normal(A.shape)
        fd = central_difference(lambda X: inner(gB, cur_of(X, I, J)), A, V)
        assert inner(dA, V) == pytest.approx(fd, rel=1e-6)


def test_masked_loss_with_target_matches_finite_difference():
    A, rng = _problem(34, noise=0.05)
    Y = A + 0.01 * rng.standard_normal(A.shape)
    I, J = [1, 2, 6, 10], [0, 5, 7, 9]
    mask = (rng.random(A.shape[1:]) < 0.5).astype(np.uint8)
    g = masked_loss_grad(A, I, J, mask, Y=Y)
    V = rng.standard_normal(A.shape)
    fd = central_difference(lambda X: masked_loss(X, I, J, mask, Y=Y), A, V)
    assert inner(g, V) == pytest.approx(fd, rel=1e-6)


def test_masked_self_loss_with_noise_matches_finite_difference():
    A, rng = _problem(35, noise=0.05)
    I, J = [0, 1, 4, 7, 11], [2, 3, 5, 8]
    mask = (rng.random(A.shape[1:]) < 0.5).astype(np.uint8)
    g = masked_loss_grad(A, I, J, mask)
    V = rng.standard_normal(A.shape)
    fd = central_difference(lambda X: masked_loss(X, I, J, mask), A, V)
    assert inner(g, V) == pytest.approx(fd, rel=1e-6)


def test_empty_mask_and_exact_rank_give_zero_gradient():
    A, rng = _problem(36)
    I, J = [0, 3, 6, 9], [1, 2, 5, 7]
    g0 = masked_loss_grad(A, I, J, np.zeros(A.shape[1:], np.uint8))
    assert not g0.any()
    mask = (rng.random(A.shape[1:]) < 0.5).astype(np.uint8)
    g = masked_loss_grad(A, I, J, mask, max_rank=2)
    assert np.sqrt(fro2(g)) < 1e-10 * np.sqrt(fro2(A))
    assert masked_loss(A, I, J, mask, max_rank=2) < 1e-20 * fro2(A)


def test_vjp_dot_product_with_jvp():
    # <VJP(gB), V> = <gB, JVP(V)>, with the JVP dB = dC U R + C dU R + C U dR
    A, rng = _problem(37, noise=0.1)
    I, J = [1, 4, 8, 10], [0, 3, 6, 9]
    from oracle.cur import gather
    C, R, W = gather(A, I, J)
    U, _ = pinv(W)
    V = rng.standard_normal(A.shape)
    dC, dR, dW = gather(V, I, J)
    # dU from the constant-rank derivative of the pseudoinverse
    from oracle.quat import qH, eye
    r, c = W.shape[1], W.shape[2]
    dU = (-qmul(qmul(U, dW), U)
          + qmul(qmul(qmul(U, qH(U)), qH(dW)), eye(r) - qmul(W, U))
          + qmul(qmul(eye(c) - qmul(U, W), qH(dW)), qmul(qH(U), U)))
    dB = qmul(qmul(dC, U), R) + qmul(qmul(C, dU), R) + qmul(qmul(C, U), dR)
    gB = rng.standard_normal(A.shape)
    assert inner(cur_vjp(A, I, J, gB), V) == pytest.approx(inner(gB, dB), rel=1e-10)
