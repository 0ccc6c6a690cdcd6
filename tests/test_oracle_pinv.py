"""Pins of the checker's Moore-Penrose inverse (Section 2.1 notation; the
projector facts used in the proof of Lemma 2)."""
import numpy as np
import pytest

from oracle.quat import qmul, qH, fro2, real_rep, eye
from oracle.pinv import pinv, singular_values
from tests.qhelp import random_isometry, lowrank_svd_form


def _close(X, Y, tol):
    return np.sqrt(fro2(X - Y)) <= tol * max(1.0, np.sqrt(fro2(Y)))


def _penrose(X, Xp, tol=1e-10):
    assert _close(qmul(qmul(X, Xp), X), X, tol)          # X X+ X = X
    assert _close(qmul(qmul(Xp, X), Xp), Xp, tol)        # X+ X X+ = X+
    XXp = qmul(X, Xp)
    XpX = qmul(Xp, X)
    assert _close(qH(XXp), XXp, tol)                     # (X X+)^H = X X+
    assert _close(qH(XpX), XpX, tol)                     # (X+ X)^H = X+ X


@pytest.mark.parametrize("shape", [(6, 6), (9, 4), (4, 9), (1, 5), (5, 1), (13, 7)])
def test_penrose_conditions_full_rank(shape):
    rng = np.random.default_rng(sum(shape))
    X = rng.standard_normal((4, *shape))
    Xp, k = pinv(X)
    assert Xp.shape == (4, shape[1], shape[0])
    assert k == min(shape)
    _penrose(X, Xp)


@pytest.mark.parametrize("m,n,k", [(8, 8, 3), (10, 6, 2), (5, 12, 4)])
def test_penrose_conditions_rank_deficient(m, n, k):
    rng = np.random.default_rng(100 + m * n + k)
    X = qmul(rng.standard_normal((4, m, k)), rng.standard_normal((4, k, n)))
    Xp, r = pinv(X)
    assert r == k
    _penrose(X, Xp)


def test_invertible_is_inverse():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((4, 7, 7))
    Xp, _ = pinv(X)
    assert _close(qmul(X, Xp), eye(7), 1e-11)
    assert _close(qmul(Xp, X), eye(7), 1e-11)


def test_rank_one_closed_form():
    # (x y^H)^+ = y x^H / (|x|^2 |y|^2)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((4, 6, 1))
    y = rng.standard_normal((4, 5, 1))
    X = qmul(x, qH(y))
    Xp, k = pinv(X)
    assert k == 1
    expect = qmul(y, qH(x)) / (fro2(x) * fro2(y))
    assert _close(Xp, expect, 1e-12)


def test_isometry_pinv_is_conjugate_transpose():
    rng = np.random.default_rng(5)
    Q = random_isometry(9, 4, rng)
    assert _close(qmul(qH(Q), Q), eye(4), 1e-12)
    Qp, _ = pinv(Q)
    assert _close(Qp, qH(Q), 1e-12)


def test_agrees_with_real_representation_pinv():
    # a different route: NumPy's real SVD pseudoinverse of the 4m x 4n matrix
    rng = np.random.default_rng(6)
    X = qmul(rng.standard_normal((4, 8, 3)), rng.standard_normal((4, 3, 6)))
    Xp, _ = pinv(X)
    ref = np.linalg.pinv(real_rep(X), rcond=1e-10)
    assert np.allclose(real_rep(Xp), ref, atol=1e-10)


def test_truncation_rules():
    rng = np.random.default_rng(7)
    X, _, _ = lowrank_svd_form(10, 8, [5.0, 2.0, 1e-3, 1e-20], rng)
    sv = singular_values(X)
    assert sv[:3] == pytest.approx([5.0, 2.0, 1e-3], rel=1e-9)
    _, k = pinv(X)
    assert k == 3                      # 1e-20 is below max(p,q) * 2^-52 * 5
    _, k = pinv(X, rtol=1e-2)
    assert k == 2
    Xp, k = pinv(X, max_rank=1)
    assert k == 1
    # keeping one singular value gives the pseudoinverse of the best rank-1 part
    X1, _, _ = lowrank_svd_form(10, 8, [5.0], np.random.default_rng(7))
    assert np.sqrt(fro2(Xp)) == pytest.approx(1 / 5.0, rel=1e-9)


def test_zero_and_empty():
    Xp, k = pinv(np.zeros((4, 3, 2)))
    assert k == 0 and Xp.shape == (4, 2, 3) and not Xp.any()
    Xp, k = pinv(np.zeros((4, 0, 3)))
    assert k == 0 and Xp.shape == (4, 3, 0)
