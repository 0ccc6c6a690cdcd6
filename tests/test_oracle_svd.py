"""Pins of the checker's quaternion singular values (through the complex
adjoint, Section 2.1): the cases with closed forms or textbook routines."""
import numpy as np

from oracle.pinv import singular_values
from oracle.quat import qmul, fro2


def test_real_matrices_reduce_to_the_real_svd():
    rng = np.random.default_rng(1)
    for p, q in ((7, 5), (5, 7), (12, 12)):
        X = np.zeros((4, p, q))
        X[0] = rng.standard_normal((p, q))
        assert np.allclose(singular_values(X), np.linalg.svd(X[0], compute_uv=False), rtol=1e-13, atol=0)


def test_diagonal_quaternion_matrix():
    # diag(d_1..d_n) with quaternion d_i: singular values are |d_i|, sorted
    rng = np.random.default_rng(2)
    d = rng.standard_normal((4, 6))
    X = np.zeros((4, 6, 6))
    for i in range(6):
        X[:, i, i] = d[:, i]
    assert np.allclose(singular_values(X), np.sort(np.linalg.norm(d, axis=0))[::-1], rtol=1e-13, atol=0)


def test_frobenius_and_rank():
    rng = np.random.default_rng(3)
    X = qmul(rng.standard_normal((4, 30, 4)), rng.standard_normal((4, 4, 20)))
    s = singular_values(X)
    assert s.shape == (20,)
    assert abs((s ** 2).sum() - fro2(X)) < 1e-11 * fro2(X)
    assert (s[:4] > 1e-8 * s[0]).all() and (s[4:] < 1e-12 * s[0]).all()


def test_unitary_invariance():
    # a quaternion rotation u X v with unit quaternions u, v on the left and
    # right keeps every singular value
    rng = np.random.default_rng(4)
    X = rng.standard_normal((4, 9, 7))
    u = rng.standard_normal(4); u /= np.linalg.norm(u)
    v = rng.standard_normal(4); v /= np.linalg.norm(v)
    U = np.zeros((4, 9, 9)); V = np.zeros((4, 7, 7))
    for i in range(9):
        U[:, i, i] = u
    for i in range(7):
        V[:, i, i] = v
    assert np.allclose(singular_values(qmul(qmul(U, X), V)), singular_values(X), rtol=1e-12, atol=0)
