"""Pins of the checker's quaternion algebra (Section 2.2)."""
import os

import numpy as np
import pytest

from oracle.quat import qmul, qH, fro2, chi, unchi, real_rep, stack, unstack, inner, spectral_norm
from tests.qhelp import basis


def _table(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "hamilton_table.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            a, b, s, c = line.split()
            rows.append((a, b, int(s), c))
    return rows


def test_hamilton_table_all_sixteen_products(golden_dir):
    rows = _table(golden_dir)
    assert len(rows) == 16
    for a, b, s, c in rows:
        got = qmul(basis(a), basis(b))
        assert np.array_equal(got, s * basis(c)), (a, b)


def test_ijk_is_minus_one():
    ijk = qmul(qmul(basis("i"), basis("j")), basis("k"))
    assert np.array_equal(ijk, -basis("1"))


def test_scalar_product_by_hand():
    # (1 + 2i + 3j + 4k)(5 + 6i + 7j + 8k) expanded by hand with the table
    a = np.array([1.0, 2, 3, 4]).reshape(4, 1, 1)
    b = np.array([5.0, 6, 7, 8]).reshape(4, 1, 1)
    # real: 5 - 12 - 21 - 32 = -60
    # i:    6 + 10 + (3*8: jk=i) 24 - (4*7: kj=-i) 28 = 12
    # j:    7 - (2*8: ik=-j) 16 + 15 + (4*6: ki=j) 24 = 30
    # k:    8 + (2*7: ij=k) 14 - (3*6: ji=-k) 18 + 20 = 24
    assert qmul(a, b).ravel().tolist() == [-60.0, 12.0, 30.0, 24.0]


def test_complex_adjoint_is_multiplicative():
    rng = np.random.default_rng(11)
    A = rng.standard_normal((4, 7, 5))
    B = rng.standard_normal((4, 5, 6))
    assert np.allclose(chi(qmul(A, B)), chi(A) @ chi(B), rtol=0, atol=1e-12)


def test_complex_adjoint_roundtrip_and_hermitian():
    rng = np.random.default_rng(12)
    A = rng.standard_normal((4, 6, 3))
    assert np.array_equal(unchi(chi(A), 6, 3), A)
    assert np.allclose(chi(qH(A)), chi(A).conj().T, atol=0)


def test_real_representation_is_multiplicative():
    rng = np.random.default_rng(13)
    A = rng.standard_normal((4, 4, 3))
    B = rng.standard_normal((4, 3, 5))
    assert np.allclose(real_rep(qmul(A, B)), real_rep(A) @ real_rep(B), atol=1e-12)
    assert np.allclose(stack(qmul(A, B)), real_rep(A) @ stack(B), atol=1e-12)
    assert np.array_equal(unstack(stack(B)), B)
    assert np.array_equal(real_rep(qH(A)), real_rep(A).T)


def test_conjugate_transpose_reverses_products():
    rng = np.random.default_rng(14)
    A = rng.standard_normal((4, 4, 6))
    B = rng.standard_normal((4, 6, 3))
    assert np.allclose(qH(qmul(A, B)), qmul(qH(B), qH(A)), atol=1e-12)


def test_noncommutative_and_associative():
    rng = np.random.default_rng(15)
    A, B, C = (rng.standard_normal((4, 3, 3)) for _ in range(3))
    assert not np.allclose(qmul(A, B), qmul(B, A))
    assert np.allclose(qmul(qmul(A, B), C), qmul(A, qmul(B, C)), atol=1e-12)


def test_frobenius_norm_three_ways():
    rng = np.random.default_rng(16)
    A = rng.standard_normal((4, 5, 4))
    by_loop = 0.0
    for s in range(5):
        for t in range(4):
            by_loop += sum(A[c, s, t] ** 2 for c in range(4))   # |a_st|^2
    tr = qmul(qH(A), A)[0].trace()                             # Re Tr(A^H A)
    assert fro2(A) == pytest.approx(by_loop, rel=1e-14)
    assert fro2(A) == pytest.approx(tr, rel=1e-13)
    # chi doubles the squared Frobenius norm
    assert np.linalg.norm(chi(A)) ** 2 == pytest.approx(2 * fro2(A), rel=1e-13)
    assert inner(A, A) == pytest.approx(fro2(A), rel=1e-15)


def test_spectral_norm_is_unitarily_invariant_and_bounded():
    rng = np.random.default_rng(17)
    A = rng.standard_normal((4, 6, 4))
    s2 = spectral_norm(A)
    assert s2 <= np.sqrt(fro2(A)) + 1e-12
    x = rng.standard_normal((4, 4, 1))
    assert np.sqrt(fro2(qmul(A, x))) <= s2 * np.sqrt(fro2(x)) + 1e-12


def test_residual_identity_of_a_refined_core():
    # The algebra the library's refined solve relies on for its residual:
    # with D = Q_C^H E Q_R and G = Q^H Q, for any Q_C, Q_R (not only
    # orthonormal ones),
    #   ||E - Q_C D Q_R^H||_F^2 = ||E||^2 - 2 ||D||^2 + Re Tr(D^H G_C D G_R),
    # because the real part of a quaternion trace is cyclic.  Near-orthonormal
    # factors (defect delta) make the last term ||D||^2 (1 + O(delta)).
    rng = np.random.default_rng(31)
    m, n, c, r = 30, 26, 7, 6
    E = rng.standard_normal((4, m, n))
    Qc = rng.standard_normal((4, m, c))
    Qr = rng.standard_normal((4, n, r))
    D = qmul(qmul(qH(Qc), E), Qr)
    lhs = fro2(E - qmul(qmul(Qc, D), qH(Qr)))
    Gc, Gr = qmul(qH(Qc), Qc), qmul(qH(Qr), Qr)
    rhs = fro2(E) - 2 * fro2(D) + qmul(qmul(qmul(qH(D), Gc), D), Gr)[0].trace()
    assert lhs == pytest.approx(rhs, rel=1e-11)
    # cyclic real trace, the step the identity takes
    X, Y = rng.standard_normal((4, 5, 3)), rng.standard_normal((4, 3, 5))
    assert qmul(X, Y)[0].trace() == pytest.approx(qmul(Y, X)[0].trace(), rel=1e-12)
    # with orthonormal factors (polar factors of the random ones) the last
    # term is ||D||^2 and the residual is ||E||^2 - ||D||^2
    def orth(Z):
        U, _, Vh = np.linalg.svd(chi(Z), full_matrices=False)
        return unchi(U @ Vh, Z.shape[1], Z.shape[2])
    Qc, Qr = orth(Qc), orth(Qr)
    D = qmul(qmul(qH(Qc), E), Qr)
    assert fro2(E - qmul(qmul(Qc, D), qH(Qr))) == pytest.approx(fro2(E) - fro2(D), rel=1e-11)
    # and a defect delta moves it by at most about 3 delta ||D||^2
    Qc2 = Qc * (1 + 1e-4)  # Q^H Q = (1 + 1e-4)^2 I: defect about 2e-4 per column
    D2 = qmul(qmul(qH(Qc2), E), Qr)
    exact = fro2(E - qmul(qmul(Qc2, D2), qH(Qr)))
    approx = fro2(E) - fro2(D2)
    assert abs(exact - approx) <= 3 * 2.0001e-4 * fro2(D2)
