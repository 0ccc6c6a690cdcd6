"""Quaternion scalar and matrix algebra (Section 2.2, "Quaternion and
quaternion matrices").

Part of the FP64 reference checker (test infrastructure only).
"""
from __future__ import annotations

import numpy as np


def qmul(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Quaternion matrix product D = A B, written out as sixteen real products.

    Uses the multiplication laws of the basis (Section 2.2):
    i^2 = j^2 = k^2 = ijk = -1, ij = -ji = k, jk = -kj = i, ki = -ik = j.
    Expanding (A0 + A1 i + A2 j + A3 k)(B0 + B1 i + B2 j + B3 k) and
    collecting the coefficient of each basis element gives the four planes
    below.  A is (4, m, k), B is (4, k, n); the result is (4, m, n).
    """
    A0, A1, A2, A3 = A[0], A[1], A[2], A[3]
    B0, B1, B2, B3 = B[0], B[1], B[2], B[3]
    D0 = A0 @ B0 - A1 @ B1 - A2 @ B2 - A3 @ B3
    D1 = A0 @ B1 + A1 @ B0 + A2 @ B3 - A3 @ B2   # j*k = i, k*j = -i
    D2 = A0 @ B2 - A1 @ B3 + A2 @ B0 + A3 @ B1   # k*i = j, i*k = -j
    D3 = A0 @ B3 + A1 @ B2 - A2 @ B1 + A3 @ B0   # i*j = k, j*i = -k
    return np.stack([D0, D1, D2, D3])


def qconj(A: np.ndarray) -> np.ndarray:
    """Entrywise conjugate a* = a0 - a1 i - a2 j - a3 k (Section 2.2)."""
    return np.stack([A[0], -A[1], -A[2], -A[3]])


def qH(A: np.ndarray) -> np.ndarray:
    """Conjugate transpose A^H = (a*_ts) (Section 2.2)."""
    return np.ascontiguousarray(qconj(A).transpose(0, 2, 1))


def fro2(A: np.ndarray) -> float:
    """Squared Frobenius norm: the sum of |a_st|^2 over all entries (Section 2.2)."""
    return float(np.sum(A * A))


def fro(A: np.ndarray) -> float:
    return float(np.sqrt(fro2(A)))


def inner(X: np.ndarray, Y: np.ndarray) -> float:
    """Real inner product Re Tr(X^H Y); equals the sum over planes of X_c . Y_c."""
    return float(np.sum(X * Y))


def eye(n: int) -> np.ndarray:
    Z = np.zeros((4, n, n))
    Z[0] = np.eye(n)
    return Z


def chi(A: np.ndarray) -> np.ndarray:
    """Complex adjoint of A = a + b j with a = A0 + A1 i and b = A2 + A3 i.

    chi(A) = [[a, b], [-conj(b), conj(a)]] is a (2m x 2n) complex matrix;
    chi is an injective *-homomorphism, so products, conjugate transposes,
    Moore-Penrose inverses and spectral norms carry over to complex matrices.
    """
    a = A[0] + 1j * A[1]
    b = A[2] + 1j * A[3]
    return np.block([[a, b], [-b.conj(), a.conj()]])


def unchi(M: np.ndarray, rows: int, cols: int) -> np.ndarray:
    """Inverse of chi on its image: read a and b from the top blocks."""
    a = M[:rows, :cols]
    b = M[:rows, cols:]
    return np.stack([a.real, a.imag, b.real, b.imag])


def real_rep(A: np.ndarray) -> np.ndarray:
    """Left real representation L(A) (4m x 4k), with stack(AB) = L(A) stack(B).

    Block row p of L(A) holds the signed planes that multiply B_0..B_3 in
    plane p of the product (see qmul).
    """
    A0, A1, A2, A3 = A
    return np.block([
        [A0, -A1, -A2, -A3],
        [A1, A0, -A3, A2],
        [A2, A3, A0, -A1],
        [A3, -A2, A1, A0],
    ])


def stack(B: np.ndarray) -> np.ndarray:
    """Component stack [B0; B1; B2; B3] (4k x n)."""
    return np.concatenate([B[0], B[1], B[2], B[3]], axis=0)


def unstack(S: np.ndarray) -> np.ndarray:
    k = S.shape[0] // 4
    return np.stack([S[c * k:(c + 1) * k] for c in range(4)])


def spectral_norm(A: np.ndarray) -> float:
    """||A||_2 (Section 2.2) as the largest singular value of chi(A)."""
    if A.size == 0:
        return 0.0
    return float(np.linalg.norm(chi(A), 2))


def qrank(A: np.ndarray, rtol: float = 1e-10) -> int:
    """Quaternion rank: half the rank of chi(A)."""
    s = np.linalg.svd(chi(A), compute_uv=False)
    if s.size == 0 or s[0] == 0:
        return 0
    return int(np.sum(s > rtol * s[0]) // 2)
