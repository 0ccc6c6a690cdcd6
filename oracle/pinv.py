"""Moore-Penrose inverse of a quaternion matrix (the (.)^dagger of Section 2.1).

Part of the FP64 reference checker (test infrastructure only).

Reading used where the paper is silent: singular values at or below
rtol * sigma_max are treated as zero, rtol < 0 selects
max(rows, cols) * 2^-52, and max_rank > 0 keeps at most that many
quaternion singular values (the predefined rank k of Algorithm 1).
"""
from __future__ import annotations

import numpy as np

from .quat import chi, unchi


def pinv(X: np.ndarray, rtol: float = -1.0, max_rank: int = 0):
    """Return (X^dagger, rank) for X of shape (4, p, q); X^dagger is (4, q, p).

    chi(X^dagger) = chi(X)^dagger, and every singular value of X appears twice
    among those of chi(X).  The SVD of chi(X) (LAPACK) is taken, quaternion
    singular values are read as every other value of the sorted list, and the
    kept ones are inverted pair by pair.
    """
    _, p, q = X.shape
    if rtol < 0:
        rtol = max(p, q) * 2.0 ** -52
    if p == 0 or q == 0:
        return np.zeros((4, q, p)), 0
    M = chi(X)
    U, s, Vh = np.linalg.svd(M, full_matrices=False)
    sq = s[0::2]
    smax = sq[0]
    if smax == 0.0:
        return np.zeros((4, q, p)), 0
    k = int(np.sum(sq > rtol * smax))
    if max_rank > 0:
        k = min(k, max_rank)
    kc = 2 * k
    Mp = (Vh[:kc].conj().T / s[:kc]) @ U[:, :kc].conj().T
    return unchi(Mp, q, p), k


def singular_values(X: np.ndarray) -> np.ndarray:
    """Quaternion singular values of X in descending order."""
    if X.shape[1] == 0 or X.shape[2] == 0:
        return np.zeros(0)
    return np.linalg.svd(chi(X), compute_uv=False)[0::2]
