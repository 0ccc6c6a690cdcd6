"""Perturbation estimate of the QMCUR approximation (Section 3.2, Theorem 1)
and the experiment that illustrates it (Example 4.1).

Part of the FP64 reference checker (test infrastructure only).

Theorem 1: for X~ = X + E with X = W_k Sigma_k V_k^H of rank k, index sets
I (rows) and J (columns), C~ = X~(:, J), R~ = X~(I, :) and the least-squares
core U~ = C~^+ X~ R~^+, the spectral-norm error satisfies

    ||X - C~ U~ R~||_2 <= ||E||_2 (||W_{k,I}^+||_2 + ||V_{k,J}^+||_2 + 3),

with W_{k,I} = W_k(I, :) and V_{k,J} = V_k(J, :).  Example 4.1 builds X from
unitary W_k, V_k (m x k) and a positive diagonal Sigma_k, adds Gaussian noise
and plots the error against ||E||_2.

Readings where the paper leaves a choice open: the unitary factors are the
polar factors of Gaussian quaternion matrices (unique, so two independent
implementations build the same X); the noise level sigma of the example is
read as the standard deviation of every component, E = sigma * E0 with E0
standard Gaussian; C and R have ceil(k ln k) columns and rows (the sizing of
Section 3.1).
"""
from __future__ import annotations

import numpy as np

from .cur import cur_product, solve
from .pinv import singular_values
from .quat import chi, qH, qmul, spectral_norm, unchi


def polar_factor(G: np.ndarray) -> np.ndarray:
    """Unitary polar factor Q of a full-column-rank G (4, p, q): G = Q H with
    Q^H Q = I and H Hermitian positive definite.

    Through the complex adjoint: chi is multiplicative and maps ^H to the
    conjugate transpose, so chi(Q) is the polar factor of chi(G), i.e.
    U V^H from the thin SVD chi(G) = U S V^H (LAPACK)."""
    _, p, q = G.shape
    U, _, Vh = np.linalg.svd(chi(G), full_matrices=False)
    return unchi(U @ Vh, p, q)


def lowrank_product(W: np.ndarray, sig: np.ndarray, V: np.ndarray) -> np.ndarray:
    """X = W diag(sig) V^H for real sig (Example 4.1)."""
    k = sig.shape[0]
    S = np.zeros((4, k, k))
    S[0] = np.diag(sig)
    return qmul(qmul(W, S), qH(V))


def perturbation_errors(X: np.ndarray, E: np.ndarray, W: np.ndarray, V: np.ndarray, c: int, r: int,
                        sampling: str = "length", seed: int = 0) -> dict:
    """One noise level of Example 4.1: Algorithm 1 (least-squares core) on
    X~ = X + E, then the quantities of Theorem 1 in the spectral norm.

    Returns err = ||X - C~ U~ R~||_2, norm_E = ||E||_2, w_pinv =
    ||W_{k,I}^+||_2 and v_pinv = ||V_{k,J}^+||_2 (the reciprocal of the
    smallest singular value, infinite when the sampled rows or columns lose
    rank), bound = norm_E (w_pinv + v_pinv + 3), and the index sets."""
    Xt = X + E
    sol = solve(Xt, c, r, sampling, "car", seed)
    D = X - cur_product(sol["C"], sol["U"], sol["R"])
    err = spectral_norm(D)
    norm_E = spectral_norm(E)
    k = W.shape[2]

    def pinv_norm(F):
        s = singular_values(F)
        return 1.0 / s[-1] if s.size == k and s[-1] > 0 else np.inf

    w_pinv = pinv_norm(W[:, sol["I"], :])
    v_pinv = pinv_norm(V[:, sol["J"], :])
    return dict(err=err, norm_E=norm_E, w_pinv=w_pinv, v_pinv=v_pinv,
                bound=norm_E * (w_pinv + v_pinv + 3.0), I=sol["I"], J=sol["J"])
