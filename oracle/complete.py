"""Quaternion matrix completion with QMCUR (Algorithm 2; Example 4.4).

Part of the FP64 reference checker (test infrastructure only).

Starting from the observed entries X^0 = P_Omega(Y) (zeros elsewhere), each
step replaces X^t by its QMCUR approximation M^{t+1} = C U R computed with
Algorithm 1 on the fixed index sets I and J (C = X^t(:, J), R = X^t(I, :),
U = C^+ X^t R^+), then restores the observed entries,
X^{t+1} = P_Omega(Y) + P_Omega^c(M^{t+1})  (the masking step of Example 4.4),
and stops when ||X^{t+1} - X^t||_F / ||X^t||_F <= tol or after max_iter
steps.  The paper writes the iterates with a dot and sizes them |I| x |J|;
both are read as the m x n iterate itself.

Variant (resampled index sets): step t draws J and I afresh from the
sampling probabilities of X^t (Section 3.1, length or uniform) with seed
seed + t, J as set 0 and I as set 1, as Algorithm 1 does for one matrix.

sample_size: Section 3.1 sizes C and R as k log k; read as ceil(k ln k)
(natural logarithm), at least k and at most the available count.
"""
from __future__ import annotations

import math

import numpy as np

from .cur import gather, core_car, cur_product
from .quat import fro2
from .sampling import draw, probs_length, probs_uniform, MASK64


def complete(Y: np.ndarray, mask: np.ndarray, I, J, max_iter: int = 200, tol: float = 1e-4, rtol: float = -1.0,
             max_rank: int = 0):
    """Returns dict(X, iters, rel): the last iterate, the number of steps and
    the last relative change."""
    keep = np.asarray(mask, dtype=bool)[None]
    X = np.where(keep, Y, 0.0)
    rel = np.inf
    t = 0
    while t < max_iter:
        C, R, _ = gather(X, I, J)
        U, _, _ = core_car(X, C, R, rtol, max_rank)
        M = cur_product(C, U, R)
        Xn = np.where(keep, Y, M)
        d2, o2 = fro2(Xn - X), fro2(X)
        rel = np.sqrt(d2 / o2) if o2 > 0 else (np.inf if d2 > 0 else 0.0)
        X = Xn
        t += 1
        if rel <= tol:
            break
    return dict(X=X, iters=t, rel=rel)


def sample_size(k: int, limit: int) -> int:
    """ceil(k ln k) clipped to [k, limit] (k = 1 gives 1)."""
    if k < 1 or limit < 1:
        raise ValueError("k and limit must be positive")
    s = math.ceil(k * math.log(k)) if k > 1 else 1
    return int(min(limit, max(k, s)))


def complete_resampled(Y: np.ndarray, mask: np.ndarray, r: int, c: int, sampling: str = "length", seed: int = 0,
                       max_iter: int = 200, tol: float = 1e-4, rtol: float = -1.0, max_rank: int = 0):
    """Algorithm 2 with the index sets drawn again at every step from the
    probabilities of the current iterate.  Returns dict(X, iters, rel, I, J)
    with the index sets of the last step."""
    keep = np.asarray(mask, dtype=bool)[None]
    X = np.where(keep, Y, 0.0)
    _, m, n = X.shape
    rel = np.inf
    I = J = None
    t = 0
    while t < max_iter:
        if sampling == "length":
            p, q, _ = probs_length(X)
        elif sampling == "uniform":
            p, q = probs_uniform(m, n)
        else:
            raise ValueError("sampling is 'length' or 'uniform'")
        st = (seed + t) & MASK64
        J = draw(p, c, st, 0)
        I = draw(q, r, st, 1)
        C, R, _ = gather(X, I, J)
        U, _, _ = core_car(X, C, R, rtol, max_rank)
        M = cur_product(C, U, R)
        Xn = np.where(keep, Y, M)
        d2, o2 = fro2(Xn - X), fro2(X)
        rel = np.sqrt(d2 / o2) if o2 > 0 else (np.inf if d2 > 0 else 0.0)
        X = Xn
        t += 1
        if rel <= tol:
            break
    return dict(X=X, iters=t, rel=rel, I=I, J=J)
