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
"""
from __future__ import annotations

import numpy as np

from .cur import gather, core_car, cur_product
from .quat import fro2


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
