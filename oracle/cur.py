"""The QMCUR approximation itself (Algorithm 1 and Section 3.1).

Part of the FP64 reference checker (test infrastructure only).

Readings used where the paper is silent or inconsistent:
  * U is |J| x |I| (c x r): Section 3.1 and the least-squares problem give
    this shape; the |I| x |J| in Algorithm 1, step 3 is read as a typo.
  * The intersection core U = W^dagger with W = A(I, J) is the classical
    cross approximation of the real-matrix CUR literature the paper builds
    on; it is provided next to the least-squares core U = C^dagger A R^dagger.
  * Sampled columns and rows are used as they are, without rescaling.
  * Products are associated as T = A R^dagger, U = C^dagger T and
    B = (C U) R.
"""
from __future__ import annotations

import numpy as np

from .quat import qmul, fro2
from .pinv import pinv
from .sampling import probs_length, probs_uniform, draw


def gather(A: np.ndarray, I: np.ndarray, J: np.ndarray):
    """C = A(:, J), R = A(I, :) and W = A(I, J) (Section 2.1 notation,
    Algorithm 1 steps 1-2)."""
    I = np.asarray(I, dtype=np.int64)
    J = np.asarray(J, dtype=np.int64)
    C = A[:, :, J]
    R = A[:, I, :]
    W = A[:, I][:, :, J]
    return C, R, W


def core_wpinv(W: np.ndarray, rtol: float = -1.0, max_rank: int = 0):
    """Intersection core U = W^dagger; returns (U, rank)."""
    return pinv(W, rtol, max_rank)


def core_car(A: np.ndarray, C: np.ndarray, R: np.ndarray, rtol: float = -1.0, max_rank: int = 0):
    """Least-squares core U = C^dagger X R^dagger (Algorithm 1 step 3, and the
    arg-min characterisation in Section 3.1); returns (U, rank_C, rank_R)."""
    Cp, kc = pinv(C, rtol, max_rank)
    Rp, kr = pinv(R, rtol, max_rank)
    T = qmul(A, Rp)
    U = qmul(Cp, T)
    return U, kc, kr


def cur_product(C: np.ndarray, U: np.ndarray, R: np.ndarray) -> np.ndarray:
    """B = C U R (Algorithm 1 output), associated as (C U) R."""
    return qmul(qmul(C, U), R)


def residual(A: np.ndarray, C: np.ndarray, U: np.ndarray, R: np.ndarray, mask=None) -> float:
    """||P_Omega(A - C U R)||_F; without a mask this is ||A - CUR||_F, the
    numerator of the relative error of Example 4.2."""
    D = A - cur_product(C, U, R)
    if mask is not None:
        D = D * np.asarray(mask, dtype=np.float64)[None]
    return float(np.sqrt(fro2(D)))


def solve(A: np.ndarray, c: int, r: int, sampling: str = "length", core: str = "car",
          seed: int = 0, rtol: float = -1.0, max_rank: int = 0, with_replacement: bool = False):
    """Algorithm 1 end to end: probabilities, draws J (set 0) and I (set 1),
    gathers, core and the relative error ||A - CUR||_F / ||A||_F."""
    _, m, n = A.shape
    if sampling == "length":
        p, q, _ = probs_length(A)
    elif sampling == "uniform":
        p, q = probs_uniform(m, n)
    else:
        raise ValueError(sampling)
    J = draw(p, c, seed, 0, with_replacement)
    I = draw(q, r, seed, 1, with_replacement)
    C, R, W = gather(A, I, J)
    if core == "wpinv":
        U, rank = core_wpinv(W, rtol, max_rank)
    elif core == "car":
        U, rank, _ = core_car(A, C, R, rtol, max_rank)
    else:
        raise ValueError(core)
    res = residual(A, C, U, R)
    return dict(p=p, q=q, I=I, J=J, C=C, R=R, W=W, U=U, rank=rank, residual=res,
                rel_err=res / np.sqrt(fro2(A)))
