"""Derivatives of B = CUR(A) with the intersection core U = W^dagger, and of
the masked data-fit loss ||P_Omega(A - CUR(A))||_F^2 (the objective of the
completion problem in Example 4.4, restricted to the observed set Omega).

Part of the FP64 reference checker (test infrastructure only).

Gradients are with respect to the four real planes: dL = <G, dA> with
<X, Y> = Re Tr(X^H Y).  Because Re Tr(XY) = Re Tr(YX) also holds for
quaternion matrices, the usual matrix-calculus rules carry over:
  B = C U R:  gC = gB R^H U^H,  gU = C^H gB R^H,  gR = U^H C^H gB.
  U = W^dagger (constant rank, Golub-Pereyra 1973):
      gW = -U^H gU U^H + (I - W U) gU^H U U^H + U^H U gU^H (I - U W).
  C = A(:, J), R = A(I, :), W = A(I, J): the gradients scatter back into
  the sampled columns, rows and intersection.
"""
from __future__ import annotations

import numpy as np

from .quat import qmul, qH, eye, fro2
from .pinv import pinv
from .cur import gather


def pinv_vjp(W: np.ndarray, U: np.ndarray, gU: np.ndarray) -> np.ndarray:
    """Cotangent of W from the cotangent gU of U = W^dagger (constant rank)."""
    r, c = W.shape[1], W.shape[2]
    UH = qH(U)
    gUH = qH(gU)
    t1 = -qmul(qmul(UH, gU), UH)
    t2 = qmul(qmul(eye(r) - qmul(W, U), gUH), qmul(U, UH))
    t3 = qmul(qmul(qmul(UH, U), gUH), eye(c) - qmul(U, W))
    return t1 + t2 + t3


def cur_vjp(A: np.ndarray, I, J, gB: np.ndarray, rtol: float = -1.0, max_rank: int = 0) -> np.ndarray:
    """d<gB, CUR(A)>/dA for U = W^dagger: the vector-Jacobian product."""
    I = np.asarray(I, dtype=np.int64)
    J = np.asarray(J, dtype=np.int64)
    C, R, W = gather(A, I, J)
    U, _ = pinv(W, rtol, max_rank)
    gC = qmul(qmul(gB, qH(R)), qH(U))
    gU = qmul(qmul(qH(C), gB), qH(R))
    gR = qmul(qmul(qH(U), qH(C)), gB)
    gW = pinv_vjp(W, U, gU)
    dA = np.zeros_like(A)
    dA[:, :, J] += gC
    dA[:, I, :] += gR
    for s, i in enumerate(I):
        dA[:, i, J] += gW[:, s, :]
    return dA


def cur_of(A: np.ndarray, I, J, rtol: float = -1.0, max_rank: int = 0) -> np.ndarray:
    C, R, W = gather(A, I, J)
    U, _ = pinv(W, rtol, max_rank)
    return qmul(qmul(C, U), R)


def masked_loss(A: np.ndarray, I, J, mask, Y=None, rtol: float = -1.0, max_rank: int = 0) -> float:
    """L = ||P_Omega(Y - CUR(A))||_F^2 with Y = A unless a target is given."""
    T = A if Y is None else Y
    D = (T - cur_of(A, I, J, rtol, max_rank)) * np.asarray(mask, dtype=np.float64)[None]
    return fro2(D)


def masked_loss_grad(A: np.ndarray, I, J, mask, Y=None, rtol: float = -1.0, max_rank: int = 0) -> np.ndarray:
    """dL/dA for masked_loss.  With G = 2 P_Omega(Y - CUR(A)) the cotangent of
    B is -G; when Y is A itself the direct term +G is added."""
    Mk = np.asarray(mask, dtype=np.float64)[None]
    T = A if Y is None else Y
    G = 2.0 * (T - cur_of(A, I, J, rtol, max_rank)) * Mk
    dA = cur_vjp(A, I, J, -G, rtol, max_rank)
    if Y is None:
        dA = dA + G
    return dA


def central_difference(f, A: np.ndarray, V: np.ndarray, h: float = 1e-6) -> float:
    """(f(A + hV) - f(A - hV)) / (2h), the directional derivative along V."""
    return (f(A + h * V) - f(A - h * V)) / (2.0 * h)
