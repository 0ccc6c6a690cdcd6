"""Perturbation estimate of QMCUR (Section 3.2, Theorem 1) and the experiment
of Example 4.1, on the GPU.

Theorem 1 bounds the spectral-norm error of the least-squares CUR of a noisy
rank-k matrix X~ = X + E, X = W_k Sigma_k V_k^H, by
||E||_2 (||W_{k,I}^+||_2 + ||V_{k,J}^+||_2 + 3).  Every step below is a call
into libqcur: the polar factors and spectral norms come from the Jacobi QSVD
(qcur_svd), products from qcur_gemm, X - C~U~R~ from the residual kernel's
difference output, the sampled rows of W_k and V_k from qcur_gather.  The
unitary factors are the polar factors U V^H of Gaussian quaternion matrices
(unique for full column rank, so any implementation builds the same X).
"""
from __future__ import annotations

import torch

from . import qcur as _q


def polar_factor(G: torch.Tensor) -> torch.Tensor:
    """Unitary polar factor Q = U V^H of a full-column-rank FP64 G (4, p, q)
    from its thin QSVD G = U diag(s) V^H."""
    _, U, V = _q.svd(G)
    return _q.gemm(U, V, _q.OP_N, _q.OP_H)


def lowrank_product(W: torch.Tensor, sig: torch.Tensor, V: torch.Tensor) -> torch.Tensor:
    """X = W diag(sig) V^H (Example 4.1) for a real vector sig."""
    k = sig.numel()
    S = torch.zeros((4, k, k), dtype=torch.float64, device=W.device)
    S[0] = torch.diag(sig.to(device=W.device, dtype=torch.float64))
    return _q.gemm(_q.gemm(W, S), V, _q.OP_N, _q.OP_H)


def spectral_norm(A: torch.Tensor) -> float:
    """||A||_2: the largest quaternion singular value (Jacobi QSVD, FP64)."""
    s, _, _ = _q.svd(A, vectors=False)
    return float(s[0]) if s.numel() else 0.0


def _pinv_norm(F: torch.Tensor, k: int) -> float:
    s, _, _ = _q.svd(F, vectors=False)
    lo = float(s[-1]) if s.numel() == k else 0.0
    return 1.0 / lo if lo > 0 else float("inf")


def perturbation_errors(X: torch.Tensor, E0: torch.Tensor, scale: float, W: torch.Tensor, V: torch.Tensor,
                        c: int, r: int, sampling: int = _q.LENGTH, seed: int = 0,
                        norm_E0: float | None = None) -> dict:
    """One noise level of Example 4.1 with E = scale * E0 (FP64 throughout).

    X~ = X + scale E0 (one product-accumulate), Algorithm 1 with the
    least-squares core on X~, D = X - C~ U~ R~, and the quantities of
    Theorem 1: err = ||D||_2, norm_E = ||E||_2 (scale times norm_E0 when it
    is given), w_pinv = ||W_k(I,:)^+||_2, v_pinv = ||V_k(J,:)^+||_2 and
    bound = norm_E (w_pinv + v_pinv + 3).  Index sets I, J are returned
    as device tensors."""
    _, m, n = X.shape
    k = W.shape[2]
    eye = torch.zeros((4, n, n), dtype=torch.float64, device=X.device)
    eye[0] = torch.eye(n, dtype=torch.float64, device=X.device)
    Xt = _q.gemm(E0, eye, alpha=scale, beta=1.0, D=_q.cast(X, torch.float64))
    sol = _q.solve(Xt, c, r, sampling, _q.CORE_CAR, _q.F64, seed)
    _, D = _q.residual(X, sol["C"], sol["U"], sol["R"], want_E=True)
    err = spectral_norm(D)
    if norm_E0 is None:
        norm_E0 = spectral_norm(E0)
    norm_E = abs(scale) * norm_E0
    cols = torch.arange(k, dtype=torch.int64, device=X.device)
    _, WI, _ = _q.gather(W, sol["I"], cols, want=("R",))
    _, VJ, _ = _q.gather(V, sol["J"], cols, want=("R",))
    w_pinv, v_pinv = _pinv_norm(WI, k), _pinv_norm(VJ, k)
    return dict(err=err, norm_E=norm_E, w_pinv=w_pinv, v_pinv=v_pinv, bound=norm_E * (w_pinv + v_pinv + 3.0),
                I=sol["I"], J=sol["J"])
