"""The benchmark workloads at full size on the MI355X against the FP64
reference checker: the colour-image-shaped 1024 x 1024 solve (FP64, FP32,
BF16 operands with one refinement step) and the dense 4096 x 4096 solve
(FP32 products with one refinement step, FP64 pseudoinverses).  Draws are
compared bit for bit and C U R element by element: FP64 within 1e-12
(widened by the conditioning of C and R, which limits how well the FP64
projectors themselves are determined), FP32 products within 1e-5, BF16
operands within 2e-2 and split BF16 within 1e-4 relative Frobenius error."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from oracle.quat import qmul, fro2
from oracle.pinv import singular_values

pytestmark = pytest.mark.gpu

q = pytest.importorskip("paper_2402_19147_amd")
Q = q.qcur
DEV = torch.device("cuda:0")


def T(x, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


def N(t):
    return t.detach().to(torch.float64).cpu().numpy()


def kappa(X):
    s = singular_values(X)
    return float(s[0] / s[-1])


def tolerance(compute, C, R):
    if compute == Q.F64:
        return max(1e-12, 10 * 2.0 ** -52 * (kappa(C) + kappa(R)))
    return {Q.F32: 1e-5, Q.BF16: 2e-2, Q.BF16X3: 1e-4}[compute]


@pytest.fixture(scope="module")
def color():
    cfg = workloads.WORKLOADS["color_1024"]
    A = workloads.color_like(cfg["m"], cfg["n"], cfg["k"], cfg["seed"], cfg["noise"])
    ref = oracle.solve(A, cfg["c"], cfg["r"], "length", "car", seed=cfg["seed"])
    return cfg, A, ref


@pytest.mark.parametrize("compute,refine", [(Q.F64, 0), (Q.F32, 0), (Q.F32, 1), (Q.BF16, 1), (Q.BF16X3, 0)])
def test_color_workload(color, compute, refine):
    cfg, A, ref = color
    m, n = cfg["m"], cfg["n"]
    dt = torch.float64 if compute == Q.F64 else torch.float32
    Ad = N(T(A, dt))
    # the native solve (qcur_solve) with its C U R output
    S = Q.Solver(m, n, cfg["c"], cfg["r"], core=Q.CORE_CAR, compute=compute)
    B = torch.empty((4, m, n), dtype=dt, device=DEV)
    S(T(A, dt), sampling=Q.LENGTH, seed=cfg["seed"], refine_steps=refine, B=B)
    q.sync_status()
    if compute == Q.F64:
        refd = ref
    else:  # the checker on the same (rounded) input
        refd = oracle.solve(Ad, cfg["c"], cfg["r"], "length", "car", seed=cfg["seed"])
    assert N(S.J).astype(np.int64).tolist() == refd["J"].tolist()
    assert N(S.I).astype(np.int64).tolist() == refd["I"].tolist()
    Bref = oracle.cur_product(refd["C"], refd["U"], refd["R"])
    err = np.sqrt(fro2(N(B) - Bref) / fro2(Bref))
    tol = tolerance(compute, refd["C"], refd["R"])
    assert err < tol, err
    res = float(N(S.residual)[0])
    assert abs(res - refd["residual"]) <= tol * np.sqrt(fro2(Ad))


@pytest.mark.slow
def test_dense_workload_f32_refined():
    cfg = workloads.WORKLOADS["dense_4096"]
    m, n = cfg["m"], cfg["n"]
    L, Rt, E = workloads.lowrank_gaussian_factors(m, n, cfg["k"], cfg["seed"], cfg["noise"])
    A = qmul(L, Rt) + E
    A32 = N(T(A, torch.float32))
    del A, L, Rt, E
    S = Q.Solver(m, n, cfg["c"], cfg["r"], core=Q.CORE_CAR, compute=Q.F32)
    B = torch.empty((4, m, n), dtype=torch.float32, device=DEV)
    S(T(A32, torch.float32), sampling=Q.LENGTH, seed=cfg["seed"], refine_steps=1, B=B)
    q.sync_status()
    ref = oracle.solve(A32, cfg["c"], cfg["r"], "length", "car", seed=cfg["seed"])
    assert N(S.J).astype(np.int64).tolist() == ref["J"].tolist()
    assert N(S.I).astype(np.int64).tolist() == ref["I"].tolist()
    assert N(S.ranks).tolist() == [cfg["c"], cfg["r"]]
    tol = tolerance(Q.F32, ref["C"], ref["R"])
    res = float(N(S.residual)[0])
    assert abs(res - ref["residual"]) <= tol * np.sqrt(fro2(A32))
    # all of C U R, element by element, against the checker's
    Bref = oracle.cur_product(ref["C"], ref["U"], ref["R"])
    err = np.sqrt(fro2(N(B) - Bref) / fro2(Bref))
    assert err < tol, err
