"""The benchmark workloads at full size on the MI355X against the FP64
reference checker: the colour-image-shaped 1024 x 1024 solve (FP64, FP32,
BF16 operands with one refinement step) and the dense 4096 x 4096 solve
(FP32 products with one refinement step, FP64 pseudoinverses).  Draws are
compared bit for bit; products within tolerances that follow the
conditioning of C and R (rounding of the operands is amplified by kappa)."""
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
    k = kappa(C) + kappa(R)
    u = {Q.F64: 2.0 ** -52, Q.F32: 2.0 ** -24, Q.BF16: 2.0 ** -9, Q.BF16X3: 2.0 ** -16}[compute]
    floor = {Q.F64: 1e-12, Q.F32: 1e-5, Q.BF16: 2e-2, Q.BF16X3: 1e-4}[compute]
    return max(floor, 10 * u * k)


@pytest.fixture(scope="module")
def color():
    cfg = workloads.WORKLOADS["color_1024"]
    A = workloads.color_like(cfg["m"], cfg["n"], cfg["k"], cfg["seed"], cfg["noise"])
    ref = oracle.solve(A, cfg["c"], cfg["r"], "length", "car", seed=cfg["seed"])
    return cfg, A, ref


@pytest.mark.parametrize("compute,refine", [(Q.F64, 0), (Q.F32, 0), (Q.F32, 1), (Q.BF16, 1), (Q.BF16X3, 0)])
def test_color_workload(color, compute, refine):
    cfg, A, ref = color
    dt = torch.float64 if compute == Q.F64 else torch.float32
    Ad = N(T(A, dt))
    out = q.solve(T(A, dt), cfg["c"], cfg["r"], sampling=Q.LENGTH, core=Q.CORE_CAR, compute=compute,
                  seed=cfg["seed"], refine_steps=refine, want_B=True)
    q.sync_status()
    if compute == Q.F64:
        refd = ref
    else:  # the checker on the same (rounded) input
        refd = oracle.solve(Ad, cfg["c"], cfg["r"], "length", "car", seed=cfg["seed"])
    assert N(out["J"]).astype(np.int64).tolist() == refd["J"].tolist()
    assert N(out["I"]).astype(np.int64).tolist() == refd["I"].tolist()
    Bref = oracle.cur_product(refd["C"], refd["U"], refd["R"])
    err = np.sqrt(fro2(N(out["B"]) - Bref) / fro2(Bref))
    assert err < tolerance(compute, refd["C"], refd["R"]), err
    res = float(N(out["residual"])[0])
    assert abs(res - refd["residual"]) <= tolerance(compute, refd["C"], refd["R"]) * np.sqrt(fro2(Ad))


@pytest.mark.slow
def test_dense_workload_f32_refined():
    cfg = workloads.WORKLOADS["dense_4096"]
    L, Rt, E = workloads.lowrank_gaussian_factors(cfg["m"], cfg["n"], cfg["k"], cfg["seed"], cfg["noise"])
    A = qmul(L, Rt) + E
    A32 = N(T(A, torch.float32))
    S = Q.Solver(cfg["m"], cfg["n"], cfg["c"], cfg["r"], core=Q.CORE_CAR, compute=Q.F32)
    S(T(A32, torch.float32), sampling=Q.LENGTH, seed=cfg["seed"], refine_steps=1)
    q.sync_status()
    ref = oracle.solve(A32, cfg["c"], cfg["r"], "length", "car", seed=cfg["seed"])
    assert N(S.J).astype(np.int64).tolist() == ref["J"].tolist()
    assert N(S.I).astype(np.int64).tolist() == ref["I"].tolist()
    assert N(S.ranks).tolist() == [cfg["c"], cfg["r"]]
    tol = tolerance(Q.F32, ref["C"], ref["R"])
    res = float(N(S.residual)[0])
    assert abs(res - ref["residual"]) <= tol * np.sqrt(fro2(A32))
    # the core itself, compared through C U R on a sample of 4096 entries
    rng = np.random.default_rng(0)
    ii = rng.integers(0, cfg["m"], 4096)
    jj = rng.integers(0, cfg["n"], 4096)
    U = N(S.U)
    CU = qmul(ref["C"][:, ii, :], U)          # (4, 4096, r) rows of C U
    CUr = qmul(ref["C"][:, ii, :], ref["U"])
    Rj = ref["R"][:, :, jj]
    def entries(X):
        out = np.empty((4, len(ii)))
        for t in range(len(ii)):
            out[:, t] = qmul(X[:, t:t + 1, :], Rj[:, :, t:t + 1])[:, 0, 0]
        return out
    b, br = entries(CU), entries(CUr)
    assert np.sqrt(np.sum((b - br) ** 2) / np.sum(br ** 2)) < tol
