"""Completion from partially observed entries (Algorithm 2) on the GPU
against the checker's loop (MI355X only)."""
import numpy as np
import pytest
import torch

import workloads
from oracle.complete import complete as ref_complete
from oracle.quat import qmul, fro2

pytestmark = pytest.mark.gpu

Q = pytest.importorskip("paper_2402_19147_amd.qcur")
DEV = torch.device("cuda:0")


def T(x, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


def N(t):
    return t.detach().to(torch.float64).cpu().numpy()


def problem(m, n, k, p_obs, c, seed, full_cross=False, noise=0.0):
    L, Rt, E = workloads.lowrank_gaussian_factors(m, n, k, seed, noise)
    A = qmul(L, Rt) + E
    rng = np.random.default_rng(seed)
    mask = (rng.random((m, n)) < p_obs).astype(np.uint8)
    I = np.sort(rng.choice(m, c, replace=False)).astype(np.int64)
    J = np.sort(rng.choice(n, c, replace=False)).astype(np.int64)
    if full_cross:
        mask[I, :] = 1
        mask[:, J] = 1
    Y = np.where(mask[None] == 1, A, rng.standard_normal(A.shape))
    return A, Y, mask, I, J


@pytest.fixture(autouse=True)
def _status_clean():
    Q.sync_status()
    yield
    Q.sync_status()


@pytest.mark.parametrize("compute,tol", [(Q.F64, 1e-9), (Q.F32, 2e-4)])
def test_fixed_steps_match_checker(compute, tol):
    # 150 x 130 (several 64-tiles with ragged edges), rank 4, half observed
    A, Y, mask, I, J = problem(150, 130, 4, 0.5, 12, seed=31, noise=1e-3)
    dt = torch.float64 if compute == Q.F64 else torch.float32
    Yg = T(Y, dt)
    Yc = N(Yg)
    X, iters, rel = Q.complete(Yg, T(mask, torch.uint8), T(I, torch.int64), T(J, torch.int64), compute=compute,
                               max_iter=6, tol=0.0)
    Q.sync_status()
    ref = ref_complete(Yc, mask, I, J, max_iter=6, tol=0.0)
    assert iters == 6
    Xg = N(X)
    assert np.sqrt(fro2(Xg - ref["X"]) / fro2(ref["X"])) < tol
    assert abs(rel - ref["rel"]) <= tol * 10 * max(ref["rel"], 1e-300) + tol
    # observed entries are the observations, bit for bit
    keep = np.broadcast_to(mask[None] == 1, Y.shape)
    assert np.array_equal(Xg[keep], Yc[keep])


def test_stop_between_host_round_trips_matches_checker():
    # Several steps run between host round trips; the stopping rule must
    # still take the first step that meets it (here step 11, inside the
    # second group of steps) and leave that step's iterate in X.
    A, Y, mask, I, J = problem(150, 130, 4, 0.5, 12, seed=34, noise=1e-3)
    rels = [ref_complete(Y, mask, I, J, max_iter=t, tol=0.0)["rel"] for t in range(1, 12)]
    assert rels[10] < 0.99 * min(rels[:10])
    tol = float(np.sqrt(rels[10] * min(rels[:10])))
    ref = ref_complete(Y, mask, I, J, max_iter=100, tol=tol)
    assert ref["iters"] == 11
    X, iters, rel = Q.complete(T(Y), T(mask, torch.uint8), T(I, torch.int64), T(J, torch.int64), compute=Q.F64,
                               max_iter=100, tol=tol)
    Q.sync_status()
    assert iters == 11
    assert abs(rel - ref["rel"]) <= 1e-9 * ref["rel"]
    assert np.sqrt(fro2(N(X) - ref["X"]) / fro2(ref["X"])) < 1e-9


def test_exact_recovery_with_observed_cross():
    A, Y, mask, I, J = problem(130, 110, 3, 0.25, 8, seed=32, full_cross=True)
    X, iters, rel = Q.complete(T(Y), T(mask, torch.uint8), T(I, torch.int64), T(J, torch.int64), compute=Q.F64,
                               max_iter=400, tol=1e-12)
    Q.sync_status()
    ref = ref_complete(Y, mask, I, J, max_iter=400, tol=1e-12)
    assert rel <= 1e-12 and iters < 400
    assert abs(iters - ref["iters"]) <= 1
    assert np.sqrt(fro2(N(X) - A) / fro2(A)) < 1e-9


def test_stopping_and_degenerate_cases():
    A, Y, mask, I, J = problem(90, 70, 3, 0.4, 8, seed=33, full_cross=True)
    X, iters, rel = Q.complete(T(Y), T(mask, torch.uint8), T(I, torch.int64), T(J, torch.int64), max_iter=200,
                               tol=1e-4)
    assert iters < 200 and rel <= 1e-4
    # every entry observed: one step, X = Y
    full = np.ones_like(mask)
    X, iters, rel = Q.complete(T(A), T(full, torch.uint8), T(I, torch.int64), T(J, torch.int64), max_iter=50,
                               tol=1e-4)
    assert iters == 1 and rel == 0.0
    assert np.array_equal(N(X), A)
    # no step: the observed entries with zeros elsewhere
    X, iters, rel = Q.complete(T(Y), T(mask, torch.uint8), T(I, torch.int64), T(J, torch.int64), max_iter=0)
    assert iters == 0
    assert np.array_equal(N(X), np.where(mask[None] == 1, Y, 0.0))
    Q.sync_status()


@pytest.mark.parametrize("sampling,name", [(Q.LENGTH, "length"), (Q.UNIFORM, "uniform")])
def test_resampled_steps_match_checker(sampling, name):
    # index sets drawn again from every iterate: the same draws as the
    # checker's (exact integer sampler) and the same iterates
    from oracle.complete import complete_resampled as ref_resampled
    A, Y, mask, _, _ = problem(150, 130, 4, 0.5, 12, seed=41, noise=1e-3)
    X, iters, rel, I, J = Q.complete_resampled(T(Y), T(mask, torch.uint8), 14, 12, sampling=sampling, seed=77,
                                               compute=Q.F64, max_iter=5, tol=0.0)
    Q.sync_status()
    ref = ref_resampled(Y, mask, 14, 12, name, seed=77, max_iter=5, tol=0.0)
    assert iters == 5
    assert np.array_equal(N(I).astype(np.int64), ref["I"]) and np.array_equal(N(J).astype(np.int64), ref["J"])
    assert np.sqrt(fro2(N(X) - ref["X"]) / fro2(ref["X"])) < 1e-9
    assert abs(rel - ref["rel"]) <= 1e-8 * ref["rel"] + 1e-12


def test_resampled_fp32_first_step_and_convergence():
    from oracle.complete import complete_resampled as ref_resampled
    A, Y, mask, _, _ = problem(130, 110, 3, 0.6, 10, seed=42)
    Yg = T(Y, torch.float32)
    X, iters, rel, I, J = Q.complete_resampled(Yg, T(mask, torch.uint8), 10, 10, seed=5, compute=Q.F32, max_iter=1,
                                               tol=0.0)
    Q.sync_status()
    ref = ref_resampled(N(Yg), mask, 10, 10, "length", seed=5, max_iter=1, tol=0.0)
    assert np.array_equal(N(I).astype(np.int64), ref["I"]) and np.array_equal(N(J).astype(np.int64), ref["J"])
    assert np.sqrt(fro2(N(X) - ref["X"]) / fro2(ref["X"])) < 2e-4
    # the rank-3 matrix with 40% of its entries missing is recovered
    X, iters, rel, I, J = Q.complete_resampled(T(Y), T(mask, torch.uint8), 10, 10, seed=5, compute=Q.F64,
                                               max_iter=300, tol=1e-10)
    Q.sync_status()
    miss = np.broadcast_to(mask[None] == 0, A.shape)
    assert np.linalg.norm((N(X) - A)[miss]) / np.linalg.norm(A[miss]) < 1e-6
