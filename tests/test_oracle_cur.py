"""Pins of the checker's CUR steps: exact recovery (Lemma 1 and the cross
approximation), the least-squares optimality of C^+ X R^+ (Section 3.1),
Theorem 1 and Lemma 3 (Section 3.2), and the residual."""
import itertools

import numpy as np
import pytest

from oracle.quat import qmul, qH, fro2, qrank, spectral_norm, eye
from oracle.pinv import pinv
from oracle.cur import gather, core_wpinv, core_car, cur_product, residual, solve
from tests.qhelp import lowrank_svd_form
import workloads


def _rel(X, Y):
    return np.sqrt(fro2(X - Y)) / np.sqrt(fro2(Y))


def test_cross_approximation_brute_force_6x6_rank2():
    # every (I, J) with |I| = |J| = 2: A = C W^+ R exactly iff rank W = rank A
    rng = np.random.default_rng(21)
    A = qmul(rng.standard_normal((4, 6, 2)), rng.standard_normal((4, 2, 6)))
    assert qrank(A) == 2
    ok = bad = 0
    for I in itertools.combinations(range(6), 2):
        for J in itertools.combinations(range(6), 2):
            C, R, W = gather(A, I, J)
            U, k = core_wpinv(W)
            err = _rel(cur_product(C, U, R), A)
            if qrank(W) == 2:
                assert err < 1e-10, (I, J, err)
                ok += 1
            else:
                bad += 1
    assert ok == 225 and bad == 0   # generic data: every 2x2 intersection has rank 2


def test_cross_approximation_fails_when_intersection_rank_drops():
    rng = np.random.default_rng(22)
    L = rng.standard_normal((4, 6, 2))
    L[:, 4:, 1] = 0          # rows 4 and 5 see only the first factor
    A = qmul(L, rng.standard_normal((4, 2, 6)))
    C, R, W = gather(A, [4, 5], [0, 1])
    assert qrank(W) == 1
    U, k = core_wpinv(W, rtol=1e-10)
    assert k == 1
    assert _rel(cur_product(C, U, R), A) > 1e-3
    # with |I| = |J| = 3 (rank W = 2 again) recovery returns
    C, R, W = gather(A, [0, 4, 5], [0, 1, 2])
    U, k = core_wpinv(W, rtol=1e-10)
    assert k == 2 and _rel(cur_product(C, U, R), A) < 1e-10


def test_lemma1_least_squares_core_recovers_exact_rank():
    rng = np.random.default_rng(23)
    A = qmul(rng.standard_normal((4, 30, 4)), rng.standard_normal((4, 4, 25)))
    I, J = [1, 5, 8, 13, 17, 22, 29], [0, 3, 7, 11, 19, 24]
    C, R, _ = gather(A, I, J)
    assert qrank(C) == qrank(R) == qrank(A) == 4
    U, kc, kr = core_car(A, C, R, rtol=1e-10)
    assert U.shape == (4, len(J), len(I))       # c x r
    assert _rel(cur_product(C, U, R), A) < 1e-11


def test_least_squares_stationarity_and_optimality():
    # C^+ X R^+ minimises ||X - C U R||_F: the gradient C^H (X - CUR) R^H vanishes
    rng = np.random.default_rng(24)
    A = qmul(rng.standard_normal((4, 20, 3)), rng.standard_normal((4, 3, 18)))
    A = A + 0.05 * rng.standard_normal(A.shape)
    C, R, _ = gather(A, [0, 2, 4, 6, 9], [1, 3, 5, 7])
    U, _, _ = core_car(A, C, R)
    G = qmul(qmul(qH(C), A - cur_product(C, U, R)), qH(R))
    assert np.sqrt(fro2(G)) < 1e-10 * np.sqrt(fro2(A))
    base = residual(A, C, U, R)
    for _ in range(5):
        dU = 1e-3 * rng.standard_normal(U.shape)
        assert residual(A, C, U + dU, R) > base


def test_theorem1_and_lemma3_on_noisy_low_rank():
    rng = np.random.default_rng(25)
    m, k = 40, 4
    X, Wk, Vk = lowrank_svd_form(m, m, [10.0, 7.0, 3.0, 1.0], rng)
    I, J = [0, 3, 7, 12, 19, 25, 33], [2, 5, 9, 14, 21, 30]
    C, R, _ = gather(X, I, J)
    # Lemma 3: ||X R^+|| = ||Wk(I,:)^+||,  ||C^+ X|| = ||(Vk(J,:)^H)^+||
    Rp, _ = pinv(R, rtol=1e-10)
    Cp, _ = pinv(C, rtol=1e-10)
    WkI = Wk[:, I, :]
    VkJ = Vk[:, J, :]
    assert spectral_norm(qmul(X, Rp)) == pytest.approx(spectral_norm(pinv(WkI)[0]), rel=1e-8)
    assert spectral_norm(qmul(Cp, X)) == pytest.approx(spectral_norm(pinv(qH(VkJ))[0]), rel=1e-8)
    for sigma in [1e-1, 1e-3, 1e-5]:
        E = sigma * rng.standard_normal(X.shape)
        Xt = X + E
        Ct, Rt, _ = gather(Xt, I, J)
        Ut, _, _ = core_car(Xt, Ct, Rt)
        lhs = spectral_norm(X - cur_product(Ct, Ut, Rt))
        nE = spectral_norm(E)
        bound1 = (spectral_norm(E[:, I, :]) * spectral_norm(qmul(X, Rp))
                  + spectral_norm(E[:, :, J]) * spectral_norm(qmul(Cp, X)) + 3 * nE)
        bound2 = nE * (spectral_norm(pinv(WkI)[0]) + spectral_norm(pinv(VkJ)[0]) + 3)
        assert lhs <= bound1 * (1 + 1e-9)
        assert lhs <= bound2 * (1 + 1e-9)


def test_residual_expansion_identity():
    rng = np.random.default_rng(26)
    A = rng.standard_normal((4, 9, 8))
    C, R, _ = gather(A, [1, 4, 6], [0, 2, 5])
    U = rng.standard_normal((4, 3, 3))
    B = cur_product(C, U, R)
    lhs = residual(A, C, U, R) ** 2
    rhs = fro2(A) - 2 * np.sum(A * B) + fro2(B)
    assert lhs == pytest.approx(rhs, rel=1e-12)
    mask = (rng.random((9, 8)) < 0.5).astype(np.uint8)
    assert residual(A, C, U, R, mask) ** 2 == pytest.approx(fro2((A - B) * mask[None]), rel=1e-13)
    assert residual(A, C, U, R, np.zeros((9, 8), np.uint8)) == 0.0


def test_plain_workload_recovers_to_rounding():
    cfg = workloads.WORKLOADS["plain_f64_256"]
    L, Rt, _ = workloads.lowrank_gaussian_factors(cfg["m"], cfg["n"], cfg["k"], cfg["seed"])
    A = qmul(L, Rt)
    out = solve(A, cfg["c"], cfg["r"], "uniform", "wpinv", seed=cfg["seed"])
    assert out["rank"] == 10
    assert out["rel_err"] < 1e-12
    assert len(np.unique(out["I"])) == 40 and len(np.unique(out["J"])) == 40
