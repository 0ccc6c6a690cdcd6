"""Theorem 1 experiment (Section 3.2, Example 4.1) on the GPU against the
checker (MI355X only): the construction of X = W_k Sigma_k V_k^H from polar
factors, the errors and bound terms of one noise level on identical inputs,
and at the example's full size (500 x 500, k = 50) the bound and the linear
growth of the error with ||E||_2."""
import math

import numpy as np
import pytest
import torch

import workloads
from oracle.perturbation import lowrank_product as ref_lowrank
from oracle.perturbation import perturbation_errors as ref_errors
from oracle.perturbation import polar_factor as ref_polar
from oracle.quat import fro2

pytestmark = pytest.mark.gpu

Q = pytest.importorskip("paper_2402_19147_amd.qcur")
P = pytest.importorskip("paper_2402_19147_amd.perturbation")
DEV = torch.device("cuda:0")


def T(x, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


def N(t):
    return t.detach().to(torch.float64).cpu().numpy()


@pytest.fixture(autouse=True)
def _status_clean():
    Q.sync_status()
    yield
    Q.sync_status()


def test_construction_matches_checker():
    # 70 x 61 with k = 6: ragged against every tile size
    GW, GV, sig, _ = workloads.perturbation_factors(70, 61, 6, seed=21)
    W, V = P.polar_factor(T(GW)), P.polar_factor(T(GV))
    X = P.lowrank_product(W, torch.tensor(sig), V)
    Wr, Vr = ref_polar(GW), ref_polar(GV)
    Xr = ref_lowrank(Wr, sig, Vr)
    assert np.abs(N(W) - Wr).max() < 1e-12
    assert np.abs(N(V) - Vr).max() < 1e-12
    assert math.sqrt(fro2(N(X) - Xr) / fro2(Xr)) < 1e-12


@pytest.mark.parametrize("sampling,sigma", [("length", 1e-1), ("length", 1e-3), ("uniform", 3e-2)])
def test_one_noise_level_matches_checker(sampling, sigma):
    m, n, k = 72, 66, 6
    GW, GV, sig, E0 = workloads.perturbation_factors(m, n, k, seed=22)
    Wr, Vr = ref_polar(GW), ref_polar(GV)
    Xr = ref_lowrank(Wr, sig, Vr)
    c = r = Q.sample_size(k, min(m, n))
    s = sigma
    smode = Q.LENGTH if sampling == "length" else Q.UNIFORM
    out = P.perturbation_errors(T(Xr), T(E0), s, T(Wr), T(Vr), c, r, smode, seed=5)
    Q.sync_status()
    ref = ref_errors(Xr, s * E0, Wr, Vr, c, r, sampling, seed=5)
    assert np.array_equal(N(out["I"]).astype(np.int64), ref["I"])
    assert np.array_equal(N(out["J"]).astype(np.int64), ref["J"])
    for key in ("err", "norm_E", "w_pinv", "v_pinv", "bound"):
        assert out[key] == pytest.approx(ref[key], rel=1e-9), key
    assert out["err"] <= out["bound"]


def test_example_4_1_full_size():
    # X = W_k Sigma_k V_k^H, 500 x 500, k = 50, c = r = ceil(50 ln 50) = 196,
    # noise levels (standard deviations) 1e-1 .. 1e-6
    m = n = 500
    k = 50
    GW, GV, sig, E0 = workloads.perturbation_factors(m, n, k, seed=11)
    W, V = P.polar_factor(T(GW)), P.polar_factor(T(GV))
    X = P.lowrank_product(W, torch.tensor(sig), V)
    c = r = Q.sample_size(k, m)
    assert c == 196
    E0g = T(E0)
    nE0 = P.spectral_norm(E0g)
    rows = []
    for sigma in (1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6):
        out = P.perturbation_errors(X, E0g, sigma, W, V, c, r, Q.LENGTH, seed=3, norm_E0=nE0)
        Q.sync_status()
        assert out["err"] <= out["bound"], sigma
        rows.append((out["norm_E"], out["err"]))
    # linear in ||E||_2: the log-log slope over the six levels is one
    x = np.log([a for a, _ in rows])
    y = np.log([b for _, b in rows])
    slope = np.polyfit(x, y, 1)[0]
    assert 0.9 < slope < 1.1
