"""Parity of every libqcur call with the FP64 CPU reference checker on the
same seeded inputs (MI355X only).  Integer, index and copy results are
compared bit for bit; floating-point results within the stated relative
Frobenius tolerances (FP64 1e-12 unless conditioning says otherwise, FP32
1e-5, BF16 operands 2e-2)."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import workloads
from oracle.quat import qmul, qH, fro2

pytestmark = pytest.mark.gpu

Q = pytest.importorskip("paper_2402_19147_amd.qcur")
DEV = torch.device("cuda:0")


def T(x, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


def N(t):
    return t.detach().to(torch.float64).cpu().numpy()


def rel(x, ref):
    d = np.sqrt(fro2(np.asarray(x, dtype=np.float64) - ref))
    return d / max(np.sqrt(fro2(ref)), 1e-300)


def kappa(X):
    from oracle.pinv import singular_values
    sv = singular_values(X)
    sv = sv[sv > sv[0] * 1e-13]
    return float(sv[0] / sv[-1])


def cur_tol(C, R, floor=1e-12):
    """FP64 tolerance for U-invariant products: the projectors C C^+ and
    R^+ R are only determined to about eps * kappa."""
    return max(floor, 10 * 2.0 ** -52 * (kappa(C) + kappa(R)))


def bf16_round(x):
    return torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()


@pytest.fixture(autouse=True)
def _status_clean():
    Q.sync_status()
    yield
    Q.sync_status()


# ---------------------------------------------------------------- qgemm
GEMM_SHAPES = [(1, 1, 1), (16, 4, 16), (70, 37, 45), (130, 50, 70), (64, 1024, 64), (200, 96, 33), (72, 40, 88),
               (136, 200, 104)]


@pytest.mark.parametrize("M,K,Nn", GEMM_SHAPES)
@pytest.mark.parametrize("compute", [Q.F64, Q.F32, Q.BF16, Q.BF16X3])
@pytest.mark.parametrize("opA,opB", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm_small_integers_bit_exact(M, K, Nn, compute, opA, opB):
    rng = np.random.default_rng(M * 1000 + K * 10 + Nn + opA * 3 + opB)
    lim = 2 if K > 64 else 4
    A = workloads.small_int_quat(M, K, rng, lim) if opA == 0 else workloads.small_int_quat(K, M, rng, lim)
    B = workloads.small_int_quat(K, Nn, rng, lim) if opB == 0 else workloads.small_int_quat(Nn, K, rng, lim)
    Ae = A if opA == 0 else qH(A)
    Be = B if opB == 0 else qH(B)
    ref = qmul(Ae, Be)
    tdt = {Q.F64: torch.float64, Q.F32: torch.float32, Q.BF16: torch.bfloat16, Q.BF16X3: torch.float32}[compute]
    D = Q.gemm(T(A, tdt), T(B, tdt), opA=opA, opB=opB, compute=compute)
    assert np.array_equal(N(D), ref)


@pytest.mark.parametrize("M,K,Nn", [(896, 72, 960), (900, 64, 963), (896, 70, 960)])
@pytest.mark.parametrize("opA,opB", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm_bf16_64_tiles_bit_exact(M, K, Nn, opA, opB):
    # enough 64-tiles to select them: interior tiles take the unconditional
    # vector loads (K = 72: a last K slice of 8 valid columns; K = 70: only
    # the x-contiguous operands qualify), ragged M and N the guarded loads
    rng = np.random.default_rng(M + K + Nn + 2 * opA + opB)
    A = workloads.small_int_quat(M, K, rng, 4) if opA == 0 else workloads.small_int_quat(K, M, rng, 4)
    B = workloads.small_int_quat(K, Nn, rng, 4) if opB == 0 else workloads.small_int_quat(Nn, K, rng, 4)
    ref = qmul(A if opA == 0 else qH(A), B if opB == 0 else qH(B))
    D = Q.gemm(T(A, torch.bfloat16), T(B, torch.bfloat16), opA=opA, opB=opB, compute=Q.BF16)
    assert np.array_equal(N(D), ref)


@pytest.mark.parametrize("M,K,Nn", [(200, 1024, 200), (37, 301, 45), (256, 1024, 256), (1, 64, 1), (16, 4099, 16),
                                    (200, 800, 13), (400, 4096, 400), (512, 2051, 300)])
@pytest.mark.parametrize("compute,tol", [(Q.F64, 1e-13), (Q.F32, 1e-5)])
def test_gemm_thin_hn(M, K, Nn, compute, tol):
    # A^H B with a long K and a small output: the fragment-streaming kernel
    # (ragged 16-blocks, K not a multiple of 4, several K splits)
    rng = np.random.default_rng(M + K + Nn)
    dt = torch.float64 if compute == Q.F64 else torch.float32
    A = N(T(rng.standard_normal((4, K, M)), dt))
    B = N(T(rng.standard_normal((4, K, Nn)), dt))
    D0 = N(T(rng.standard_normal((4, M, Nn)), dt))
    Dt = T(D0, dt)
    Q.gemm(T(A, dt), T(B, dt), opA=1, opB=0, alpha=0.75, beta=-1.5, D=Dt, compute=compute)
    ref = 0.75 * qmul(qH(A), B) - 1.5 * D0
    assert rel(N(Dt), ref) < tol
    Ai = workloads.small_int_quat(K, M, rng, 2)
    Bi = workloads.small_int_quat(K, Nn, rng, 2)
    assert np.array_equal(N(Q.gemm(T(Ai, dt), T(Bi, dt), opA=1, opB=0, compute=compute)), qmul(qH(Ai), Bi))


@pytest.mark.parametrize("M,K,Nn", [(1024, 200, 200), (1000, 64, 37), (777, 256, 250), (512, 4, 16), (600, 70, 40),
                                    (4096, 400, 400), (900, 512, 512), (700, 300, 333), (1500, 128, 64),
                                    (2000, 36, 50)])
def test_gemm_f64_tall_nh(M, K, Nn):
    # FP64 A B^H with a tall output and a short K: the run-streaming kernel
    # (ragged 16-blocks, K at its limit; K = 70 is not a multiple of 4 and
    # takes the tiled kernel)
    rng = np.random.default_rng(M + 3 * K + Nn)
    A = rng.standard_normal((4, M, K))
    B = rng.standard_normal((4, Nn, K))
    D0 = rng.standard_normal((4, M, Nn))
    Dt = T(D0)
    Q.gemm(T(A), T(B), opA=0, opB=1, alpha=-0.5, beta=0.25, D=Dt, compute=Q.F64)
    assert rel(N(Dt), -0.5 * qmul(A, qH(B)) + 0.25 * D0) < 1e-13
    Ai = workloads.small_int_quat(M, K, rng, 3)
    Bi = workloads.small_int_quat(Nn, K, rng, 3)
    assert np.array_equal(N(Q.gemm(T(Ai), T(Bi), opA=0, opB=1, compute=Q.F64)), qmul(Ai, qH(Bi)))


@pytest.mark.parametrize("M,K,Nn", [(2048, 1024, 400), (2100, 1030, 333), (4096, 4096, 400)])
@pytest.mark.parametrize("compute", [Q.F32, Q.F64])
def test_gemm_tall_long_k_plans(M, K, Nn, compute):
    # tall outputs with a long K take 64 x 80 tiles (FP32) and more K slices:
    # ragged edges in both directions, bit-exact on small integers
    rng = np.random.default_rng(M + K + Nn)
    dt = torch.float64 if compute == Q.F64 else torch.float32
    Ai = workloads.small_int_quat(M, K, rng, 1)
    Bi = workloads.small_int_quat(K, Nn, rng, 1)
    D = Q.gemm(T(Ai, dt), T(Bi, dt), compute=compute)
    assert np.array_equal(N(D), qmul(Ai, Bi))
    if M * K <= 4 * 10 ** 6:
        A = rng.standard_normal((4, M, K))
        B = rng.standard_normal((4, K, Nn))
        D0 = rng.standard_normal((4, M, Nn))
        Dt = T(D0, dt)
        Q.gemm(T(A, dt), T(B, dt), alpha=0.5, beta=2.0, D=Dt, compute=compute)
        ref = 0.5 * qmul(N(T(A, dt)), N(T(B, dt))) + 2.0 * N(T(D0, dt))
        assert rel(N(Dt), ref) < (1e-13 if compute == Q.F64 else 1e-5)


@pytest.mark.parametrize("compute,tol", [(Q.F64, 1e-13), (Q.F32, 1e-5), (Q.BF16, 2e-2), (Q.BF16X3, 1e-4)])
def test_gemm_gaussian_alpha_beta(compute, tol):
    rng = np.random.default_rng(7)
    A = rng.standard_normal((4, 150, 90))
    B = rng.standard_normal((4, 90, 77))
    D0 = rng.standard_normal((4, 150, 77))
    tdt = {Q.F64: torch.float64, Q.F32: torch.float32, Q.BF16: torch.bfloat16, Q.BF16X3: torch.float32}[compute]
    odt = torch.float64 if compute == Q.F64 else torch.float32
    Dt = T(D0, odt)
    Q.gemm(T(A, tdt), T(B, tdt), alpha=-0.5, beta=2.0, D=Dt, compute=compute)
    if compute == Q.BF16:
        ref = -0.5 * qmul(bf16_round(A), bf16_round(B)) + 2.0 * D0
    elif compute == Q.BF16X3:
        ref = -0.5 * qmul(N(T(A, torch.float32)), N(T(B, torch.float32))) + 2.0 * N(T(D0, torch.float32))
    else:
        ref = -0.5 * qmul(A, B) + 2.0 * D0
    assert rel(N(Dt), ref) < tol


@pytest.mark.parametrize("opA,opB", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm_split_bf16_error(opA, opB):
    # hi + lo halves carry about 16 bits of each FP32 operand: the product
    # error stays near 2^-16, far below BF16's 2^-9, at split-K sizes
    rng = np.random.default_rng(70 + 2 * opA + opB)
    M, K, Nn = 300, 1024, 200
    A = rng.standard_normal((4, M, K) if opA == 0 else (4, K, M))
    B = rng.standard_normal((4, K, Nn) if opB == 0 else (4, Nn, K))
    A32, B32 = N(T(A, torch.float32)), N(T(B, torch.float32))
    ref = qmul(A32 if opA == 0 else qH(A32), B32 if opB == 0 else qH(B32))
    D = Q.gemm(T(A, torch.float32), T(B, torch.float32), opA=opA, opB=opB, compute=Q.BF16X3)
    err = rel(N(D), ref)
    assert err < 4e-5, err
    Db = Q.gemm(T(A, torch.bfloat16), T(B, torch.bfloat16), opA=opA, opB=opB, compute=Q.BF16)
    assert err < rel(N(Db), ref) / 20


def test_gemm_strided_views():
    rng = np.random.default_rng(8)
    big = rng.standard_normal((4, 100, 120))
    A = big[:, 10:80, 5:65]            # 70 x 60 view with ld 120
    B = rng.standard_normal((4, 60, 40))
    At = T(big)[:, 10:80, 5:65]
    D = Q.gemm(At, T(B))
    assert rel(N(D), qmul(A, B)) < 1e-13


# ---------------------------------------------------------------- probs / draw / gather
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_probs_length_and_uniform(dtype):
    A = workloads.color_like(300, 517, 7, seed=3)
    Ad = N(T(A, dtype))
    p, q, f2 = Q.probs(T(A, dtype), Q.LENGTH)
    pr, qr, fr = oracle.probs_length(Ad)
    assert np.allclose(N(p), pr, rtol=1e-12, atol=0)
    assert np.allclose(N(q), qr, rtol=1e-12, atol=0)
    assert abs(float(N(f2)[0]) - fr) <= 1e-13 * fr
    p, q, _ = Q.probs(T(A, dtype), Q.UNIFORM)
    pu, qu = oracle.probs_uniform(300, 517)
    assert np.array_equal(N(p), pu) and np.array_equal(N(q), qu)


def test_probs_deterministic():
    A = T(workloads.color_like(257, 1000, 5, seed=4))
    p1, q1, _ = Q.probs(A)
    p2, q2, _ = Q.probs(A)
    assert torch.equal(p1, p2) and torch.equal(q1, q2)


def test_draw_golden_cases():
    with open(os.path.join(os.path.dirname(__file__), "golden", "draws.json")) as f:
        cases = json.load(f)
    for c in cases:
        p = np.array([float.fromhex(x) for x in c["p"]])
        idx = Q.draw(T(p), c["count"], c["seed"], c["set_id"], c["with_replacement"])
        assert N(idx).astype(np.int64).tolist() == c["idx"], c["name"]


@pytest.mark.parametrize("n,count,repl", [(1, 1, False), (64, 64, False), (65, 3, False), (4096, 400, False),
                                          (5000, 4999, False), (16384, 100, False), (777, 2000, True),
                                          (8192, 50, True)])
def test_draw_matches_checker(n, count, repl):
    rng = np.random.default_rng(n + count)
    w = rng.random(n) ** 3
    w[rng.random(n) < 0.1] = 0.0
    if not repl and (w > 0).sum() < count:
        w[:count] = 1.0
    p = w / w.sum()
    idx = Q.draw(T(p), count, seed=n, set_id=3, with_replacement=repl)
    ref = oracle.draw(p, count, n, 3, repl)
    assert torch.equal(idx.cpu(), torch.tensor(ref))


def test_draw_errors_raise_sample_status():
    p = T(np.array([0.5, 0.0, 0.5]))
    idx = Q.draw(p, 3, 1, 0)           # only two positive weights
    with pytest.raises(Q.QcurError) as e:
        Q.sync_status()
    assert e.value.status == 5
    assert (N(idx) == -1).all()
    Q.draw(T(np.array([0.5, np.nan, 0.5])), 1, 1, 0)
    with pytest.raises(Q.QcurError):
        Q.sync_status()


def test_probs_zero_matrix_raises_numeric():
    Q.probs(torch.zeros((4, 5, 6), dtype=torch.float64, device=DEV))
    with pytest.raises(Q.QcurError) as e:
        Q.sync_status()
    assert e.value.status == 6


@pytest.mark.parametrize("compute", [Q.F64, Q.F32])
def test_approx_nonfinite_factor_raises_numeric(compute):
    # C large enough for the CholeskyQR group, whose FP64 cast checks every
    # element; one NaN must reach the status word
    rng = np.random.default_rng(31)
    A = rng.standard_normal((4, 300, 260))
    C = np.ascontiguousarray(A[:, :, :40])
    R = np.ascontiguousarray(A[:, :40, :])
    C[2, 17, 5] = np.nan
    dt = torch.float64 if compute == Q.F64 else torch.float32
    Q.approx(T(A, dt), T(C, dt), T(R, dt), None, core=Q.CORE_CAR, compute=compute)
    with pytest.raises(Q.QcurError) as e:
        Q.sync_status()
    assert e.value.status == 6


@pytest.mark.parametrize("out_dt", [torch.float64, torch.float32, torch.bfloat16])
def test_gather_bit_exact(out_dt):
    rng = np.random.default_rng(9)
    A = rng.standard_normal((4, 123, 301))
    I = np.sort(rng.choice(123, 17, replace=False))
    J = np.sort(rng.choice(301, 29, replace=False))
    C, R, W = Q.gather(T(A), T(I, torch.int64), T(J, torch.int64), dtype=out_dt)
    Cr, Rr, Wr = oracle.gather(A, I, J)
    conv = (lambda x: x) if out_dt == torch.float64 else (
        lambda x: torch.tensor(x).to(out_dt).to(torch.float64).numpy())
    assert np.array_equal(N(C), conv(Cr)) and np.array_equal(N(R), conv(Rr)) and np.array_equal(N(W), conv(Wr))


def test_gather_out_of_range_flags_arg():
    A = T(np.ones((4, 5, 5)))
    Q.gather(A, T(np.array([0, 7]), torch.int64), T(np.array([1]), torch.int64))
    with pytest.raises(Q.QcurError) as e:
        Q.sync_status()
    assert e.value.status == 1


# ---------------------------------------------------------------- pinv
@pytest.mark.parametrize("p,q", [(1, 1), (7, 7), (40, 40), (60, 13), (13, 60), (300, 70), (70, 300), (257, 129)])
def test_pinv_full_rank(p, q):
    rng = np.random.default_rng(p * q)
    X = rng.standard_normal((4, p, q))
    Xp, rank = Q.pinv(T(X))
    ref, k = oracle.qpinv(X)
    assert int(N(rank)[0]) == k == min(p, q)
    assert rel(N(Xp), ref) < 1e-11


@pytest.mark.parametrize("p,q,k", [(40, 40, 10), (90, 50, 7), (50, 90, 7), (200, 150, 30)])
def test_pinv_exact_rank(p, q, k):
    rng = np.random.default_rng(p + q + k)
    X = qmul(rng.standard_normal((4, p, k)), rng.standard_normal((4, k, q)))
    Xp, rank = Q.pinv(T(X))
    ref, kr = oracle.qpinv(X)
    assert int(N(rank)[0]) == kr == k
    assert rel(N(Xp), ref) < 1e-10
    G = N(Xp)
    assert rel(qmul(qmul(X, G), X), X) < 1e-11


def test_pinv_max_rank_and_rtol():
    rng = np.random.default_rng(12)
    from tests.qhelp import lowrank_svd_form
    X, _, _ = lowrank_svd_form(30, 20, [9.0, 5.0, 2.0, 1e-2, 1e-9], rng)
    from oracle.pinv import singular_values
    sv = singular_values(X)
    for rtol, mr in [(-1.0, 0), (1e-5, 0), (1e-1, 0), (-1.0, 2)]:
        Xp, rank = Q.pinv(T(X), rtol, mr)
        ref, k = oracle.qpinv(X, rtol, mr)
        assert int(N(rank)[0]) == k
        # both sides carry ~eps * kappa error in the smallest kept singular pair
        tol = max(1e-11, 64 * 2.0 ** -52 * sv[0] / sv[k - 1])
        assert rel(N(Xp), ref) < tol


@pytest.mark.parametrize("p,q", [(1024, 200), (200, 1024), (2048, 256)])
def test_pinv_fast_path_shapes(p, q):
    # numerically full rank: the CholeskyQR2 path with its certificate
    rng = np.random.default_rng(p + 7 * q)
    X = qmul(rng.standard_normal((4, p, 40)), rng.standard_normal((4, 40, q))) + 0.05 * rng.standard_normal((4, p, q))
    Xp, rank = Q.pinv(T(X))
    ref, k = oracle.qpinv(X)
    assert int(N(rank)[0]) == k == min(p, q)
    assert rel(N(Xp), ref) < max(1e-11, 64 * 2.0 ** -52 * kappa(X))


def test_pinv_ill_conditioned_falls_back():
    # kappa = 1e9 > the CholeskyQR2 limit: the Jacobi path must take over
    rng = np.random.default_rng(14)
    from tests.qhelp import lowrank_svd_form
    X, _, _ = lowrank_svd_form(300, 70, np.logspace(0, -9, 70), rng)
    Xp, rank = Q.pinv(T(X))
    ref, k = oracle.qpinv(X)
    assert int(N(rank)[0]) == k == 70
    assert rel(N(Xp), ref) < 64 * 2.0 ** -52 * 1e9
    Xp2, rank2 = Q.pinv(T(X), max_rank=20)      # no gap at the cap: subspace iteration gives way to Jacobi
    ref2, k2 = oracle.qpinv(X, max_rank=20)
    assert int(N(rank2)[0]) == k2 == 20
    assert rel(N(Xp2), ref2) < 1e-9


@pytest.mark.parametrize("p,q,k,mr", [(256, 256, 64, 0), (300, 230, 45, 0)])
def test_pinv_rank_deficient_deflated_jacobi(p, q, k, mr):
    # exact-rank products of Gaussian factors (the differentiation workload's
    # W = A(I, J)): multi-launch Jacobi sweeps with the pairs of rounding-noise
    # columns left unrotated
    rng = np.random.default_rng(p + q + k)
    X = qmul(rng.standard_normal((4, p, k)), rng.standard_normal((4, k, q)))
    Xp, rank = Q.pinv(T(X), max_rank=mr)
    ref, kr = oracle.qpinv(X, max_rank=mr)
    assert int(N(rank)[0]) == kr == k
    assert rel(N(Xp), ref) < 1e-10
    assert rel(qmul(qmul(X, N(Xp)), X), X) < 1e-11


@pytest.mark.parametrize("p,q,k,mr,noise", [
    (256, 256, 64, 64, 0.0),      # the differentiation workload's W = A(I, J): exact rank 64
    (256, 256, 64, 64, "f32"),    # the same with FP32-rounded entries (a tail near 1e-7 of sigma_1)
    (400, 300, 40, 40, 1e-9),     # tall, rank 40 plus a small full-rank tail
    (200, 520, 30, 30, 0.0),      # wide
    (256, 256, 64, 20, 0.0),      # a cap below the rank cuts into the spectrum
    (256, 256, 40, 64, 0.0),      # rank below the cap: the sketch is rank-deficient, Jacobi takes over
])
def test_pinv_rank_capped_subspace_route(p, q, k, mr, noise):
    # a rank cap k with 2k <= min(p, q): subspace iteration with its a posteriori
    # bound, else the Jacobi SVD; either way the truncated pseudoinverse
    rng = np.random.default_rng(p + 3 * q + k + mr)
    X = qmul(rng.standard_normal((4, p, k)), rng.standard_normal((4, k, q)))
    if noise == "f32":
        X = X.astype(np.float32).astype(np.float64)
    elif noise:
        X = X + noise * rng.standard_normal(X.shape)
    Xp, rank = Q.pinv(T(X), max_rank=mr)
    ref, kr = oracle.qpinv(X, max_rank=mr)
    assert int(N(rank)[0]) == kr == min(k, mr)
    from oracle.pinv import singular_values
    sv = singular_values(X)
    # the kept pairs carry ~eps * sigma_1 / sigma_k; a cut inside the spectrum
    # also moves the subspace by ~eps * sigma_1 / (sigma_k - sigma_{k+1})
    gap = sv[kr - 1] - sv[kr] if kr < len(sv) else sv[kr - 1]
    tol = max(1e-10, 64 * 2.0 ** -52 * sv[0] ** 2 / (sv[kr - 1] * gap))
    assert rel(N(Xp), ref) < tol


@pytest.mark.parametrize("shape,k,mr", [((256, 256), 64, 64), ((300, 230), 45, 0), ((1024, 200), 0, 0),
                                        ((300, 70), 0, 20)])
def test_pinv_and_svd_run_twice_bitwise(shape, k, mr):
    # the same input twice gives the same bits: the CholeskyQR path (fixed-order
    # reductions), the multi-launch Jacobi sweeps of a rank-deficient matrix
    # (every workgroup of a round reads the same negligible-pair bound) and
    # the rank-capped route; the thin SVD likewise
    p, q = shape
    rng = np.random.default_rng(p + 7 * q + k)
    X = (qmul(rng.standard_normal((4, p, k)), rng.standard_normal((4, k, q))) if k
         else rng.standard_normal((4, p, q)))
    Xt = T(X)
    runs = [Q.pinv(Xt, max_rank=mr) for _ in range(2)]
    Q.sync_status()
    assert torch.equal(runs[0][0], runs[1][0]) and torch.equal(runs[0][1], runs[1][1])
    svds = [Q.svd(Xt) for _ in range(2)]
    Q.sync_status()
    for a, b in zip(svds[0], svds[1]):
        assert torch.equal(a, b)


# ---------------------------------------------------------------- thin QSVD
def _qH(X):
    Y = np.swapaxes(X, 1, 2).copy()
    Y[1:] *= -1
    return Y


@pytest.mark.parametrize("p,q,k", [(1, 1, 0), (7, 5, 0), (40, 40, 0), (60, 13, 0), (13, 60, 0), (300, 70, 0),
                                   (70, 300, 0), (257, 129, 0), (200, 150, 30)])
def test_svd_matches_checker(p, q, k):
    # singular values against the checker; U, V orthonormal on the nonzero
    # singular values and U diag(s) V^H = X
    from oracle.pinv import singular_values
    rng = np.random.default_rng(p * 1000 + q + k)
    X = (qmul(rng.standard_normal((4, p, k)), rng.standard_normal((4, k, q))) if k
         else rng.standard_normal((4, p, q)))
    s, U, V = Q.svd(T(X))
    Q.sync_status()
    s, U, V = N(s), N(U), N(V)
    sv = singular_values(X)
    n = min(p, q)
    assert s.shape == (n,) and np.all(np.diff(s) <= 0)
    keep = sv > 1e-10 * sv[0]
    assert np.max(np.abs(s[keep] - sv[keep]) / sv[keep]) < 1e-12
    assert np.all(s[~keep] < 1e-10 * sv[0])
    nk = int(keep.sum())
    G = qmul(_qH(U[:, :, :nk]), U[:, :, :nk])
    H = qmul(_qH(V[:, :, :nk]), V[:, :, :nk])
    E = np.zeros_like(G)
    E[0] = np.eye(nk)
    assert np.abs(G - E).max() < 1e-12 and np.abs(H - E).max() < 1e-12
    B = qmul(U * s[None, None, :], _qH(V))
    assert rel(B, X) < 1e-12


def test_svd_zero_matrix_and_values_only():
    # p >= q: the left factor comes from the (zero) orthogonalised columns,
    # the right factor stays unitary
    s, U, V = Q.svd(torch.zeros((4, 9, 6), dtype=torch.float64, device=DEV))
    Q.sync_status()
    assert not N(s).any() and not N(U).any()
    H = qmul(_qH(N(V)), N(V))
    assert np.abs(H[0] - np.eye(6)).max() < 1e-15 and not H[1:].any()
    rng = np.random.default_rng(8)
    X = rng.standard_normal((4, 50, 30))
    s, U, V = Q.svd(T(X), vectors=False)
    Q.sync_status()
    from oracle.pinv import singular_values
    assert U is None and V is None
    assert np.max(np.abs(N(s) - singular_values(X)) / singular_values(X)) < 1e-12


def test_pinv_zero_matrix():
    Xp, rank = Q.pinv(torch.zeros((4, 6, 4), dtype=torch.float64, device=DEV))
    assert int(N(rank)[0]) == 0 and not N(Xp).any()


# ---------------------------------------------------------------- approx / residual
def _noisy(m, n, k, seed, noise=1e-3):
    L, Rt, E = workloads.lowrank_gaussian_factors(m, n, k, seed, noise)
    return qmul(L, Rt) + E


def test_approx_car_f64_matches_checker():
    A = _noisy(150, 130, 6, 21)
    rng = np.random.default_rng(1)
    I = np.sort(rng.choice(150, 24, replace=False))
    J = np.sort(rng.choice(130, 20, replace=False))
    C, R, W = oracle.gather(A, I, J)
    U, B, ranks = Q.approx(T(A), T(C), T(R), T(W), core=Q.CORE_CAR, compute=Q.F64, want_B=True)
    Ur, kc, kr = oracle.core_car(A, C, R)
    assert N(ranks).tolist() == [kc, kr]
    assert rel(N(U), Ur) < 1e-10
    assert rel(N(B), oracle.cur_product(C, Ur, R)) < cur_tol(C, R)


@pytest.mark.parametrize("compute,tol", [(Q.F64, None), (Q.F32, 1e-5)])
def test_approx_car_ragged_pair_fast_path(compute, tol):
    # C (700 x 90) and R^H (500 x 110) share one padded CholeskyQR group
    A = _noisy(700, 500, 12, 51, 1e-2)
    rng = np.random.default_rng(6)
    I = np.sort(rng.choice(700, 110, replace=False))
    J = np.sort(rng.choice(500, 90, replace=False))
    C, R, W = oracle.gather(A, I, J)
    Ur, kc, kr = oracle.core_car(A, C, R)
    Br = oracle.cur_product(C, Ur, R)
    dt = torch.float64 if compute == Q.F64 else torch.float32
    U, B, ranks = Q.approx(T(A, dt), T(C, dt), T(R, dt), None, core=Q.CORE_CAR, compute=compute, want_B=True)
    assert N(ranks).tolist() == [kc, kr] == [90, 110]
    assert rel(N(B), Br) < (cur_tol(C, R) if tol is None else tol)


def test_approx_wpinv_plain_workload_full_size():
    cfg = workloads.WORKLOADS["plain_f64_256"]
    L, Rt, _ = workloads.lowrank_gaussian_factors(256, 256, 10, cfg["seed"])
    A = qmul(L, Rt)
    out = Q.solve(T(A), 40, 40, sampling=Q.UNIFORM, core=Q.CORE_WPINV, compute=Q.F64, seed=cfg["seed"])
    ref = oracle.solve(A, 40, 40, "uniform", "wpinv", seed=cfg["seed"])
    assert N(out["J"]).astype(np.int64).tolist() == ref["J"].tolist()
    assert N(out["I"]).astype(np.int64).tolist() == ref["I"].tolist()
    assert N(out["ranks"]).tolist() == [10, 10]
    relerr = float(N(out["residual"])[0]) / np.sqrt(fro2(A))
    assert relerr < 1e-12
    # U is unique for the truncated rank; compare the U-invariant product
    assert rel(qmul(qmul(ref["C"], N(out["U"])), ref["R"]), A) < 1e-12


@pytest.mark.parametrize("compute,tol", [(Q.F32, 1e-5), (Q.BF16, 2e-2), (Q.BF16X3, 1e-4)])
@pytest.mark.parametrize("refine", [0, 1])
def test_approx_car_mixed_precision(compute, tol, refine):
    A = workloads.color_like(200, 180, 8, seed=5)
    rng = np.random.default_rng(2)
    I = np.sort(rng.choice(200, 32, replace=False))
    J = np.sort(rng.choice(180, 32, replace=False))
    C, R, W = oracle.gather(A, I, J)
    Ur, _, _ = oracle.core_car(A, C, R)
    Br = oracle.cur_product(C, Ur, R)
    U, B, _ = Q.approx(T(A, torch.float32), T(C, torch.float32), T(R, torch.float32), None,
                       core=Q.CORE_CAR, compute=compute, refine_steps=refine, want_B=True)
    assert rel(N(B), Br) < tol


@pytest.mark.parametrize("compute", [Q.F64, Q.F32])
def test_approx_car_rejected_fast_path_recomputes(compute):
    # exact rank 5 with 12 sampled columns and rows: the Gram matrices of C
    # and R are singular, the certificate rejects the fast path after its
    # products were enqueued, and the Jacobi factors replace it
    L, Rt, _ = workloads.lowrank_gaussian_factors(90, 80, 5, 61)
    A = qmul(L, Rt)
    rng = np.random.default_rng(8)
    I = np.sort(rng.choice(90, 12, replace=False))
    J = np.sort(rng.choice(80, 12, replace=False))
    C, R, W = oracle.gather(A, I, J)
    dt = torch.float64 if compute == Q.F64 else torch.float32
    # FP32 inputs carry rounding of relative size 2^-24: truncate below it
    rtol = -1.0 if compute == Q.F64 else 1e-5
    U, B, ranks = Q.approx(T(A, dt), T(C, dt), T(R, dt), None, core=Q.CORE_CAR, compute=compute, rtol=rtol,
                           want_B=True)
    assert N(ranks).tolist() == [5, 5]
    # Lemma 1: C U R = A when rank C = rank R = rank A
    assert rel(N(B), A) < (1e-10 if compute == Q.F64 else 1e-5)


def test_approx_car_f32_second_pass_matches_checker():
    # columns graded over five decades: kappa(C), kappa(R) near 1e5 keep the
    # fast path but leave the first CholeskyQR pass non-orthogonal beyond
    # 2^-22, so the second pass runs after the speculative products
    rng = np.random.default_rng(9)
    m, n = 160, 120
    A = rng.standard_normal((4, m, n)) * (10.0 ** (-5.0 * np.arange(n) / (n - 1)))[None, None, :]
    I = np.sort(rng.choice(m, 40, replace=False))
    J = np.sort(rng.choice(n, 30, replace=False))
    J[0], J[-1] = 0, n - 1
    C, R, W = oracle.gather(A, I, J)
    Ur, kc, kr = oracle.core_car(A, C, R)
    Br = oracle.cur_product(C, Ur, R)
    U, B, ranks = Q.approx(T(A, torch.float32), T(C, torch.float32), T(R, torch.float32), None,
                           core=Q.CORE_CAR, compute=Q.F32, want_B=True)
    assert N(ranks).tolist() == [kc, kr] == [30, 40]
    assert rel(N(B), Br) < 1e-5


def test_residual_masked_matches_checker():
    rng = np.random.default_rng(3)
    A = _noisy(140, 150, 5, 31, 1e-2)
    C = A[:, :, :18]
    R = A[:, :20, :]
    U = rng.standard_normal((4, 18, 20)) * 1e-3
    mask = (rng.random((140, 150)) < 0.5).astype(np.uint8)
    fro, E = Q.residual(T(A), T(C), T(U), T(R), mask=torch.tensor(mask, device=DEV), want_E=True, e_scale=2.0)
    ref = oracle.residual(A, C, U, R, mask)
    assert abs(float(N(fro)[0]) - ref) <= 1e-12 * ref
    Er = 2.0 * (A - oracle.cur_product(C, U, R)) * mask[None]
    assert rel(N(E), Er) < 1e-12


# ---------------------------------------------------------------- backward
@pytest.mark.parametrize("dtype,tol,noise,r,c", [(torch.float64, 1e-9, 1e-2, 12, 10),
                                                 (torch.float32, 1e-4, 3.0, 16, 8)])
def test_backward_vjp_and_masked_loss(dtype, tol, noise, r, c):
    # FP32: a well-conditioned W (noise-dominated), since the pinv adjoint
    # amplifies rounding by about kappa(W)^2
    from oracle.grad import cur_vjp, masked_loss_grad, masked_loss
    rng = np.random.default_rng(4)
    A = _noisy(96, 80, 4, 41, noise)
    I = np.sort(rng.choice(96, r, replace=False))
    J = np.sort(rng.choice(80, c, replace=False))
    gB = rng.standard_normal(A.shape)
    mask = (rng.random((96, 80)) < 0.5).astype(np.uint8)
    It, Jt = T(I, torch.int64), T(J, torch.int64)
    dA, _ = Q.backward(T(A, dtype), It, Jt, gB=T(gB, dtype))
    assert rel(N(dA), cur_vjp(A, I, J, gB)) < tol
    dA, loss = Q.backward(T(A, dtype), It, Jt, mask=torch.tensor(mask, device=DEV))
    assert rel(N(dA), masked_loss_grad(A, I, J, mask)) < tol
    lr = masked_loss(A, I, J, mask)
    assert abs(float(N(loss)[0]) - lr) <= max(tol, 1e-12) * lr


def test_backward_repeated_index_flags_arg():
    A = T(np.random.default_rng(5).standard_normal((4, 10, 10)))
    Q.backward(A, T(np.array([1, 1, 2]), torch.int64), T(np.array([0, 3, 4]), torch.int64))
    with pytest.raises(Q.QcurError):
        Q.sync_status()


# ---------------------------------------------------------------- the native solve
@pytest.mark.parametrize("compute", [Q.F64, Q.F32, Q.BF16, Q.BF16X3])
@pytest.mark.parametrize("exact", [False, True])
def test_refined_residual_without_the_product(compute, exact):
    # with one refinement step and no C U R requested, the residual comes
    # from the step's own residual E and correction D (exact identity, taken
    # when ||D|| is small next to ||E||: the noisy case); exact-rank inputs
    # leave E and D both at rounding level and take the explicit product.
    # Either way it matches the residual of C U R formed explicitly and the
    # checker's.
    if exact:
        L, Rt, _ = workloads.lowrank_gaussian_factors(300, 260, 6, 17)
        A = qmul(L, Rt)
    else:
        A = workloads.color_like(300, 260, 12, seed=9, noise=0.01)
    c, r = 48, 40
    dt = torch.float64 if compute == Q.F64 else torch.float32
    S = Q.Solver(A.shape[1], A.shape[2], c, r, core=Q.CORE_CAR, compute=compute)
    At = T(A, dt)
    B = torch.empty((4, A.shape[1], A.shape[2]), dtype=dt, device=DEV)
    S(At, sampling=Q.LENGTH, seed=21, refine_steps=1, B=B)
    res_explicit = float(N(S.residual)[0])
    S(At, sampling=Q.LENGTH, seed=21, refine_steps=1)
    res = float(N(S.residual)[0])
    Q.sync_status()
    Ad = np.asarray(N(At))
    nA = np.sqrt(fro2(Ad))
    ref = oracle.solve(Ad, c, r, "length", "car", seed=21)
    tol = {Q.F64: cur_tol(ref["C"], ref["R"]), Q.F32: 1e-5, Q.BF16: 2e-2, Q.BF16X3: 1e-4}[compute]
    assert abs(res - ref["residual"]) <= tol * nA
    assert abs(res - res_explicit) <= tol * nA
    if not exact:
        # the noise floor: the residual is of the noise's size, not rounding
        assert res > 1e-3 * nA


@pytest.mark.parametrize("sampling,core,compute", [(Q.UNIFORM, Q.CORE_WPINV, Q.F64), (Q.LENGTH, Q.CORE_CAR, Q.F64),
                                                   (Q.LENGTH, Q.CORE_CAR, Q.F32), (Q.LENGTH, Q.CORE_CAR, Q.BF16),
                                                   (Q.LENGTH, Q.CORE_CAR, Q.BF16X3)])
def test_native_solve_matches_checker(sampling, core, compute):
    if core == Q.CORE_WPINV:
        L, Rt, _ = workloads.lowrank_gaussian_factors(256, 240, 10, 1)
        A = qmul(L, Rt)
        c = r = 40
    else:
        A = workloads.color_like(320, 288, 12, seed=8, noise=0.01)
        c, r = 60, 72
    dt = torch.float64 if compute == Q.F64 else torch.float32
    S = Q.Solver(A.shape[1], A.shape[2], c, r, core=core, compute=compute)
    B = torch.empty((4, A.shape[1], A.shape[2]), dtype=torch.float64 if compute == Q.F64 else torch.float32,
                    device=DEV)
    S(T(A, dt), sampling=sampling, seed=13, refine_steps=1 if compute == Q.BF16 else 0, B=B)
    Ad = np.asarray(N(T(A, dt)))
    ref = oracle.solve(Ad, c, r, "uniform" if sampling == Q.UNIFORM else "length",
                       "wpinv" if core == Q.CORE_WPINV else "car", seed=13)
    Q.sync_status()
    assert N(S.J).astype(np.int64).tolist() == ref["J"].tolist()
    assert N(S.I).astype(np.int64).tolist() == ref["I"].tolist()
    tol = {Q.F64: cur_tol(ref["C"], ref["R"]), Q.F32: 1e-5, Q.BF16: 2e-2, Q.BF16X3: 1e-4}[compute]
    # C U R element by element against the checker's
    Bref = oracle.cur_product(ref["C"], ref["U"], ref["R"])
    assert rel(N(B), Bref) < tol
    # |res - res_ref| <= ||CUR - (CUR)_ref||_F
    res = float(N(S.residual)[0])
    assert abs(res - ref["residual"]) <= tol * np.sqrt(fro2(Ad))
