"""Batched QMCUR (qcur_solve_batched): every problem of an uneven batch
against the FP64 reference checker and against the single-matrix solve on
the same inputs, the Jacobi fallback inside the batch, graph replay, and the
512-problem workload (MI355X only)."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from oracle.cur import cur_product
from oracle.quat import fro2
from oracle.sampling import draw, probs_length

pytestmark = pytest.mark.gpu

Q = pytest.importorskip("paper_2402_19147_amd.qcur")
DEV = torch.device("cuda:0")
U32 = 2.0 ** -24


def T(x, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


def N(t):
    return t.detach().to(torch.float64).cpu().numpy()


def rel(x, ref):
    return np.sqrt(fro2(np.asarray(x, dtype=np.float64) - ref)) / max(np.sqrt(fro2(ref)), 1e-300)


def kappa(X):
    from oracle.pinv import singular_values
    sv = singular_values(X)
    sv = sv[sv > sv[0] * 1e-13]
    return float(sv[0] / sv[-1])


def tol_for(compute, C, R):
    """Relative tolerance (w.r.t. ||A||_F) of CUR products and residuals:
    FP64 1e-12, widened by the conditioning of the sampled C and R (which
    limits how well the FP64 projectors are determined); FP32 products 1e-5;
    BF16 operands 2e-2."""
    if compute == Q.F64:
        return max(1e-12, 10 * 2.0 ** -52 * (kappa(C) + kappa(R)))
    return {Q.F32: 1e-5, Q.BF16: 2e-2}[compute]


def make_batch(count, seed, mn=(20, 150), k=(2, 8), noise=1e-3):
    probs = workloads.batch_problems(count, seed, mn_range=mn, k_range=k, noise=noise)
    dims = [(P["m"], P["n"], 2 * P["k"], 2 * P["k"]) for P in probs]
    return probs, dims


def tdt(compute):
    return torch.float64 if compute == Q.F64 else torch.float32


@pytest.fixture(autouse=True)
def _status_clean():
    Q.sync_status()
    yield
    Q.sync_status()


def check_problem(bs, A, b, dims, seed, compute, sampling="length", max_rank=0):
    m, n, c, r = dims[b]
    Ab = N(A[b, :, :m, :n])  # the values the kernels saw
    pg, qg = N(bs.p[b, :n]), N(bs.q[b, :m])
    if sampling == "length":
        p_ref, q_ref, _ = probs_length(Ab)
        assert np.allclose(pg, p_ref, rtol=1e-13, atol=0)
        assert np.allclose(qg, q_ref, rtol=1e-13, atol=0)
    else:
        assert np.all(pg == 1.0 / n) and np.all(qg == 1.0 / m)
    # draws are bit-exact given the probabilities the kernels used
    J = N(bs.J[b, :c]).astype(np.int64)
    I = N(bs.I[b, :r]).astype(np.int64)
    assert J.tolist() == draw(pg, c, seed + b, 0).tolist()
    assert I.tolist() == draw(qg, r, seed + b, 1).tolist()
    ref = oracle.solve(Ab, c, r, sampling, "car", seed=seed + b, max_rank=max_rank)
    # the checker's own probabilities differ from the kernels' only by rounding
    assert ref["J"].tolist() == J.tolist() and ref["I"].tolist() == I.tolist()
    nA = np.sqrt(fro2(Ab))
    tol = tol_for(compute, ref["C"], ref["R"])
    res = float(N(bs.residual)[b])
    assert abs(res - ref["residual"]) <= tol * nA, (b, res, ref["residual"])
    Bref = cur_product(ref["C"], ref["U"], ref["R"])
    if bs.B is not None:
        # the batch's own C U R, element by element
        B = N(bs.B[b, :, :m, :n])
    else:
        # C U R from the returned U (FP64 U only: an FP32 U carries its own
        # rounding, amplified by the conditioning of C and R)
        assert compute == Q.F64
        B = cur_product(ref["C"], N(bs.U[b, :, :c, :r]), ref["R"])
    assert np.sqrt(fro2(B - Bref)) <= tol * nA, b
    if compute == Q.F64:
        # and the core itself through C U R in FP64
        Bu = cur_product(ref["C"], N(bs.U[b, :, :c, :r]), ref["R"])
        assert np.sqrt(fro2(Bu - Bref)) <= tol * nA, b
    return ref


@pytest.mark.parametrize("compute", [Q.F64, Q.F32, Q.BF16])
def test_batch_matches_checker(compute):
    probs, dims = make_batch(10, seed=21)
    dt = tdt(compute)
    bs = Q.BatchSolver(dims, compute=compute, refine_steps=1 if compute == Q.BF16 else 0, a_dtype=dt,
                       want_B=True)
    A = Q.pack_batch([P["A"] for P in probs], dtype=dt, device=DEV)
    bs(A, seed=5)
    Q.sync_status()
    for b in range(len(dims)):
        check_problem(bs, A, b, dims, 5, compute)
        assert N(bs.ranks[b]).astype(int).tolist() == [dims[b][2], dims[b][3]]


@pytest.mark.parametrize("compute", [Q.F64, Q.F32])
def test_batch_factors_wider_than_one_block(compute):
    # c = r = 2k > 64: the factors' Gram matrices exceed one 64 x 64 block, so
    # the batch takes the multi-launch CholeskyQR route (tile-task Cholesky
    # with identity padding) instead of the one-workgroup-per-factor kernel
    probs, dims = make_batch(4, seed=29, mn=(150, 260), k=(33, 40))
    assert max(max(d[2], d[3]) for d in dims) > 64
    dt = tdt(compute)
    bs = Q.BatchSolver(dims, compute=compute, a_dtype=dt, want_B=True)
    A = Q.pack_batch([P["A"] for P in probs], dtype=dt, device=DEV)
    bs(A, seed=8)
    Q.sync_status()
    for b in range(len(dims)):
        check_problem(bs, A, b, dims, 8, compute)


def test_batch_uniform_sampling():
    probs, dims = make_batch(7, seed=24)
    bs = Q.BatchSolver(dims, compute=Q.F64, sampling=Q.UNIFORM, a_dtype=torch.float64)
    A = Q.pack_batch([P["A"] for P in probs], dtype=torch.float64, device=DEV)
    bs(A, seed=77)
    Q.sync_status()
    for b in range(len(dims)):
        check_problem(bs, A, b, dims, 77, Q.F64, sampling="uniform")


@pytest.mark.parametrize("compute", [Q.F64, Q.F32])
def test_batch_equals_single_solve(compute):
    probs, dims = make_batch(6, seed=22, mn=(64, 200), k=(4, 12))
    dt = tdt(compute)
    bs = Q.BatchSolver(dims, compute=compute, a_dtype=dt, want_B=True)
    A = Q.pack_batch([P["A"] for P in probs], dtype=dt, device=DEV)
    bs(A, seed=9)
    for b, (m, n, c, r) in enumerate(dims):
        Ab = A[b, :, :m, :n].contiguous()
        S = Q.Solver(m, n, c, r, core=Q.CORE_CAR, compute=compute)
        Bs = torch.empty((4, m, n), dtype=bs.B.dtype, device=DEV)
        S(Ab, seed=9 + b, B=Bs)
        Q.sync_status()
        assert torch.equal(S.I, bs.I[b, :r]) and torch.equal(S.J, bs.J[b, :c])
        C, R, _ = oracle.gather(N(Ab), N(S.I), N(S.J))
        tol = tol_for(compute, C, R)
        nA = np.sqrt(fro2(N(Ab)))
        assert abs(float(N(S.residual)[0]) - float(N(bs.residual)[b])) <= tol * nA
        assert np.sqrt(fro2(N(Bs) - N(bs.B[b, :, :m, :n]))) <= tol * nA


@pytest.mark.parametrize("compute", [Q.F64, Q.F32])
def test_batch_rank_deficient_falls_back_to_jacobi(compute):
    # exact rank k with c = r = 2k: every C_b and R_b is rank deficient, the
    # CholeskyQR certificate fails and the in-batch Jacobi SVD takes over;
    # Lemma 1 (exact recovery) then makes the residual vanish
    probs, dims = make_batch(6, seed=23, mn=(30, 90), k=(2, 5), noise=0.0)
    dt = tdt(compute)
    bs = Q.BatchSolver(dims, compute=compute, a_dtype=dt)
    A = Q.pack_batch([P["A"] for P in probs], dtype=dt, device=DEV)
    # FP32 inputs carry rounding noise near 1e-7 relative: cut there
    rtol = -1.0 if compute == Q.F64 else 1e-5
    bs(A, seed=3, rtol=rtol)
    Q.sync_status()
    floor = 1e-10 if compute == Q.F64 else 1e-5
    for b, P in enumerate(probs):
        m, n, c, r = dims[b]
        assert N(bs.ranks[b]).astype(int).tolist() == [P["k"], P["k"]]
        Ab = N(A[b, :, :m, :n])
        assert float(N(bs.residual)[b]) <= floor * np.sqrt(fro2(Ab))
        ref = oracle.solve(Ab, c, r, "length", "car", seed=3 + b, rtol=rtol)
        assert ref["rank"] == P["k"]
        B = cur_product(ref["C"], N(bs.U[b, :, :c, :r]), ref["R"])
        assert rel(B, Ab) <= floor


def test_batch_max_rank():
    # k = 4 for every problem, c = r = 8, noise 1e-3: capping the rank at 4
    # keeps the signal and drops the noise directions (a wide gap)
    probs, dims = make_batch(5, seed=25, mn=(40, 120), k=(4, 4))
    bs = Q.BatchSolver(dims, compute=Q.F64, a_dtype=torch.float64)
    A = Q.pack_batch([P["A"] for P in probs], dtype=torch.float64, device=DEV)
    bs(A, seed=11, max_rank=4)
    Q.sync_status()
    for b in range(len(dims)):
        assert N(bs.ranks[b]).astype(int).tolist() == [4, 4]
        m, n, c, r = dims[b]
        Ab = N(A[b, :, :m, :n])
        ref = oracle.solve(Ab, c, r, "length", "car", seed=11 + b, max_rank=4)
        nA = np.sqrt(fro2(Ab))
        assert abs(float(N(bs.residual)[b]) - ref["residual"]) <= 1e-9 * nA
        B = cur_product(ref["C"], N(bs.U[b, :, :c, :r]), ref["R"])
        assert np.sqrt(fro2(B - cur_product(ref["C"], ref["U"], ref["R"]))) <= 1e-9 * nA


@pytest.mark.parametrize("compute", [Q.F64, Q.F32, Q.BF16])
@pytest.mark.parametrize("noise", [1e-2, 0.0])
def test_batch_refined_residual_without_the_product(compute, noise):
    # one refinement step and no C U R asked for: each problem's residual
    # comes from its step's ||E_b||^2 - ||D_b||^2 when D_b is small next to
    # E_b (the noisy batch) and from the explicit product otherwise (exact
    # rank: E_b and D_b both rounding); either way it matches the residual
    # of the run that forms C U R, and the checker's
    probs, dims = make_batch(10, seed=41, mn=(40, 200), k=(3, 9), noise=noise)
    dt = tdt(compute)
    A = Q.pack_batch([P["A"] for P in probs], dtype=dt, device=DEV)
    with_B = Q.BatchSolver(dims, compute=compute, refine_steps=1, a_dtype=dt, want_B=True)
    with_B(A, seed=7)
    plain = Q.BatchSolver(dims, compute=compute, refine_steps=1, a_dtype=dt)
    plain(A, seed=7)
    Q.sync_status()
    tol = {Q.F64: 1e-9, Q.F32: 1e-5, Q.BF16: 2e-2}[compute]
    for b in range(len(dims)):
        m, n, c, r = dims[b]
        Ab = N(A[b, :, :m, :n])
        nA = np.sqrt(fro2(Ab))
        res, res_B = float(N(plain.residual)[b]), float(N(with_B.residual)[b])
        assert abs(res - res_B) <= tol * nA, b
        ref = oracle.solve(Ab, c, r, "length", "car", seed=7 + b)
        assert abs(res - ref["residual"]) <= tol * nA, b
        if noise > 0:
            assert res > 1e-3 * nA, b


def test_batch_graph_replay():
    probs, dims = make_batch(9, seed=26, mn=(40, 160), k=(3, 9))
    bs = Q.BatchSolver(dims, compute=Q.F32, refine_steps=1, a_dtype=torch.float32)
    A = Q.pack_batch([P["A"] for P in probs], dtype=torch.float32, device=DEV)
    bs(A, seed=31)
    torch.cuda.synchronize()
    ref = [t.clone() for t in (bs.I, bs.J, bs.U, bs.residual, bs.ranks)]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        bs(A, seed=31)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        bs(A, seed=31)
    for _ in range(3):
        for t in (bs.I, bs.J):
            t.fill_(-1)  # the entries past c_b / r_b are never written
        bs.U.zero_()
        bs.residual.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for t, r in zip((bs.I, bs.J, bs.U, bs.residual, bs.ranks), ref):
            assert torch.equal(t, r)
    Q.sync_status()


def test_batch_rejects_unprepared_workspace():
    probs, dims = make_batch(3, seed=27)
    bs = Q.BatchSolver(dims, compute=Q.F32, a_dtype=torch.float32)
    A = Q.pack_batch([P["A"] for P in probs], dtype=torch.float32, device=DEV)
    bs.dims = bs.dims.copy()
    bs.dims[0, 2] -= 1  # sizes that differ from the prepared ones
    with pytest.raises(Q.QcurError):
        bs(A, seed=1)


@pytest.mark.slow
@pytest.mark.parametrize("compute", [Q.F32, Q.BF16])
def test_batch_512_workload(compute):
    # 512 problems, m, n ~ U{64..512}, k ~ U{8..32}, c = r = 2k
    probs = workloads.batch_problems(512, 4)
    dims = [(P["m"], P["n"], 2 * P["k"], 2 * P["k"]) for P in probs]
    bs = Q.BatchSolver(dims, compute=compute, refine_steps=1, a_dtype=torch.float32, want_B=True)
    A = Q.pack_batch([P["A"] for P in probs], dtype=torch.float32, device=DEV)
    bs(A, seed=40)
    Q.sync_status()
    res = N(bs.residual)
    assert np.all(np.isfinite(res))
    # every problem: sorted distinct in-range draws, full ranks
    for b, (m, n, c, r) in enumerate(dims):
        J = N(bs.J[b, :c]).astype(np.int64)
        I = N(bs.I[b, :r]).astype(np.int64)
        assert np.all(np.diff(J) > 0) and J[0] >= 0 and J[-1] < n
        assert np.all(np.diff(I) > 0) and I[0] >= 0 and I[-1] < m
    assert np.all(N(bs.ranks)[:, 0] == np.array([d[2] for d in dims]))
    # every problem against the checker, element by element
    for b in range(len(dims)):
        check_problem(bs, A, b, dims, 40, compute)


@pytest.mark.parametrize("compute", [Q.F32, Q.BF16])
def test_batch_autotuned_plans(compute):
    probs, dims = make_batch(12, seed=28, mn=(40, 260), k=(3, 12))
    A = Q.pack_batch([P["A"] for P in probs], dtype=torch.float32, device=DEV)
    bs = Q.BatchSolver(dims, compute=compute, refine_steps=1, a_dtype=torch.float32, autotune=True, want_B=True)
    assert bs.plans() is None
    bs(A, seed=6)  # measures the candidate plans
    Q.sync_status()
    plans = bs.plans()
    assert plans is not None and len(plans) == 13
    # the FP64 factor stages run in the one-workgroup-per-factor CholeskyQR2
    # kernel (reported as 16-blocks, fixed); the others on tuned 32- or 64-tiles
    fixed = ("gram_C", "gram_R", "q1_C", "q1_R", "gram2", "p2p1", "q1p2")
    assert all(plans[k] == (16, 1) for k in fixed)
    assert all(t in (32, 64) for name, (t, s) in plans.items() if name not in fixed)
    assert all(1 <= s <= 4 for name, (t, s) in plans.items() if name != "residual")
    first = [t.clone() for t in (bs.I, bs.J, bs.U, bs.residual)]
    for b in range(len(dims)):
        check_problem(bs, A, b, dims, 6, compute)
    # later calls reuse the plans: bitwise repeatable, also from a captured graph
    bs(A, seed=6)
    torch.cuda.synchronize()
    for t, r in zip((bs.I, bs.J, bs.U, bs.residual), first):
        assert torch.equal(t, r)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        bs(A, seed=6)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        bs(A, seed=6)
    bs.U.zero_()
    bs.residual.zero_()
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    for t, r in zip((bs.I, bs.J, bs.U, bs.residual), first):
        assert torch.equal(t, r)
    Q.sync_status()
