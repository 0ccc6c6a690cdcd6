"""Benchmark of the QMCUR hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one whole QMCUR solve (Algorithm 1) of the colour-image-shaped
workload: a 1024 x 1024 pure quaternion matrix of rank 50 plus N(0, 0.01^2)
noise, length sampling of c = r = 200 columns and rows, the least-squares
core U = C^+ A R^+ and the residual ||A - CUR||_F.  Every step runs
probabilities -> draws -> gathers -> FP64 factors of C and R -> core
products -> residual on the GPU, with the input already resident in HBM.

Variants: plain FP64 (the reference rate), FP32 matrix-core products
(with and without one refinement step) and BF16-operand products with one
refinement step.  The headline value is the fastest mixed variant whose CUR
product is within 1e-3 relative Frobenius error of the FP64 one.

Also reported on the same JSON line: the roofline of the dominant
matrix-core kernel (T = A Q_R, timed alone with HIP events on the stream
the library launches on), the quaternion GEMM rate at the 4096 x 400 x 4096
shapes in each dtype, the 512-problem uneven batch (graph replay) against
plain FP64 solves one at a time, the 4096 x 4096 dense workload, and the
FP64 reference checker timed on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "color_1024"
T_AQR_F32_HBM_BYTES = 54.7e6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--gemm-reps", type=int, default=20)
    ap.add_argument("--no-extra", action="store_true", help="skip the batch and dense workloads")
    return ap.parse_args()


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(how the path would shard is described in DESIGN.md).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import workloads
    import paper_2402_19147_amd as q

    cfg = workloads.WORKLOADS[WORKLOAD]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    A_host = workloads.color_like(cfg["m"], cfg["n"], cfg["k"], cfg["seed"], cfg["noise"])
    A64 = torch.tensor(A_host, device=dev)
    A32 = A64.to(torch.float32)
    c, r, seed = cfg["c"], cfg["r"], cfg["seed"]
    m, n = cfg["m"], cfg["n"]

    variants = {
        "plain_f64": dict(A=A64, compute=q.F64, refine=0),
        "f32": dict(A=A32, compute=q.F32, refine=0),
        "f32_refine1": dict(A=A32, compute=q.F32, refine=1),
        "bf16_refine1": dict(A=A32, compute=q.BF16, refine=1),
        "bf16x3": dict(A=A32, compute=q.BF16X3, refine=0),
    }
    solvers = {name: q.Solver(m, n, c, r, core=q.CORE_CAR, compute=v["compute"]) for name, v in variants.items()}

    def step(name, v):
        return solvers[name](v["A"], sampling=q.LENGTH, seed=seed, refine_steps=v["refine"])

    results = {}
    for name, v in variants.items():
        for _ in range(args.warmup):
            step(name, v)
        q.sync_status()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(name, v)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        q.sync_status()
        results[name] = dict(ms_per_step=dt * 1e3, solves_per_s=1.0 / dt)
        log(f"{name}: {dt * 1e3:.3f} ms/solve")

    # accuracy of each variant: CUR product against the FP64 one (same draws)
    ref = q.solve(A64, c, r, sampling=q.LENGTH, core=q.CORE_CAR, compute=q.F64, seed=seed, want_B=True)
    Bref = ref["B"].to(torch.float64)
    nA = float(torch.linalg.vector_norm(A64))
    B_host = {}
    for name, v in variants.items():
        out = q.solve(v["A"], c, r, sampling=q.LENGTH, core=q.CORE_CAR, compute=v["compute"], seed=seed,
                      refine_steps=v["refine"], want_B=True)
        B = out["B"].to(torch.float64)
        B_host[name] = (B.cpu().numpy(), out["I"].cpu().numpy(), out["J"].cpu().numpy())
        results[name]["cur_rel_err_vs_f64"] = float(torch.linalg.vector_norm(B - Bref) / torch.linalg.vector_norm(Bref))
        results[name]["rel_residual"] = float(out["residual"].cpu()[0]) / nA
        results[name]["same_draws"] = bool(torch.equal(out["I"], ref["I"]) and torch.equal(out["J"], ref["J"]))
    q.sync_status()

    # the headline is taken among the FP32 and BF16 variants, whose matrix-core
    # kernel is the one profiled for the roofline; split BF16 is reported
    # beside them
    mixed = [k for k in ("f32", "f32_refine1", "bf16_refine1") if results[k]["cur_rel_err_vs_f64"] <= 1e-3]
    head = max(mixed, key=lambda k: results[k]["solves_per_s"]) if mixed else "plain_f64"

    def time_gemm(Aop, Bop, compute, reps, opB=q.OP_N):
        D = q.gemm(Aop, Bop, opB=opB, compute=compute)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            q.gemm(Aop, Bop, opB=opB, D=D, compute=compute)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    # dominant matrix-core kernel of the solve: T = A Q_R with A 1024 x 1024
    # and the orthonormal factor Q_R 1024 x 200, in the headline's dtype
    rng = np.random.default_rng(0)
    hd = variants[head]["compute"]
    tdt = {q.F64: torch.float64, q.F32: torch.float32, q.BF16: torch.bfloat16}[hd]
    Qr = torch.tensor(rng.standard_normal((4, n, r)), dtype=tdt, device=dev)
    t_gemm = time_gemm(A64.to(tdt), Qr, hd, args.gemm_reps)
    flops = 32.0 * m * n * r
    peak = {q.F64: 78.6, q.F32: 157.3, q.BF16: 2500.0}[hd]
    achieved = flops / t_gemm / 1e12
    # HBM bytes per GEMM of this kernel (FP32 split-K partials + reduction),
    # FETCH_SIZE + WRITE_SIZE from rocprofv3 --pmc runs of this script scaled
    # by a copy of known size (profiles/qgemm_f32_T_AQr_color_1024.md, taken
    # on the two-stage LDS pipeline of k_qgemm); only valid for that kernel
    traffic = T_AQR_F32_HBM_BYTES if hd == q.F32 else None
    roofline = dict(bound="mfma", kernel=f"qgemm T = A Q_R ({m}x{n} . {n}x{r})", achieved=achieved, peak=peak,
                    unit="TFLOP/s", frac=achieved / peak, traffic=traffic, avg_launch_us=t_gemm * 1e6,
                    algorithmic_flop_per_launch=flops, algorithmic_bytes_per_launch=4.0 * (m * n + n * r + m * r) *
                    {q.F64: 8, q.F32: 4, q.BF16: 2}[hd])
    ceil = measured_ceilings(torch, dev)
    mkey = {q.F64: "f64", q.F32: "f32", q.BF16: "bf16"}[hd]
    roofline["measured_peak"] = ceil["mfma_tflops"][mkey]
    roofline["frac_of_measured"] = achieved / ceil["mfma_tflops"][mkey] if ceil["mfma_tflops"][mkey] else None
    log("measured ceilings: MFMA " + ", ".join(f"{k} {v:.1f}" for k, v in ceil["mfma_tflops"].items()) +
        f" TFLOP/s, copy {ceil['copy_gbps']:.0f} GB/s")

    # quaternion GEMM rate at the dense shapes, every dtype
    qg = {}
    for dname, dcode, dt in (("f64", q.F64, torch.float64), ("f32", q.F32, torch.float32),
                             ("bf16", q.BF16, torch.bfloat16)):
        pk = {q.F64: 78.6, q.F32: 157.3, q.BF16: 2500.0}[dcode]
        for shape in ((4096, 400, 4096), (4096, 4096, 400)):
            M, K, N = shape
            X = torch.tensor(rng.standard_normal((4, M, K)), dtype=dt, device=dev)
            Y = torch.tensor(rng.standard_normal((4, K, N)), dtype=dt, device=dev)
            t = time_gemm(X, Y, dcode, 5)
            tf = 32.0 * M * K * N / t / 1e12
            qg[f"{dname}_{M}x{K}x{N}"] = dict(tflops=tf, frac_of_peak=tf / pk, ms=t * 1e3,
                                              frac_of_measured=tf / ceil["mfma_tflops"][dname])
            del X, Y
    # split BF16: FP32 operands, three BF16 products; tflops counts the
    # quaternion product once, the fraction counts the three MFMA products
    for shape in ((4096, 400, 4096), (4096, 4096, 400)):
        M, K, N = shape
        X = torch.tensor(rng.standard_normal((4, M, K)), dtype=torch.float32, device=dev)
        Y = torch.tensor(rng.standard_normal((4, K, N)), dtype=torch.float32, device=dev)
        t = time_gemm(X, Y, q.BF16X3, 5)
        tf = 32.0 * M * K * N / t / 1e12
        qg[f"bf16x3_{M}x{K}x{N}"] = dict(tflops=tf, mfma_frac_of_bf16_peak=3 * tf / 2500.0, ms=t * 1e3)
        del X, Y
    log("qgemm: " + ", ".join(f"{k} {v['tflops']:.1f}" for k, v in qg.items()))

    extra = {"measured_ceilings": ceil, "hbm_kernels": bench_hbm(q, torch, dev, A32, ceil)}
    if not args.no_extra:
        extra["batch_512"] = bench_batch(q, torch, workloads, dev, args)
        extra["dense_4096"] = bench_dense(q, torch, workloads, dev, args)
        extra["complete_512x768"] = bench_complete(q, torch, workloads, dev)
        extra["adjoint_2048"] = bench_adjoint(q, torch, workloads, dev, args)
        extra["qsvd_500"] = bench_qsvd(q, torch, workloads, dev)
        extra["theorem1_500"] = bench_theorem1(q, torch, workloads, dev)
    # a plain copy of known size, for scaling HBM byte counters of profiled runs
    src = torch.empty(64 * 2 ** 20, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst

    cpu = None
    if not args.no_cpu_baseline:
        cpu, ref_cpu = cpu_baseline(A_host, c, r, seed, args.cpu_seconds)
        # every variant's C U R against the oracle's (same draws required)
        for name, (Bv, Iv, Jv) in B_host.items():
            same = bool(np.array_equal(Iv, ref_cpu["I"]) and np.array_equal(Jv, ref_cpu["J"]))
            results[name]["oracle_same_draws"] = same
            results[name]["cur_rel_err_vs_oracle"] = (float(np.linalg.norm(Bv - ref_cpu["B"]) /
                                                            np.linalg.norm(ref_cpu["B"])) if same else None)

    line = {
        "metric": "QMCUR solves/s (mixed precision, rel. err <= 1e-3 vs FP64)",
        "value": results[head]["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": results[head]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"plain_f64": "f64", "f32": "f32", "f32_refine1": "f32", "bf16_refine1": "bf16"}[head],
        "data": "synthetic",
        "config": {"workload": "color_1024: 1024x1024 pure quaternion, rank 50 + N(0,0.01^2), length "
                               "sampling c=r=200, U=C^+AR^+, FP64 factors of C and R", "variant": head},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "variants": results,
        "plain_f64_solves_per_s": results["plain_f64"]["solves_per_s"],
        "speedup_vs_plain_f64": results[head]["solves_per_s"] / results["plain_f64"]["solves_per_s"],
        "qgemm": qg,
    }
    line.update(extra)
    print(json.dumps(line))


def bench_batch(q, torch, workloads, dev, args):
    """512 uneven problems (m, n ~ U{64..512}, k ~ U{8..32}, c = r = 2k):
    the batched solve (GEMM launch plans chosen by the autotuner on the first
    call, and with fixed plans for comparison) replayed from a captured
    graph, against plain FP64 solves of the same problems one at a time."""
    cfg = workloads.WORKLOADS["batch_512"]
    probs = workloads.batch_problems(cfg["count"], cfg["seed"], cfg["mn_range"], cfg["k_range"], cfg["noise"])
    dims = [(P["m"], P["n"], 2 * P["k"], 2 * P["k"]) for P in probs]
    A32 = q.pack_batch([P["A"] for P in probs], dtype=torch.float32, device=dev)
    out = {"workload": "512 pure quaternion problems, m,n ~ U{64..512}, rank k ~ U{8..32} + N(0,1e-3^2), "
                       "length sampling c=r=2k, U=C^+AR^+", "problems": len(dims)}
    seed = cfg["seed"]
    ref_res = None
    for name, comp, refine, tune in (("f32", q.F32, 0, True), ("f32_fixed_plans", q.F32, 0, False),
                                     ("f32_refine1", q.F32, 1, True), ("bf16_refine1", q.BF16, 1, True)):
        bs = q.BatchSolver(dims, compute=comp, refine_steps=refine, a_dtype=torch.float32, autotune=tune)
        bs(A32, seed=seed)  # with autotune: times the candidate plans of every GEMM stage
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            bs(A32, seed=seed)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            bs(A32, seed=seed)
        for _ in range(args.warmup):
            g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g.replay()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        q.sync_status()
        res = bs.residual.cpu().numpy()
        out[name] = dict(ms_per_batch=dt * 1e3, solves_per_s=len(dims) / dt, residual_sum=float(res.sum()))
        if tune:
            out[name]["plans"] = {k: list(v) for k, v in bs.plans().items()}
        if ref_res is None:
            ref_res = res
        log(f"batch {name}: {dt * 1e3:.3f} ms per {len(dims)} solves")
        del bs, g
    # plain FP64: one qcur_solve per problem, no graph
    A64 = A32.to(torch.float64)
    t_total = 0.0
    for b, (m, n, c, r) in enumerate(dims):
        S = q.Solver(m, n, c, r, core=q.CORE_CAR, compute=q.F64)
        Ab = A64[b, :, :m, :n].contiguous()
        S(Ab, seed=seed + b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S(Ab, seed=seed + b)
        torch.cuda.synchronize()
        t_total += time.perf_counter() - t0
    q.sync_status()
    out["plain_f64_single"] = dict(ms_per_batch=t_total * 1e3, solves_per_s=len(dims) / t_total)
    out["speedup_f32_vs_plain_f64"] = out["f32"]["solves_per_s"] / out["plain_f64_single"]["solves_per_s"]
    log(f"batch plain f64 one at a time: {t_total * 1e3:.1f} ms")
    return out


def bench_dense(q, torch, workloads, dev, args):
    """4096 x 4096, rank 100 N(0,1) factors + N(0, 1e-3^2), c = r = 400:
    FP32 products (without and with one refinement step) against plain FP64."""
    cfg = workloads.WORKLOADS["dense_4096"]
    L, Rt, E = workloads.lowrank_gaussian_factors(cfg["m"], cfg["n"], cfg["k"], cfg["seed"], cfg["noise"])
    Lt = torch.tensor(L, device=dev)
    Rtt = torch.tensor(Rt, device=dev)
    # A = L Rt (quaternion product, formed with torch matmuls) + E
    A64 = quaternion_product_torch(torch, Lt, Rtt) + torch.tensor(E, device=dev)
    del Lt, Rtt
    A32 = A64.to(torch.float32)
    m, n, c, r, seed = cfg["m"], cfg["n"], cfg["c"], cfg["r"], cfg["seed"]
    out = {"workload": "4096x4096 quaternion, rank 100 N(0,1) factors + N(0,1e-3^2), length sampling c=r=400, "
                       "U=C^+AR^+"}
    Bs = {}
    for name, A, comp, refine in (("plain_f64", A64, q.F64, 0), ("f32", A32, q.F32, 0), ("f32_refine1", A32, q.F32, 1),
                                  ("bf16x3", A32, q.BF16X3, 0)):
        S = q.Solver(m, n, c, r, core=q.CORE_CAR, compute=comp)
        S(A, seed=seed, refine_steps=refine)
        torch.cuda.synchronize()
        reps = max(2, args.steps // 2)
        t0 = time.perf_counter()
        for _ in range(reps):
            S(A, seed=seed, refine_steps=refine)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        q.sync_status()
        out[name] = dict(ms_per_step=dt * 1e3, solves_per_s=1.0 / dt,
                         rel_residual=float(S.residual.cpu()[0]) / float(torch.linalg.vector_norm(A64)))
        sol = q.solve(A, c, r, core=q.CORE_CAR, compute=comp, seed=seed, refine_steps=refine, want_B=True)
        Bs[name] = sol["B"].to(torch.float64)
        log(f"dense {name}: {dt * 1e3:.2f} ms/solve")
        del S, sol
    for name in ("f32", "f32_refine1", "bf16x3"):
        out[name]["cur_rel_err_vs_f64"] = float(torch.linalg.vector_norm(Bs[name] - Bs["plain_f64"]) /
                                                torch.linalg.vector_norm(Bs["plain_f64"]))
        out[f"speedup_{name}_vs_plain_f64"] = out[name]["solves_per_s"] / out["plain_f64"]["solves_per_s"]
    q.sync_status()
    return out


def quaternion_product_torch(torch, L, Rt):
    """A = L Rt with the sixteen plane products of the Hamilton table
    (input generation for the benchmark only)."""
    terms = {(0, 0, 0, 1), (1, 1, 0, -1), (2, 2, 0, -1), (3, 3, 0, -1), (1, 0, 1, 1), (0, 1, 1, 1), (3, 2, 1, -1),
             (2, 3, 1, 1), (2, 0, 2, 1), (3, 1, 2, 1), (0, 2, 2, 1), (1, 3, 2, -1), (3, 0, 3, 1), (2, 1, 3, -1),
             (1, 2, 3, 1), (0, 3, 3, 1)}
    out = torch.zeros((4, L.shape[1], Rt.shape[2]), dtype=L.dtype, device=L.device)
    for a, b, d, sg in terms:
        out[d] += sg * (L[a] @ Rt[b])
    return out


def bench_adjoint(q, torch, workloads, dev, args):
    """Masked CUR loss and its gradient through the adjoint kernels at
    2048 x 2048 (rank-64 N(0,1) factors, c = r = 256 fixed index sets,
    U = W^+ capped at rank 64, Bernoulli(0.5) mask): one forward + backward."""
    cfg = workloads.WORKLOADS["adjoint_2048"]
    m, k, c = cfg["m"], cfg["k"], cfg["c"]
    L, Rt, _ = workloads.lowrank_gaussian_factors(m, m, k, cfg["seed"])
    A64 = quaternion_product_torch(torch, torch.tensor(L, device=dev), torch.tensor(Rt, device=dev))
    I = torch.tensor(workloads.uniform_index_set(m, c, cfg["seed"], 0), device=dev)
    J = torch.tensor(workloads.uniform_index_set(m, c, cfg["seed"], 1), device=dev)
    mask = torch.tensor(workloads.bernoulli_mask(m, m, cfg["mask_p"], cfg["seed"]), device=dev)
    out = {"workload": "2048x2048 quaternion, rank-64 N(0,1) factors, c=r=256 fixed uniform index sets, U=W^+ "
                       "(max_rank 64), Bernoulli(0.5) mask, loss ||P_Omega(A - CUR(A))||_F^2, forward + backward"}
    for name, dt in (("f64", torch.float64), ("f32", torch.float32)):
        A = A64.to(dt)

        def step():
            At = A.detach().requires_grad_(True)
            loss = q.cur_loss(At, I, J, mask, max_rank=cfg["max_rank"])
            loss.backward()
            return At.grad

        step()
        torch.cuda.synchronize()
        reps = max(2, args.steps // 2)
        t0 = time.perf_counter()
        for _ in range(reps):
            step()
        torch.cuda.synchronize()
        dt_s = (time.perf_counter() - t0) / reps
        q.sync_status()
        out[name] = dict(ms_per_step=dt_s * 1e3, steps_per_s=1.0 / dt_s)
        log(f"adjoint {name}: {dt_s * 1e3:.2f} ms per forward+backward")
    return out


def bench_complete(q, torch, workloads, dev):
    """Completion from 30% observed entries (Algorithm 2) of a 512 x 768
    colour-image-shaped matrix: time per step, next to the paper's reported
    seconds per iteration for its 512 x 768 test images (hardware not
    stated; context only)."""
    import numpy as np
    cfg = workloads.WORKLOADS["complete_512x768"]
    m, n, k, seed = cfg["m"], cfg["n"], cfg["k"], cfg["seed"]
    A = workloads.color_like(m, n, k, seed, cfg["noise"])
    truth = workloads.color_like(m, n, k, seed, 0.0)
    mask = workloads.bernoulli_mask(m, n, cfg["mask_p"], seed)
    I = workloads.uniform_index_set(m, cfg["r"], seed, 0)
    J = workloads.uniform_index_set(n, cfg["c"], seed, 1)
    out = {"workload": "512x768 pure quaternion, rank 20 + N(0,0.01^2), 70% of entries missing, c=r=60 fixed "
                       "uniform index sets, t_max=200, tol=1e-4",
           "paper_s_per_iter_range": [0.135, 0.351]}
    miss = mask == 0
    for name, comp, dt in (("f64", q.F64, torch.float64), ("f32", q.F32, torch.float32)):
        Y = torch.tensor(A, dtype=dt, device=dev)
        Mk = torch.tensor(mask, device=dev)
        It = torch.tensor(I, device=dev)
        Jt = torch.tensor(J, device=dev)
        q.complete(Y, Mk, It, Jt, compute=comp, max_iter=2, tol=0.0)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X, iters, rel = q.complete(Y, Mk, It, Jt, compute=comp, max_iter=cfg["max_iter"], tol=cfg["tol"])
        torch.cuda.synchronize()
        dt_s = time.perf_counter() - t0
        q.sync_status()
        Xh = X.to(torch.float64).cpu().numpy()
        err = float(np.sqrt(((Xh - truth)[:, miss] ** 2).sum() / ((truth[:, miss]) ** 2).sum()))
        out[name] = dict(iterations=iters, last_rel_change=rel, ms_per_iter=dt_s * 1e3 / max(iters, 1),
                         total_ms=dt_s * 1e3, rel_err_missing_vs_noiseless=err)
        log(f"complete {name}: {iters} steps, {dt_s * 1e3 / max(iters, 1):.3f} ms/step")
    # the same problem with I, J drawn again from every iterate (length
    # probabilities), c = r = ceil(k ln k)
    cr = q.sample_size(k, min(m, n))
    Y = torch.tensor(A, dtype=torch.float32, device=dev)
    Mk = torch.tensor(mask, device=dev)
    q.complete_resampled(Y, Mk, cr, cr, sampling=q.LENGTH, seed=seed, compute=q.F32, max_iter=2, tol=0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X, iters, rel, _, _ = q.complete_resampled(Y, Mk, cr, cr, sampling=q.LENGTH, seed=seed, compute=q.F32,
                                               max_iter=cfg["max_iter"], tol=cfg["tol"])
    torch.cuda.synchronize()
    dt_s = time.perf_counter() - t0
    q.sync_status()
    Xh = X.to(torch.float64).cpu().numpy()
    err = float(np.sqrt(((Xh - truth)[:, miss] ** 2).sum() / ((truth[:, miss]) ** 2).sum()))
    out["f32_resampled_length"] = dict(c=cr, r=cr, iterations=iters, last_rel_change=rel,
                                       ms_per_iter=dt_s * 1e3 / max(iters, 1), total_ms=dt_s * 1e3,
                                       rel_err_missing_vs_noiseless=err)
    log(f"complete f32 resampled: {iters} steps, {dt_s * 1e3 / max(iters, 1):.3f} ms/step, err {err:.4f}")
    return out


def bench_qsvd(q, torch, workloads, dev):
    """Example 4.2's comparison on one 500 x 500 rank-10 + N(0, 1e-4^2)
    quaternion matrix: QMCUR (length sampling, c = r = ceil(k ln k), FP64,
    least-squares core) against the thin QSVD of the whole matrix (Jacobi,
    FP64) and its rank-k truncation."""
    cfg = workloads.WORKLOADS["qsvd_500"]
    m, n, k, seed = cfg["m"], cfg["n"], cfg["k"], cfg["seed"]
    L, Rt, E = workloads.lowrank_gaussian_factors(m, n, k, seed, cfg["noise"])
    A = quaternion_product_torch(torch, torch.tensor(L, device=dev), torch.tensor(Rt, device=dev))
    A = A + torch.tensor(E, device=dev)
    nA = float(torch.linalg.vector_norm(A))
    c = q.sample_size(k, min(m, n))
    S = q.Solver(m, n, c, c, core=q.CORE_CAR, compute=q.F64)
    for _ in range(3):
        S(A, seed=seed)
    torch.cuda.synchronize()
    reps = 20
    t0 = time.perf_counter()
    for i in range(reps):
        S(A, seed=seed + i)
    torch.cuda.synchronize()
    t_cur = (time.perf_counter() - t0) / reps
    res = float(S.residual.cpu()[0]) / nA
    q.svd(A)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s, U, V = q.svd(A)
    torch.cuda.synchronize()
    t_svd = time.perf_counter() - t0
    q.sync_status()
    sv = s.cpu().numpy()
    err_k = float((sv[k:] ** 2).sum() ** 0.5 / nA)
    out = {"workload": "500x500 quaternion, rank 10 N(0,1) factors + N(0,1e-4^2); QMCUR length sampling "
                       f"c=r={c}, FP64, U=C^+AR^+; QSVD: thin Jacobi SVD of A, FP64",
           "qmcur_ms": t_cur * 1e3, "qmcur_rel_err": res, "qsvd_ms": t_svd * 1e3, "qsvd_rank_k_rel_err": err_k,
           "qsvd_over_qmcur_time": t_svd / t_cur}
    log(f"qsvd 500: {t_svd * 1e3:.1f} ms (rank-10 err {err_k:.2e}) vs QMCUR {t_cur * 1e3:.3f} ms (err {res:.2e})")
    return out


def bench_theorem1(q, torch, workloads, dev):
    """Example 4.1 (Theorem 1): X = W_k Sigma_k V_k^H (500 x 500, k = 50,
    polar factors of Gaussian matrices, Sigma_k ~ U(1, 10)) plus Gaussian
    noise of standard deviation sigma per component, sigma = 1e-1 .. 1e-6; QMCUR with
    length sampling, c = r = ceil(k ln k), FP64, least-squares core.  Per
    level: ||E||_2, ||X - C~U~R~||_2 and Theorem 1's bound; the log-log
    slope of the error against ||E||_2 (one for linear growth)."""
    from paper_2402_19147_amd import perturbation as pt
    import math
    import numpy as np
    cfg = workloads.WORKLOADS["theorem1_500"]
    m, n, k, seed = cfg["m"], cfg["n"], cfg["k"], cfg["seed"]
    GW, GV, sig, E0 = workloads.perturbation_factors(m, n, k, seed)
    t0 = time.perf_counter()
    W = pt.polar_factor(torch.tensor(GW, device=dev))
    V = pt.polar_factor(torch.tensor(GV, device=dev))
    X = pt.lowrank_product(W, torch.tensor(sig), V)
    E0g = torch.tensor(E0, device=dev)
    nE0 = pt.spectral_norm(E0g)
    c = q.sample_size(k, min(m, n))
    levels = []
    for sigma in cfg["sigmas"]:
        out = pt.perturbation_errors(X, E0g, sigma, W, V, c, c, q.LENGTH, seed, norm_E0=nE0)
        levels.append({"sigma": sigma, "norm_E": out["norm_E"], "err": out["err"], "bound": out["bound"],
                       "err_over_norm_E": out["err"] / out["norm_E"], "w_pinv": out["w_pinv"],
                       "v_pinv": out["v_pinv"]})
    torch.cuda.synchronize()
    q.sync_status()
    elapsed = time.perf_counter() - t0
    slope = float(np.polyfit(np.log([v["norm_E"] for v in levels]), np.log([v["err"] for v in levels]), 1)[0])
    ok = all(v["err"] <= v["bound"] for v in levels)
    log(f"theorem1 500: slope {slope:.3f}, bound holds {ok}, err/|E| " +
        " ".join(f"{v['err_over_norm_E']:.2f}" for v in levels) + f" ({elapsed:.2f} s)")
    return {"workload": f"500x500, X = W_k Sigma_k V_k^H, k={k}, Gaussian noise N(0, sigma^2), sigma=1e-1..1e-6; QMCUR "
                        f"length sampling c=r={c}, FP64, U=C^+AR^+", "levels": levels, "loglog_slope": slope,
            "bound_holds": ok, "seconds": elapsed}


def cpu_baseline(A, c, r, seed, seconds):
    """The FP64 reference checker timed on the host cores, whole solves: with
    the BLAS threads it starts with, then with one thread.  Also returns one
    solve's I, J and C U R for the accuracy comparison."""
    import numpy as np
    import oracle
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        threadpool_limits = None
        threads = os.cpu_count()
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
    except OSError:
        pass

    def timed(budget, cap):
        times, out = [], None
        t_end = time.perf_counter() + budget
        while True:
            t0 = time.perf_counter()
            out = oracle.solve(A, c, r, "length", "car", seed=seed)
            times.append(time.perf_counter() - t0)
            if time.perf_counter() > t_end or len(times) >= cap:
                return times, out

    times, ref = timed(seconds, 50)
    med = float(np.median(times))
    one = None
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            t1, _ = timed(seconds / 2, 10)
        one = {"value": 1.0 / float(np.median(t1)), "cores": 1, "sample": f"{len(t1)} solves, median"}
    B = oracle.cur_product(ref["C"], ref["U"], ref["R"])
    cpu = {"value": 1.0 / med, "unit": "solves/s", "cores": threads, "kind": "oracle",
           "sample": f"{len(times)} full FP64 solves of the same 1024x1024 workload, median",
           "host_cpus": os.cpu_count(), "cpu_model": model, "one_thread": one}
    return cpu, {"I": ref["I"], "J": ref["J"], "B": B}


def measured_ceilings(torch, dev):
    """Achievable MFMA rate per dtype and streaming-copy bandwidth on this
    device (libqcur_probe: a loop of independent MFMAs, a 1 GiB copy)."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2402_19147_amd", "libqcur_probe.so"))
    lib.qcur_probe_mfma.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.qcur_probe_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_double)]
    torch.cuda.synchronize()
    out = {"mfma_tflops": {}}
    for name, code in (("f64", 0), ("f32", 1), ("bf16", 2)):
        v = ctypes.c_double(0.0)
        rc = lib.qcur_probe_mfma(code, 4096, ctypes.byref(v))
        if rc != 0:
            raise RuntimeError(f"qcur_probe_mfma({name}) failed: {rc}")
        out["mfma_tflops"][name] = v.value
    src = torch.empty(2 ** 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    src.fill_(1.0)
    torch.cuda.synchronize()
    g = ctypes.c_double(0.0)
    rc = lib.qcur_probe_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), 2 ** 30, 10,
                             ctypes.byref(g))
    if rc != 0:
        raise RuntimeError(f"qcur_probe_copy failed: {rc}")
    out["copy_gbps"] = g.value
    out["copy_bytes"] = 2 ** 30
    del src, dst
    return out


def bench_hbm(q, torch, dev, A32, ceil):
    """Achieved HBM bandwidth of the HBM-bound steps: the probabilities (a1,
    one read of A) on the 1024^2 workload and on a 4096^2 FP32 matrix, and the
    gathers (a3) at 4096^2 with c = r = 400.  Algorithmic bytes over the time
    of one call (all of its launches), against 8 TB/s and the measured copy."""
    import numpy as np

    def timed(fn, reps=20):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    out = {}
    big = torch.randn((4, 4096, 4096), dtype=torch.float32, device=dev)
    for name, X in (("probs_f32_1024x1024", A32), ("probs_f32_4096x4096", big)):
        _, mm, nn = X.shape
        t = timed(lambda: q.probs(X, q.LENGTH))
        byt = 4.0 * mm * nn * 4
        out[name] = {"bytes": byt, "us": t * 1e6, "gbps": byt / t / 1e9, "frac_of_peak": byt / t / 8e12,
                     "frac_of_measured": byt / t / 1e9 / ceil["copy_gbps"]}
    rng = np.random.default_rng(3)
    I = torch.tensor(np.sort(rng.choice(4096, 400, replace=False)), device=dev)
    J = torch.tensor(np.sort(rng.choice(4096, 400, replace=False)), device=dev)
    t = timed(lambda: q.gather(big, I, J))
    byt = 2.0 * 4 * (4096 * 400 + 400 * 4096 + 400 * 400) * 4
    out["gather_f32_4096_c400"] = {"bytes": byt, "us": t * 1e6, "gbps": byt / t / 1e9, "frac_of_peak": byt / t / 8e12,
                                   "frac_of_measured": byt / t / 1e9 / ceil["copy_gbps"]}
    del big
    log("hbm: " + ", ".join(f"{k} {v['gbps']:.0f} GB/s" for k, v in out.items()))
    return out


if __name__ == "__main__":
    main()
