"""Benchmark of the QMCUR hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one whole QMCUR solve (Algorithm 1) of the large dense workload:
a 4096 x 4096 quaternion matrix, the quaternion product of rank-100 N(0,1)
factors plus N(0, 1e-3^2) noise, length sampling of c = r = 400 columns and
rows, the least-squares core U = C^+ A R^+ with FP32 matrix-core products,
one refinement step on the core and FP64 pseudoinverses, and the residual
||A - CUR||_F.  Every step runs probabilities -> draws -> gathers -> FP64
factors of C and R -> core products -> refinement -> residual on the GPU,
with the input already resident in HBM.

Also on the same JSON line: the same solve as plain FP64 (the reference
rate) and in the other product precisions; the roofline of the dominant
matrix-core kernel (T = A Q_R at 4096 x 4096 x 400 in FP32, timed alone
with HIP events on the stream the library launches on); the quaternion GEMM
rate at the 4096 x 400 x 4096 shapes in each dtype; the 1024 x 1024
colour-image-shaped workload; the 512-problem uneven batch (graph replay);
the completion loop; the adjoint; the QSVD comparison and the Theorem 1
experiment; and the FP64 reference checker timed on the host cores.  Every
result carries its error against the checker on the same input.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "dense_4096"
HEAD = "f32_refine1"
# HBM bytes per launch of the roofline kernel (FETCH_SIZE + WRITE_SIZE of the
# FP32 T = A Q_R product at 4096 x 4096 x 400 and its split-K reduction,
# scaled by a copy of known size), from profiles/qgemm_f32_T_AQr_dense_4096.md
T_AQR_F32_HBM_BYTES = 998.8e6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip every use of the FP64 checker")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--gemm-reps", type=int, default=10)
    ap.add_argument("--no-extra", action="store_true", help="only the headline workload and its roofline")
    ap.add_argument("--only", default="", help="comma-separated extra workloads to run (default all)")
    return ap.parse_args()


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def rel_err(x, ref):
    import numpy as np
    return float(np.sqrt(np.sum((np.asarray(x, dtype=np.float64) - ref) ** 2) / np.sum(ref ** 2)))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: the workloads run on "
              "a single GPU, and no multi-GPU path is built.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import workloads
    import paper_2402_19147_amd as q

    cfg = workloads.WORKLOADS[WORKLOAD]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    m, n, c, r, seed = cfg["m"], cfg["n"], cfg["c"], cfg["r"], cfg["seed"]
    L, Rt, E = workloads.lowrank_gaussian_factors(m, n, cfg["k"], seed, cfg["noise"])
    # A = L Rt (quaternion product formed with torch matmuls, input generation
    # only) + E; the FP32 runs and the checker see the FP32 rounding of it
    A64 = quaternion_product_torch(torch, torch.tensor(L, device=dev), torch.tensor(Rt, device=dev))
    A64 += torch.tensor(E, device=dev)
    del L, Rt, E
    A32 = A64.to(torch.float32)
    A64r = A32.to(torch.float64)  # the same values in FP64 for the plain FP64 solve
    del A64

    variants = {
        "plain_f64": dict(A=A64r, compute=q.F64, refine=0),
        "f32": dict(A=A32, compute=q.F32, refine=0),
        "f32_refine1": dict(A=A32, compute=q.F32, refine=1),
        "bf16x3": dict(A=A32, compute=q.BF16X3, refine=0),
    }
    solvers = {name: q.Solver(m, n, c, r, core=q.CORE_CAR, compute=v["compute"]) for name, v in variants.items()}
    results = {}
    for name, v in variants.items():
        S = solvers[name]
        for _ in range(args.warmup):
            S(v["A"], sampling=q.LENGTH, seed=seed, refine_steps=v["refine"])
        q.sync_status()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            S(v["A"], sampling=q.LENGTH, seed=seed, refine_steps=v["refine"])
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        q.sync_status()
        results[name] = dict(ms_per_step=dt * 1e3, solves_per_s=1.0 / dt)
        log(f"dense {name}: {dt * 1e3:.3f} ms/solve")
    # C U R of every variant (one more solve each, untimed) for the accuracy
    nA = float(torch.linalg.vector_norm(A64r))
    B_host = {}
    for name, v in variants.items():
        S = solvers[name]
        B = torch.empty((4, m, n), dtype=torch.float64 if v["compute"] == q.F64 else torch.float32, device=dev)
        S(v["A"], sampling=q.LENGTH, seed=seed, refine_steps=v["refine"], B=B)
        q.sync_status()
        B_host[name] = B.cpu().numpy()
        results[name]["rel_residual"] = float(S.residual.cpu()[0]) / nA
        results[name]["ranks"] = S.ranks.cpu().tolist()
        IJ = (S.I.cpu().numpy().copy(), S.J.cpu().numpy().copy())
        results[name]["_IJ"] = IJ
        del B
    for name in variants:
        if name != "plain_f64":
            results[name]["cur_rel_err_vs_gpu_f64"] = rel_err(B_host[name], B_host["plain_f64"].astype(np.float64))
            results[name]["speedup_vs_plain_f64"] = results[name]["solves_per_s"] / results["plain_f64"]["solves_per_s"]

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

    # dominant matrix-core kernel of the solve: T = A Q_R with A 4096 x 4096
    # and the orthonormal factor Q_R 4096 x 400, FP32 (the refinement repeats
    # the same shape for E Q_R, and the residual products have the transposed
    # shape 4096 x 400 x 4096)
    rng = np.random.default_rng(0)
    Qr = torch.tensor(rng.standard_normal((4, n, r)) / np.sqrt(4.0 * n), dtype=torch.float32, device=dev)
    t_gemm = time_gemm(A32, Qr, q.F32, args.gemm_reps)
    flops = 32.0 * m * n * r
    achieved = flops / t_gemm / 1e12
    roofline = dict(bound="mfma", kernel=f"qgemm T = A Q_R ({m}x{n} . {n}x{r}, FP32)", achieved=achieved,
                    peak=157.3, unit="TFLOP/s", frac=achieved / 157.3, traffic=T_AQR_F32_HBM_BYTES,
                    avg_launch_us=t_gemm * 1e6, algorithmic_flop_per_launch=flops,
                    algorithmic_bytes_per_launch=4.0 * (m * n + n * r + m * r) * 4)
    del Qr
    ceil = measured_ceilings(torch, dev)
    roofline["measured_peak"] = ceil["mfma_tflops"]["f32"]
    roofline["frac_of_measured"] = achieved / ceil["mfma_tflops"]["f32"] if ceil["mfma_tflops"]["f32"] else None
    log(f"roofline T = A Q_R: {achieved:.1f} TFLOP/s ({achieved / 157.3:.3f} of peak), {t_gemm * 1e6:.1f} us")
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
    for shape in ((4096, 400, 4096), (4096, 4096, 400)):
        M, K, N = shape
        X = torch.tensor(rng.standard_normal((4, M, K)), dtype=torch.float32, device=dev)
        Y = torch.tensor(rng.standard_normal((4, K, N)), dtype=torch.float32, device=dev)
        t = time_gemm(X, Y, q.BF16X3, 5)
        tf = 32.0 * M * K * N / t / 1e12
        qg[f"bf16x3_{M}x{K}x{N}"] = dict(tflops=tf, mfma_frac_of_bf16_peak=3 * tf / 2500.0, ms=t * 1e3)
        del X, Y
    log("qgemm: " + ", ".join(f"{k} {v['tflops']:.1f}" for k, v in qg.items()))

    use_oracle = not args.no_cpu_baseline
    only = set(x for x in args.only.split(",") if x)
    want = (lambda name: not args.no_extra and (not only or name in only))
    extra = {"measured_ceilings": ceil}
    if want("hbm_kernels"):
        extra["hbm_kernels"] = bench_hbm(q, torch, dev, A32, ceil)
    del solvers, variants
    A32_host = A32.cpu().numpy().astype(np.float64)
    del A32, A64r
    torch.cuda.empty_cache()
    if want("color_1024"):
        extra["color_1024"] = bench_color(q, torch, workloads, dev, args, use_oracle)
    if want("batch_512"):
        extra["batch_512"] = bench_batch(q, torch, workloads, dev, args, use_oracle)
    if want("complete_512x768"):
        extra["complete_512x768"] = bench_complete(q, torch, workloads, dev, use_oracle)
    if want("adjoint_2048"):
        extra["adjoint_2048"] = bench_adjoint(q, torch, workloads, dev, args, use_oracle)
    if want("qsvd_500"):
        extra["qsvd_500"] = bench_qsvd(q, torch, workloads, dev, use_oracle)
    if want("theorem1_500"):
        extra["theorem1_500"] = bench_theorem1(q, torch, workloads, dev)
    # a plain copy of known size, for scaling HBM byte counters of profiled runs
    src = torch.empty(64 * 2 ** 20, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst

    cpu = None
    if use_oracle:
        cpu, ref = cpu_baseline(A32_host, c, r, seed, args.cpu_seconds)
        for name in results:
            Iv, Jv = results[name]["_IJ"]
            same = bool(np.array_equal(Iv, ref["I"]) and np.array_equal(Jv, ref["J"]))
            results[name]["oracle_same_draws"] = same
            results[name]["cur_rel_err_vs_oracle"] = rel_err(B_host[name], ref["B"]) if same else None
        log("dense vs oracle: " + ", ".join(f"{k} {v['cur_rel_err_vs_oracle']:.2e}" for k, v in results.items()
                                            if v.get("cur_rel_err_vs_oracle") is not None))
    for v in results.values():
        v.pop("_IJ", None)

    hd = results[HEAD]
    line = {
        "metric": "QMCUR solves/s (mixed precision, rel. err <= 1e-3 vs FP64)",
        "value": hd["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hd["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "dense_4096: 4096x4096 quaternion, rank-100 N(0,1) factors + N(0,1e-3^2), length "
                               "sampling c=r=400, U=C^+AR^+ with FP32 products, one refinement step, FP64 pinv "
                               "of C and R",
                   "variant": HEAD},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "variants": results,
        "plain_f64_solves_per_s": results["plain_f64"]["solves_per_s"],
        "speedup_vs_plain_f64": hd["solves_per_s"] / results["plain_f64"]["solves_per_s"],
        "qgemm": qg,
    }
    line.update(extra)
    print(json.dumps(line))


def bench_color(q, torch, workloads, dev, args, use_oracle):
    """The 1024 x 1024 colour-image-shaped workload (pure quaternion, rank 50
    + N(0, 0.01^2), length sampling c = r = 200, U = C^+ A R^+): plain FP64,
    FP32 products with and without refinement, BF16 operands with
    refinement, split BF16; errors against the checker on the same input."""
    import numpy as np
    cfg = workloads.WORKLOADS["color_1024"]
    m, n, c, r, seed = cfg["m"], cfg["n"], cfg["c"], cfg["r"], cfg["seed"]
    A_host = workloads.color_like(m, n, cfg["k"], seed, cfg["noise"])
    A64 = torch.tensor(A_host, device=dev)
    A32 = A64.to(torch.float32)
    variants = {
        "plain_f64": dict(A=A64, compute=q.F64, refine=0),
        "f32": dict(A=A32, compute=q.F32, refine=0),
        "f32_refine1": dict(A=A32, compute=q.F32, refine=1),
        "bf16_refine1": dict(A=A32, compute=q.BF16, refine=1),
        "bf16x3": dict(A=A32, compute=q.BF16X3, refine=0),
    }
    out = {"workload": "1024x1024 pure quaternion, rank 50 + N(0,0.01^2), length sampling c=r=200, U=C^+AR^+"}
    Bs = {}
    for name, v in variants.items():
        S = q.Solver(m, n, c, r, core=q.CORE_CAR, compute=v["compute"])
        for _ in range(args.warmup):
            S(v["A"], seed=seed, refine_steps=v["refine"])
        torch.cuda.synchronize()
        reps = max(args.steps, 20)
        t0 = time.perf_counter()
        for _ in range(reps):
            S(v["A"], seed=seed, refine_steps=v["refine"])
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        B = torch.empty((4, m, n), dtype=torch.float64 if v["compute"] == q.F64 else torch.float32, device=dev)
        S(v["A"], seed=seed, refine_steps=v["refine"], B=B)
        q.sync_status()
        Bs[name] = (B.cpu().numpy(), S.I.cpu().numpy().copy(), S.J.cpu().numpy().copy())
        out[name] = dict(ms_per_step=dt * 1e3, solves_per_s=1.0 / dt)
        log(f"color {name}: {dt * 1e3:.3f} ms/solve")
    for name in variants:
        if name != "plain_f64":
            out[name]["speedup_vs_plain_f64"] = out[name]["solves_per_s"] / out["plain_f64"]["solves_per_s"]
    if use_oracle:
        import oracle
        A32h = A32.cpu().numpy().astype(np.float64)
        refs = {}
        for key, Ah in (("f64", A_host), ("f32", A32h)):
            t0 = time.perf_counter()
            ref = oracle.solve(Ah, c, r, "length", "car", seed=seed)
            refs[key] = (oracle.cur_product(ref["C"], ref["U"], ref["R"]), ref["I"], ref["J"])
            out[f"oracle_s_per_solve_{key}_input"] = time.perf_counter() - t0
        for name, (B, I, J) in Bs.items():
            Bref, Ir, Jr = refs["f64" if name == "plain_f64" else "f32"]
            same = bool(np.array_equal(I, Ir) and np.array_equal(J, Jr))
            out[name]["oracle_same_draws"] = same
            out[name]["cur_rel_err_vs_oracle"] = rel_err(B, Bref) if same else None
        log("color vs oracle: " + ", ".join(f"{k} {out[k]['cur_rel_err_vs_oracle']:.2e}" for k in variants
                                            if out[k].get("cur_rel_err_vs_oracle") is not None))
        settle()
    return out


def bench_batch(q, torch, workloads, dev, args, use_oracle):
    """512 uneven problems (m, n ~ U{64..512}, k ~ U{8..32}, c = r = 2k):
    the batched solve (GEMM launch plans chosen by the autotuner on the first
    call, and with fixed plans for comparison) replayed from a captured
    graph, against plain FP64 solves of the same problems one at a time.
    As with the single solves, the timed replays return U, I, J and the
    residuals without forming C U R; one more solve per variant (untimed)
    forms it, and every problem's C U R is held against the checker's."""
    import numpy as np
    cfg = workloads.WORKLOADS["batch_512"]
    probs = workloads.batch_problems(cfg["count"], cfg["seed"], cfg["mn_range"], cfg["k_range"], cfg["noise"])
    dims = [(P["m"], P["n"], 2 * P["k"], 2 * P["k"]) for P in probs]
    A32 = q.pack_batch([P["A"] for P in probs], dtype=torch.float32, device=dev)
    out = {"workload": "512 pure quaternion problems, m,n ~ U{64..512}, rank k ~ U{8..32} + N(0,1e-3^2), "
                       "length sampling c=r=2k, U=C^+AR^+", "problems": len(dims)}
    seed = cfg["seed"]
    Bs = {}
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
        reps = max(args.steps, 10)
        t0 = time.perf_counter()
        for _ in range(reps):
            g.replay()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        q.sync_status()
        out[name] = dict(ms_per_batch=dt * 1e3, solves_per_s=len(dims) / dt)
        if tune:
            out[name]["plans"] = {k: list(v) for k, v in bs.plans().items()}
        log(f"batch {name}: {dt * 1e3:.3f} ms per {len(dims)} solves")
        if name != "f32_fixed_plans":
            # C U R from one more solve of the same variant (untimed)
            bsB = q.BatchSolver(dims, compute=comp, refine_steps=refine, a_dtype=torch.float32, autotune=tune,
                                want_B=True)
            bsB(A32, seed=seed)
            q.sync_status()
            nA = torch.linalg.vector_norm(A32.double(), dim=(1, 2, 3))
            out[name]["residual_max_rel_diff_vs_B_run"] = float(
                ((bs.residual.double() - bsB.residual.double()).abs() / nA).max())
            Bs[name] = (bsB.B.cpu().numpy(), bsB.I.cpu().numpy(), bsB.J.cpu().numpy())
            del bsB
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
    if use_oracle:
        import oracle
        A32h = A32.cpu().numpy().astype(np.float64)
        errs = {k: [] for k in Bs}
        t0 = time.perf_counter()
        for b, (m, n, c, r) in enumerate(dims):
            Ab = A32h[b, :, :m, :n]
            ref = oracle.solve(Ab, c, r, "length", "car", seed=seed + b)
            Bref = oracle.cur_product(ref["C"], ref["U"], ref["R"])
            for k, (B, I, J) in Bs.items():
                same = np.array_equal(I[b, :r], ref["I"]) and np.array_equal(J[b, :c], ref["J"])
                errs[k].append(rel_err(B[b, :, :m, :n], Bref) if same else float("nan"))
        out["oracle_seconds"] = time.perf_counter() - t0
        for k, e in errs.items():
            e = np.asarray(e)
            out[k]["cur_rel_err_vs_oracle"] = dict(max=float(np.max(e)), median=float(np.median(e)),
                                                   problems=int(len(e)), draws_differ=int(np.isnan(e).sum()))
        log("batch vs oracle (max over problems): " +
            ", ".join(f"{k} {out[k]['cur_rel_err_vs_oracle']['max']:.2e}" for k in errs))
        settle()
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


def bench_adjoint(q, torch, workloads, dev, args, use_oracle):
    """Masked CUR loss and its gradient through the adjoint kernels at
    2048 x 2048 (rank-64 N(0,1) factors, c = r = 256 fixed index sets,
    U = W^+ capped at rank 64, Bernoulli(0.5) mask): one forward + backward.
    At this exact-rank point C U R = A, so the loss and its gradient vanish;
    the accuracy check is the vector-Jacobian product of B = CUR(A) for a
    seeded N(0,1) cotangent, against the checker's."""
    import numpy as np
    cfg = workloads.WORKLOADS["adjoint_2048"]
    m, k, c = cfg["m"], cfg["k"], cfg["c"]
    L, Rt, _ = workloads.lowrank_gaussian_factors(m, m, k, cfg["seed"])
    A64 = quaternion_product_torch(torch, torch.tensor(L, device=dev), torch.tensor(Rt, device=dev))
    I = torch.tensor(workloads.uniform_index_set(m, c, cfg["seed"], 0), device=dev)
    J = torch.tensor(workloads.uniform_index_set(m, c, cfg["seed"], 1), device=dev)
    mask = torch.tensor(workloads.bernoulli_mask(m, m, cfg["mask_p"], cfg["seed"]), device=dev)
    gB_host = workloads.rng_for(cfg["seed"], 11).standard_normal((4, m, m))
    out = {"workload": "2048x2048 quaternion, rank-64 N(0,1) factors, c=r=256 fixed uniform index sets, U=W^+ "
                       "(max_rank 64), Bernoulli(0.5) mask, loss ||P_Omega(A - CUR(A))||_F^2, forward + backward"}
    vjp = {}
    for name, dt in (("f64", torch.float64), ("f32", torch.float32)):
        A = A64.to(dt)

        def step():
            At = A.detach().requires_grad_(True)
            loss = q.cur_loss(At, I, J, mask, max_rank=cfg["max_rank"])
            loss.backward()
            return loss, At.grad

        step()
        torch.cuda.synchronize()
        reps = max(2, args.steps // 2)
        t0 = time.perf_counter()
        for _ in range(reps):
            loss, g = step()
        torch.cuda.synchronize()
        dt_s = (time.perf_counter() - t0) / reps
        q.sync_status()
        nA = float(torch.linalg.vector_norm(A.to(torch.float64)))
        out[name] = dict(ms_per_step=dt_s * 1e3, steps_per_s=1.0 / dt_s,
                         loss_over_normA2=float(loss.detach()) / nA ** 2,
                         grad_norm_over_normA=float(torch.linalg.vector_norm(g.to(torch.float64))) / nA)
        dA, _ = q.backward(A, I, J, gB=torch.tensor(gB_host, dtype=dt, device=dev), max_rank=cfg["max_rank"])
        q.sync_status()
        vjp[name] = dA.to(torch.float64).cpu().numpy()
        log(f"adjoint {name}: {dt_s * 1e3:.2f} ms per forward+backward")
    if use_oracle:
        import oracle
        t0 = time.perf_counter()
        ref = oracle.grad.cur_vjp(A64.cpu().numpy(), I.cpu().numpy(), J.cpu().numpy(), gB_host,
                                  max_rank=cfg["max_rank"])
        out["oracle_vjp_seconds"] = time.perf_counter() - t0
        for name in vjp:
            out[name]["vjp_rel_err_vs_oracle"] = rel_err(vjp[name], ref)
        log("adjoint VJP vs oracle: " + ", ".join(f"{k} {out[k]['vjp_rel_err_vs_oracle']:.2e}" for k in vjp))
    return out


def bench_complete(q, torch, workloads, dev, use_oracle):
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

    def N64(t):
        return t.to(torch.float64).cpu().numpy()

    checks = []  # the checker runs after all timed runs (its host threads would compete with the launches)
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
        checks.append((name, N64(Y), iters, Xh))
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
    if use_oracle:
        # the checker's Algorithm 2 on the same inputs for the same numbers of steps
        import oracle
        for name, Yh, iters, Xh in checks:
            t1 = time.perf_counter()
            ref = oracle.complete.complete(Yh, mask, I, J, max_iter=iters, tol=0.0)
            out[name]["oracle_seconds"] = time.perf_counter() - t1
            out[name]["iterate_rel_err_vs_oracle"] = rel_err(Xh, ref["X"])
        settle()
    return out


def settle():
    """A pause after a checker run, so that its host threads have gone idle
    before the next timed GPU run (they would compete with its launches)."""
    time.sleep(1.0)


def bench_qsvd(q, torch, workloads, dev, use_oracle):
    """Example 4.2's comparison on one 500 x 500 rank-10 + N(0, 1e-4^2)
    quaternion matrix: QMCUR (length sampling, c = r = ceil(k ln k), FP64,
    least-squares core) against the thin QSVD of the whole matrix (Jacobi,
    FP64) and its rank-k truncation."""
    import numpy as np
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
    if use_oracle:
        import oracle
        ref = oracle.pinv.singular_values(A.cpu().numpy())
        out["singular_values_max_rel_err_vs_oracle"] = float(np.max(np.abs(sv - ref)) / ref[0])
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
    """The FP64 reference checker timed on the host cores: whole solves of
    the same 4096 x 4096 input (probabilities, draws, pseudoinverses through
    LAPACK, the core products), with the BLAS threads it starts with; a
    bounded sample of about `seconds` of CPU time (at least one solve).  Also
    returns the checker's I, J and C U R for the accuracy comparison."""
    import numpy as np
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
    except OSError:
        pass
    times, ref = [], None
    t_end = time.perf_counter() + seconds
    while True:
        t0 = time.perf_counter()
        ref = oracle.solve(A, c, r, "length", "car", seed=seed)
        times.append(time.perf_counter() - t0)
        if time.perf_counter() > t_end or len(times) >= 10:
            break
    med = float(np.median(times))
    B = oracle.cur_product(ref["C"], ref["U"], ref["R"])
    cpu = {"value": 1.0 / med, "unit": "solves/s", "cores": threads, "kind": "oracle",
           "sample": f"{len(times)} whole FP64 solves of the same 4096x4096 input (median "
                     f"{med:.2f} s each)", "host_cpus": os.cpu_count(), "cpu_model": model}
    log(f"oracle: {med:.2f} s per 4096x4096 solve on {threads} threads")
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
