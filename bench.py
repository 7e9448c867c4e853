#!/usr/bin/env python3
"""Throughput of the exact-GP hot path on one MI355X.

One step = covariance assembly + tiled Cholesky + predictive mean + full
posterior covariance (n = 16384 training points, n_test = 4096, D = 8,
tile 512, FP64), inputs resident in HBM. Reported as GFLOP/s with the flop
convention n^3/3 (Cholesky) + n^2 n_test (V solve) + n_test^2 n (W) + 2 n^2
(vector solves) + 2 n n_test (mean); assembly time counts, its flops do not.

Prints one JSON line. `--gpus` above 1 is refused: this path runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Cholesky+predict GFLOP/s & % peak at n=16384, FP64 vs mixed, at stated error"
FP64_PEAK_TFLOPS = 78.6     # MI355X dense FP64 (vector = matrix)
# the tile-update kernel of each precision and the dense matrix peak of its
# operand type (TFLOP/s)
UPDATE_KERNEL = {"fp64": ("k_update_f64 (GEMM/SYRK tile updates)", FP64_PEAK_TFLOPS),
                 "fp32": ("k_update_f32 (GEMM/SYRK tile updates, FP32 operands and "
                          "accumulator)", 157.3),
                 "bf16": ("k_update_bf16 (GEMM/SYRK tile updates, BF16 operands, FP32 "
                          "accumulator)", 2500.0)}

# HBM bytes per dispatch of the tile-update kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs scaled by a 1 GiB copy (profiles/fp64_c3_hbm_traffic.md); only
# valid for the kernel source they were taken on (k_update.hip + k_update_dev.h).
UPDATE_TRAFFIC = {"k_update_sha256_16": "d33c82f84f89af05", "bytes_per_launch": 972816478}


def update_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("k_update.hip", "k_update_dev.h"):
        h.update(open(os.path.join(ROOT, "paper_2602_19683_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def update_traffic():
    ok = update_source_hash() == UPDATE_TRAFFIC["k_update_sha256_16"]
    return UPDATE_TRAFFIC["bytes_per_launch"] if ok else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def path_flops(n, ns):
    return n ** 3 / 3 + n * n * ns + ns * ns * n + 2 * n * n + 2 * n * ns


def host_info():
    """Host CPU model and the logical CPUs this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    return model, nproc


def oracle_run(X, y, Xs, h, log):
    """The oracle (plain C, OpenMP, FP64) on the same workload, timed once:
    L, alpha, the mean and the full covariance from the plain definitions.
    Gives both the CPU baseline and the reference for the errors."""
    import oracle
    n, ns = X.shape[0], Xs.shape[0]
    log(f"oracle predict n={n} n_test={ns} on the host cores ...")
    t = time.perf_counter()
    ref = oracle.predict(X, y, Xs, h, want=("L", "alpha", "mean", "cov"))
    dt = time.perf_counter() - t
    model, nproc = host_info()
    cpu = {"value": round(path_flops(n, ns) / dt / 1e9, 3), "unit": "GFLOP/s",
           "cores": oracle.num_threads(), "kind": "oracle",
           "sample": f"the full workload: oracle predict (L, alpha, mean, full covariance), "
                     f"n={n}, n_test={ns}, D={X.shape[1]}, one run of {dt:.1f} s",
           "seconds": round(dt, 2), "nproc": nproc, "cpu_model": model}
    log(f"cpu baseline: {cpu}")
    return ref, cpu


def gpu_outputs(ctx, K, yd, mean, cov):
    """Host copies of the factor (dense, lower), alpha = K^{-1} y through the
    factor, the mean and the covariance of the last timed step."""
    import torch
    alpha = ctx.solve(K, yd)
    Ld = ctx.to_dense(K)
    torch.cuda.synchronize()
    out = {"L": Ld.cpu().numpy(), "alpha": alpha.cpu().numpy(), "mean": mean.cpu().numpy(),
           "cov": cov.cpu().numpy()}
    del Ld
    torch.cuda.empty_cache()
    return out


def errors_vs_oracle(got, ref):
    """Normwise relative errors against the oracle (lower triangle for L,
    2-norm for vectors, Frobenius for the covariance) and max|A-B|/max|B|
    for the covariance."""
    import oracle
    out = {}
    if got.get("L") is not None:
        out["rel_L"] = oracle.rel_err_lower(got["L"], ref["L"])
    if got.get("alpha") is not None:
        out["rel_alpha"] = oracle.rel_err(got["alpha"], ref["alpha"])
    out["rel_mean"] = oracle.rel_err(got["mean"], ref["mean"])
    if got.get("cov") is not None:
        out["rel_cov"] = oracle.rel_err(got["cov"], ref["cov"])
        out["max_rel_cov"] = oracle.max_rel(got["cov"], ref["cov"])
    return out


def mixed_runs(ctx, K, step, mean64, cov64, ms64, flops, args, log, ref=None):
    """FP32 / BF16 tile updates (FP64 POTRF, TRSM, solves, refinement): time
    per step, and errors against the oracle (ref, when it was run) and
    against the FP64 results of the same GPU run."""
    import torch
    L64 = ctx.to_dense(K)
    m64, c64 = mean64.clone(), cov64.clone()
    out = {}
    for prec in ("fp32", "bf16"):
        mean = torch.empty_like(m64)
        cov = torch.empty_like(c64)
        step(prec, mean, cov)
        ctx.sync()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            st = step(prec, mean, cov)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        L = ctx.to_dense(K)
        rel = lambda a, b: float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
        out[prec] = {
            "ms_per_step": round(ms, 4),
            "value": round(flops / (ms * 1e-3) / 1e9, 2),
            "speedup_vs_fp64": round(ms64 / ms, 3),
            "precision_used": {0: "fp64", 1: "fp32", 2: "bf16"}[st["precision"]],
            "ir_steps": st["iters"], "ir_method": st["method"],
            "ir_rel_residual": st["rel_residual"],
            "rel_mean_vs_fp64": rel(mean, m64),
            "rel_cov_vs_fp64": rel(cov, c64),
            "rel_L_vs_fp64": rel(torch.tril(L), torch.tril(L64)),
        }
        if ref is not None:
            torch.cuda.synchronize()
            got = {"L": L.cpu().numpy(), "mean": mean.cpu().numpy(), "cov": cov.cpu().numpy()}
            out[prec]["vs_oracle"] = errors_vs_oracle(got, ref)
            del got
        del L
        torch.cuda.empty_cache()
        log(f"mixed {prec}: {out[prec]}")
    del L64
    torch.cuda.empty_cache()
    return out


def persistent_run(Xd, yd, Xsd, h, tile, mean64, cov64, ms64, flops, args, log):
    """The same FP64 step with the persistent executor (one launch per sweep):
    time per step, and whether mean and covariance equal the stream
    executor's bit for bit."""
    import torch
    from paper_2602_19683_amd import GPR_EXEC_PERSISTENT, Context
    ctx = Context(0, executor=GPR_EXEC_PERSISTENT)
    mean = torch.empty_like(mean64)
    cov = torch.empty_like(cov64)
    K = None
    for _ in range(max(args.warmup, 1)):
        _, _, K, _ = ctx.fit_predict(Xd, yd, Xsd, h, tile, "fp64", K=K, mean=mean, cov=cov,
                                     ir_stats=True)
        ctx.sync()
    ctx.profile(True)
    ctx.profile_read(reset=True)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        ctx.fit_predict(Xd, yd, Xsd, h, tile, "fp64", K=K, mean=mean, cov=cov, ir_stats=True)
    e1.record()
    torch.cuda.synchronize()
    ctx.sync()
    ms = e0.elapsed_time(e1) / args.steps
    prof = ctx.profile_read(reset=True)
    ctx.profile(False)
    nl, tms, fl, _ = prof["persist"]
    out = {"ms_per_step": round(ms, 4), "value": round(flops / (ms * 1e-3) / 1e9, 2),
           "speedup_vs_streams": round(ms64 / ms, 3),
           "sweep_kernel_ms": round(tms / max(nl, 1), 4),
           "sweep_kernel_tflops": round(fl / (tms * 1e-3) / 1e12, 3) if tms else None,
           "bitwise_equal_to_streams": bool(torch.equal(mean, mean64) and torch.equal(cov, cov64))}
    K.free()
    ctx.close()
    log(f"persistent executor: {out}")
    return out


def mixed_mid_run(ctx, args, log):
    """Mixed precision where BF16 factors: n = 8192, n_test = 2048, tile 256,
    (l, v, sigma^2) = (1, 1, 0.1). Plain refinement does not contract with
    BF16 updates here, and conjugate gradients preconditioned by the BF16
    factor take over. Time per fused call (mean + full covariance), the
    refinement used, and errors against the FP64 call."""
    import torch
    from gpr_inputs import DEFAULT_HYPER, nfir_train_test
    n, ns, tile = 8192, 2048, 256
    X, y, Xs = nfir_train_test(n, ns)
    d = lambda a: torch.from_numpy(a).to("cuda:0")
    Xd, yd, Xsd = d(X), d(y), d(Xs)
    out, ref = {}, None
    for prec in ("fp64", "fp32", "bf16"):
        mean = torch.empty(ns, dtype=torch.float64, device="cuda:0")
        cov = torch.empty(ns, ns, dtype=torch.float64, device="cuda:0")
        _, _, K, st = ctx.fit_predict(Xd, yd, Xsd, DEFAULT_HYPER, tile, prec, mean=mean, cov=cov,
                                      ir_stats=True)
        ctx.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, _, _, st = ctx.fit_predict(Xd, yd, Xsd, DEFAULT_HYPER, tile, prec, K=K, mean=mean,
                                          cov=cov, ir_stats=True)
        ctx.sync()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        rel = lambda a, b: float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
        r = {"ms_per_call": round(ms, 4)}
        if prec == "fp64":
            ref = (mean.clone(), cov.clone())
        else:
            r.update({"precision_used": {0: "fp64", 1: "fp32", 2: "bf16"}[st["precision"]],
                      "refinement": st["method"], "refinement_steps": st["iters"],
                      "rel_residual": st["rel_residual"],
                      "rel_mean_vs_fp64": rel(mean, ref[0]), "rel_cov_vs_fp64": rel(cov, ref[1])})
        out[prec] = r
        K.free()
    out["config"] = f"n={n}, n_test={ns}, D=8, tile {tile}, (l, v, sigma^2) = {DEFAULT_HYPER}"
    log(f"mixed at n=8192: {out}")
    return out


def timed_calls(fn, steps, warm=1):
    """Mean ms per call of fn() over `steps` calls after `warm` untimed ones
    (device time between two events on the current stream)."""
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def left_looking_run(Xd, yd, Xsd, h, tile, ms64, mean64, cov64, flops, args, log):
    """The left-looking task order: the benchmarked FP64 step and the FP32 /
    BF16 forms at the same size, and the three precisions at n = 8192,
    n_test = 2048, tile 256; errors against the right-looking FP64 results."""
    import torch
    from gpr_inputs import DEFAULT_HYPER, nfir_train_test
    from paper_2602_19683_amd import Context
    rel = lambda a, b: float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
    out = {}
    ctx = Context(0, variant="left")
    ns = Xsd.shape[0]
    mean = torch.empty_like(mean64)
    cov = torch.empty_like(cov64)
    K = None
    for prec in ("fp64", "fp32", "bf16"):
        st = {}

        def call():
            nonlocal K
            _, _, K, s_ = ctx.fit_predict(Xd, yd, Xsd, h, tile, prec, K=K, mean=mean, cov=cov,
                                          ir_stats=True)
            st.update(s_)
        ms = timed_calls(call, args.steps)
        ctx.sync()
        out[prec] = {"ms_per_step": round(ms, 4), "value": round(flops / (ms * 1e-3) / 1e9, 2),
                     "vs_right_looking_fp64": round(ms64 / ms, 3),
                     "rel_mean_vs_fp64": rel(mean, mean64), "rel_cov_vs_fp64": rel(cov, cov64)}
        if prec != "fp64":
            out[prec].update({"precision_used": {0: "fp64", 1: "fp32", 2: "bf16"}[st["precision"]],
                              "refinement": st["method"], "refinement_steps": st["iters"]})
        log(f"left-looking {prec}: {out[prec]}")
    K.free()
    n2, ns2, tile2 = 8192, 2048, 256
    X, y, Xs = nfir_train_test(n2, ns2)
    d = lambda a: torch.from_numpy(a).to("cuda:0")
    X2, y2, Xs2 = d(X), d(y), d(Xs)
    mid = {}
    ref = None
    for variant in ("right", "left"):
        ctx.set_variant(variant)
        for prec in ("fp64", "fp32", "bf16"):
            m2 = torch.empty(ns2, dtype=torch.float64, device="cuda:0")
            c2 = torch.empty(ns2, ns2, dtype=torch.float64, device="cuda:0")
            K2 = None
            st = {}

            def call2():
                nonlocal K2
                _, _, K2, s_ = ctx.fit_predict(X2, y2, Xs2, DEFAULT_HYPER, tile2, prec, K=K2,
                                               mean=m2, cov=c2, ir_stats=True)
                st.update(s_)
            ms = timed_calls(call2, args.steps)
            ctx.sync()
            r = {"ms_per_call": round(ms, 4)}
            if ref is None:
                ref = (m2.clone(), c2.clone())
            else:
                r.update({"rel_mean_vs_fp64": rel(m2, ref[0]), "rel_cov_vs_fp64": rel(c2, ref[1])})
            if prec != "fp64":
                r.update({"precision_used": {0: "fp64", 1: "fp32", 2: "bf16"}[st["precision"]],
                          "refinement": st["method"], "refinement_steps": st["iters"]})
            mid[f"{variant}_{prec}"] = r
            K2.free()
    mid["config"] = f"n={n2}, n_test={ns2}, D=8, tile {tile2}, (l, v, sigma^2) = {DEFAULT_HYPER}"
    out["n8192_tile256"] = mid
    log(f"left-looking at n=8192: {mid}")
    ctx.close()
    return out


def sweep_runs(args, log):
    """Smaller configurations: n = 4096, n_test = 1024 over tiles 128 / 256 /
    512 (time per fused FP64 call, and the assembly and factorisation-sweep
    parts from the per-launch timers), and the latency of n = 128,
    n_test = 128, tile 32 in microseconds on the stream executor and on an
    automatic-executor context (which picks the persistent one here)."""
    import torch
    from gpr_inputs import DEFAULT_HYPER, nfir_train_test
    from paper_2602_19683_amd import GPR_EXEC_AUTO, Context
    d = lambda a: torch.from_numpy(a).to("cuda:0")
    out = {}
    n, ns = 4096, 1024
    X, y, Xs = nfir_train_test(n, ns)
    Xd, yd, Xsd = d(X), d(y), d(Xs)
    with Context(0) as ctx:
        for tile in (128, 256, 512):
            mean = torch.empty(ns, dtype=torch.float64, device="cuda:0")
            cov = torch.empty(ns, ns, dtype=torch.float64, device="cuda:0")
            K = None

            def call():
                nonlocal K
                K = ctx.fit_predict(Xd, yd, Xsd, DEFAULT_HYPER, tile, "fp64", K=K, mean=mean,
                                    cov=cov)[2]
            ms = timed_calls(call, max(args.steps, 10))
            ctx.profile(True)
            ctx.profile_read(reset=True)
            reps = max(args.steps, 10)
            for _ in range(reps):
                call()
            prof = ctx.profile_read(reset=True)
            ctx.profile(False)
            part = lambda *ks: round(sum(prof[k][1] for k in ks) / reps, 4)
            out[f"tile{tile}"] = {
                "ms_per_call": round(ms, 4),
                "gflops": round(path_flops(n, ns) / (ms * 1e-3) / 1e9, 1),
                "assembly_ms": part("assemble"),
                "sweep_kernels_ms": part("potrf", "trsm", "update"),
                "solves_mean_export_ms": part("trtri", "trsv", "matvec", "export")}
            K.free()
        out["c2_config"] = f"n={n}, n_test={ns}, D=8, fp64, gpr_fit_predict; kernel times are " \
                           f"sums over launches (the streams overlap)"
        X1, y1, Xs1 = nfir_train_test(128, 128)
        X1d, y1d, Xs1d = d(X1), d(y1), d(Xs1)
        mean = torch.empty(128, dtype=torch.float64, device="cuda:0")
        cov = torch.empty(128, 128, dtype=torch.float64, device="cuda:0")
        K = None

        def small():
            nonlocal K
            K = ctx.fit_predict(X1d, y1d, Xs1d, DEFAULT_HYPER, 32, "fp64", K=K, mean=mean,
                                cov=cov)[2]
        ms = timed_calls(small, 50, warm=5)
        out["c1_latency_us"] = round(ms * 1e3, 1)
        out["c1_config"] = "n=128, n_test=128, D=8, tile 32, fp64, gpr_fit_predict (mean + full " \
                           "covariance), mean of 50 calls"
        K.free()
        ref = (mean.clone(), cov.clone())
    # the same call on a GPR_EXEC_AUTO context, which runs this sweep on the
    # persistent executor (one launch instead of the per-step launches)
    with Context(0, executor=GPR_EXEC_AUTO) as actx:
        K = None

        def small_auto():
            nonlocal K
            K = actx.fit_predict(X1d, y1d, Xs1d, DEFAULT_HYPER, 32, "fp64", K=K, mean=mean,
                                 cov=cov)[2]
        ms = timed_calls(small_auto, 50, warm=5)
        out["c1_latency_us_auto"] = round(ms * 1e3, 1)
        out["c1_auto_bitwise_equal"] = bool(torch.equal(mean, ref[0]) and torch.equal(cov, ref[1]))
        K.free()
    log(f"sweeps: {out}")
    return out


def large_run(args, log):
    """The large configuration: n = 32768, n_test = 8192, D = 8, tile 1024.
    FP32-update factorisation with FP64 refinement and the full covariance
    (one fused call), and the FP64 NLML with its gradient, on the stream
    executor and on the persistent executor; errors of the mixed mean and
    covariance against the FP64 streams result of the same run."""
    import torch
    from gpr_inputs import DEFAULT_HYPER, nfir_train_test
    from paper_2602_19683_amd import GPR_EXEC_PERSISTENT, GPR_EXEC_STREAMS, Context
    n, ns, tile = 32768, 8192, 1024
    X, y, Xs = nfir_train_test(n, ns)
    d = lambda a: torch.from_numpy(a).to("cuda:0")
    Xd, yd, Xsd = d(X), d(y), d(Xs)
    rel = lambda a, b: float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
    out, ref = {}, None
    steps = max(1, min(args.steps, 3))
    for name, ex in (("streams", GPR_EXEC_STREAMS), ("persistent", GPR_EXEC_PERSISTENT)):
        with Context(0, executor=ex) as ctx:
            r = {}
            for prec in ("fp64", "fp32"):
                mean = torch.empty(ns, dtype=torch.float64, device="cuda:0")
                cov = torch.empty(ns, ns, dtype=torch.float64, device="cuda:0")
                K = None
                st = {}

                def call():
                    nonlocal K
                    _, _, K, s_ = ctx.fit_predict(Xd, yd, Xsd, DEFAULT_HYPER, tile, prec, K=K,
                                                  mean=mean, cov=cov, ir_stats=True)
                    st.update(s_)
                ms = timed_calls(call, steps)
                ctx.sync()
                r[prec] = {"ms_per_call": round(ms, 2),
                           "gflops": round(path_flops(n, ns) / (ms * 1e-3) / 1e9, 1)}
                if ref is None:
                    ref = (mean.clone(), cov.clone())
                else:
                    r[prec].update({"rel_mean_vs_fp64_streams": rel(mean, ref[0]),
                                    "rel_cov_vs_fp64_streams": rel(cov, ref[1])})
                if prec != "fp64":
                    r[prec].update({"precision_used": {0: "fp64", 1: "fp32", 2: "bf16"}[st["precision"]],
                                    "refinement": st["method"], "refinement_steps": st["iters"]})
                K.free()
                del mean, cov
                torch.cuda.empty_cache()
                log(f"large {name} {prec}: {r[prec]}")
            res = {}

            def nl():
                res["v"] = ctx.nlml_grad(Xd, yd, DEFAULT_HYPER, tile)
            ms = timed_calls(nl, 1)
            ctx.sync()
            r["nlml_grad_ms"] = round(ms, 2)
            r["nlml"] = float(res["v"][0].cpu()[0])
            r["grad"] = [float(v) for v in res["v"][1].cpu()]
            log(f"large {name} nlml+grad: {ms:.1f} ms")
            out[name] = r
            torch.cuda.empty_cache()
    out["config"] = f"n={n}, n_test={ns}, D=8, tile {tile}, (l, v, sigma^2) = {DEFAULT_HYPER}"
    return out


def variants_run(ctx, K, Xd, yd, Xsd, h, tile, args, log):
    """The prediction variants of the same fit (FP64, one fused call each):
    mean only (no test rows swept) and mean + predictive variances (V^T
    formed, the test block skipped), time per call."""
    import torch
    ns = Xsd.shape[0]
    mean = torch.empty(ns, dtype=torch.float64, device="cuda:0")
    var = torch.empty(ns, dtype=torch.float64, device="cuda:0")
    calls = {
        "mean_only": lambda: ctx.fit_predict(Xd, yd, Xsd, h, tile, "fp64", full_cov=False, K=K,
                                             mean=mean),
        "mean_and_variance": lambda: ctx.fit_predict_var(Xd, yd, Xsd, h, tile, "fp64", K=K,
                                                         mean=mean, var=var),
    }
    out = {}
    for name, call in calls.items():
        call()
        ctx.sync()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            call()
        e1.record()
        torch.cuda.synchronize()
        ctx.sync()
        out[name + "_ms"] = round(e0.elapsed_time(e1) / args.steps, 4)
    log(f"variants: {out}")
    return out


def isolated_update_run(Xd, yd, Xsd, h, tile, precision, args, log):
    """The same step with every launch on one stream (no overlap between
    launches): per-launch time and rate of the tile-update kernel alone, so
    that its roofline fraction is not shared with concurrent launches."""
    import torch
    from paper_2602_19683_amd import Context
    ctx = Context(0, n_streams=1)
    K = None
    mean = torch.empty(Xsd.shape[0], dtype=torch.float64, device="cuda:0")
    cov = torch.empty(Xsd.shape[0], Xsd.shape[0], dtype=torch.float64, device="cuda:0")
    for _ in range(max(args.warmup, 1)):
        _, _, K = ctx.fit_predict(Xd, yd, Xsd, h, tile, precision, K=K, mean=mean, cov=cov)
        ctx.sync()
    ctx.profile(True)
    ctx.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.fit_predict(Xd, yd, Xsd, h, tile, precision, K=K, mean=mean, cov=cov)
    ctx.sync()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    prof = ctx.profile_read(reset=True)
    ctx.profile(False)
    nl, tms, fl, _ = prof["update"]
    out = {"streams": 1, "ms_per_step": round(ms, 4),
           "update_launches_per_step": nl / args.steps,
           "update_avg_launch_ms": round(tms / max(nl, 1), 4),
           "update_ms_per_step": round(tms / args.steps, 4),
           "achieved": round(fl / (tms * 1e-3) / 1e12, 3) if tms else None,
           "frac": round(fl / (tms * 1e-3) / 1e12 / UPDATE_KERNEL[precision][1], 4)
           if tms else None}
    K.free()
    ctx.close()
    log(f"isolated update kernel (one stream): {out}")
    return out


def library_run(ctx, K, Xd, h, tile, args, log):
    """The single-tile analogue: the vendor dense Cholesky (torch.linalg.cholesky
    on the assembled n x n FP64 matrix, rocSOLVER through hipSOLVER) against this
    library's assembly + tiled Cholesky of the same matrix, and the normwise
    difference between the two factors."""
    import torch
    torch.backends.cuda.preferred_linalg_library("cusolver")
    ctx.assemble(Xd, h, tile, K=K)
    A = ctx.to_dense(K)
    ctx.sync()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    ms_lib = timed(lambda: torch.linalg.cholesky(A))
    ms_asm = timed(lambda: ctx.assemble(Xd, h, tile, K=K))
    ms_ours = timed(lambda: (ctx.assemble(Xd, h, tile, K=K), ctx.cholesky(K)))
    ctx.sync()
    L_ours = torch.tril(ctx.to_dense(K))
    L_lib = torch.linalg.cholesky(A)
    torch.cuda.synchronize()
    diff = float(torch.linalg.norm(L_ours - L_lib) / torch.linalg.norm(L_lib))
    n = A.shape[0]
    out = {"vendor_cholesky_ms": round(ms_lib, 4),
           "vendor_gflops": round(n ** 3 / 3 / (ms_lib * 1e-3) / 1e9, 1),
           "tiled_cholesky_ms": round(ms_ours - ms_asm, 4),
           "tiled_gflops": round(n ** 3 / 3 / ((ms_ours - ms_asm) * 1e-3) / 1e9, 1),
           "rel_diff_factor": diff,
           "vendor": "torch.linalg.cholesky (hipSOLVER / rocSOLVER), one n x n FP64 matrix"}
    del A, L_ours, L_lib
    torch.cuda.empty_cache()
    log(f"library comparator: {out}")
    return out


def nlml_run(ctx, args, log):
    """The gradient workload: NLML and its gradient in (l, v, sigma^2) at
    n = 8192, D = 8, tile 256, from (0.3, 2.0, 0.5): time per evaluation
    (forward factorisation + reverse sweep + reduction) and per NLML-only
    evaluation, with GFLOP/s over n^3/3 (forward) + 2 n^3/3 (adjoint)."""
    import torch
    from gpr_inputs import nfir
    n, tile, h = 8192, 256, (0.3, 2.0, 0.5)
    X, y = nfir(n)
    Xd, yd = torch.from_numpy(X).to("cuda:0"), torch.from_numpy(y).to("cuda:0")
    out = {}
    for grad in (True, False):
        ctx.nlml_grad(Xd, yd, h, tile, grad=grad)
        ctx.sync()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            nl, g, _ = ctx.nlml_grad(Xd, yd, h, tile, grad=grad)
        e1.record()
        torch.cuda.synchronize()
        ctx.sync()
        ms = e0.elapsed_time(e1) / args.steps
        if grad:
            out["ms_nlml_and_grad"] = round(ms, 4)
            out["gflops_nlml_and_grad"] = round(n ** 3 / ms * 1e-6, 2)  # (1/3 + 2/3) n^3
            out["nlml"] = float(nl.cpu()[0])
            out["grad"] = [float(v) for v in g.cpu()]
        else:
            out["ms_nlml_only"] = round(ms, 4)
    # the hyperparameter fit (gpr_fit_hyper): Adam steps, each one NLML and
    # gradient evaluation plus the Adam step on the device (the host reads the
    # stop flag every few steps)
    import time
    ctx.fit_hyper(Xd, yd, h, tile, max_steps=1)
    t0 = time.perf_counter()
    th, tr, k = ctx.fit_hyper(Xd, yd, h, tile, max_steps=args.steps)
    out["ms_per_adam_step"] = round((time.perf_counter() - t0) * 1e3 / k, 4)
    out["adam_nlml_first_last"] = [float(tr[0]), float(tr[-1])]
    out["config"] = f"n={n}, D=8, tile {tile}, (l, v, sigma^2) = {h}, fp64"
    log(f"nlml: {out}")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--n-test", type=int, default=4096)
    ap.add_argument("--tile", type=int, default=512)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the FP32 / BF16 comparison runs after the FP64 line")
    ap.add_argument("--path", default="fused", choices=["fused", "calls"],
                    help="fused: gpr_fit_predict (one sweep); calls: assemble + cholesky + predict")
    ap.add_argument("--streams", type=int, default=3,
                    help="1 = no overlap between launches (isolated kernel timings)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-nlml", action="store_true",
                    help="skip the NLML-gradient timing (n = 8192, tile 256) after the line")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-isolated", action="store_true",
                    help="skip the one-stream run that times the update kernel alone")
    ap.add_argument("--no-persistent", action="store_true",
                    help="skip the persistent-executor timing of the same FP64 step")
    ap.add_argument("--no-library", action="store_true",
                    help="skip the vendor dense-Cholesky comparator")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the mean-only and mean + variance timings")
    ap.add_argument("--executor", default="streams", choices=["streams", "persistent"],
                    help="executor of the timed line (persistent: one launch per sweep)")
    ap.add_argument("--variant", default="right", choices=["right", "left"],
                    help="task order of the timed line (right- or left-looking Cholesky)")
    ap.add_argument("--no-left", action="store_true",
                    help="skip the left-looking timings after the line")
    ap.add_argument("--no-sweeps", action="store_true",
                    help="skip the n = 4096 tile sweep and the n = 128 latency")
    ap.add_argument("--large", action="store_true",
                    help="only the n = 32768, n_test = 8192, tile 1024 runs (streams vs "
                         "persistent; FP32-update prediction and the NLML gradient)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run one device-to-device copy of MIB MiB (for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the GP hot path runs on one GPU only here; "
              "multi-GPU sharding is a design note, not a measured path (use --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        nel = args.calibrate_copy * (1 << 20) // 8
        a = torch.ones(nel, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"copied {args.calibrate_copy} MiB (read {args.calibrate_copy} MiB, write {args.calibrate_copy} MiB)")
        return
    if args.large:
        print(json.dumps({"large": large_run(args, log)}), flush=True)
        return
    from gpr_inputs import DEFAULT_HYPER, nfir_train_test
    from paper_2602_19683_amd import GPR_EXEC_PERSISTENT, GPR_EXEC_STREAMS, Context, _lib

    n, ns, tile, D = args.n, args.n_test, args.tile, 8
    h = DEFAULT_HYPER
    log(f"bench: path={args.path} n={n} n_test={ns} tile={tile} precision={args.precision} "
        f"steps={args.steps} warmup={args.warmup}")
    X, y, Xs = nfir_train_test(n, ns, D)
    dev = lambda a: torch.from_numpy(a).to("cuda:0")
    Xd, yd, Xsd = dev(X), dev(y), dev(Xs)
    mean = torch.empty(ns, dtype=torch.float64, device="cuda:0")
    cov = torch.empty(ns, ns, dtype=torch.float64, device="cuda:0")
    persistent_line = args.executor == "persistent"
    ctx = Context(0, n_streams=args.streams,
                  executor=GPR_EXEC_PERSISTENT if persistent_line else GPR_EXEC_STREAMS,
                  variant=args.variant)
    K = ctx.assemble(Xd, h, tile)

    def step(prec=args.precision, out_mean=mean, out_cov=cov):
        if args.path == "fused":
            return ctx.fit_predict(Xd, yd, Xsd, h, tile, prec, K=K, mean=out_mean, cov=out_cov,
                                   ir_stats=True)[3]
        ctx.assemble(Xd, h, tile, K=K)
        ctx.cholesky(K, prec)
        return ctx.predict(K, Xd, yd, Xsd, h, mean=out_mean, cov=out_cov, ir_stats=True)[2]

    for i in range(args.warmup):
        step()
        ctx.sync()
        log(f"warmup step {i + 1}/{args.warmup} done")
    ctx.profile(True)
    ctx.profile_read(reset=True)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t_wall = time.perf_counter()
    e0.record()
    marks[0].record()
    for i in range(args.steps):
        step()
        marks[i + 1].record()
    e1.record()
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ctx.sync()
    ms = e0.elapsed_time(e1) / args.steps
    per = [marks[i].elapsed_time(marks[i + 1]) for i in range(args.steps)]
    sd = (sum((x - ms) ** 2 for x in per) / max(len(per) - 1, 1)) ** 0.5
    ci95 = 1.96 * sd / max(len(per), 1) ** 0.5
    prof = ctx.profile_read(reset=True)
    ctx.profile(False)
    log(f"timed {args.steps} steps: {ms:.3f} ms/step (wall {t_wall / args.steps * 1e3:.3f})")
    for k, (nl, tms, fl, by) in prof.items():
        rate = f"{fl / (tms * 1e-3) / 1e12:7.2f} TFLOP/s" if fl and tms else \
               (f"{by / (tms * 1e-3) / 1e9:7.1f} GB/s" if by and tms else "")
        log(f"  {k:9s} launches/step {nl / args.steps:7.1f}  ms/step {tms / args.steps:8.3f}  {rate}")

    flops = path_flops(n, ns)
    value = flops / (ms * 1e-3) / 1e9
    nl, tms, fl, _ = prof["persist" if persistent_line else "update"]
    achieved = fl / (tms * 1e-3) / 1e12 if tms else 0.0
    kname, peak = UPDATE_KERNEL[args.precision]
    if persistent_line:
        kname = "k_persist (the whole sweep: POTRF panels, TRSM strips, update blocks)"
    roofline = {"bound": "mfma",
                "kernel": kname,
                "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4),
                # counters were taken for the FP64 kernel only
                "traffic": update_traffic() if args.precision == "fp64" and not persistent_line
                           else None,
                "traffic_unit": "bytes per launch",
                "avg_launch_ms": round(tms / max(nl, 1), 4),
                "flops_per_launch": round(fl / max(nl, 1), 1),
                "note": "launches of the timed region overlap across three streams, so "
                        "avg_launch_ms is shared compute; 'isolated' runs the same step on "
                        "one stream, 'step_level' divides the kernel's algorithmic flops "
                        "per step by the whole step time",
                "step_level": {"achieved": round(fl / args.steps / (ms * 1e-3) / 1e12, 3),
                               "frac": round(fl / args.steps / (ms * 1e-3) / 1e12
                                             / peak, 4)}}
    if not args.no_isolated and not persistent_line:
        roofline["isolated"] = isolated_update_run(Xd, yd, Xsd, h, tile, args.precision, args,
                                                   log)
    ref = cpu = errors = None
    if not (args.no_check and args.no_cpu_baseline):
        got = gpu_outputs(ctx, K, yd, mean, cov)
        ref, cpu = oracle_run(X, y, Xs, h, log)
        if not args.no_check:
            errors = errors_vs_oracle(got, ref)
            errors["reference"] = "oracle (full, same workload)"
            log(f"errors: {errors}")
        if args.no_cpu_baseline:
            cpu = None
        del got
    persistent = None
    if (not args.no_persistent and not persistent_line and args.precision == "fp64"
            and args.path == "fused"):
        persistent = persistent_run(Xd, yd, Xsd, h, tile, mean, cov, ms, flops, args, log)
    library = None
    if not args.no_library and args.precision == "fp64":
        library = library_run(ctx, K, Xd, h, tile, args, log)
    variants = None
    if not args.no_variants and args.path == "fused":
        variants = variants_run(ctx, K, Xd, yd, Xsd, h, tile, args, log)
    mixed = None
    if not args.no_mixed and args.precision == "fp64":
        mixed = mixed_runs(ctx, K, step, mean, cov, ms, flops, args, log,
                           ref)
        mixed["n8192_tile256"] = mixed_mid_run(ctx, args, log)
    nlml = None
    if not args.no_nlml:
        nlml = nlml_run(ctx, args, log)
    left = None
    if not args.no_left and args.precision == "fp64" and args.path == "fused" \
            and args.variant == "right" and not persistent_line:
        left = left_looking_run(Xd, yd, Xsd, h, tile, ms, mean, cov, flops, args, log)
    sweeps = None
    if not args.no_sweeps:
        sweeps = sweep_runs(args, log)
    del ref
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "ms_per_step_ci95": round(ci95, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else
                 f"f64 with {args.precision} tile updates",
        "data": "synthetic",
        "config": {"workload": f"exact GP, SE kernel: assembly + tiled Cholesky + mean + full "
                               f"covariance, n={n}, n_test={ns}, D={D}, tile {tile}, "
                               f"{args.precision}",
                   "n": n, "n_test": ns, "D": D, "tile": tile, "precision": args.precision,
                   "entry": "gpr_fit_predict" if args.path == "fused" else
                            "gpr_assemble + gpr_cholesky + gpr_predict",
                   "executor": args.executor, "variant": args.variant,
                   "parallelism": "single GPU"},
        "pct_fp64_peak": round(100 * value / (FP64_PEAK_TFLOPS * 1e3), 2),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "errors": errors,
        "mixed": mixed,
        "persistent_executor": persistent,
        "prediction_variants": variants,
        "library_comparator": library,
        "nlml_grad": nlml,
        "left_looking": left,
        "sweeps": sweeps,
        "phases_ms_per_step": {k: round(v[1] / args.steps, 4) for k, v in prof.items()},
        "lib_source_hash": _lib.library_hash(),
    }
    print(json.dumps(out), flush=True)
    K.free()
    ctx.close()


if __name__ == "__main__":
    main()
