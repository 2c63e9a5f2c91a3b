"""Benchmark: PCG time-to-solve at 1e-8 relative residual on one MI355X.

Workload (the 3D case the metric is quoted on): thick quarter ring
F(xi) = ((1+xi1) cos(pi xi2/2), (1+xi1) sin(pi xi2/2), xi3), p = 3, 128^3
elements (n = 129 per direction, N = 2,146,689 dofs), f = 3 pi^2 prod sin(pi x_i),
x0 = 0, stop at ||r|| <= 1e-8 ||b||, FD preconditioner in FP64.

A step is one full PCG solve (init, iterations, FP64 true-residual check) with
A, U_d and b resident in HBM.  Also reported: the FP32 and BF16 flexible
solves, preconditioner applies per second, per-kernel timings from HIP events
on the library's stream, the roofline of the dominant kernel (the banded A
product) and the FP64 oracle timed on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
FP64_PEAK_TF = 78.6


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def event_time(torch, fn, reps):
    """Average device time (ms) of `fn` over `reps` back-to-back calls,
    bracketed by HIP events on the current stream (the library's stream)."""
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


def cpu_baseline(target_iters, n_full, p, nnz_full):
    """The FP64 oracle (NumPy/SciPy, as it stands) on a bounded sample of the
    same workload: the thick ring at 32^3 elements, p = 3.  Its time per CG
    iteration is scaled by the ratio of FLOPs per iteration (A product
    2 nnz, FD apply 4 N sum n_d) to the full workload and multiplied by the
    GPU's iteration count."""
    import synth
    from oracle import assembly, fd, pcg
    E = 32
    prob = synth.thick_ring(E=E, p=p)
    A = assembly.assemble_matrix(prob)
    F = fd.setup(prob)
    b = assembly.assemble_load(prob, synth.RHS_SINPROD)
    t0 = time.perf_counter()
    reps = 0
    iters = 0
    while time.perf_counter() - t0 < 10.0 or reps < 3:
        _, info = pcg.solve(prob, A, F, b, rtol=1e-8)
        iters += info["iters"]
        reps += 1
    dt = time.perf_counter() - t0
    n_s = E + p - 2
    N_s = n_s ** 3
    per_iter = dt / iters
    flops_s = 2 * A.nnz + 4 * N_s * 3 * n_s
    N_f = n_full ** 3
    flops_f = 2 * nnz_full + 4 * N_f * 3 * n_full
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    return {"value": per_iter * flops_f / flops_s * target_iters, "unit": "s", "cores": int(cores),
            "kind": "oracle",
            "sample": f"oracle PCG on the thick ring at {E}^3 elements p={p} (N={N_s}), {reps} solves, "
                      f"{per_iter * 1e3:.2f} ms/iteration, scaled by FLOPs/iteration to {n_full}^3 dofs "
                      f"and x {target_iters} iterations",
            "sample_s_per_iter": per_iter}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--elements", type=int, default=128)
    ap.add_argument("--degree", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the solver runs on a single device and has no "
              "multi-GPU path in this build (--gpus must be 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    import paper_1602_01636_amd as api

    torch.cuda.set_device(0)
    E, p = args.elements, args.degree
    prob = synth.thick_ring(E=E, p=p)
    t0 = time.perf_counter()
    ctx = api.igafd_setup(prob)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    N = ctx.N
    n = ctx.n[0]
    log(f"setup {t_setup:.2f}s N={N} nnz={ctx.nnz} band={ctx.band_bytes / 1e9:.2f} GB")
    b = torch.zeros(N, dtype=torch.float64, device="cuda")
    api.igafd_load_vector(ctx, synth.RHS_SINPROD, b)
    u = torch.zeros_like(b)

    def solve(prec="fp64"):
        return api.igafd_solve(ctx, b, u, rtol=1e-8, precision=prec)

    for _ in range(args.warmup):
        solve()
    torch.cuda.synchronize()
    times, infos = [], []
    t_all = time.perf_counter()
    for k in range(args.steps):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        info = solve()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
        infos.append(info)
        log(f"step {k}: {times[-1] * 1e3:.2f} ms iters {info['iters']} true_relres {info['true_relres']:.2e}")
    wall = time.perf_counter() - t_all
    u64 = u.clone()
    ms_per_step = 1e3 * sum(times) / len(times)
    iters = infos[-1]["iters"]

    # per-kernel device times (HIP events on the library stream)
    x = torch.randn(N, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    t_spmv = event_time(torch, lambda: api.igafd_apply_A(ctx, x, y), 50)
    t_fd = {pr: event_time(torch, lambda pr=pr: api.igafd_apply_precond(ctx, pr, x, y), 50)
            for pr in ("fp64", "fp32", "bf16")}
    applies_per_s = {pr: 1e3 / t for pr, t in t_fd.items()}
    # algorithmic bytes of one A product: each stored (symmetric) value once,
    # x read once, y written once
    unique_vals = (ctx.nnz + N) // 2
    spmv_bytes = 8 * unique_vals + 16 * N
    spmv_gbs = spmv_bytes / (t_spmv * 1e-3) / 1e9
    fd_flops = 4 * N * 3 * n + N
    log(f"spmv {t_spmv * 1e3:.1f} us = {spmv_gbs:.0f} GB/s; FD fp64 {t_fd['fp64'] * 1e3:.1f} us "
        f"({fd_flops / t_fd['fp64'] / 1e9:.1f} TFLOP/s) fp32 {t_fd['fp32'] * 1e3:.1f} us bf16 {t_fd['bf16'] * 1e3:.1f} us")

    variants = {}
    if not args.no_variants:
        for prec in ("fp32", "bf16"):
            solve(prec)
            ts = []
            for _ in range(max(2, args.steps // 2)):
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                inf = solve(prec)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t1)
            err = float(torch.linalg.norm(u - u64) / torch.linalg.norm(u64))
            variants[prec] = {"s": float(np.median(ts)), "iters": inf["iters"], "true_relres": inf["true_relres"],
                              "rel_err_vs_fp64": err}
            log(f"{prec}: {variants[prec]}")

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(iters, n, p, ctx.nnz)
        log(f"cpu baseline {cpu['value']:.2f} s ({cpu['sample']})")

    out = {
        "metric": "PCG time-to-solve @1e-8 rel. residual (s) + iters; precond applies/sec",
        "value": ms_per_step / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"thick quarter ring, p={p}, {E}^3 elements, n={n}/dir, N={N} dofs, "
                               f"f=3pi^2 prod sin(pi x_i), FP64 FD-preconditioned CG, rtol 1e-8",
                   "elements": E, "degree": p, "N": N, "nnz": ctx.nnz},
        "iters": iters,
        "true_relres": infos[-1]["true_relres"],
        "precond_applies_per_s": applies_per_s,
        "kernel_ms": {"spmv": t_spmv, "fd_fp64": t_fd["fp64"], "fd_fp32": t_fd["fp32"], "fd_bf16": t_fd["bf16"]},
        "variants": variants,
        "setup_s": t_setup,
        "wall_s_timed": wall,
        "roofline": {"bound": "hbm", "achieved": spmv_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": spmv_gbs / HBM_PEAK_GBS, "traffic": None, "kernel": "k_spmv (A x)",
                     "algorithmic_bytes": spmv_bytes},
        "fd_roofline": {"bound": "mfma", "achieved": fd_flops / t_fd["fp64"] / 1e9, "peak": FP64_PEAK_TF,
                        "unit": "TFLOP/s", "frac": fd_flops / t_fd["fp64"] / 1e9 / FP64_PEAK_TF},
        "cpu_baseline": cpu,
    }
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
