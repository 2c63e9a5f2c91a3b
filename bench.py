"""Benchmark: PCG time-to-solve at 1e-8 relative residual on one MI355X.

Default workload (the 3D case the metric is quoted on): thick quarter ring
F(xi) = ((1+xi1) cos(pi xi2/2), (1+xi1) sin(pi xi2/2), xi3), p = 3, 128^3
elements (n = 129 per direction, N = 2,146,689 dofs), f = 3 pi^2 prod sin(pi x_i),
x0 = 0, stop at ||r|| <= 1e-8 ||b||, FD preconditioner in FP64.

A step is one full PCG solve (init, iterations, FP64 true-residual check) with
A, U_d and b resident in HBM.  Also reported: the FP32 and BF16 flexible
solves, preconditioner applies per second, per-kernel timings from HIP events
on the library's stream, the roofline of the dominant kernel (the banded A
product) and the FP64 oracle timed on the host cores.

Other workloads (--workload), each printing one JSON line of the same form:
  warped   unit cube warped by 8 seeded sine modes, kappa = 1 + 0.5 sin(2 pi x) cos(2 pi y),
           p = 5, 96^3 elements; BF16 FD inside flexible PCG (FP64 and FP32 reported beside it)
  batch    64 uneven problems (m_d ~ U{32..96}, p ~ U{2..5}, ring or warped), one batched call
  learned  learned diagonal scaling: trained on 2000 small warped cubes, evaluated on the
           p = 4, 112^3 warped cube: plain P, learned S P^-1 S, exact diagonal-ratio S
  square   2D unit square, identity map, p = 3, 64^2 elements (one iteration: launch latency)
  lshape   L-shaped domain of three square patches with C0 interfaces (Sec. 6, Table L),
           h^-1 = 1024 elements per patch and direction, p = 3: CG + additive Schwarz P_IAS
  adi      thick ring 128^3, p = 3: CG + the three-variable ADI preconditioner P_J (eps = 0.1)
           beside CG + the exact FD apply (the paper's FD-vs-ADI comparison)
  annulus  2D quarter annulus (the paper's Table quarterofring), h^-1 = 1024, p = 3: CG + P with
           the FD apply by tiled MFMA products (FP64; FP32 beside it)
  cube     unit cube, P = A: the FD apply as the direct solver (the paper's Table cube) at
           h^-1 = 128, 256, 512 (--elements 1024 for the 10^9-unknown case), p = 3 (--degree)

The default run (ring) also carries, as sub-objects, the warped-cube BF16
comparison ("warped_bf16") and the learned-scaling comparison
("learned_scaling": training on 2000 small warped cubes, evaluation at 112^3).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]
                       [--no-extras]
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
FP32_PEAK_TF = 157.3
BF16_PEAK_TF = 2500.0
METRIC = "PCG time-to-solve @1e-8 rel. residual (s) + iters; precond applies/sec"


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


def spmv_bytes(ctx):
    """Algorithmic bytes of one A product: each stored (symmetric) value once,
    x read once, y written once."""
    return 8 * ((ctx.nnz + ctx.N) // 2) + 16 * ctx.N


def fd_flops(ctx):
    return 4 * ctx.N * sum(ctx.n[:ctx.dim]) + ctx.N


def kernel_report(api, torch, ctx, reps=50, precisions=("fp64", "fp32", "bf16", "bf16x3")):
    """Event-timed A product and FD applies of one context."""
    x = torch.randn(ctx.N, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    t_spmv = event_time(torch, lambda: api.igafd_apply_A(ctx, x, y), reps)
    t_fd = {pr: event_time(torch, lambda pr=pr: api.igafd_apply_precond(ctx, pr, x, y), reps) for pr in precisions}
    by = spmv_bytes(ctx)
    gbs = by / (t_spmv * 1e-3) / 1e9
    fl = fd_flops(ctx)
    name, tag = spmv_kernel_name(api, ctx)
    log(f"spmv [{name}] {t_spmv * 1e3:.1f} us = {gbs:.0f} GB/s; FD " +
        " ".join(f"{pr} {t * 1e3:.1f} us" for pr, t in t_fd.items()))
    return {"t_spmv": t_spmv, "t_fd": t_fd, "bytes": by, "gbs": gbs, "fd_flops": fl, "kernel": name,
            "kernel_tag": tag}


def spmv_kernel_name(api, ctx):
    s = api.igafd_get_shape(ctx)
    if s["tile_b2"] > 0:
        return (f"igafd_apply_A: k_copy (x into the zero-halo buffer) + k_spmv_tile<p={ctx.p}> "
                f"({s['tile_b2']}x{s['tile_b3']} lines, {s['tile_threads']} threads) + k_spmv_combine"), \
            f"tile {s['tile_b2']}x{s['tile_b3']}x{s['tile_threads']}"
    return f"igafd_apply_A: k_copy (x into the zero-halo buffer) + k_spmv<R={s['spmv_rows']}>", "row"


def profiled_traffic(kernel_tag, workload_tag):
    """HBM/fabric bytes per A product (one igafd_apply_A: the copy into the
    zero-halo buffer and the product kernels) from the committed counter
    summaries (FETCH_SIZE and WRITE_SIZE, calibrated against a 1 GiB copy),
    used only while the A-product source and the kernel's launch shape (the
    tag: tile lines x threads per block) are the ones that were measured."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_1602_01636_amd", "csrc", "spmv.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        fields = {}
        for line in open(path):
            key, _, val = line.strip().partition(": ")
            if key.startswith("traffic_"):
                fields[key] = val.strip()
        if (fields.get("traffic_kernel") == kernel_tag and fields.get("traffic_workload") == workload_tag
                and fields.get("traffic_source_sha256_16") == sha):
            return int(fields["traffic_bytes_per_launch"]), os.path.relpath(path, ROOT)
    return None, None


def roofline(kr, workload_tag=None):
    traffic, source = profiled_traffic(kr["kernel_tag"], workload_tag) if workload_tag else (None, None)
    out = {"bound": "hbm", "achieved": kr["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": kr["gbs"] / HBM_PEAK_GBS, "traffic": traffic, "kernel": kr["kernel"],
           "algorithmic_bytes": kr["bytes"]}
    if traffic:
        out["traffic_source"] = source
        out["traffic_over_algorithmic"] = traffic / kr["bytes"]
    return out


def fd_roofline(kr, prec="fp64"):
    peak = {"fp64": FP64_PEAK_TF, "fp32": FP32_PEAK_TF, "bf16": BF16_PEAK_TF, "bf16x3": BF16_PEAK_TF}[prec]
    tf = kr["fd_flops"] / kr["t_fd"][prec] / 1e9
    return {"bound": "mfma", "precision": prec, "achieved": tf, "peak": peak, "unit": "TFLOP/s", "frac": tf / peak}


def timed_solves(api, torch, ctx, b, u, steps, warmup, **kw):
    for _ in range(warmup):
        api.igafd_solve(ctx, b, u, rtol=1e-8, **kw)
    torch.cuda.synchronize()
    times, infos = [], []
    for k in range(steps):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        info = api.igafd_solve(ctx, b, u, rtol=1e-8, **kw)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
        infos.append(info)
        log(f"step {k}: {times[-1] * 1e3:.3f} ms iters {info['iters']} true_relres {info['true_relres']:.2e}")
    return times, infos


def oracle_fd_apply_times(prob, reps=3):
    """The oracle's FD apply (numpy mode products, FP64) at the full size, on
    one host thread (as the paper's single core) and on all of them: best of
    `reps` per thread count."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import fd
    F = fd.setup(prob)
    n = [len(f["lam"]) for f in F]
    r = np.random.default_rng(2).standard_normal(int(np.prod(n)))
    out = {}
    for label, limit in (("1_thread", 1), ("all_threads", None)):
        with threadpool_limits(limits=limit):
            threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
            best = float("inf")
            for _ in range(reps):
                t0 = time.perf_counter()
                fd.fd_apply(F, r)
                best = min(best, time.perf_counter() - t0)
        out[label] = {"s": best, "threads": int(threads)}
    return out


def cpu_baseline(prob, u_gpu=None, f=None):
    """The FP64 oracle (NumPy/SciPy, as it stands) on the whole workload: its
    PCG on the same thick-ring (or 2D quarter-annulus) problem, with A applied
    in its Kronecker form (the ring's Q is diagonal and depends on xi1 only),
    the FD apply by numpy
    mode products and b assembled by sum factorisation.  As for the GPU, the
    setup (univariate eigendecompositions, b) is outside the timed solve.
    Returns the baseline and the distance of the GPU's solution to the
    oracle's."""
    import synth
    from oracle import assembly, fd, pcg
    from threadpoolctl import threadpool_info
    t0 = time.perf_counter()
    F = fd.setup(prob)
    Aop = assembly.ring_operator(prob)
    b = assembly.assemble_load_tensor(prob, f or synth.RHS_SINPROD)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    u, info = pcg.pcg(Aop, lambda r: fd.fd_apply(F, r), b, rtol=1e-8)
    dt = time.perf_counter() - t0
    cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    n = [len(f["lam"]) for f in F]
    out = {"value": dt, "unit": "s", "cores": int(cores), "kind": "oracle", "iters": info["iters"],
           "true_relres": info["true_relres"], "setup_s": t_setup,
           "sample": f"the whole workload, one solve: oracle PCG on the {'thick ring' if len(n) == 3 else 'quarter annulus'}, "
                     f"{n[0]}^{len(n)} dofs, p={prob['degree']}, "
                     f"rtol 1e-8 (A in Kronecker form, FD by numpy mode products, BLAS on {cores} threads; "
                     f"b and the eigendecompositions set up beforehand in {t_setup:.1f} s)",
           "fd_apply_s": oracle_fd_apply_times(prob)}
    if u_gpu is not None:
        d = u_gpu - u
        out["gpu_vs_oracle"] = {"rel_2norm": float(np.linalg.norm(d) / np.linalg.norm(u)),
                                "rel_max_entry": float(np.abs(d).max() / np.abs(u).max())}
    return out


def result(args, value, ms_per_step, dtype, workload, extra):
    out = {"metric": METRIC, "value": value, "unit": "s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": False, "scaling": "strong",
           "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": workload}
    out.update(extra)
    return out


def copy_calibration(torch):
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log("copy calibration: 1 GiB read + 1 GiB written")


def autotune(args, api, torch, ctx):
    """igafd_autotune after setup (times the A-product candidates, among them
    512-thread tiles, and the FD shapes on this problem): returns the seconds
    it took, None when --no-autotune keeps the setup's shapes."""
    if args.no_autotune:
        return None
    t0 = time.perf_counter()
    api.igafd_autotune(ctx)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    log(f"autotune {t:.2f}s: {api.igafd_get_shape(ctx)}")
    return t


def rhs(api, torch, synth, ctx):
    b = torch.zeros(ctx.N, dtype=torch.float64, device="cuda")
    api.igafd_load_vector(ctx, synth.RHS_SINPROD, b)
    return b


# The paper's Table thick_ring (CG + P): iterations and seconds on one core of
# an i7-5820K (MATLAB R2015a, FP64 implied), setup included; its map, right-hand
# side and tolerance are not stated, so this is context, not a like-for-like figure
PAPER_RING = {
    (128, 2): {"iters": 28, "s": 14.14}, (128, 3): {"iters": 28, "s": 32.01}, (128, 4): {"iters": 28, "s": 61.22},
    (64, 3): {"iters": 27, "s": 3.35}, (32, 3): {"iters": 26, "s": 0.38},
}
for _v in PAPER_RING.values():
    _v.update(hardware="one core of an i7-5820K, MATLAB R2015a", source="Table thick_ring (CG + P)")


def run_ring(args, api, torch, synth):
    E, p = args.elements or 128, args.degree or 3
    prob = synth.thick_ring(E=E, p=p)
    t0 = time.perf_counter()
    ctx = api.igafd_setup(prob)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    N, n = ctx.N, ctx.n[0]
    log(f"setup {t_setup:.2f}s N={N} nnz={ctx.nnz} band={ctx.band_bytes / 1e9:.2f} GB")
    t_tune = autotune(args, api, torch, ctx)
    b = rhs(api, torch, synth, ctx)
    u = torch.zeros_like(b)
    t_all = time.perf_counter()
    times, infos = timed_solves(api, torch, ctx, b, u, args.steps, args.warmup)
    wall = time.perf_counter() - t_all
    u64 = u.clone()
    ms_per_step = 1e3 * sum(times) / len(times)
    iters = infos[-1]["iters"]
    kr = kernel_report(api, torch, ctx)
    variants = {}
    if not args.no_variants:
        for prec in ("fp32", "bf16", "bf16x3"):
            ts, inf = timed_solves(api, torch, ctx, b, u, max(2, args.steps // 2), 1, precision=prec)
            err = float(torch.linalg.norm(u - u64) / torch.linalg.norm(u64))
            variants[prec] = {"s": float(np.median(ts)), "iters": inf[-1]["iters"],
                              "true_relres": inf[-1]["true_relres"], "rel_err_vs_fp64": err}
            log(f"{prec}: {variants[prec]}")
    if args.copy_calibration:
        copy_calibration(torch)
    # the same solve with the phase timers on (events between the kernels)
    tinfo = api.igafd_solve(ctx, b, u, rtol=1e-8, timers=True)
    torch.cuda.synchronize()
    phases = {"spmv": tinfo["t_spmv_ms"], "fd": tinfo["t_fd_ms"], "vec": tinfo["t_vec_ms"],
              "solve": tinfo["t_solve_ms"]}
    phases["host_wait"] = phases["solve"] - phases["spmv"] - phases["fd"] - phases["vec"]
    fd_share = phases["fd"] / phases["solve"]
    log(f"phases (ms): {phases}; FD share {100 * fd_share:.1f}%")
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(prob, u64.cpu().numpy())
        log(f"cpu baseline {cpu['value']:.2f} s, {cpu['iters']} iterations ({cpu['sample']}); "
            f"GPU vs oracle {cpu['gpu_vs_oracle']}")
    qlo, qhi = api.igafd_spectral_bounds(ctx)
    workload = {"workload": f"thick quarter ring, p={p}, {E}^3 elements, n={n}/dir, N={N} dofs, "
                            f"f=3pi^2 prod sin(pi x_i), FP64 FD-preconditioned CG, rtol 1e-8",
                "elements": E, "degree": p, "N": N, "nnz": ctx.nnz}
    out = result(args, ms_per_step / 1e3, ms_per_step, "f64", workload, {
        "iters": iters, "true_relres": infos[-1]["true_relres"],
        "precond_applies_per_s": {pr: 1e3 / t for pr, t in kr["t_fd"].items()},
        "kernel_ms": {"spmv": kr["t_spmv"], **{f"fd_{pr}": t for pr, t in kr["t_fd"].items()}},
        "variants": variants, "setup_s": t_setup, "autotune_s": t_tune, "wall_s_timed": wall,
        "solve_ms": {"median": 1e3 * float(np.median(times)), "min": 1e3 * min(times), "max": 1e3 * max(times)},
        "phases_ms": phases, "fd_share": fd_share,
        "paper_fd_share": {"value": 0.1309, "source": "Table percentage, revolved ring h^-1 = 128, p = 3, "
                                                      "one core of an i7-5820K (MATLAB)"},
        "spectral_bounds": [qlo, qhi], "kappa_bound": qhi / qlo, "paper": PAPER_RING.get((E, p)),
        "roofline": roofline(kr, f"thick_ring E={E} p={p}"), "fd_roofline": fd_roofline(kr),
        "cpu_baseline": cpu})
    ctx.close()
    return out


def run_warped(args, api, torch, synth):
    E, p = args.elements or 96, args.degree or 5
    prob = synth.warped_cube(E=E, p=p, seed=3)
    t0 = time.perf_counter()
    ctx = api.igafd_setup(prob)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    log(f"setup {t_setup:.2f}s N={ctx.N} nnz={ctx.nnz} band={ctx.band_bytes / 1e9:.2f} GB")
    t_tune = autotune(args, api, torch, ctx)
    b = rhs(api, torch, synth, ctx)
    u = torch.zeros_like(b)
    ts64, inf64 = timed_solves(api, torch, ctx, b, u, max(2, args.steps // 2), 1)
    u64 = u.clone()
    variants = {"fp64": {"s": float(np.median(ts64)), "iters": inf64[-1]["iters"],
                         "true_relres": inf64[-1]["true_relres"]}}
    ts32, inf32 = timed_solves(api, torch, ctx, b, u, max(2, args.steps // 2), 1, precision="fp32")
    variants["fp32"] = {"s": float(np.median(ts32)), "iters": inf32[-1]["iters"],
                        "true_relres": inf32[-1]["true_relres"],
                        "rel_err_vs_fp64": float(torch.linalg.norm(u - u64) / torch.linalg.norm(u64))}
    tsx, infx = timed_solves(api, torch, ctx, b, u, max(2, args.steps // 2), 1, precision="bf16x3")
    variants["bf16x3"] = {"s": float(np.median(tsx)), "iters": infx[-1]["iters"],
                          "true_relres": infx[-1]["true_relres"],
                          "rel_err_vs_fp64": float(torch.linalg.norm(u - u64) / torch.linalg.norm(u64))}
    times, infos = timed_solves(api, torch, ctx, b, u, args.steps, args.warmup, precision="bf16")
    err = float(torch.linalg.norm(u - u64) / torch.linalg.norm(u64))
    ms_per_step = 1e3 * sum(times) / len(times)
    kr = kernel_report(api, torch, ctx)
    workload = {"workload": f"warped unit cube (8 sine modes, seed 3), kappa=1+0.5 sin(2pi x)cos(2pi y), p={p}, "
                            f"{E}^3 elements, N={ctx.N} dofs, BF16 FD in flexible PCG, rtol 1e-8",
                "elements": E, "degree": p, "N": ctx.N, "nnz": ctx.nnz}
    out = result(args, ms_per_step / 1e3, ms_per_step, "f64 (FD mode products bf16, fp32 accumulation)", workload, {
        "iters": infos[-1]["iters"], "true_relres": infos[-1]["true_relres"], "rel_err_vs_fp64": err,
        "precond_applies_per_s": {pr: 1e3 / t for pr, t in kr["t_fd"].items()},
        "kernel_ms": {"spmv": kr["t_spmv"], **{f"fd_{pr}": t for pr, t in kr["t_fd"].items()}},
        "variants": variants, "setup_s": t_setup, "autotune_s": t_tune, "roofline": roofline(kr),
        "fd_roofline": fd_roofline(kr, "bf16"),
        "cpu_baseline": None})
    ctx.close()
    return out


def run_batch(args, api, torch, synth):
    probs = synth.batch_problems(seed=4)
    t0 = time.perf_counter()
    ctxs = [api.igafd_setup(pr) for pr in probs]
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    for c in ctxs:
        api.igafd_autotune(c)
    t_tune = time.perf_counter() - t0
    bs = [rhs(api, torch, synth, c) for c in ctxs]
    us = [torch.zeros_like(b) for b in bs]
    band = sum(c.band_bytes for c in ctxs)
    log(f"setup {t_setup:.2f}s autotune {t_tune:.2f}s, {len(ctxs)} problems, band {band / 1e9:.1f} GB")
    for _ in range(args.warmup):
        api.igafd_solve_batched(ctxs, bs, us)
    walls, infos = [], None
    for k in range(args.steps):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        infos, wall_ms = api.igafd_solve_batched(ctxs, bs, us)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t1)
        log(f"step {k}: {walls[-1] * 1e3:.2f} ms (library wall {wall_ms:.2f} ms)")
    assert all(i["status"] == "OK" and i["true_relres"] <= 1e-8 for i in infos)
    iters = [i["iters"] for i in infos]
    alg = sum((it + 2) * spmv_bytes(c) for it, c in zip(iters, ctxs))
    ms_per_step = 1e3 * sum(walls) / len(walls)
    # one-at-a-time solves of the same problems, for comparison
    t1 = time.perf_counter()
    for c, b, u in zip(ctxs, bs, us):
        api.igafd_solve(c, b, u)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t1
    big = max(range(len(ctxs)), key=lambda k: ctxs[k].band_bytes)
    kr = kernel_report(api, torch, ctxs[big], precisions=("fp64",))
    workload = {"workload": "64 uneven 3D problems (seed 4): m_d ~ U{32..96} per direction, p ~ U{2..5}, "
                            "thick ring or warped cube, FP64 FD PCG, rtol 1e-8, one batched call",
                "count": len(ctxs), "N_total": sum(c.N for c in ctxs), "band_GB": band / 1e9}
    out = result(args, ms_per_step / 1e3, ms_per_step, "f64", workload, {
        "iters": iters, "sequential_s": t_seq, "spmv_equiv_GBps": alg / (ms_per_step * 1e-3) / 1e9,
        "setup_s": t_setup, "autotune_s": t_tune,
        "roofline": dict(roofline(kr), note=f"largest problem of the batch (#{big})"), "cpu_baseline": None})
    for c in ctxs:
        c.close()
    return out


def run_learned(args, api, torch, synth):
    from paper_1602_01636_amd import scaling
    t0 = time.perf_counter()
    mlp, hist, total = scaling.train_default(n_train=args.train, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"trained on {total} dofs of {args.train} problems in {t_train:.1f}s, loss {hist[0]:.3e} -> {hist[-1]:.3e}")
    E, p = args.elements or 112, args.degree or 4
    prob = synth.learned_eval_problem(E=E, p=p)
    # the setup's cost of the features: the same setup without and with them,
    # alternating, three times each (medians; one setup varies by a few ms)
    t_plain, t_feat = [], []
    ctx = None
    for rep in range(3):
        t0 = time.perf_counter()
        api.igafd_setup(prob).close()
        torch.cuda.synchronize()
        t_plain.append(time.perf_counter() - t0)
        if ctx is not None:
            ctx.close()
        t0 = time.perf_counter()
        ctx = api.igafd_setup(prob, features=True)
        torch.cuda.synchronize()
        t_feat.append(time.perf_counter() - t0)
    t_setup_plain, t_setup_feat = float(np.median(t_plain)), float(np.median(t_feat))
    t_tune = autotune(args, api, torch, ctx)
    b = rhs(api, torch, synth, ctx)
    u = torch.zeros_like(b)
    res = {}
    ts, inf = timed_solves(api, torch, ctx, b, u, max(2, args.steps // 2), 1)
    res["plain"] = {"s": float(np.median(ts)), "iters": inf[-1]["iters"], "true_relres": inf[-1]["true_relres"]}
    scaling.predict_scaling(mlp, ctx)  # warm-up (first launches of the network kernels)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    scaling.predict_scaling(mlp, ctx)
    torch.cuda.synchronize()
    t_pred = time.perf_counter() - t1
    feat_setup = max(0.0, t_setup_feat - t_setup_plain)
    times, infos = timed_solves(api, torch, ctx, b, u, args.steps, args.warmup, use_scaling=True)
    res["learned"] = {"s": float(np.median(times)), "iters": infos[-1]["iters"],
                      "true_relres": infos[-1]["true_relres"], "fallback": infos[-1]["fallback"],
                      "predict_s": t_pred, "features_setup_s": feat_setup,
                      "setup_s": {"without_features": t_setup_plain, "with_features": t_setup_feat}}
    api.igafd_set_scaling_diag_ratio(ctx)
    ts, inf = timed_solves(api, torch, ctx, b, u, max(2, args.steps // 2), 1, use_scaling=True)
    res["exact_ratio"] = {"s": float(np.median(ts)), "iters": inf[-1]["iters"], "true_relres": inf[-1]["true_relres"]}
    log(f"plain {res['plain']['iters']} learned {res['learned']['iters']} exact {res['exact_ratio']['iters']}")
    qlo, qhi = api.igafd_spectral_bounds(ctx)
    res["plain"]["kappa_bound"] = qhi / qlo
    use, kq, kl = api.igafd_scaling_gate(ctx)
    res["gate"] = {"use_scaling": use, "kappa_q": kq, "kappa_loc": kl, "gain": 2.0,
                   "rule": "scale when (qmax/qmin)/qloc >= gain (Prop. 1 bound vs pointwise anisotropy)"}
    kr = kernel_report(api, torch, ctx, precisions=("fp64",))
    ms_per_step = 1e3 * sum(times) / len(times)
    workload = {"workload": f"warped unit cube (seed 10000), kappa=1+0.5 sin(2pi x)cos(2pi y), p={p}, {E}^3 elements, "
                            f"N={ctx.N}, FP64 PCG with learned S P^-1 S (network trained on {args.train} small "
                            f"warped cubes)", "elements": E, "degree": p, "N": ctx.N}
    out = result(args, ms_per_step / 1e3, ms_per_step, "f64 (network bf16, fp32 accumulation)", workload, {
        "iters": infos[-1]["iters"], "variants": res, "train_s": t_train, "train_dofs": total,
        "loss_first_last": [hist[0], hist[-1]], "autotune_s": t_tune, "roofline": roofline(kr), "cpu_baseline": None})
    ctx.close()
    mlp.close()
    return out


def run_square(args, api, torch, synth):
    E, p = args.elements or 64, args.degree or 3
    ctx = api.igafd_setup(synth.square_2d(E=E, p=p))
    b = rhs(api, torch, synth, ctx)
    u = torch.zeros_like(b)
    times, infos = timed_solves(api, torch, ctx, b, u, max(args.steps, 20), args.warmup)
    ms_per_step = 1e3 * float(np.median(times))
    kr = kernel_report(api, torch, ctx, reps=200)
    workload = {"workload": f"2D unit square, identity map, p={p}, {E}^2 elements, N={ctx.N}, FP64 FD PCG "
                            f"(P = A: one iteration; launch-latency bound)", "elements": E, "degree": p, "N": ctx.N}
    out = result(args, ms_per_step / 1e3, ms_per_step, "f64", workload, {
        "iters": infos[-1]["iters"], "true_relres": infos[-1]["true_relres"],
        "kernel_ms": {"spmv": kr["t_spmv"], **{f"fd_{pr}": t for pr, t in kr["t_fd"].items()}},
        "roofline": roofline(kr), "cpu_baseline": None})
    ctx.close()
    return out


def lshape_nnz(n, hole, p):
    """Stored nonzeros of A over the unknowns of the L-shaped grid: pairs of
    unknowns whose indices differ by at most p in both directions."""
    mask = np.ones((n, n), dtype=bool)
    mask[hole:, hole:] = False
    pad = np.pad(mask, p)
    cnt = np.zeros((n, n), dtype=np.int64)
    for o2 in range(2 * p + 1):
        for o1 in range(2 * p + 1):
            cnt += pad[o2:o2 + n, o1:o1 + n]
    return int(cnt[mask].sum())


def lshape_cpu_baseline(target_iters, E_full, p, flops_iter_full):
    """The oracle's CG + P_IAS (glued three-patch matrix, FD local solves) on
    a bounded sample: h^-1 = 128, same p; time per iteration scaled by the
    FLOPs per iteration (A product 2 nnz, P_IAS 8 h n (h + n)) to the full
    mesh, times the GPU's iteration count."""
    import synth
    from oracle import multipatch as mp
    E = 128
    L = mp.LShape(synth.uniform_knots(E, p), p)
    S = mp.Schwarz(L)
    A = S.A
    b = L.load(synth.RHS_PAPER_POLY)
    t0 = time.perf_counter()
    reps = iters = 0
    while time.perf_counter() - t0 < 10.0 or reps < 3:
        _, info = S.solve(b, "ias")
        iters += info["iters"]
        reps += 1
    dt = time.perf_counter() - t0
    h = L.m - 2
    n = 2 * h + 1
    per_iter = dt / iters
    flops_s = 2 * A.nnz + 8 * h * n * (h + n)
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    return {"value": per_iter * flops_iter_full / flops_s * target_iters, "unit": "s", "cores": int(cores),
            "kind": "oracle",
            "sample": f"oracle CG + P_IAS on the L-shaped domain at h^-1={E} p={p} (N={L.N}), {reps} solves, "
                      f"{per_iter * 1e3:.2f} ms/iteration, scaled by FLOPs/iteration to h^-1={E_full} "
                      f"and x {target_iters} iterations",
            "sample_s_per_iter": per_iter}


def run_lshape(args, api, torch, synth):
    E, p = args.elements or 1024, args.degree or 3
    knots = synth.uniform_knots(E, p)
    t0 = time.perf_counter()
    ctx = api.igafd_lshape_setup(knots, p)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    n, h = ctx.n[0], ctx.hole
    b = torch.zeros(ctx.N, dtype=torch.float64, device="cuda")
    api.igafd_load_vector(ctx, synth.RHS_PAPER_POLY, b)
    u = torch.zeros_like(b)
    times, infos = timed_solves(api, torch, ctx, b, u, args.steps, args.warmup)
    ms_per_step = 1e3 * float(np.median(times))
    variants = {}
    if not args.no_variants:
        for prec in ("fp32", "bf16", "bf16x3"):
            tv, iv = timed_solves(api, torch, ctx, b, u, 3, 1, precision=prec)
            variants[prec] = {"ms": 1e3 * float(np.median(tv)), "iters": iv[-1]["iters"],
                              "true_relres": iv[-1]["true_relres"]}
    x = torch.randn(ctx.N, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    t_spmv = event_time(torch, lambda: api.igafd_apply_A(ctx, x, y), 20)
    t_fd = {pr: event_time(torch, lambda pr=pr: api.igafd_apply_precond(ctx, pr, x, y), 10)
            for pr in ("fp64", "fp32", "bf16", "bf16x3")}
    nnz_L = lshape_nnz(n, h, p)
    by = 8 * ((nnz_L + ctx.ndofs) // 2) + 16 * ctx.ndofs
    fl = 8 * h * n * (h + n)
    log(f"A product {t_spmv * 1e3:.1f} us ({by / t_spmv / 1e6:.0f} GB/s); P_IAS " +
        " ".join(f"{pr} {t * 1e3:.1f} us ({fl / t / 1e9:.1f} TF/s)" for pr, t in t_fd.items()))
    tf = fl / t_fd["fp64"] / 1e9
    roof = {"bound": "mfma", "achieved": tf, "peak": FP64_PEAK_TF, "unit": "TFLOP/s", "frac": tf / FP64_PEAK_TF,
            "traffic": None, "kernel": "P_IAS apply: two subdomain FD applies (FP64 mode products) + combine",
            "algorithmic_flops": fl}
    spmv_roof = {"bound": "hbm", "achieved": by / t_spmv / 1e6, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": by / t_spmv / 1e6 / HBM_PEAK_GBS, "algorithmic_bytes": by}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = lshape_cpu_baseline(infos[-1]["iters"], E, p, 2 * nnz_L + fl)
    workload = {"workload": f"L-shaped domain, 3 square patches with C0 interfaces, h^-1={E} per patch, p={p}, "
                            f"{ctx.ndofs} unknowns (grid {n}^2), f = 2 sum(x_i^2 - x_i), CG + additive Schwarz "
                            f"P_IAS with FP64 FD local solves", "elements_per_patch": E, "degree": p,
                "unknowns": ctx.ndofs}
    out = result(args, ms_per_step / 1e3, ms_per_step, "f64", workload, {
        "iters": infos[-1]["iters"], "true_relres": infos[-1]["true_relres"], "setup_s": t_setup,
        "variants": variants, "kernel_ms": {"spmv": t_spmv, **{f"schwarz_{pr}": t for pr, t in t_fd.items()}},
        "roofline": roof, "spmv_roofline": spmv_roof, "cpu_baseline": cpu})
    ctx.close()
    return out


def run_adi(args, api, torch, synth):
    """CG with the three-variable ADI preconditioner P_J (eps = 0.1) beside CG
    with the exact FD apply, on the thick ring (the paper's FD-vs-ADI
    comparison of Sec. 7)."""
    E, p = args.elements or 128, args.degree or 3
    eps = 0.1
    ctx = api.igafd_setup(synth.thick_ring(E=E, p=p))
    b = rhs(api, torch, synth, ctx)
    u = torch.zeros_like(b)
    t0 = time.perf_counter()
    J, rho = api.igafd_set_adi(ctx, eps)
    t_params = time.perf_counter() - t0
    times, infos = timed_solves(api, torch, ctx, b, u, args.steps, args.warmup)
    ms_per_step = 1e3 * float(np.median(times))
    x = torch.randn(ctx.N, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    t_adi = event_time(torch, lambda: api.igafd_apply_precond(ctx, "fp64", x, y), 10)
    t_spmv = event_time(torch, lambda: api.igafd_apply_A(ctx, x, y), 20)
    # the greedy parameters (eq. greedy1/2) beside the geometric ones
    t0 = time.perf_counter()
    Jg, rhog = api.igafd_set_adi_greedy(ctx, eps)
    t_params_g = time.perf_counter() - t0
    t_adi_g = event_time(torch, lambda: api.igafd_apply_precond(ctx, "fp64", x, y), 10)
    tg, infg = timed_solves(api, torch, ctx, b, u, 3, 1)
    log(f"ADI greedy: J = {Jg}, rho = {rhog:.3f}, apply {t_adi_g * 1e3:.1f} us, solve {1e3 * float(np.median(tg)):.1f} ms, "
        f"{infg[-1]['iters']} iterations")
    greedy = {"J": Jg, "rho": rhog, "param_setup_s": t_params_g, "apply_ms": t_adi_g,
              "solve_ms": 1e3 * float(np.median(tg)), "iters": infg[-1]["iters"],
              "true_relres": infg[-1]["true_relres"]}
    api.igafd_set_adi(ctx, 0)
    t_fd = event_time(torch, lambda: api.igafd_apply_precond(ctx, "fp64", x, y), 20)
    tf, inf = timed_solves(api, torch, ctx, b, u, 3, 1)
    # bytes one ADI step moves in the kernels as written (vector passes of N doubles):
    # 2 + 4 (u), 3 + 4 (r*), 4 (s*), 3 + 4 (s**), 3 + 4 (s), 4 (v) = 35 passes
    by = 35 * 8 * ctx.N * J + 4 * 8 * ctx.N * 2
    gbs = by / (t_adi * 1e-3) / 1e9
    log(f"ADI: J = {J}, rho = {rho:.3f}, apply {t_adi * 1e3:.1f} us ({gbs:.0f} GB/s); FD apply {t_fd * 1e3:.1f} us; "
        f"A product {t_spmv * 1e3:.1f} us")
    workload = {"workload": f"thick quarter ring, p={p}, {E}^3 elements, N={ctx.N}, CG + three-variable ADI "
                            f"preconditioner P_J (eps={eps}, J={J})", "elements": E, "degree": p, "N": ctx.N}
    out = result(args, ms_per_step / 1e3, ms_per_step, "f64", workload, {
        "iters": infos[-1]["iters"], "true_relres": infos[-1]["true_relres"],
        "adi": {"J": J, "rho": rho, "eps": eps, "param_setup_s": t_params},
        "fd_comparison": {"ms": 1e3 * float(np.median(tf)), "iters": inf[-1]["iters"]}, "greedy": greedy,
        "kernel_ms": {"adi_apply": t_adi, "fd_apply": t_fd, "spmv": t_spmv},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                     "traffic": None, "kernel": "P_J apply (banded line products and solves)",
                     "algorithmic_bytes": by},
        "cpu_baseline": None})
    ctx.close()
    return out


# The paper's Table quarterofring (CG + P, upper part): 2D quarter annulus,
# f = 2 sum(x_i^2 - x_i), iterations and seconds on one core of an i7-5820K
# (MATLAB), preconditioner setup included
PAPER_ANNULUS = {
    (128, 2): (25, 0.04), (128, 3): (25, 0.06), (128, 4): (25, 0.07), (128, 5): (25, 0.09),
    (256, 2): (25, 0.20), (256, 3): (25, 0.26), (256, 4): (25, 0.34), (256, 5): (25, 0.40),
    (512, 2): (26, 1.13), (512, 3): (26, 1.36), (512, 4): (26, 1.62), (512, 5): (26, 2.00),
    (1024, 2): (26, 7.30), (1024, 3): (26, 8.13), (1024, 4): (26, 9.09), (1024, 5): (26, 10.52),
}


def run_annulus(args, api, torch, synth):
    """2D quarter annulus (the paper's Table quarterofring): CG + P with the
    FD apply by tiled MFMA products (n = 1025 per direction at h^-1 = 1024),
    FP64 and FP32 mode products."""
    E, p = args.elements or 1024, args.degree or 3
    t0 = time.perf_counter()
    ctx = api.igafd_setup(synth.quarter_annulus_2d(E=(E, E), p=p))
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    b = torch.zeros(ctx.N, dtype=torch.float64, device="cuda")
    api.igafd_load_vector(ctx, synth.RHS_PAPER_POLY, b)
    u = torch.zeros_like(b)
    times, infos = timed_solves(api, torch, ctx, b, u, args.steps, args.warmup)
    u64 = u.clone()
    ms_per_step = 1e3 * float(np.median(times))
    variants = {}
    if not args.no_variants:
        for prec in ("fp32", "bf16", "bf16x3"):
            ts, inf = timed_solves(api, torch, ctx, b, u, max(2, args.steps // 2), 1, precision=prec)
            variants[prec] = {"s": float(np.median(ts)), "iters": inf[-1]["iters"],
                              "true_relres": inf[-1]["true_relres"],
                              "rel_err_vs_fp64": float(torch.linalg.norm(u - u64) / torch.linalg.norm(u64))}
            log(f"{prec}: {variants[prec]}")
    kr = kernel_report(api, torch, ctx, reps=20)
    iters = infos[-1]["iters"]
    paper = PAPER_ANNULUS.get((E, p))
    log(f"annulus h^-1={E} p={p} N={ctx.N}: setup {t_setup:.2f} s, solve {ms_per_step:.2f} ms, {iters} iterations" +
        (f"; paper {paper[0]} iterations, {paper[1]} s" if paper else ""))
    cpu = None if args.no_cpu_baseline else cpu_baseline(synth.quarter_annulus_2d(E=(E, E), p=p), u64.cpu().numpy(),
                                                           synth.RHS_PAPER_POLY)
    workload = {"workload": f"2D quarter annulus F = ((1+xi1) cos(pi xi2/2), (1+xi1) sin(pi xi2/2)), p={p}, "
                            f"{E}^2 elements, N={ctx.N}, f = 2 sum(x_i^2 - x_i), FP64 FD-preconditioned CG "
                            f"(FD by tiled MFMA products), rtol 1e-8", "elements": E, "degree": p, "N": ctx.N}
    out = result(args, ms_per_step / 1e3, ms_per_step, "f64", workload, {
        "iters": iters, "true_relres": infos[-1]["true_relres"], "setup_s": t_setup, "variants": variants,
        "solve_ms": {"median": ms_per_step, "min": 1e3 * min(times), "max": 1e3 * max(times)},
        "kernel_ms": {"spmv": kr["t_spmv"], **{f"fd_{pr}": t for pr, t in kr["t_fd"].items()}},
        "paper": ({"iters": paper[0], "s": paper[1], "hardware": "one core of an i7-5820K, MATLAB R2015a",
                   "source": "Table quarterofring (CG + P)"} if paper else None),
        "roofline": dict(fd_roofline(kr), kernel="k_gemm (four FP64 mode products, tiled MFMA)",
                         algorithmic_flops=kr["fd_flops"], traffic=None),
        "spmv_roofline": roofline(kr), "cpu_baseline": cpu})
    ctx.close()
    return out


# The paper's Table cube (upper part): FD direct solver on the unit cube,
# P = A, b = randn, seconds per solve including the 1D eigendecompositions, one
# core of an i7-5820K (MATLAB); h^-1 -> seconds, per degree
PAPER_CUBE_FD_S = {
    1: {128: 0.19, 256: 1.80, 512: 23.02, 1024: 331.01}, 2: {128: 0.15, 256: 1.87, 512: 22.58, 1024: 316.15},
    3: {128: 0.17, 256: 2.05, 512: 23.45, 1024: 328.65}, 4: {128: 0.17, 256: 1.90, 512: 23.26, 1024: 318.42},
    5: {128: 0.18, 256: 2.10, 512: 23.65, 1024: 331.06}, 6: {128: 0.17, 256: 1.82, 512: 21.89, 1024: 310.31},
}


def cube_cpu_baseline(E, p):
    """The oracle's FD apply (FP64, numpy on the host cores) at the same size
    when it is at most 512^3 elements, else at 512^3 scaled by the FLOPs."""
    from threadpoolctl import threadpool_info

    import synth
    from oracle import fd
    Es = min(E, 512)
    F = fd.setup(synth.unit_cube(Es, p))
    n = len(F[0]["lam"])
    r = np.random.default_rng(1).standard_normal(n ** 3)
    t0 = time.perf_counter()
    fd.fd_apply(F, r)
    t = time.perf_counter() - t0
    nf = E + p - 2
    scale = (nf ** 4) / (n ** 4)
    cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    log(f"cpu baseline: oracle FD apply at {Es}^3 elements: {t:.2f} s on {cores} threads")
    return {"value": t * scale, "unit": "s", "cores": cores, "kind": "oracle",
            "sample": f"one oracle FD apply (numpy, FP64) at h^-1={Es}, p={p}" +
                      (f", scaled by the FLOPs (n^4) to h^-1={E}" if Es != E else "")}


def run_cube(args, api, torch, synth):
    """Unit cube, P = A: the FD apply is the direct solver (the paper's Table
    cube, right-hand side randn).  Preconditioner-only contexts (no A) at
    h^-1 = 128, 256, 512 (or --elements); per size the host setup (1D
    eigendecompositions + upload) and the event-timed applies in FP64, FP32 and
    BF16.  The timed steps are FP64 direct solves at the largest size."""
    p = args.degree or 3
    sizes = [args.elements] if args.elements else [128, 256, 512]
    gen = torch.Generator(device="cuda")
    per_size = []
    for E in sizes:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx = api.igafd_setup_precond(synth.unit_cube(E, p))
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        gen.manual_seed(E)
        r = torch.randn(ctx.N, dtype=torch.float64, device="cuda", generator=gen)
        s = torch.empty_like(r)
        fl = fd_flops(ctx)
        reps = 20 if ctx.N < 5e7 else 5
        t_fd = {pr: event_time(torch, lambda pr=pr: api.igafd_apply_precond(ctx, pr, r, s), reps)
                for pr in ("fp64", "fp32", "bf16", "bf16x3")}
        tf = {pr: fl / t / 1e9 for pr, t in t_fd.items()}
        paper = PAPER_CUBE_FD_S.get(p, {}).get(E)
        log(f"cube h^-1={E} p={p} n={ctx.n[0]} N={ctx.N}: setup {t_setup:.2f} s; apply " +
            ", ".join(f"{pr} {t:.2f} ms ({tf[pr]:.1f} TF)" for pr, t in t_fd.items()) +
            (f"; paper {paper} s" if paper else ""))
        per_size.append({"elements": E, "n": ctx.n[0], "N": ctx.N, "setup_s": t_setup,
                         "apply_ms": t_fd, "tflops": tf, "applies_per_s": {pr: 1e3 / t for pr, t in t_fd.items()},
                         "fp64_mfma_frac": tf["fp64"] / FP64_PEAK_TF,
                         "solve_s_setup_plus_fp64_apply": t_setup + t_fd["fp64"] / 1e3, "paper_s": paper})
        if E != sizes[-1]:
            ctx.close()
            del r, s
    for _ in range(args.warmup):
        api.igafd_apply_precond(ctx, "fp64", r, s)
    torch.cuda.synchronize()
    times = []
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        api.igafd_apply_precond(ctx, "fp64", r, s)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    if args.copy_calibration:
        copy_calibration(torch)
    ms_per_step = 1e3 * float(np.median(times))
    last = per_size[-1]
    E = last["elements"]
    cpu = None if args.no_cpu_baseline else cube_cpu_baseline(E, p)
    workload = {"workload": f"unit cube, identity map, kappa = 1 (P = A), p={p}, {E}^3 elements, N={ctx.N}, "
                            f"FD direct solve (one FP64 apply of P^-1 to a randn right-hand side)",
                "elements": E, "degree": p, "N": ctx.N}
    out = result(args, ms_per_step / 1e3, ms_per_step, "f64", workload, {
        "iters": 0, "sizes": per_size,
        "roofline": {"bound": "mfma", "achieved": last["tflops"]["fp64"], "peak": FP64_PEAK_TF, "unit": "TFLOP/s",
                     "frac": last["fp64_mfma_frac"], "traffic": None,
                     "kernel": "k_gemm (six FP64 mode products, tiled MFMA)", "algorithmic_flops": fd_flops(ctx)},
        "cpu_baseline": cpu})
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ring", choices=["ring", "warped", "batch", "learned", "square", "lshape", "adi",
                                                             "cube", "annulus"])
    ap.add_argument("--elements", type=int, default=0)
    ap.add_argument("--degree", type=int, default=0)
    ap.add_argument("--train", type=int, default=2000, help="training problems (learned workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the setup's default kernel shapes (ring, warped, learned workloads)")
    ap.add_argument("--no-extras", action="store_true",
                    help="ring workload only: skip the warped-cube BF16 and learned-scaling sub-objects")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed region, one plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the solver runs on a single device and has no "
              "multi-GPU path in this build (--gpus must be 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    import paper_1602_01636_amd as api

    torch.cuda.set_device(0)
    run = {"ring": run_ring, "warped": run_warped, "batch": run_batch, "learned": run_learned,
           "square": run_square, "lshape": run_lshape, "adi": run_adi, "cube": run_cube,
           "annulus": run_annulus}[args.workload]
    out = run(args, api, torch, synth)
    if args.workload == "ring" and not args.no_extras:
        # the two extensions' comparisons (mixed-precision FD on the warped
        # cube, learned scaling), on their own workloads (fewer timed solves;
        # each sub-object carries its own config)
        sub = argparse.Namespace(**vars(args))
        sub.steps, sub.warmup, sub.elements, sub.degree = max(3, args.steps // 4), 1, 0, 0
        log("== warped cube, p = 5, 96^3: BF16 / split-BF16 / FP32 / FP64 FD")
        w = run_warped(sub, api, torch, synth)
        v = w["variants"]
        fp64_s = v["fp64"]["s"]
        out["warped_bf16"] = {
            "config": w["config"], "bf16_s": w["value"], "bf16_iters": w["iters"],
            "bf16_rel_err_vs_fp64": w["rel_err_vs_fp64"], "variants": v,
            "speedup_vs_fp64": {pr: fp64_s / (w["value"] if pr == "bf16" else v[pr]["s"])
                                for pr in ("bf16", "bf16x3", "fp32")},
            "fd_roofline_bf16": w["fd_roofline"], "kernel_ms": w["kernel_ms"]}
        log("== learned scaling: train on the small warped cubes, evaluate at 112^3, p = 4")
        ln = run_learned(sub, api, torch, synth)
        lv = ln["variants"]
        saving = lv["plain"]["s"] - lv["learned"]["s"]
        cost = lv["learned"]["predict_s"] + lv["learned"]["features_setup_s"]
        out["learned_scaling"] = {
            "config": ln["config"], "variants": lv, "train_s": ln["train_s"], "train_dofs": ln["train_dofs"],
            "loss_first_last": ln["loss_first_last"], "saving_per_solve_s": saving,
            "prediction_cost_s": cost, "pays_off_first_solve": bool(cost < saving),
            # solves of one setup (right-hand sides) after which the features and
            # the prediction have paid for themselves
            "pays_off_after_solves": (int(np.ceil(cost / saving)) if saving > 0 else None)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
