#!/usr/bin/env python3
"""Benchmark: H^2 x X throughput (algorithmic GB/s) and block-CG time to 1e-8.

One step = one H^2 x X product (forward transformation, coupling, backward
transformation, near field) on the FP64 throughput workload: n = 65536 points
on the unit sphere, kernel exp(-r/0.5) + 1.0 delta, leaf <= 64, eta = 1,
Chebyshev order 4 (k = 64), m = 32 right-hand sides N(0, 1).  Inputs are
resident in HBM before the timed region starts.  After the timed products the
same operator solves A X = B with block CG to relative residual 1e-8.

Prints one JSON line on stdout; progress goes to stderr.
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

PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_BF16_TFLOPS = 2500.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def alg_bytes(plan, m, s_b=8, s_n=8, s_v=8, beta_nonzero=False):
    """Algorithmic HBM bytes of one product: V, E, S once, near field once, X read, Y written."""
    k = plan.k
    op = s_b * (plan.n * k + (plan.C - 1) * k * k + plan.n_adm * k * k)
    return op + s_n * plan.near_entries + s_v * plan.n * m * (2 + (1 if beta_nonzero else 0))


def alg_flops(plan, m):
    k = plan.k
    return 2 * m * (2 * plan.n * k + 2 * (plan.C - 1) * k * k + plan.n_adm * k * k + plan.near_entries)


def coupling_bytes(plan, s_b=8):
    """Algorithmic bytes of the coupling stage: every S_b once (k^2 s_b per admissible block)."""
    return s_b * plan.n_adm * plan.k * plan.k


def coupling_intermediate_bytes(plan, m, s_h=8):
    """The coupling's intermediate traffic, reported apart: x-hat read once, y-hat written once."""
    return 2 * s_h * plan.C * plan.k * m


def coupling_flops(plan, m):
    return 2 * plan.n_adm * plan.k * plan.k * m


def measured_traffic(kernel_profile):
    """HBM bytes per launch from a committed rocprofv3 PMC summary (FETCH_SIZE and WRITE_SIZE
    scaled by a plain-copy calibration), or None when the kernel source has changed since."""
    import hashlib

    path = os.path.join(ROOT, "profiles", kernel_profile)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    src = os.path.join(ROOT, kv.get("kernel_source", ""))
    if not os.path.isfile(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != kv.get("kernel_source_sha256"):
        return None
    return int(1024 * (float(kv["fetch_size_kib_per_launch"]) * float(kv["fetch_scale"]) +
                       float(kv["write_size_kib_per_launch"]) * float(kv["write_scale"])))


def host_info():
    """CPU model, logical CPUs and RAM of the host, from /proc."""
    model, ram = "unknown", 0.0
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                ram = int(line.split()[1]) / 2**20
                break
    except OSError:
        pass
    return dict(cpu_model=model, nproc=os.cpu_count(), ram_gib=round(ram, 1))


def host_copy_gbs(threads, nbytes=1 << 30, reps=5):
    """STREAM-like copy bandwidth of the host: `threads` threads each copy their slice of a
    nbytes array (numpy copies release the GIL); bytes counted as read + write."""
    import concurrent.futures as cf

    a = np.ones(nbytes // 8)
    b = np.empty_like(a)
    bounds = np.linspace(0, a.size, threads + 1).astype(np.int64)

    def part(i):
        np.copyto(b[bounds[i]:bounds[i + 1]], a[bounds[i]:bounds[i + 1]])

    with cf.ThreadPoolExecutor(threads) as ex:
        list(ex.map(part, range(threads)))
        best = 0.0
        for _ in range(reps):
            t0 = time.perf_counter()
            list(ex.map(part, range(threads)))
            best = max(best, 2 * a.nbytes / (time.perf_counter() - t0) / 1e9)
    return round(best, 2)


def cpu_baseline(w, P, X, plan, budget_s):
    """The oracle (the paper's CPU method: parallel forward / list-wise multiplication /
    backward) timed on the host's cores, then with one thread, beside the host's copy
    bandwidth."""
    import oracle

    o = oracle.OracleH2(P, **w.params())
    o.matmul(X[:, :1])  # warm the code path
    cores = oracle.num_threads()

    def timed(budget, min_runs=1):
        times = []
        t_end = time.perf_counter() + budget
        while True:
            t0 = time.perf_counter()
            o.matmul(X)
            times.append(time.perf_counter() - t0)
            if time.perf_counter() > t_end and len(times) >= min_runs:
                break
        return float(np.median(times)), len(times)

    t, runs = timed(budget_s)
    oracle.set_threads(1)
    try:
        t1, runs1 = timed(0.0)
    finally:
        oracle.set_threads(cores)
    b = alg_bytes(plan, X.shape[1])
    return dict(value=round(b / t / 1e9, 3), unit="GB/s", cores=cores, kind="oracle",
                sample=f"{runs} full products, {w.name}, median {t * 1e3:.1f} ms each "
                       f"(OpenMP, forward / list-wise multiplication / backward of the paper)",
                one_thread=dict(value=round(b / t1 / 1e9, 3), unit="GB/s", ms=round(t1 * 1e3, 1), runs=runs1),
                host_copy_gbs=host_copy_gbs(cores), host=host_info())


def time_products(h2x, torch, A, X, Y, steps):
    h2x.h2_matmul(A, X, out=Y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        h2x.h2_matmul(A, X, out=Y)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def lambda_max(torch, h2x, A, n, iters=40, seed=7):
    """Largest eigenvalue of the (symmetric) FP64 operator by power iteration (Rayleigh quotient)."""
    g = torch.Generator(device="cuda:0").manual_seed(seed)
    v = torch.randn((n, 1), dtype=torch.float64, device="cuda:0", generator=g)
    v /= v.norm()
    lam = 0.0
    for _ in range(iters):
        w = h2x.h2_matmul(A, v)
        lam = float((v * w).sum())
        v = w / w.norm()
    return lam


def precision_record(torch, h2x, W, max_iter):
    """The precision workload (n = 262144 uniform in the unit cube, exp(-r/0.25) + 0.5 I, k = 64,
    m = 64): time to an FP64 true residual of 1e-10 with plain FP64 block CG against block CG
    with FP32-storage iterations and FP64 residual replacement; true residuals with the FP64
    product; lambda_max by power iteration (lambda_min >= the shift, so kappa <= lambda_max / shift)."""
    w = W.WORKLOADS["cube-n262144-k64-m64"]
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    plan = h2x.Plan(w.points(), **w.params())
    A = h2x.H2Matrix(plan, storage="f64", device=dev)
    A32 = h2x.H2Matrix(plan, storage="f32", device=dev)
    B = torch.from_numpy(w.rhs()).to(dev)
    # first launches and workspace allocations outside the timed solves
    h2x.block_cg_solve(A, B, rtol=1e-10, max_iter=2)
    h2x.block_cg_mixed(A, A32, B, rtol=1e-10, max_iter=2, graph=True)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    rec = {"workload": w.name, "rtol": 1e-10, "setup_s": round(setup, 2)}

    def true_rel(X):
        return ((B - h2x.h2_matmul(A, X)).norm(dim=0) / B.norm(dim=0)).max().item()

    log(f"[precision] FP64 block CG to 1e-10 on {w.name}")
    t0 = time.perf_counter()
    X, info = h2x.block_cg_solve(A, B, rtol=1e-10, max_iter=max_iter)
    torch.cuda.synchronize()
    rec["fp64_cg"] = {"time_s": round(time.perf_counter() - t0, 3), "iters": info.iters, "status": info.status,
                      "max_true_relres": true_rel(X)}
    log(f"[precision] {rec['fp64_cg']}")
    log("[precision] FP32 iterations with FP64 residual replacement to 1e-10")
    t0 = time.perf_counter()
    X, info = h2x.block_cg_mixed(A, A32, B, rtol=1e-10, delta=0.1, max_iter=max_iter, graph=True)
    torch.cuda.synchronize()
    rec["fp32_residual_replacement"] = {"time_s": round(time.perf_counter() - t0, 3), "iters": info.iters,
                                        "replacements": info.outer_iters, "status": info.status,
                                        "max_true_relres": true_rel(X)}
    log(f"[precision] {rec['fp32_residual_replacement']}")
    rec["speedup_fp32_vs_fp64"] = round(rec["fp64_cg"]["time_s"] / rec["fp32_residual_replacement"]["time_s"], 3)
    lam = lambda_max(torch, h2x, A, plan.n)
    rec["lambda_max"] = round(lam, 2)
    rec["kappa_bound"] = round(lam / w.shift, 1)
    del A, A32
    torch.cuda.empty_cache()
    return rec


def precision_report(args, torch, h2x, W):
    """FP64, FP32 and BF16 operators on the precision workload (n = 262144 in the unit cube,
    exp(-r/0.25) + 0.5 I, k = 64, m = 64): product time and algorithmic GB/s, error of each
    product against the FP64 product, FP64 block CG to 1e-8 and FP64-refined solves to 1e-10."""
    w = W.WORKLOADS["cube-n262144-k64-m64"]
    dev = torch.device("cuda:0")
    P = w.points()
    t0 = time.perf_counter()
    plan = h2x.Plan(P, **w.params())
    log(f"[precision] plan {time.perf_counter() - t0:.1f} s: C={plan.C} adm={plan.n_adm} near={plan.near_entries}")
    X = torch.from_numpy(w.rhs()).to(dev)
    m = w.m
    out = {"workload": w.name, "n": w.n, "k": w.k, "m": m, "n_adm": plan.n_adm, "near_entries": plan.near_entries}
    ops = {}
    Y64 = None
    for prec, s_b, s_n in (("f64", 8, 8), ("f32", 4, 4), ("bf16", 2, 4)):
        t0 = time.perf_counter()
        A = h2x.H2Matrix(plan, storage=prec, device=dev)
        tune = A.autotune(m) if args.autotune else None
        torch.cuda.synchronize()
        Y = torch.empty_like(X)
        ms = time_products(h2x, torch, A, X, Y, args.steps)
        B_alg = alg_bytes(plan, m, s_b=s_b, s_n=s_n)
        rec = {"setup_s": round(time.perf_counter() - t0, 2), "autotune": tune, "ms_per_product": round(ms, 3),
               "alg_gbs": round(B_alg / (ms * 1e-3) / 1e9, 1), "alg_bytes": int(B_alg)}
        if prec == "f64":
            Y64 = Y.clone()
        else:
            rec["max_col_rel_err_vs_f64"] = ((Y - Y64).norm(dim=0) / Y64.norm(dim=0)).max().item()
        ops[prec] = A
        out[prec] = rec
        log(f"[precision] {prec}: {rec}")
    B = X
    if not args.cg:
        print(json.dumps(out), flush=True)
        return
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Xs, info = h2x.block_cg_solve(ops["f64"], B, rtol=1e-8, max_iter=args.max_cg_iter)
    torch.cuda.synchronize()
    out["cg_f64_1e-8"] = {"time_s": round(time.perf_counter() - t0, 3), "iters": info.iters, "status": info.status}
    log(f"[precision] FP64 block CG to 1e-8: {out['cg_f64_1e-8']}")
    t0 = time.perf_counter()
    Xs, info = h2x.block_cg_solve(ops["f64"], B, rtol=1e-10, max_iter=args.max_cg_iter)
    torch.cuda.synchronize()
    out["cg_f64_1e-10"] = {"time_s": round(time.perf_counter() - t0, 3), "iters": info.iters, "status": info.status}
    log(f"[precision] FP64 block CG to 1e-10: {out['cg_f64_1e-10']}")
    for prec, inner in (("f32", 1e-6), ("bf16", 1e-2)):
        t0 = time.perf_counter()
        log(f"[precision] refining with the {prec} operator (inner rtol {inner})")
        Xr, info = h2x.block_cg_refine(ops["f64"], ops[prec], B, rtol=1e-10, inner_rtol=inner, max_outer=6,
                                       max_inner=args.max_cg_iter)
        torch.cuda.synchronize()
        R = torch.empty_like(B)
        h2x.h2_matmul(ops["f64"], Xr, out=R)
        res = ((B - R).norm(dim=0) / B.norm(dim=0)).max().item()
        out[f"refine_{prec}_1e-10"] = {"time_s": round(time.perf_counter() - t0, 3), "outer": info.outer_iters,
                                       "inner_iters": info.iters, "status": info.status, "true_relres": res,
                                       "inner_rtol": inner}
        log(f"[precision] refined {prec}: {out[f'refine_{prec}_1e-10']}")
    for prec in ("f32", "bf16"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        log(f"[precision] CG with {prec} iterations and FP64 residual replacement")
        Xr, info = h2x.block_cg_mixed(ops["f64"], ops[prec], B, rtol=1e-10, delta=0.1, max_iter=args.max_cg_iter,
                                      graph=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        R = torch.empty_like(B)
        h2x.h2_matmul(ops["f64"], Xr, out=R)
        res = ((B - R).norm(dim=0) / B.norm(dim=0)).max().item()
        out[f"mixed_{prec}_1e-10"] = {"time_s": round(dt, 3), "iters": info.iters, "replacements": info.outer_iters,
                                      "status": info.status, "true_relres": res}
        log(f"[precision] mixed {prec}: {out[f'mixed_{prec}_1e-10']}")
    print(json.dumps(out), flush=True)


def grad_report(args, torch, h2x, W):
    """Differentiation workload (n = 131072 on the sphere, exp(-r/0.5) + I, k = 64, m = 16, FP64):
    forward product, adjoint product, gradients (dS and dell; dell only), block-CG solve to
    1e-8 and its implicit-adjoint backward (a second solve plus the gradient kernels)."""
    from paper_2509_17257_amd.autograd import h2_solve
    w = W.WORKLOADS["sphere-n131072-k64-m16"]
    dev = torch.device("cuda:0")
    A = h2x.H2Matrix(w.points(), device=dev, **w.params())
    plan = A.plan
    m = w.m
    X = torch.from_numpy(w.rhs()).to(dev)
    dY = torch.from_numpy(W.rhs(w.n, m, 2100 + w.index)).to(dev)
    out = {"workload": w.name, "n": w.n, "k": w.k, "m": m, "n_adm": plan.n_adm, "near_entries": plan.near_entries}
    log(f"[grad] {w.name}: C={plan.C} adm={plan.n_adm} near entries={plan.near_entries}")

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    Y = torch.empty_like(X)
    reps = max(3, min(args.steps, 50))
    B_alg = alg_bytes(plan, m)
    ms = timed(lambda: h2x.h2_matmul(A, X, out=Y), reps)
    out["forward"] = {"ms": round(ms, 4), "alg_gbs": round(B_alg / (ms * 1e-3) / 1e9, 1)}
    ms = timed(lambda: h2x.h2_matmul_adjoint(A, dY, out=Y), reps)
    out["adjoint"] = {"ms": round(ms, 4), "alg_gbs": round(B_alg / (ms * 1e-3) / 1e9, 1)}
    dS_bytes = 8 * plan.n_adm * plan.k * plan.k
    ms = timed(lambda: h2x.h2_grad(A, X, dY, want_dS=True, want_dell=True), reps)
    out["grad_dS_dell"] = {"ms": round(ms, 4), "dS_bytes": dS_bytes, "dS_write_gbs": round(dS_bytes / (ms * 1e-3) / 1e9, 1)}
    ms = timed(lambda: h2x.h2_grad(A, X, dY, want_dS=True, want_dell=False), reps)
    out["grad_dS"] = {"ms": round(ms, 4), "dS_write_gbs": round(dS_bytes / (ms * 1e-3) / 1e9, 1)}
    ms = timed(lambda: h2x.h2_grad(A, X, dY, want_dS=False, want_dell=True), reps)
    out["grad_dell"] = {"ms": round(ms, 4)}
    log(f"[grad] {out}")
    B = X
    ell = torch.tensor(w.ell, dtype=torch.float64, requires_grad=True)
    Bg = B.clone().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Xs = h2_solve(A, Bg, ell, rtol=1e-8, max_iter=args.max_cg_iter)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    (dY * Xs).sum().backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    out["solve_1e-8"] = {"time_s": round(t1 - t0, 3)}
    out["implicit_adjoint_backward"] = {"time_s": round(t2 - t1, 3), "dell": float(ell.grad)}
    log(f"[grad] solve {t1 - t0:.3f} s, implicit-adjoint backward {t2 - t1:.3f} s")
    print(json.dumps(out), flush=True)


def batch_report(args, torch, h2x, W):
    """Batching workload: 64 independent systems (n log-uniform in [2048, 32768] on spheres,
    ell ~ U[0.2, 1], shift 1, k = 27 or 64, m = 1..32).  Batched product (one merged
    operator per Chebyshev order) against a loop of per-system products; batched block CG
    to 1e-8 with and without the HIP-graph step against a loop of per-system solves; the
    batched product with FP32 storage."""
    systems = W.batch_systems()
    dev = torch.device("cuda:0")
    pts = [s.points() for s in systems]
    prms = [dict(ell=s.ell, shift=s.shift, eta=1.0, leaf=s.leaf, p=s.p) for s in systems]
    t0 = time.perf_counter()
    batch = h2x.Batch(list(zip(pts, prms)), device=dev)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    m = max(s.m for s in systems)
    Bh = np.zeros((batch.n, m))
    for i, s in enumerate(systems):
        r0, r1 = batch.rows(i)
        Bh[r0:r1, :s.m] = s.rhs()
    B = torch.from_numpy(Bh).to(dev)
    Y = torch.empty_like(B)
    parts = {i: p for grp, ps in zip(batch.order, batch._parts) for i, p in zip(grp, ps)}
    alg = sum(alg_bytes(parts[i], s.m) for i, s in enumerate(systems))
    alg_pad = sum(alg_bytes(parts[i], m) for i in range(len(systems)))
    out = {"workload": f"batch-{len(systems)}-spheres", "systems": len(systems), "n_total": batch.n,
           "m_max": m, "setup_s": round(setup_s, 2),
           "n_adm_total": int(sum(p.n_adm for p in batch.plans)),
           "near_entries_total": int(sum(p.near_entries for p in batch.plans)),
           "alg_bytes_per_product": int(alg), "alg_bytes_padded_m": int(alg_pad)}
    log(f"[batch] {len(systems)} systems, n total {batch.n}, setup {setup_s:.1f} s")
    if args.autotune:
        out["autotune"] = batch.autotune(m)
        log(f"[batch] autotuned: {out['autotune']}")

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    reps = max(3, min(args.steps, 50))
    ms = timed(lambda: h2x.batch_matmul(batch, B, out=Y), reps)
    out["batched_product"] = {"ms": round(ms, 4), "alg_gbs": round(alg / (ms * 1e-3) / 1e9, 1),
                              "products_per_s": round(1e3 / ms, 1)}
    # the same products one system at a time (each with its own m)
    mats = [h2x.H2Matrix(parts[i], device=dev) for i in range(len(systems))]
    Xs = [B[batch.rows(i)[0]:batch.rows(i)[1], :s.m].contiguous() for i, s in enumerate(systems)]
    Ys = [torch.empty_like(x) for x in Xs]

    def loop():
        for A, x, y in zip(mats, Xs, Ys):
            h2x.h2_matmul(A, x, out=y)
    ms_loop = timed(loop, max(3, reps // 4))
    out["per_system_loop"] = {"ms": round(ms_loop, 4), "alg_gbs": round(alg / (ms_loop * 1e-3) / 1e9, 1)}
    log(f"[batch] product: batched {ms:.3f} ms, per-system loop {ms_loop:.3f} ms")
    for graph in ((True, False) if args.cg else ()):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X, info = h2x.batch_block_cg_solve(batch, B, rtol=1e-8, max_iter=args.max_cg_iter, graph=graph)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[f"batched_cg_graph{int(graph)}"] = {"time_s": round(dt, 3), "iters": info.iters, "status": info.status,
                                               "sys_iters_min": int(info.sys_iters.min()),
                                               "sys_iters_max": int(info.sys_iters.max())}
        log(f"[batch] batched CG graph={graph}: {dt:.3f} s, {info.iters} iterations")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tot = 0
    for A, b in zip(mats, Xs if args.cg else ()):
        _, info = h2x.block_cg_solve(A, b, rtol=1e-8, max_iter=args.max_cg_iter)
        tot += info.iters
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if args.cg:
        out["per_system_cg_loop"] = {"time_s": round(dt, 3), "iters_total": tot}
    log(f"[batch] per-system CG loop: {dt:.3f} s")
    del mats
    b32 = h2x.Batch(list(zip(pts, prms)), storage="f32", device=dev)
    Y32 = torch.empty_like(B)
    ms32 = timed(lambda: h2x.batch_matmul(b32, B, out=Y32), reps)
    h2x.batch_matmul(batch, B, out=Y)
    err = 0.0
    for i, s in enumerate(systems):
        r0, r1 = batch.rows(i)
        a, b = Y32[r0:r1, :s.m], Y[r0:r1, :s.m]
        err = max(err, ((a - b).norm(dim=0) / b.norm(dim=0)).max().item())
    alg32 = sum(alg_bytes(parts[i], s.m, s_b=4, s_n=4) for i, s in enumerate(systems))
    out["batched_product_f32"] = {"ms": round(ms32, 4), "alg_gbs": round(alg32 / (ms32 * 1e-3) / 1e9, 1),
                                  "max_col_rel_err_vs_f64": err}
    log(f"[batch] {out}")
    print(json.dumps(out), flush=True)


def mm_report(args, torch, h2x, W):
    """Multi-vector product against repeated single-vector products (the paper's
    H^2-MM experiment, section 4): on the FP64 sphere workload (n = 65536, k = 64), one
    product with m columns against m products with one column each, for
    m = 1, 10, 50, 100, 200; and the single-vector bandwidth for growing n.  Both byte
    conventions: algorithmic bytes (matrix once, X read, Y written) and the paper's
    effective bytes, m times (matrix + 3 n doubles)."""
    dev = torch.device("cuda:0")
    out = {"workload": "sphere, exp(-r/0.5) + I, leaf 64, eta 1, k 64 (FP64)", "mm_vs_mvm": [], "mvm_vs_n": []}

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def matrix_bytes(plan):
        k = plan.k
        return 8 * (plan.n * k + (plan.C - 1) * k * k + plan.n_adm * k * k) + 8 * plan.near_entries

    P = W.sphere_points(65536, 1001)
    A = h2x.H2Matrix(P, device=dev, ell=0.5, shift=1.0, eta=1.0, leaf=64, p=4)
    plan = A.plan
    mb = matrix_bytes(plan)
    reps = max(3, min(args.steps, 20))
    for m in (1, 10, 50, 100, 200):
        if args.autotune:
            A.autotune(m)
        X = torch.from_numpy(W.rhs(plan.n, m, 7000 + m)).to(dev)
        Y = torch.empty_like(X)
        ms_mm = timed(lambda: h2x.h2_matmul(A, X, out=Y), reps)
        cols = [X[:, j:j + 1].contiguous() for j in range(m)]
        outs = [torch.empty_like(c) for c in cols]

        def mvm():
            for c, o in zip(cols, outs):
                h2x.h2_matmul(A, c, out=o)
        ms_mvm = timed(mvm, max(1, reps // 4))
        rec = {"m": m, "ms_mm": round(ms_mm, 4), "ms_m_mvm": round(ms_mvm, 4), "speedup": round(ms_mvm / ms_mm, 2),
               "alg_gbs_mm": round(alg_bytes(plan, m) / (ms_mm * 1e-3) / 1e9, 1),
               "paper_convention_gbs_mm": round(m * (mb + 3 * 8 * plan.n) / (ms_mm * 1e-3) / 1e9, 1)}
        out["mm_vs_mvm"].append(rec)
        log(f"[mm] {rec}")
    del A
    for n in (4096, 16384, 65536, 262144):
        A = h2x.H2Matrix(W.sphere_points(n, 7100 + n % 97), device=dev, ell=0.5, shift=1.0, eta=1.0, leaf=64, p=4)
        x = torch.from_numpy(W.rhs(n, 1, 7200)).to(dev)
        y = torch.empty_like(x)
        ms = timed(lambda: h2x.h2_matmul(A, x, out=y), reps)
        rec = {"n": n, "ms": round(ms, 4), "alg_gbs": round(alg_bytes(A.plan, 1) / (ms * 1e-3) / 1e9, 1)}
        out["mvm_vs_n"].append(rec)
        log(f"[mm] {rec}")
        del A
    print(json.dumps(out), flush=True)


def gmres_report(args, torch, h2x, W):
    """Block GMRES(restart) (section 5.2, block form without a preconditioner) on the FP64
    sphere workload (n = 65536, k = 64, m = 32) to 1e-8, for the symmetric operator and a
    non-symmetric one (an eighth of the coupling blocks perturbed by 0.005 N(0, 1)): solve time, Arnoldi
    steps and cycles, the share of the products in the solve (the rest is Gram-Schmidt,
    rotations and updates: the paper's "GMRES time"), and the block solve against
    single-right-hand-side solves of a sample of columns (block against standard GMRES)."""
    dev = torch.device("cuda:0")
    w = W.FP64
    A = h2x.H2Matrix(w.points(), device=dev, **w.params())
    if args.autotune:
        A.autotune(w.m)
        A.autotune(1)
    B = torch.from_numpy(w.rhs()).to(dev)
    rtol, restart, sample, cap = 1e-8, 30, 4, 3000
    out = {"workload": w.name, "rtol": rtol, "restart": restart, "runs": []}

    def wall(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    def prod_ms(m):
        X = torch.from_numpy(W.rhs(w.n, m, 7300 + m)).to(dev)
        Y = torch.empty_like(X)
        h2x.h2_matmul(A, X, out=Y)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            h2x.h2_matmul(A, X, out=Y)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 20

    for kind in ("symmetric", "nonsymmetric"):
        if kind == "nonsymmetric":
            S = A.coupling()
            g = torch.Generator(device="cpu").manual_seed(7301)
            idx = torch.randperm(S.shape[0], generator=g)[: S.shape[0] // 8].to(dev)
            S[idx] += 0.005 * torch.randn(S[idx].shape, generator=g, dtype=torch.float64).to(dev)
            A.set_coupling(S)
            del S
        h2x.block_gmres_solve(A, B[:, :1], rtol=rtol, restart=restart, max_iter=2)  # warm-up
        (X, info), t_blk = wall(lambda: h2x.block_gmres_solve(A, B, rtol=rtol, restart=restart, max_iter=cap))
        res = (torch.linalg.norm(B - h2x.h2_matmul(A, X), dim=0) / torch.linalg.norm(B, dim=0)).max().item()
        pm = prod_ms(w.m)
        products = info.iters + info.cycles + 1  # steps, one residual per cycle, the final check
        singles = []
        for j in range(sample):
            (x1, i1), t1 = wall(lambda: h2x.block_gmres_solve(A, B[:, j:j + 1].contiguous(), rtol=rtol,
                                                              restart=restart, max_iter=cap))
            singles.append((t1, i1.iters))
        t1m = sum(t for t, _ in singles) / sample
        rec = {"operator": kind, "m": w.m, "time_s": round(t_blk, 4), "steps": info.iters, "cycles": info.cycles,
               "status": info.status, "max_true_relres": res, "product_ms_m32": round(pm, 4),
               "product_share": round(products * pm * 1e-3 / t_blk, 3),
               "gmres_ms_per_step": round((t_blk - products * pm * 1e-3) / max(1, info.iters) * 1e3, 4),
               "single_rhs_time_s": round(t1m, 4), "single_rhs_steps": [s for _, s in singles],
               "single_rhs_sample": f"columns 0..{sample - 1}, mean time",
               "block_speedup_est": round(w.m * t1m / t_blk, 2)}
        out["runs"].append(rec)
        log(f"[gmres] {rec}")
    print(json.dumps(out), flush=True)


def chunk_report(args, torch, h2x, W):
    """Right-hand-side chunking (section 5, memory-footprint remarks): on the FP64 sphere
    workload (n = 65536, k = 64) with m = 128 right-hand sides, the measured product-time
    curve, the chunk the policy picks under three workspace budgets, and block CG to 1e-8
    solved in chunks of every candidate size that fits, to see whether the pick is the
    fastest."""
    dev = torch.device("cuda:0")
    w = W.FP64
    A = h2x.H2Matrix(w.points(), device=dev, **w.params())
    m, rtol = 128, 1e-8
    cands = [8, 16, 32, 64, 128]
    if args.autotune:
        for c in cands:
            A.autotune(c)
    curve = dict(zip(cands, A.product_times(cands, reps=10)))
    B = torch.from_numpy(W.rhs(w.n, m, 7400)).to(dev)
    ws = {c: h2x.solve_workspace_bytes(A.plan, c, solver="cg") for c in cands}
    out = {"workload": w.name, "m": m, "rtol": rtol, "curve_ms_per_product": {str(c): round(t, 4) for c, t in curve.items()},
           "workspace_bytes": {str(c): ws[c] for c in cands}, "budgets": [], "solves": []}
    measured = {}
    for c in cands:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X, info = h2x.block_cg_solve_chunked(A, B, c, rtol=rtol)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        measured[c] = dt
        rec = {"m_chunk": c, "time_s": round(dt, 4), "max_iters": info.iters, "status": info.status,
               "predicted_product_s": round(-(-m // c) * curve[c] * info.iters * 1e-3, 4)}
        out["solves"].append(rec)
        log(f"[chunk] {rec}")
    for name, budget in (("unlimited", 1 << 62), ("fits 32 columns", ws[32]), ("fits 8 columns", ws[8])):
        pick = h2x.choose_chunk(A.plan, m, budget, solver="cg", curve=curve)
        fit = [c for c in cands if ws[c] <= budget]
        best = min(fit, key=lambda c: measured[c])
        rec = {"budget": name, "budget_bytes": min(budget, 2**63 - 1), "pick": pick, "fastest_measured": best,
               "pick_over_fastest": round(measured.get(pick, float("nan")) / measured[best], 3)}
        out["budgets"].append(rec)
        log(f"[chunk] {rec}")
    print(json.dumps(out), flush=True)


def complex_report(args, torch, h2x, W):
    """Complex Helmholtz operator (section 5.2's complex setting; single-layer kernel with
    equal quadrature weights) on the FP64 sphere workload's points (n = 65536, leaf 64,
    k = 64), 16 complex right-hand sides: product time and algorithmic bandwidth (S and N
    complex, 16 bytes per entry; V and E real), block GMRES(30) to 1e-8, and single-column
    GMRES of a sample of columns, for wavenumbers 1 and 4."""
    dev = torch.device("cuda:0")
    w = W.FP64
    P = w.points()
    mc, rtol, restart, sample = 16, 1e-8, 30, 4
    out = {"workload": f"helmholtz-sphere-n{w.n}-k64-m{mc}c", "runs": []}
    for kappa in (1.0, 4.0):
        A = h2x.H2Matrix(P, device=dev, kernel="helmholtz", ell=kappa, shift=1.0, eta=1.0, leaf=64, p=4)
        if args.autotune:
            A.autotune(2 * mc)
        plan = A.plan
        k = plan.k
        alg = (8 * (plan.n * k + (plan.C - 1) * k * k) + 16 * plan.n_adm * k * k + 16 * plan.near_entries
               + 16 * plan.n * mc * 2)
        X = torch.complex(torch.from_numpy(W.rhs(w.n, mc, 7500)), torch.from_numpy(W.rhs(w.n, mc, 7501))).to(dev)
        Y = torch.empty_like(X)
        h2x.h2_matmul(A, X, out=Y)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = max(5, min(args.steps, 50))
        e0.record()
        for _ in range(reps):
            h2x.h2_matmul(A, X, out=Y)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        B = torch.complex(torch.from_numpy(W.rhs(w.n, mc, 7502)), torch.from_numpy(W.rhs(w.n, mc, 7503))).to(dev)
        h2x.block_gmres_solve(A, B[:, :1].contiguous(), rtol=rtol, restart=restart, max_iter=2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Xs, info = h2x.block_gmres_solve(A, B, rtol=rtol, restart=restart, max_iter=3000)
        torch.cuda.synchronize()
        t_blk = time.perf_counter() - t0
        res = (torch.linalg.norm(B - h2x.h2_matmul(A, Xs), dim=0) / torch.linalg.norm(B, dim=0)).max().item()
        singles = []
        for j in range(sample):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, i1 = h2x.block_gmres_solve(A, B[:, j:j + 1].contiguous(), rtol=rtol, restart=restart, max_iter=3000)
            torch.cuda.synchronize()
            singles.append((time.perf_counter() - t0, i1.iters))
        t1 = sum(t for t, _ in singles) / sample
        rec = {"kappa": kappa, "complex_columns": mc, "product_ms": round(ms, 4),
               "product_alg_gbs": round(alg / (ms * 1e-3) / 1e9, 1), "alg_bytes": alg,
               "gmres_time_s": round(t_blk, 4), "gmres_steps": info.iters, "gmres_cycles": info.cycles,
               "gmres_status": info.status, "max_true_relres": res, "single_rhs_time_s": round(t1, 4),
               "single_rhs_steps": [s for _, s in singles], "block_speedup_est": round(mc * t1 / t_blk, 2)}
        out["runs"].append(rec)
        log(f"[complex] {rec}")
        del A
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="sphere-n65536-k64-m32")
    ap.add_argument("--cg", type=int, default=1, help="also time block CG to 1e-8")
    ap.add_argument("--max-cg-iter", type=int, default=5000)
    ap.add_argument("--precision-record", type=int, default=1,
                    help="also time FP64 CG against FP32 residual replacement to 1e-10 on the precision workload")
    ap.add_argument("--autotune", type=int, default=1, help="autotune the tile shapes before timing (1) or not (0)")
    ap.add_argument("--cpu-baseline-s", type=float, default=12.0, help="0 disables the oracle timing")
    ap.add_argument("--precision-report", action="store_true",
                    help="report FP64 / FP32 / BF16 products and FP64 vs refined block CG on the precision workload")
    ap.add_argument("--mm-report", action="store_true",
                    help="multi-vector product against repeated single-vector products (m = 1..200)")
    ap.add_argument("--batch-report", action="store_true",
                    help="batched products and block CG over the 64-system batching workload")
    ap.add_argument("--grad-report", action="store_true",
                    help="time the adjoint product, gradients and implicit-adjoint solve on the differentiation workload")
    ap.add_argument("--gmres-report", action="store_true",
                    help="block GMRES(30) to 1e-8 on the FP64 workload, symmetric and non-symmetric operators")
    ap.add_argument("--chunk-report", action="store_true",
                    help="right-hand-side chunk policy: product-time curve, picks under budgets, chunked CG solves")
    ap.add_argument("--complex-report", action="store_true",
                    help="complex Helmholtz operator: products and block GMRES over C on the FP64 workload's points")
    ap.add_argument("--copy-calibration-gib", type=float, default=0.0,
                    help="only run a plain device copy of this many GiB (to scale HBM traffic counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "sharding across GPUs is designed but not built", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2509_17257_amd as h2x
    from paper_2509_17257_amd import workloads as W

    if args.copy_calibration_gib > 0:
        # plain device copy of a known size (scales the HBM traffic counters) and the
        # bandwidth a copy and a read-only reduction reach on this device
        nbytes = int(args.copy_calibration_gib * 2**30) // 8 * 8
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        reps = 10
        dst.copy_(src)
        torch.cuda.synchronize()
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        for _ in range(reps):
            dst.copy_(src)
        e1.record()
        for _ in range(reps):
            src.sum()
        e2.record()
        torch.cuda.synchronize()
        copy_gbs = 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
        read_gbs = nbytes * reps / (e1.elapsed_time(e2) * 1e-3) / 1e9
        print(json.dumps({"copy_calibration_bytes": nbytes, "copies": reps + 1, "copy_gbs": round(copy_gbs, 1),
                          "read_gbs": round(read_gbs, 1)}), flush=True)
        return

    if args.precision_report:
        precision_report(args, torch, h2x, W)
        return
    if args.grad_report:
        grad_report(args, torch, h2x, W)
        return
    if args.batch_report:
        batch_report(args, torch, h2x, W)
        return
    if args.mm_report:
        mm_report(args, torch, h2x, W)
        return
    if args.gmres_report:
        gmres_report(args, torch, h2x, W)
        return
    if args.chunk_report:
        chunk_report(args, torch, h2x, W)
        return
    if args.complex_report:
        complex_report(args, torch, h2x, W)
        return

    w = W.WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    log(f"[bench] workload {w.name}: building plan and operator")
    P = w.points()
    t0 = time.perf_counter()
    A = h2x.H2Matrix(P, device=dev, **w.params())
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    plan = A.plan
    m = w.m
    Xh = w.rhs()
    X = torch.from_numpy(Xh).to(dev)
    Y = torch.empty_like(X)
    log(f"[bench] setup {setup_s:.2f} s; C={plan.C} leaves={plan.leaves} adm={plan.n_adm} near={plan.n_near} "
        f"near entries={plan.near_entries}")

    tune = A.autotune(m) if args.autotune else None
    if tune:
        log(f"[bench] autotuned tile shapes: {tune}")
    for _ in range(args.warmup):
        h2x.h2_matmul(A, X, out=Y)
    torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup} done; timing {args.steps} products")
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        h2x.h2_matmul(A, X, out=Y)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    B_alg = alg_bytes(plan, m)
    F = alg_flops(plan, m)
    gbs = B_alg / (ms * 1e-3) / 1e9
    log(f"[bench] {ms:.4f} ms/product, {gbs:.1f} GB/s algorithmic")
    # stage times: after the timed region, the same number of products, each recording its
    # stage boundaries with HIP events on the library's stream (the caller's stream), read
    # afterwards; the coupling is one kernel launch, so its stage time is that launch's
    # duration (plus the launch gap before it)
    timer = h2x.Timer(args.steps)
    for i in range(args.steps):
        h2x.h2_matmul(A, X, out=Y, timer=timer, slot=i)
    torch.cuda.synchronize()
    per = np.array([timer.read(j) for j in range(args.steps)])
    stage = per.mean(axis=0)
    log(f"[bench] stage times from {args.steps} marked products after the timed region")
    cb, cf, ci = coupling_bytes(plan), coupling_flops(plan, m), coupling_intermediate_bytes(plan, m)
    c_ms = stage[h2x.STAGES.index("coupling")]
    c_gbs = cb / (c_ms * 1e-3) / 1e9
    c_tf = cf / (c_ms * 1e-3) / 1e12
    bound = "hbm" if cb / (PEAK_HBM_GBS * 1e9) >= cf / (PEAK_FP64_TFLOPS * 1e12) else "mfma"
    if bound == "hbm":
        roof = dict(bound="hbm", achieved=round(c_gbs, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                    frac=round(c_gbs / PEAK_HBM_GBS, 4), traffic=None)
    else:
        roof = dict(bound="mfma", achieved=round(c_tf, 2), peak=PEAK_FP64_TFLOPS, unit="TFLOP/s",
                    frac=round(c_tf / PEAK_FP64_TFLOPS, 4), traffic=None)
    if w.name == "sphere-n65536-k64-m32":
        roof["traffic"] = measured_traffic("coupling_f64_sphere-n65536-k64-m32.pmc.txt")
    roof.update(kernel="coupling", kernel_ms=round(float(c_ms), 5), kernel_ms_min=round(float(per[:, 2].min()), 5),
                kernel_bytes=int(cb), intermediate_bytes=int(ci), kernel_flops=int(cf),
                bytes_rule="k^2 * 8 bytes per admissible block (S once); x-hat / y-hat apart")
    log("[bench] stages ms: " + ", ".join(f"{n}={v:.4f}" for n, v in zip(h2x.STAGES, stage)))

    out = {
        "metric": "H2*X algorithmic GB/s (FP64), n=65536 k=64 m=32",
        "value": round(gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded points on the unit sphere, N(0,1) right-hand sides)",
        "config": {"workload": w.name, "n": w.n, "k": w.k, "m": m, "leaf": w.leaf, "eta": w.eta, "ell": w.ell,
                   "shift": w.shift, "clusters": plan.C, "n_adm": plan.n_adm, "n_near": plan.n_near,
                   "near_entries": plan.near_entries},
        "products_per_s": round(1e3 / ms, 2),
        "alg_bytes_per_product": int(B_alg),
        "alg_flops_per_product": int(F),
        "hbm_frac": round(gbs / PEAK_HBM_GBS, 4),
        "fp64_frac": round(F / (ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, 4),
        "paper_convention_gbs": round(m * (B_alg - 8 * 3 * plan.n * m + 3 * 8 * plan.n) / (ms * 1e-3) / 1e9, 1),
        "stage_ms": {n: round(float(v), 5) for n, v in zip(h2x.STAGES, stage)},
        "roofline": roof,
        "setup_s": round(setup_s, 3),
        "autotune": tune,
    }

    if args.cg:
        B = X
        # a few iterations of each variant first, so that the timed solves include neither
        # the first launch of a kernel nor the first allocation of the solver's workspace
        for variant in ("independent", "shared"):
            h2x.block_cg_solve(A, B, rtol=1e-8, max_iter=3, variant=variant)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Xs, info = h2x.block_cg_solve(A, B, rtol=1e-8, max_iter=5000)
        torch.cuda.synchronize()
        cg_s = time.perf_counter() - t0
        R = torch.empty_like(B)
        h2x.h2_matmul(A, Xs, out=R)
        res = ((B - R).norm(dim=0) / B.norm(dim=0)).max().item()
        out["block_cg"] = {"rtol": 1e-8, "time_s": round(cg_s, 4), "iters": info.iters, "status": info.status,
                           "max_true_relres": res, "precision": "f64", "variant": "independent"}
        log(f"[bench] block CG: {info.iters} iterations, {cg_s:.3f} s, true rel res {res:.2e}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Xs, info = h2x.block_cg_solve(A, B, rtol=1e-8, max_iter=5000, variant="shared")
        torch.cuda.synchronize()
        cg_s = time.perf_counter() - t0
        h2x.h2_matmul(A, Xs, out=R)
        res = ((B - R).norm(dim=0) / B.norm(dim=0)).max().item()
        out["block_cg_shared"] = {"rtol": 1e-8, "time_s": round(cg_s, 4), "iters": info.iters, "status": info.status,
                                  "max_true_relres": res, "precision": "f64", "variant": "shared"}
        log(f"[bench] shared-space block CG: {info.iters} iterations, {cg_s:.3f} s, true rel res {res:.2e}")

    if args.precision_record:
        out["precision"] = precision_record(torch, h2x, W, args.max_cg_iter)

    if args.cpu_baseline_s > 0:
        log(f"[bench] timing the CPU oracle for ~{args.cpu_baseline_s:.0f} s")
        out["cpu_baseline"] = cpu_baseline(w, P, Xh, plan, args.cpu_baseline_s)
        log(f"[bench] CPU oracle: {out['cpu_baseline']}")

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
