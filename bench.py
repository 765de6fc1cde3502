"""Throughput of the FFT-accelerated multi-block Poisson solve on one GPU.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload lshape|box|cube32]
                    [--precision fp64|mixed] [--lockstep] [--no-cpu] [--no-variants]
    python bench.py --workload batch64 [--steps K] [--no-variants]  # 64 uneven problems, batched form
    python bench.py --workload serve [--requests N]    # Poisson request stream, server
    python bench.py --transform-compare                # z transform: LDS FFT vs dense matrix product
    python bench.py --copy-calibrate                   # 1 GiB copies (scale for HBM byte counters)

One step is one complete solve of the pressure-Poisson problem (Algorithm 1):
forward z-transform, the shifted 2D multigrid solves of every mode to a
relative residual of 1e-10, inverse transform.  The rhs is resident in device
memory before the timed region starts.  The default workload is the
three-block L-shaped cross-section (each block 256 x 256, tanh-stretched y,
Neumann walls) with 512 periodic z cells, solved in FP64, each mode stopped
at its own convergence test.

Output: one JSON line with grid points/s (``value``), solves/s, the roofline
record of the dominant kernel (the finest-level fused smoothing sweep, timed
with events on the solve stream) and the CPU oracle timed on a bounded sample
of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
RTOL = 1e-10


def _workload(name: str):
    if name == "lshape":
        return W.config2(), W.CONFIG_SEEDS[2], W.CONFIG_DIST[2]
    if name == "box":
        return W.config3(), W.CONFIG_SEEDS[3], W.CONFIG_DIST[3]
    if name == "cube32":
        return W.config1(), W.CONFIG_SEEDS[1], W.CONFIG_DIST[1]
    raise SystemExit(f"unknown workload {name}")


def _bytes_per_cell(precision: str) -> float:
    """Method bytes of one finest-level fused launch per plane cell and mode.

    Each launch does one red-black smoothing sweep (read p and f, write p:
    3 words) plus either the residual with its restriction (read p and f,
    write a quarter-size coarse rhs: 2.25 words) or the prolongation with its
    correction (2.25 words), so 5.25 words per cell.
    """
    w = 8.0 if precision == "fp64" else 4.0
    return 5.25 * w


def _vcycle_bytes_per_point(precision: str, nu1: int, nu2: int) -> float:
    """Method bytes of one V-cycle per fine point: (sweeps*3 + 4.5) words x 4/3."""
    w = 8.0 if precision == "fp64" else 4.0
    return ((nu1 + nu2) * 3.0 + 4.5) * w * 4.0 / 3.0


def _traffic_record(workload: str, precision: str):
    """HBM bytes per launch of the dominant kernel from the committed counter summary
    (the JSON block of profiles/traffic_fused_sweep_<workload>_<precision>.md)."""
    names = {"lshape3x256^2x512_stretch1.5": "lshape_256x3x512", "box512x512x1024_DD_NN_NN": "box_512x512x1024"}
    if workload not in names:
        return None
    path = os.path.join(HERE, "profiles", f"traffic_fused_sweep_{names[workload]}_{precision}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    if "```json" not in text:
        return None
    block = text.split("```json", 1)[1].split("```", 1)[0]
    rec = json.loads(block)
    # counters describe one build of the sweep kernels: stale once the source changed
    if rec.get("kernel_source_sha256") != _kernel_source_hash():
        return None
    return rec


def _kernel_source_hash() -> str:
    import hashlib
    path = os.path.join(HERE, "paper_2106_03583_amd", "csrc", "march.hip")
    return hashlib.sha256(open(path, "rb").read()).hexdigest()


def cpu_baseline(prob, f, budget_s: float = 20.0) -> dict:
    """The FP64 oracle (Algorithm 1 with sparse LU per mode) on a bounded sample.

    Sample: the full forward and inverse transforms, plus k factorisations and
    solves of shifted planes with distinct shifts (smallest |shift| first, as
    long as the time budget lasts); the full-solve time is extrapolated as
    transforms + factorisations x (distinct shifts)/k + plane solves x nz/k.
    """
    import oracle
    from oracle.solve import _geom, _plane_factor, _plane_solve, assemble_2d, _to_modes, _from_modes
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = 1
    g = _geom(prob)
    T = oracle.basis(g.zkind, g.nz)
    lam = oracle.eigenvalues(g.zkind, g.nz)
    key = np.round(lam, 12)
    distinct = len(set(key.tolist()))
    _, first = np.unique(key, return_index=True)
    order = sorted(first.tolist(), key=lambda q: abs(lam[q]))
    t0 = time.perf_counter()
    fp = oracle.project_compatible(prob, f) if oracle.is_singular(prob) else f
    fhat = _to_modes(g, fp, T)
    t_fwd = time.perf_counter() - t0
    A2 = assemble_2d(g)
    phat = np.zeros_like(fhat)
    t_fac = t_sol = 0.0
    k = 0
    sing_xy = not g.has_dirichlet_xy()
    spent = time.perf_counter()
    for q in order:
        t1 = time.perf_counter()
        fac = _plane_factor(g, A2, lam[q] / (g.dz * g.dz), (lam[q] == 0.0) and sing_xy)
        t2 = time.perf_counter()
        phat[q] = _plane_solve(fac, fhat[q])
        t3 = time.perf_counter()
        t_fac += t2 - t1
        t_sol += t3 - t2
        k += 1
        if time.perf_counter() - spent > budget_s or k >= 64:
            break
    t0 = time.perf_counter()
    _from_modes(g, phat, T)
    t_inv = time.perf_counter() - t0
    nz = g.nz
    t_est = t_fwd + t_inv + t_fac * distinct / k + t_sol * nz / k
    return {
        "value": float(prob.ncells / t_est),
        "unit": "grid points/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"FP64 oracle (Algorithm 1, sparse LU per shifted plane) on the same field: full forward "
                   f"and inverse transforms ({t_fwd + t_inv:.1f} s), {k} of {distinct} distinct plane "
                   f"factorisations with their solves ({t_fac + t_sol:.1f} s); full solve extrapolated as "
                   f"transforms + factorisations x {distinct}/{k} + solves x {nz}/{k} = {t_est:.1f} s; "
                   f"BLAS threads {threads}, factorisations single-threaded"),
    }


def _device_rhs(torch, n, seed):
    """Seeded uniform[-1, 1) rhs drawn on the device (throughput runs only)."""
    g = torch.Generator(device="cuda")
    g.manual_seed(int(seed))
    return torch.rand(n, generator=g, dtype=torch.float64, device="cuda") * 2.0 - 1.0


def _rel(torch, a, b):
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def bench_batch(args, torch, mbp):
    """64 independent solves of uneven size: mixed batched form vs plain FP64."""
    probs = W.config4()
    ncells = sum(p.ncells for p in probs)
    rhs = [_device_rhs(torch, p.ncells, 4000 + i) for i, p in enumerate(probs)]
    t0 = time.perf_counter()
    fast = [mbp.Plan(p, precision="mixed") for p in probs]
    plain = [] if args.no_variants else [mbp.Plan(p, precision="fp64") for p in probs]
    t_plan = time.perf_counter() - t0
    out_f = [torch.zeros_like(r) for r in rhs]
    out_p = [torch.zeros_like(r) for r in rhs]
    print(f"# batch64: {len(probs)} problems, {ncells} cells, plans {t_plan:.1f} s", file=sys.stderr, flush=True)
    # warm-up (the first call tunes the schedule), then timed calls
    mbp.solve_batch(fast, rhs, out_f, rtol=RTOL, flags=mbp.PROJECT_RHS | mbp.AUTOTUNE)
    for _ in range(max(0, args.warmup - 1)):
        mbp.solve_batch(fast, rhs, out_f, rtol=RTOL, flags=mbp.PROJECT_RHS)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for _ in range(args.steps):
        infos = mbp.solve_batch(fast, rhs, out_f, rtol=RTOL, flags=mbp.PROJECT_RHS)
    torch.cuda.synchronize()
    t_fast = (time.perf_counter() - w0) / args.steps
    sched = mbp.batch_schedule(fast)
    t_plain = t_fp64_batch = diff = None
    if plain:  # --no-variants: the batched form alone (e.g. under a profiler)
        # plain FP64: one solve at a time, all modes in lockstep, host-driven
        for pl, r, o in zip(plain, rhs, out_p):
            pl.solve(r, o, rtol=RTOL, flags=mbp.PROJECT_RHS)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for pl, r, o in zip(plain, rhs, out_p):
            pl.solve(r, o, rtol=RTOL, flags=mbp.PROJECT_RHS)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - w0
        # the FP64 batched form, for the breakdown
        w0 = time.perf_counter()
        mbp.solve_batch(plain, rhs, out_p, rtol=RTOL, flags=mbp.PROJECT_RHS)
        torch.cuda.synchronize()
        t_fp64_batch = time.perf_counter() - w0
        diff = max(_rel(torch, a, b) for a, b in zip(out_f, out_p))
    ok = all(i.status == 0 and i.rel_residual <= RTOL for i in infos)
    for pl in fast + plain:
        pl.close()
    return {
        "metric": "solves/s at 1e-10 relative residual",
        "value": len(probs) / t_fast,
        "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(t_fast * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32-in-f64", "data": "synthetic (seeded, device-drawn rhs)",
        "config": {"workload": "batch of 64 uneven boxes 64..384 x 64..384 x 64..256, all BC pairs",
                   "cells": ncells, "form": "mixed, batched graph replay, per-mode retirement",
                   "schedule_streams_cycles": sched},
        "grid_points_per_s": ncells / t_fast,
        "plain_fp64_solves_per_s": len(probs) / t_plain if t_plain else None,
        "fp64_batched_solves_per_s": len(probs) / t_fp64_batch if t_fp64_batch else None,
        "speedup_vs_plain_fp64": t_plain / t_fast if t_plain else None,
        "max_rel_diff_vs_plain": diff,
        "ok": ok,
        "plan_s": round(t_plan, 2),
    }


def bench_serve(args, torch, mbp):
    """Poisson stream of requests through the server; latency p50/p99."""
    n = args.requests
    reqs = W.config5(count=n, rate_per_s=1.0)
    cells = [r.problem.ncells for r in reqs]
    rhs = [_device_rhs(torch, c, r.seed) for c, r in zip(cells, reqs)]
    outs = [torch.zeros_like(x) for x in rhs]
    torch.cuda.synchronize()
    budget = int(args.server_gb * (1 << 30))
    srv = mbp.Server(hbm_budget=budget, slots=args.slots, precision="mixed")

    def closed_loop():
        w0 = time.perf_counter()
        ts = [srv.submit(r.problem, x, o, rtol=RTOL, flags=mbp.PROJECT_RHS) for r, x, o in zip(reqs, rhs, outs)]
        res = [srv.wait(t) for t in ts]
        return time.perf_counter() - w0, res

    closed_loop()  # warm: builds and caches plans where the budget allows
    t_cap, _ = closed_loop()
    capacity = n / t_cap
    rate = 0.7 * capacity
    print(f"# serve: {n} requests, capacity {capacity:.1f} solves/s, replay at {rate:.1f}/s",
          file=sys.stderr, flush=True)
    w0 = time.perf_counter()
    tickets = []
    for r, x, o in zip(reqs, rhs, outs):
        due = w0 + r.arrival_s / rate
        while True:
            now = time.perf_counter()
            if now >= due:
                break
            time.sleep(min(0.0005, due - now))
        tickets.append(srv.submit(r.problem, x, o, rtol=RTOL, flags=mbp.PROJECT_RHS))
    res = [srv.wait(t) for t in tickets]
    t_open = time.perf_counter() - w0
    srv.close()
    lat = np.array([ms for _, _, ms in res])
    steady = lat[n // 10:]
    ok = all(st == 0 for st, _, _ in res)
    # the same trace back to back through the plain FP64 solver (plans built beforehand)
    plans = [mbp.Plan(r.problem, precision="fp64") for r in reqs]
    ref = [torch.zeros_like(x) for x in rhs]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for pl, x, o in zip(plans, rhs, ref):
        pl.solve(x, o, rtol=RTOL, flags=mbp.PROJECT_RHS)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - w0
    diff = max(_rel(torch, a, b) for a, b in zip(outs, ref))
    for pl in plans:
        pl.close()
    return {
        "metric": "solves/s at 1e-10 relative residual; p50/p99 latency",
        "value": capacity,
        "unit": "solves/s",
        "n_gpus": 1, "steps": n, "warmup": n,
        "ms_per_step": round(1e3 / capacity, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32-in-f64", "data": "synthetic (seeded, device-drawn rhs)",
        "config": {"workload": f"Poisson request stream, {n} requests, sizes log-uniform 32..512 per axis",
                   "cells": int(sum(cells)), "slots": args.slots, "hbm_budget_gb": args.server_gb},
        "capacity_solves_per_s": capacity,
        "replay_rate_per_s": rate,
        "replay_solves_per_s": n / t_open,
        "latency_ms_p50": float(np.percentile(steady, 50)),
        "latency_ms_p99": float(np.percentile(steady, 99)),
        "plain_fp64_solves_per_s": n / t_plain,
        "speedup_vs_plain_fp64": (n / t_cap) / (n / t_plain),
        "max_rel_diff_vs_plain": diff,
        "ok": ok,
    }


def transform_compare(torch, mbp):
    """The z transform of a 256 x 256 plane stack two ways: the LDS FFT kernel
    (DCT-II, forward) and a dense nz x nz matrix times the [nz, plane] field in
    FP64 (a library GEMM on the matrix cores).  Both move the same 16 B per
    cell; the matrix form also spends 2 nz flops per cell."""
    cols = 256 * 256
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed(fn, reps=10):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(reps):
            fn()
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / reps

    rows = []
    for nz in (64, 96, 128, 192, 256, 512, 1024):
        g = torch.Generator(device="cuda").manual_seed(nz)
        T = torch.randn(nz, nz, dtype=torch.float64, device="cuda", generator=g)
        X = torch.randn(nz, cols, dtype=torch.float64, device="cuda", generator=g)
        Y = torch.empty_like(X)
        t_gemm = timed(lambda: torch.matmul(T, X, out=Y))
        prob = W.box(256, 256, nz, 1.0, 1.0, 1.0, "DD", "NN", "NN")
        plan = mbp.Plan(prob, precision="fp64")
        f = X.reshape(-1)
        fh = torch.empty_like(f)
        t_fft = timed(lambda: plan.forward(f, fh))
        plan.close()
        rows.append({"nz": nz, "cells": nz * cols, "fft_ms": round(t_fft, 4), "gemm_ms": round(t_gemm, 4),
                     "fft_GBs": round(16 * nz * cols / (t_fft * 1e-3) / 1e9, 1),
                     "gemm_TFLOPs": round(2.0 * nz * nz * cols / (t_gemm * 1e-3) / 1e12, 1),
                     "fft_over_gemm": round(t_fft / t_gemm, 3)})
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="lshape", choices=["lshape", "box", "cube32", "batch64", "serve"])
    ap.add_argument("--requests", type=int, default=200, help="serve: requests in the stream")
    ap.add_argument("--slots", type=int, default=8, help="serve: concurrent requests")
    ap.add_argument("--server-gb", type=float, default=96.0, help="serve: plan memory budget (GiB)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--lockstep", action="store_true", help="iterate all modes until the global test passes")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-variants", action="store_true", help="skip the short runs of the other forms")
    ap.add_argument("--copy-calibrate", action="store_true",
                    help="only run five 1 GiB device-to-device copies (scale for HBM byte counters)")
    ap.add_argument("--transform-compare", action="store_true",
                    help="only time the z transform as the LDS FFT kernel and as a dense FP64 matrix "
                         "product (library GEMM) for several nz")
    args = ap.parse_args(argv)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the solver runs every mode of a problem on a single "
              "device; multi-GPU sharding is not implemented (use --gpus 1).", file=sys.stderr)
        return 2

    import torch
    import paper_2106_03583_amd as mbp

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    if args.copy_calibrate:
        n = 1 << 27
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(5):
            y.copy_(x)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / 5
        print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "ms": ms,
                          "GBs": 16 * n / (ms * 1e-3) / 1e9}), flush=True)
        return 0
    if args.transform_compare:
        for row in transform_compare(torch, mbp):
            print(json.dumps(row), flush=True)
        return 0
    if args.workload in ("batch64", "serve"):
        out = (bench_batch if args.workload == "batch64" else bench_serve)(args, torch, mbp)
        print(json.dumps(out), flush=True)
        return 0 if out["ok"] else 1
    prob, seed, dist = _workload(args.workload)
    f = W.rhs(prob, seed, dist)
    fd = torch.from_numpy(f).cuda()
    flags = mbp.PROJECT_RHS | (0 if args.lockstep else mbp.RETIRE)
    t0 = time.perf_counter()
    plan = mbp.Plan(prob, precision=args.precision)
    t_plan = (time.perf_counter() - t0) * 1e3
    p = torch.zeros_like(fd)
    print(f"# workload {prob.name} cells={prob.ncells} precision={args.precision} "
          f"retire={not args.lockstep} plan_ms={t_plan:.1f}", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        plan.solve(fd, p, rtol=RTOL, flags=flags)
    torch.cuda.synchronize()

    plan.profile(True)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    infos = []
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        infos.append(plan.solve(fd, p, rtol=RTOL, flags=flags, stream=stream))
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = ev0.elapsed_time(ev1)
    prof = plan.profile_read()
    plan.profile(False)
    ms_step = ms / args.steps
    print(f"# timed {args.steps} solves: {ms_step:.2f} ms/solve (wall {wall * 1e3 / args.steps:.2f})",
          file=sys.stderr, flush=True)

    # correctness of the last solve: the solver's modal test and an
    # independent physical-space residual through the 3D operator
    last = infos[-1]
    ok = all(i.status == 0 and i.rel_residual <= RTOL for i in infos)
    Ap = torch.empty_like(fd)
    plan.apply(p, Ap)
    fpr = fd - last.removed_mean
    res3d = float(torch.linalg.vector_norm(fpr - Ap) / torch.linalg.vector_norm(fpr))

    # roofline of the dominant kernel (finest-level fused sweep)
    cls = int(np.argmax(prof["total_ms"]))
    launches = prof["launches"][cls]
    roof = None
    if launches > 0:
        avg_ms = prof["total_ms"][cls] / launches
        cells = prof["cells"][cls] / launches
        bpc = _bytes_per_cell(args.precision)
        achieved = bpc * cells / (avg_ms * 1e-3) / 1e9
        traffic = None
        tr = _traffic_record(prob.name, args.precision)
        if tr and tr.get("kernel_class") == cls and tr.get("workload") == prob.name \
                and tr.get("precision") == args.precision and not args.lockstep:
            traffic = tr.get("bytes_per_launch")
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": ["k_tile pre-smooth+residual+restrict", "k_tile correct+post-smooth+norm"][cls],
                "avg_launch_ms": round(avg_ms, 4), "launches": launches,
                "bytes_per_launch": bpc * cells}

    # all V-cycle work of the timed solves against the V-cycle byte model
    vb = _vcycle_bytes_per_point(args.precision, 1, 1)
    plane = prob.ncells // prob.nz
    mg_ms = sum(i.t_ms[1] for i in infos) / len(infos)
    cyc = sum(int(i.cycles_per_mode.sum()) if not args.lockstep else i.cycles * prob.nz for i in infos) / len(infos)
    vcycle = {"bytes_per_point": vb, "mode_cycles": cyc, "mg_ms": round(mg_ms, 3),
              "achieved_GBs": round(vb * plane * cyc / (mg_ms * 1e-3) / 1e9, 1)}
    vcycle["frac"] = round(vcycle["achieved_GBs"] / HBM_PEAK_GBS, 4)

    variants = {}
    if not args.no_variants:
        for name, prec, fl in [("fp64_lockstep", "fp64", mbp.PROJECT_RHS),
                               ("fp64_retire", "fp64", mbp.PROJECT_RHS | mbp.RETIRE),
                               ("mixed_retire", "mixed", mbp.PROJECT_RHS | mbp.RETIRE)]:
            if prec == args.precision and fl == flags:
                variants[name] = {"ms_per_solve": round(ms_step, 3), "rel_residual": last.rel_residual}
                continue
            pl = mbp.Plan(prob, precision=prec)
            q = torch.zeros_like(fd)
            pl.solve(fd, q, rtol=RTOL, flags=fl)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            n = 3
            for _ in range(n):
                inf = pl.solve(fd, q, rtol=RTOL, flags=fl, stream=stream)
            b.record(stream)
            torch.cuda.synchronize()
            variants[name] = {"ms_per_solve": round(a.elapsed_time(b) / n, 3),
                              "rel_residual": inf.rel_residual, "status": inf.status,
                              "max_abs_diff_vs_timed": float((q - p).abs().max())}
            pl.close()
            del q

    cpu = None
    if not args.no_cpu:
        print("# cpu baseline (oracle, bounded sample)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(prob, f)

    value = prob.ncells * args.steps / (ms * 1e-3)
    out = {
        "metric": "grid points/s at 1e-10 relative residual",
        "value": value,
        "unit": "grid points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-in-f64",
        "data": "synthetic (seeded)",
        "config": {"workload": prob.name, "cells": prob.ncells, "nz": prob.nz,
                   "blocks": len(prob.blocks), "precision": args.precision,
                   "mode_stop": "lockstep" if args.lockstep else "per-mode", "rtol": RTOL},
        "solves_per_s": 1e3 / ms_step,
        "ok": ok,
        "rel_residual_modal": last.rel_residual,
        "rel_residual_3d": res3d,
        "cycles_max": last.cycles,
        "t_ms_last": [round(t, 3) for t in last.t_ms],
        "plan_ms": round(t_plan, 1),
        "roofline": roof,
        "vcycle_roofline": vcycle,
        "variants": variants,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    plan.close()
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
