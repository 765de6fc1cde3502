"""Throughput of the FFT-accelerated multi-block Poisson solve on one GPU.

    python bench.py [--gpus 1] [--steps K] [--warmup W]      # headline line (see below)
    python bench.py --workload lshape|box|cube32 [--precision fp64|mixed] [--lockstep]
    python bench.py --workload batch64 | serve                # one form on its own
    python bench.py --transform-compare                       # z transform: LDS FFT vs dense product
    python bench.py --copy-calibrate                          # 1 GiB copies (scale for HBM counters)

One step is one complete solve of the pressure-Poisson problem (Algorithm 1):
forward z transform, the shifted 2D multigrid solves of every mode to a
relative residual of 1e-10, inverse transform.  The rhs is resident in device
memory before a timed region starts; plan creation is outside it.

The default run prints ONE JSON line.  Its `value` is grid points/s of the
plain FP64 solver on the 512 x 512 x 1024 box (x Dirichlet, y Neumann, z
Neumann: DCT-II), the largest single solve; beside it sit the same box in
the mixed form (FP32 V-cycles inside FP64 refinement), the roofline of the
dominant kernel (HIP events on the solve stream), the CPU oracle timed on the
same field, and sub-records for the L-shaped cross-section, the 64-problem
batch and the request stream (solves/s, p50/p99 latency, speed-up over the
plain FP64 solver, an aggregate roofline and a CPU oracle baseline each).
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
BATCH_SEED0 = 4000  # rhs seed of batch problem i


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def _workload(name: str):
    if name == "lshape":
        return W.config2(), W.CONFIG_SEEDS[2], W.CONFIG_DIST[2]
    if name == "box":
        return W.config3(), W.CONFIG_SEEDS[3], W.CONFIG_DIST[3]
    if name == "cube32":
        return W.config1(), W.CONFIG_SEEDS[1], W.CONFIG_DIST[1]
    if name == "obstacle8":  # the headline's obstacle sub-record: 64 cells per obstacle side, nz = 576
        return W.obstacle8(64, 576), 6, "normal"
    raise SystemExit(f"unknown workload {name}")


# ---------------------------------------------------------------------------
# Byte models (method bytes per point; w = word size)
# ---------------------------------------------------------------------------

def _bytes_per_cell(precision: str) -> float:
    """Method bytes of one finest-level fused launch per plane cell and mode.

    Each launch does one red-black smoothing sweep (read p and f, write p:
    3 words) plus either the residual with its restriction (read p and f,
    write a quarter-size coarse rhs: 2.25 words) or the prolongation with its
    correction (2.25 words), so 5.25 words per cell.
    """
    w = 8.0 if precision == "fp64" else 4.0
    return 5.25 * w


def _vcycle_bytes_per_point(w: float, nu1: int = 1, nu2: int = 1) -> float:
    """Method bytes of one V-cycle per fine point: (sweeps*3 + 4.5) words x 4/3."""
    return ((nu1 + nu2) * 3.0 + 4.5) * w * 4.0 / 3.0


MIXED_INNER = 4  # FP32 V-cycles per refinement step (the library's default)
SERVE_INNER = 2  # the same inside a server (its default)


def _mode_cycle_bytes(precision: str, inner: int = MIXED_INNER) -> float:
    """Method bytes per plane point and convergence step of one mode.
    FP64: one V-cycle.  Mixed: FP64 residual to FP32 (read p, f; write r:
    20 B), `inner` FP32 V-cycles, FP64 accumulation (read e, p; write p: 20 B)."""
    if precision == "fp64":
        return _vcycle_bytes_per_point(8.0)
    return 20.0 + inner * _vcycle_bytes_per_point(4.0) + 20.0


TRANSFORM_BYTES = 32.0  # forward + inverse z transform, FP64 read + write


def _solve_bytes(prob, cycles_per_mode, precision, inner: int = MIXED_INNER) -> float:
    plane = prob.ncells // prob.nz
    return prob.ncells * TRANSFORM_BYTES + float(np.sum(cycles_per_mode)) * plane * _mode_cycle_bytes(precision, inner)


# ---------------------------------------------------------------------------
# HBM counter records (committed rocprofv3 summaries)
# ---------------------------------------------------------------------------

_PROFILE_NAMES = {"lshape3x256^2x512_stretch1.5": "lshape_256x3x512", "box512x512x1024_DD_NN_NN": "box_512x512x1024"}


def _kernel_source_hash() -> str:
    import hashlib
    path = os.path.join(HERE, "paper_2106_03583_amd", "csrc", "march.hip")
    return hashlib.sha256(open(path, "rb").read()).hexdigest()


def _traffic_record(workload: str, precision: str):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary profiles/traffic_fused_sweep_<workload>_<precision>.md (its JSON
    block); None when absent or taken on another build of the kernel source."""
    if workload not in _PROFILE_NAMES:
        return None
    path = os.path.join(HERE, "profiles", f"traffic_fused_sweep_{_PROFILE_NAMES[workload]}_{precision}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    if "```json" not in text:
        return None
    rec = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    if rec.get("kernel_source_sha256") != _kernel_source_hash():
        return None
    return rec


# ---------------------------------------------------------------------------
# CPU oracle baselines
# ---------------------------------------------------------------------------

def _cpu_info():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    threads = 1
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        pass
    return model, int(threads), os.cpu_count()


def cpu_baseline_separable(probs_fs, unit: str, budget_s: float = 25.0) -> dict:
    """The oracle's separable direct solve (eigen-decomposition of the three
    1D operators, BLAS-threaded) on problems in order until ``budget_s`` of
    CPU wall time is spent; rate = cells (or solves) / time of those solved."""
    import oracle
    model, threads, ncpu = _cpu_info()
    t_all = 0.0
    cells = 0
    done = 0
    for prob, f in probs_fs:
        t0 = time.perf_counter()
        oracle.solve_separable(prob, f)
        t_all += time.perf_counter() - t0
        cells += prob.ncells
        done += 1
        if t_all > budget_s:
            break
    total = len(probs_fs)
    value = cells / t_all if unit == "grid points/s" else done / t_all
    what = "full run" if done == total else f"{done} of {total} problems (in order)"
    return {"value": value, "unit": unit, "cores": threads, "kind": "oracle",
            "sample": (f"FP64 oracle, separable direct route (1D eigen-decompositions along x, y, z; "
                       f"dense BLAS transforms), {what}: {cells} cells in {t_all:.1f} s wall; "
                       f"BLAS threads {threads} of os.cpu_count() = {ncpu}; CPU {model or 'unknown'}")}


def cpu_baseline_alg1(prob, f) -> dict:
    """The oracle's Algorithm 1 route (forward transform, one sparse LU per
    distinct modal shift, inverse transform) on the whole problem, the
    per-shift solves spread over a process pool of os.cpu_count() workers
    (at most 16)."""
    import oracle
    model, threads, ncpu = _cpu_info()
    workers = max(1, min(16, ncpu or 1))
    t0 = time.perf_counter()
    oracle.solve_alg1(prob, f, workers=workers)
    t = time.perf_counter() - t0
    return {"value": prob.ncells / t, "unit": "grid points/s", "cores": workers, "kind": "oracle",
            "sample": (f"FP64 oracle, Algorithm 1 route (sparse LU per modal shift), full run: "
                       f"{prob.ncells} cells in {t:.1f} s wall; {workers} worker processes of "
                       f"os.cpu_count() = {ncpu}; CPU {model or 'unknown'}")}


# ---------------------------------------------------------------------------
# Single problems
# ---------------------------------------------------------------------------

def _timed_solves(torch, mbp, plan, fd, p, flags, steps, warmup, profile=False):
    for _ in range(warmup):
        plan.solve(fd, p, rtol=RTOL, flags=flags)
    torch.cuda.synchronize()
    if profile:
        plan.profile(True)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    infos = []
    torch.cuda.synchronize()
    ev[0].record(stream)
    for k in range(steps):
        infos.append(plan.solve(fd, p, rtol=RTOL, flags=flags, stream=stream))
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    per = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
    total = ev[0].elapsed_time(ev[steps])
    prof = None
    if profile:
        prof = plan.profile_read()
        plan.profile(False)
    return total, per, infos, prof


def _roofline(prob, precision, prof, lockstep):
    cls = int(np.argmax(prof["total_ms"]))
    launches = prof["launches"][cls]
    if launches <= 0:
        return None
    avg_ms = prof["total_ms"][cls] / launches
    cells = prof["cells"][cls] / launches
    bpc = _bytes_per_cell(precision)
    achieved = bpc * cells / (avg_ms * 1e-3) / 1e9
    traffic = None
    tr = _traffic_record(prob.name, precision)
    if tr and tr.get("kernel_class") == cls and tr.get("workload") == prob.name \
            and tr.get("precision") == precision and not lockstep:
        traffic = tr.get("bytes_per_launch")
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": ["k_tile (pre-smoothing sweep + residual + restriction, finest level)",
                       "k_tile_corr (correction + post-smoothing sweep + residual norm, finest level)"][cls],
            "avg_launch_ms": round(avg_ms, 4), "launches": launches, "bytes_per_launch": bpc * cells,
            "bytes_model": "42 B per plane cell and mode (FP64): sweep 3 words + transfer 2.25 words"}
    if traffic:
        roof["traffic_GBs"] = round(traffic / (avg_ms * 1e-3) / 1e9, 1)
        roof["traffic_frac"] = round(roof["traffic_GBs"] / HBM_PEAK_GBS, 4)
    return roof


def run_single(torch, mbp, prob, fd, precision, lockstep, steps, warmup, profile=True):
    flags = mbp.PROJECT_RHS | (0 if lockstep else mbp.RETIRE)
    t0 = time.perf_counter()
    plan = mbp.Plan(prob, precision=precision)
    t_plan = (time.perf_counter() - t0) * 1e3
    p = torch.zeros_like(fd)
    total, per, infos, prof = _timed_solves(torch, mbp, plan, fd, p, flags, steps, warmup, profile)
    last = infos[-1]
    ok = all(i.status == 0 and i.rel_residual <= RTOL for i in infos)
    # independent physical-space residual of the last solve through the 3D operator
    Ap = torch.empty_like(fd)
    plan.apply(p, Ap)
    fpr = fd - last.removed_mean
    res3d = float(torch.linalg.vector_norm(fpr - Ap) / torch.linalg.vector_norm(fpr))
    del Ap, fpr
    ms = total / steps
    out = {"ms_per_solve": round(ms, 4), "ms_median": round(float(np.median(per)), 4),
           "ms_min": round(float(np.min(per)), 4), "grid_points_per_s": prob.ncells / (ms * 1e-3),
           "solves_per_s": 1e3 / ms, "ok": ok, "status": last.status, "rel_residual_modal": last.rel_residual,
           "rel_residual_3d": res3d, "cycles_max": last.cycles,
           "t_ms_last": [round(t, 3) for t in last.t_ms], "plan_ms": round(t_plan, 1)}
    if prof is not None:
        out["roofline"] = _roofline(prob, precision, prof, lockstep)
    # all multigrid work of the timed solves against the byte model
    plane = prob.ncells // prob.nz
    mg_ms = sum(i.t_ms[1] for i in infos) / len(infos)
    cyc = sum(int(i.cycles_per_mode.sum()) if not lockstep else i.cycles * prob.nz for i in infos) / len(infos)
    vb = _mode_cycle_bytes(precision)
    out["vcycle_roofline"] = {"bytes_per_point_and_cycle": vb, "mode_cycles": cyc, "mg_ms": round(mg_ms, 3),
                              "achieved_GBs": round(vb * plane * cyc / (mg_ms * 1e-3) / 1e9, 1)}
    out["vcycle_roofline"]["frac"] = round(out["vcycle_roofline"]["achieved_GBs"] / HBM_PEAK_GBS, 4)
    out["_p"] = p
    plan.close()
    return out


def bench_single(args, torch, mbp, prob, f, with_variants=True):
    fd = torch.from_numpy(f).cuda()
    log(f"workload {prob.name} cells={prob.ncells} precision={args.precision} lockstep={args.lockstep}")
    main = run_single(torch, mbp, prob, fd, args.precision, args.lockstep, args.steps, args.warmup)
    p_main = main.pop("_p")
    log(f"timed {args.steps} solves: {main['ms_per_solve']:.2f} ms/solve (median {main['ms_median']:.2f})")
    variants = {}
    if with_variants:
        for name, prec, lock in [("fp64_lockstep", "fp64", True), ("fp64_retire", "fp64", False),
                                 ("mixed_retire", "mixed", False)]:
            if prec == args.precision and lock == args.lockstep:
                continue
            v = run_single(torch, mbp, prob, fd, prec, lock, max(3, args.steps // 2), 1, profile=False)
            q = v.pop("_p")
            v["max_abs_diff_vs_main"] = float((q - p_main).abs().max())
            del q
            variants[name] = v
            log(f"{name}: {v['ms_per_solve']:.2f} ms/solve")
    del p_main, fd
    torch.cuda.empty_cache()
    return main, variants


# ---------------------------------------------------------------------------
# 3D multigrid without the z synthesis (the paper's comparison solver)
# ---------------------------------------------------------------------------

def bench_mg3d(args, torch, mbp, prob, f, t_fft_ms, reps=3):
    """Weighted-Jacobi V(2,2) cycles on the whole 3D system to the same 1e-10
    relative residual (the paper compares the solvers at one tolerance); the
    3D solver runs without the error-estimate test, whose global bound
    (residual over the smallest eigenvalue) would drive it far below 1e-10.
    This time over the FFT-accelerated solve's is the paper's speed-up
    figure (Sec. 4.2)."""
    fd = torch.from_numpy(f).cuda()
    plan = mbp.Plan3D(prob, etol=-1.0)
    p = torch.zeros_like(fd)
    flags = mbp.PROJECT_RHS
    plan.solve(fd, p, rtol=RTOL, flags=flags)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    infos = []
    for k in range(reps):
        infos.append(plan.solve(fd, p, rtol=RTOL, flags=flags, stream=stream))
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    per = [ev[k].elapsed_time(ev[k + 1]) for k in range(reps)]
    ms = float(np.mean(per))
    last = infos[-1]
    ok = all(i.status == 0 and i.rel_residual <= RTOL for i in infos)
    # dominant kernel: the finest-level Jacobi sweep, timed alone (read p, f; write p)
    q = torch.empty_like(p)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    plan.jacobi_sweep(p, q, fd)
    a.record(stream)
    nl = 10
    for k in range(nl):
        plan.jacobi_sweep(p if k % 2 == 0 else q, q if k % 2 == 0 else p, fd, stream=stream)
    b.record(stream)
    torch.cuda.synchronize()
    sweep_ms = a.elapsed_time(b) / nl
    sweep_bytes = 24.0 * prob.ncells
    # whole-solve byte model: per cycle and level, (nu1 + nu2) sweeps of 3 words,
    # residual + restriction (2 words + 1 coarse word), prolongation + correction
    # (2 words + 1 coarse word); plus the rhs norm and the final residual (2 + 2 words)
    cl = plan.cells_per_level
    cyc_bytes = sum(8.0 * (4 * 3 * cl[i] + 4 * cl[i] + 2 * cl[i + 1]) for i in range(len(cl) - 1))
    solve_bytes = last.cycles * cyc_bytes + 8.0 * 4 * prob.ncells
    rec = {"ms_per_solve": round(ms, 3), "ms_min": round(float(np.min(per)), 3), "cycles": last.cycles,
           "rel_residual": last.rel_residual, "grid_points_per_s": prob.ncells / (ms * 1e-3), "ok": ok,
           "levels": plan.nlevels, "nz_per_level": plan.nz_per_level,
           "fft_accelerated_speedup": ms / t_fft_ms,
           "roofline": {"bound": "hbm", "kernel": "k3_jacobi (finest weighted-Jacobi sweep)",
                        "achieved": round(sweep_bytes / (sweep_ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(sweep_bytes / (sweep_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                        "traffic": None, "avg_launch_ms": round(sweep_ms, 4),
                        "bytes_model": "24 B per cell (read p, f; write p)"},
           "solve_roofline": {"bytes_per_solve": solve_bytes,
                              "achieved_GBs": round(solve_bytes / (ms * 1e-3) / 1e9, 1),
                              "frac": round(solve_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}
    plan.close()
    del fd, p, q
    torch.cuda.empty_cache()
    log(f"mg3d {prob.name}: {ms:.1f} ms/solve, {last.cycles} cycles; FFT-accelerated is "
        f"{rec['fft_accelerated_speedup']:.2f}x faster")
    return rec


# ---------------------------------------------------------------------------
# Batched form
# ---------------------------------------------------------------------------

def _upload_host_rhs(torch, items, threads=16):
    """Seeded PCG64 uniform rhs of each (problem, seed), drawn on the host in
    parallel threads (the draws release the GIL) and copied to the device."""
    import concurrent.futures as cf

    def one(ps):
        prob, seed = ps
        return torch.from_numpy(W.rhs(prob, seed, "uniform")).to("cuda")

    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        out = list(ex.map(one, items))
    torch.cuda.synchronize()
    return out


def _solve_each(torch, mbp, probs, rhs, precision, flags, keep_plans=None, compare=None):
    """One solve at a time (plans built outside the timed intervals); returns
    the summed solve time (HIP events around each solve) and the max relative
    difference to `compare` outputs."""
    stream = torch.cuda.current_stream()
    total = 0.0
    diff = 0.0
    for i, (prob, r) in enumerate(zip(probs, rhs)):
        pl = keep_plans[i] if keep_plans is not None else mbp.Plan(prob, precision=precision)
        o = torch.zeros_like(r)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        pl.solve(r, o, rtol=RTOL, flags=flags, stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
        total += a.elapsed_time(b)
        if compare is not None:
            c = compare[i]
            diff = max(diff, float(torch.linalg.vector_norm(o - c) / torch.linalg.vector_norm(c)))
        if keep_plans is None:
            pl.close()
        del o
    return total, diff


def bench_batch(args, torch, mbp, with_cpu=True):
    """64 independent solves of uneven size: the batched mixed form against
    the plain FP64 solver (one solve at a time, lockstep modes) and against
    one-at-a-time FP64 with per-mode retirement."""
    probs = W.config4()
    ncells = sum(p.ncells for p in probs)
    rhs = _upload_host_rhs(torch, [(p, BATCH_SEED0 + i) for i, p in enumerate(probs)])
    t0 = time.perf_counter()
    fast = [mbp.Plan(p, precision="mixed") for p in probs]
    t_plan = time.perf_counter() - t0
    out_f = [torch.zeros_like(r) for r in rhs]
    log(f"batch64: {len(probs)} problems, {ncells} cells, plans {t_plan:.1f} s")
    mbp.solve_batch(fast, rhs, out_f, rtol=RTOL, flags=mbp.PROJECT_RHS | mbp.AUTOTUNE)  # tunes the schedule
    for _ in range(max(0, args.warmup - 1)):
        mbp.solve_batch(fast, rhs, out_f, rtol=RTOL, flags=mbp.PROJECT_RHS)
    torch.cuda.synchronize()
    per = []
    for _ in range(args.steps):
        w0 = time.perf_counter()
        infos = mbp.solve_batch(fast, rhs, out_f, rtol=RTOL, flags=mbp.PROJECT_RHS)
        torch.cuda.synchronize()
        per.append(time.perf_counter() - w0)
    t_fast = float(np.sum(per)) / len(per)
    sched = mbp.batch_schedule(fast)
    ok = all(i.status == 0 and i.rel_residual <= RTOL for i in infos)
    bytes_step = sum(_solve_bytes(p, i.cycles_per_mode, "mixed") for p, i in zip(probs, infos))
    for pl in fast:
        pl.close()
    log(f"batch64 mixed: {t_fast * 1e3:.1f} ms per batch")
    # plain FP64 (lockstep) and FP64 with retirement, one solve at a time
    t_lock, d_lock = _solve_each(torch, mbp, probs, rhs, "fp64", mbp.PROJECT_RHS, compare=out_f)
    t_ret, d_ret = _solve_each(torch, mbp, probs, rhs, "fp64", mbp.PROJECT_RHS | mbp.RETIRE, compare=out_f)
    log(f"batch64 plain FP64: lockstep {t_lock:.1f} ms, retire {t_ret:.1f} ms")
    # FP64 batched, for the breakdown
    plain = [mbp.Plan(p, precision="fp64") for p in probs]
    out_p = [torch.zeros_like(r) for r in rhs]
    mbp.solve_batch(plain, rhs, out_p, rtol=RTOL, flags=mbp.PROJECT_RHS)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    mbp.solve_batch(plain, rhs, out_p, rtol=RTOL, flags=mbp.PROJECT_RHS)
    torch.cuda.synchronize()
    t_fp64_batch = time.perf_counter() - w0
    for pl in plain:
        pl.close()
    del out_p, out_f, rhs
    torch.cuda.empty_cache()
    n = len(probs)
    rec = {
        "metric": "solves/s at 1e-10 relative residual",
        "value": n / t_fast, "unit": "solves/s", "steps": args.steps,
        "ms_per_step": round(t_fast * 1e3, 3), "ms_median": round(float(np.median(per)) * 1e3, 3),
        "ms_min": round(float(np.min(per)) * 1e3, 3),
        "dtype": "f32-in-f64", "data": "synthetic (seeded PCG64 rhs drawn on the host)",
        "config": {"workload": "batch of 64 uneven boxes 64..384 x 64..384 x 64..256, all BC pairs",
                   "cells": ncells, "form": "mixed, batched graph replay, per-mode retirement",
                   "schedule_streams_cycles": sched},
        "grid_points_per_s": ncells / t_fast,
        "plain_fp64_lockstep_solves_per_s": n / (t_lock * 1e-3),
        "fp64_retire_solves_per_s": n / (t_ret * 1e-3),
        "fp64_batched_solves_per_s": n / t_fp64_batch,
        "speedup_vs_plain_fp64_lockstep": (t_lock * 1e-3) / t_fast,
        "speedup_vs_fp64_retire": (t_ret * 1e-3) / t_fast,
        "max_rel_diff_vs_fp64": max(d_lock, d_ret),
        "ok": ok, "plan_s": round(t_plan, 2),
        "roofline": {"bound": "hbm", "kernel": "whole batched step (every kernel of the 64 solves)",
                     "achieved": round(bytes_step / t_fast / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(bytes_step / t_fast / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
                     "bytes_per_step": bytes_step,
                     "bytes_model": f"32 B/cell transforms + per mode and refinement step 20 + {MIXED_INNER} x 56 + "
                                    f"20 B per plane point (FP64 residual, {MIXED_INNER} FP32 V-cycles, FP64 "
                                    "accumulation)"},
    }
    if with_cpu:
        log("batch64: cpu baseline (oracle, separable route)")
        fs = [(p, W.rhs(p, BATCH_SEED0 + i, "uniform")) for i, p in enumerate(probs)]
        rec["cpu_baseline"] = cpu_baseline_separable(fs, "solves/s", budget_s=20.0)
    return rec


# ---------------------------------------------------------------------------
# Serving loop
# ---------------------------------------------------------------------------

def bench_serve(args, torch, mbp, with_cpu=True):
    """Poisson stream of requests through the server: capacity (closed loop),
    then the stream replayed at 70 % of capacity for p50/p99 latency (the
    first 10 % of requests excluded), then the same trace through the plain
    FP64 solver one request at a time (lockstep, and with retirement)."""
    n = args.requests
    reqs = W.config5(count=n, rate_per_s=1.0)
    probs = [r.problem for r in reqs]
    cells = [p.ncells for p in probs]
    log(f"serve: drawing {n} rhs on the host ({sum(cells)} cells)")
    rhs = _upload_host_rhs(torch, [(r.problem, r.seed) for r in reqs])
    outs = [torch.zeros_like(x) for x in rhs]
    torch.cuda.synchronize()
    budget = int(args.server_gb * (1 << 30))
    srv = mbp.Server(hbm_budget=budget, slots=args.slots, precision="mixed")

    def closed_loop():
        w0 = time.perf_counter()
        ts = [srv.submit(p, x, o, rtol=RTOL, flags=mbp.PROJECT_RHS) for p, x, o in zip(probs, rhs, outs)]
        res = [srv.wait(t) for t in ts]
        return time.perf_counter() - w0, res

    closed_loop()  # warm: builds and caches plans where the budget allows
    t_cap, res_cap = closed_loop()
    capacity = n / t_cap
    rate = 0.7 * capacity
    log(f"serve: capacity {capacity:.1f} solves/s, replay at {rate:.1f}/s")
    w0 = time.perf_counter()
    tickets = []
    for r, p, x, o in zip(reqs, probs, rhs, outs):
        due = w0 + r.arrival_s / rate
        while True:
            now = time.perf_counter()
            if now >= due:
                break
            time.sleep(min(0.0005, due - now))
        tickets.append(srv.submit(p, x, o, rtol=RTOL, flags=mbp.PROJECT_RHS))
    res = [srv.wait(t) for t in tickets]
    t_open = time.perf_counter() - w0
    srv.close()
    lat = np.array([ms for _, _, ms in res])
    steady = lat[n // 10:]
    ok = all(st == 0 and inf.rel_residual <= RTOL for st, inf, _ in res)
    torch.cuda.empty_cache()
    t_lock, d_lock = _solve_each(torch, mbp, probs, rhs, "fp64", mbp.PROJECT_RHS, compare=outs)
    t_ret, d_ret = _solve_each(torch, mbp, probs, rhs, "fp64", mbp.PROJECT_RHS | mbp.RETIRE, compare=outs)
    log(f"serve plain FP64: lockstep {t_lock:.0f} ms, retire {t_ret:.0f} ms for {n} requests")
    # method bytes of the capacity run: each request's transforms and mode cycles
    nbytes = 0.0
    for p, (_, inf, _) in zip(probs, res_cap):
        nbytes += _solve_bytes(p, inf.cycles_per_mode, "mixed", SERVE_INNER)
    del rhs, outs
    torch.cuda.empty_cache()
    rec = {
        "metric": "solves/s at 1e-10 relative residual; p50/p99 latency",
        "value": capacity, "unit": "solves/s", "steps": n, "warmup": n,
        "ms_per_step": round(1e3 / capacity, 3),
        "dtype": "f32-in-f64", "data": "synthetic (seeded PCG64 rhs drawn on the host)",
        "config": {"workload": f"Poisson request stream, {n} requests, sizes log-uniform 32..512 per axis, "
                               f"random BC pairs, tanh stretching 1..2",
                   "cells": int(sum(cells)), "slots": args.slots, "hbm_budget_gb": args.server_gb},
        "capacity_solves_per_s": capacity,
        "replay_rate_per_s": rate,
        "replay_solves_per_s": n / t_open,
        "latency_ms_p50": float(np.percentile(steady, 50)),
        "latency_ms_p99": float(np.percentile(steady, 99)),
        "latency_excluded_warmup": n // 10,
        "plain_fp64_lockstep_solves_per_s": n / (t_lock * 1e-3),
        "fp64_retire_solves_per_s": n / (t_ret * 1e-3),
        "speedup_vs_plain_fp64_lockstep": capacity / (n / (t_lock * 1e-3)),
        "speedup_vs_fp64_retire": capacity / (n / (t_ret * 1e-3)),
        "max_rel_diff_vs_fp64": max(d_lock, d_ret),
        "ok": ok,
        "roofline": {"bound": "hbm", "kernel": "whole served stream at capacity (every kernel)",
                     "achieved": round(nbytes / t_cap / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(nbytes / t_cap / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
                     "bytes_model": "per request: 32 B/cell transforms + per mode and refinement step "
                                    f"20 + {SERVE_INNER} x 56 + 20 B per plane point (FP64 residual, "
                                    f"{SERVE_INNER} FP32 V-cycles, FP64 accumulation)"},
    }
    if with_cpu:
        log("serve: cpu baseline (oracle, separable route)")
        fs = [(r.problem, W.rhs(r.problem, r.seed, "uniform")) for r in reqs[:200]]
        rec["cpu_baseline"] = cpu_baseline_separable(fs, "solves/s", budget_s=20.0)
    return rec


# ---------------------------------------------------------------------------
# Transform comparison and counter calibration (used for profiles/)
# ---------------------------------------------------------------------------

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


def copy_calibrate(torch):
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
    return {"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "ms": ms, "GBs": 16 * n / (ms * 1e-3) / 1e9}


# ---------------------------------------------------------------------------

def _strip(d):
    return {k: v for k, v in d.items() if not k.startswith("_")}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "lshape", "box", "cube32", "obstacle8", "batch64", "serve"])
    ap.add_argument("--requests", type=int, default=1000, help="serve: requests in the stream")
    ap.add_argument("--slots", type=int, default=8, help="serve: concurrent requests")
    ap.add_argument("--server-gb", type=float, default=96.0, help="serve: plan memory budget (GiB)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--lockstep", action="store_true", help="iterate all modes until the global test passes")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baselines")
    ap.add_argument("--no-variants", action="store_true", help="single workloads: skip the other forms")
    ap.add_argument("--no-sub", action="store_true", help="headline: skip the sub-records")
    ap.add_argument("--mg3d-only", action="store_true",
                    help="single workloads: time only the 3D multigrid comparison solver (for profiles)")
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
        print(json.dumps(copy_calibrate(torch)), flush=True)
        return 0
    if args.transform_compare:
        for row in transform_compare(torch, mbp):
            print(json.dumps(row), flush=True)
        return 0
    if args.workload in ("batch64", "serve"):
        out = (bench_batch if args.workload == "batch64" else bench_serve)(args, torch, mbp, not args.no_cpu)
        out.update({"n_gpus": 1, "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
                    "vs_baseline": None})
        print(json.dumps(out), flush=True)
        return 0 if out["ok"] else 1

    name = "box" if args.workload == "headline" else args.workload
    prob, seed, dist = _workload(name)
    f = W.rhs(prob, seed, dist)
    if args.mg3d_only:
        rec = bench_mg3d(args, torch, mbp, prob, f, 1.0, reps=args.steps)
        print(json.dumps({"workload": prob.name, "mg3d": rec}), flush=True)
        return 0 if rec["ok"] else 1
    main_rec, variants = bench_single(args, torch, mbp, prob, f, with_variants=not args.no_variants)
    mg3d = None
    if not args.no_variants and args.workload in ("headline", "box", "lshape"):
        mg3d = bench_mg3d(args, torch, mbp, prob, f, main_rec["ms_per_solve"])
    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle, full run on the same field)")
        if len(prob.blocks) == 1:
            cpu = cpu_baseline_separable([(prob, f)], "grid points/s", budget_s=1e9)
    del f
    sub = {}
    if args.workload == "headline" and not args.no_sub:
        # the L-shaped cross-section (three joined, stretched blocks), timed the same way
        lp, lseed, ldist = _workload("lshape")
        lf = W.rhs(lp, lseed, ldist)
        largs = argparse.Namespace(**{**vars(args), "precision": "fp64", "lockstep": False})
        lmain, lvar = bench_single(largs, torch, mbp, lp, lf, with_variants=True)
        lmg = bench_mg3d(largs, torch, mbp, lp, lf, lmain["ms_per_solve"])
        lcpu = None
        if not args.no_cpu:
            log("lshape: cpu baseline (oracle, Algorithm 1 route in a process pool)")
            lcpu = cpu_baseline_alg1(lp, lf)
        del lf
        sub["lshape"] = {"config": {"workload": lp.name, "cells": lp.ncells, "nz": lp.nz, "blocks": 3},
                         "fp64": _strip(lmain), **{k: _strip(v) for k, v in lvar.items()}, "mg3d": lmg,
                         "cpu_baseline": lcpu}
        # eight blocks around a square obstacle (the paper's third geometry)
        op = W.obstacle8(64, 576)
        of = W.rhs(op, 6, "normal")
        oargs = argparse.Namespace(**{**vars(args), "precision": "fp64", "lockstep": False})
        omain, ovar = bench_single(oargs, torch, mbp, op, of, with_variants=True)
        omg = bench_mg3d(oargs, torch, mbp, op, of, omain["ms_per_solve"])
        ocpu = None
        if not args.no_cpu:
            log("obstacle8: cpu baseline (oracle, Algorithm 1 route in a process pool)")
            ocpu = cpu_baseline_alg1(op, of)
        del of
        sub["obstacle8"] = {"config": {"workload": op.name, "cells": op.ncells, "nz": op.nz, "blocks": 8},
                            "fp64": _strip(omain), **{k: _strip(v) for k, v in ovar.items()}, "mg3d": omg,
                            "cpu_baseline": ocpu}
        sub["batch64"] = bench_batch(args, torch, mbp, not args.no_cpu)
        sub["serve"] = bench_serve(args, torch, mbp, not args.no_cpu)

    ms = main_rec["ms_per_solve"]
    out = {
        "metric": "grid points/s at 1e-10 relative residual (FP64; mixed beside)",
        "value": main_rec["grid_points_per_s"],
        "unit": "grid points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-in-f64",
        "data": "synthetic (seeded PCG64 rhs drawn on the host)",
        "config": {"workload": prob.name, "cells": prob.ncells, "nz": prob.nz, "blocks": len(prob.blocks),
                   "precision": args.precision, "mode_stop": "lockstep" if args.lockstep else "per-mode",
                   "rtol": RTOL},
        **{k: v for k, v in _strip(main_rec).items() if k not in ("grid_points_per_s",)},
        "variants": {k: _strip(v) for k, v in variants.items()},
        "cpu_baseline": cpu,
    }
    if "mixed_retire" in variants and args.precision == "fp64" and not args.lockstep:
        out["mixed"] = {"grid_points_per_s": variants["mixed_retire"]["grid_points_per_s"],
                        "ms_per_solve": variants["mixed_retire"]["ms_per_solve"],
                        "speedup_vs_fp64": ms / variants["mixed_retire"]["ms_per_solve"]}
    if mg3d:
        out["mg3d"] = mg3d
    if sub:
        out["sub"] = sub
    ok = main_rec["ok"] and all(v.get("ok", True) for v in variants.values()) and \
        all(v.get("ok", True) for k, v in sub.items() if k != "lshape")
    out["ok"] = ok
    print(json.dumps(out), flush=True)
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
