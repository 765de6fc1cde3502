"""Full-size parity: every cell of every full-size workload against the oracle.

Workloads (the shapes bench.py times): the three-block L-shape 3 x 256^2 x 512
(periodic z, Neumann walls, tanh-stretched y), the 512 x 512 x 1024 box
(DD / NN / NN with the DCT-II along z), the eight blocks around a square
obstacle (64 cells per side, 576 periodic z cells), the 64-problem batch (boxes
64..384 x 64..384 x 64..256, every condition pair) and a sample of the request
stream (sizes log-uniform 32..512 per axis, stretched walls).  Every rhs is
drawn on the host with NumPy's PCG64 from its seed, so the oracle sees the
same bits.

For each result, in FP64 and in the mixed form (and, for single problems, the
3D multigrid comparison solver):
  * the relative 3D residual ||f - L_h p|| / ||f|| with the ORACLE's operator
    (host, every cell) must be <= 1e-10;
  * the relative error against the oracle's direct solution (Algorithm 1 with
    a sparse LU per shift for the L-shape, the separable eigen-decomposition
    for boxes) must be <= 1e-9 in the l2 norm; the max-norm error relative to
    max |p| is printed beside it (reading R14).
"""
import os

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

RTOL = 1e-10


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def mbp():
    import paper_2106_03583_amd as m
    return m


def _workers():
    # the GPU host's CPU share is 16 cores, whatever os.cpu_count() reports
    return max(1, min(16, os.cpu_count() or 1))


def _compare(prob, f, got, ref, label):
    fp = oracle.project_compatible(prob, f) if oracle.is_singular(prob) else f
    res = oracle.rel_residual(prob, got, fp)
    err = oracle.rel_error(got, ref)
    errmax = float(np.abs(got - ref).max() / np.abs(ref).max())
    print(f"  {label} {prob.name}: residual3d={res:.2e} error_l2={err:.2e} error_max={errmax:.2e}", flush=True)
    assert res <= RTOL, (label, prob.name, res)
    assert err <= 1e-9, (label, prob.name, err)
    return res, err, errmax


def _solve_one(torch, mbp, prob, fd, precision):
    plan = mbp.Plan(prob, precision=precision)
    p = torch.zeros_like(fd)
    info = plan.solve(fd, p, rtol=RTOL, flags=mbp.PROJECT_RHS | mbp.RETIRE)
    plan.close()
    assert info.status == 0 and info.rel_residual <= RTOL
    out = p.cpu().numpy()
    del p
    return out, info


def _solve_mg3d(torch, mbp, prob, fd):
    plan = mbp.Plan3D(prob)
    p = torch.zeros_like(fd)
    info = plan.solve(fd, p, rtol=RTOL, flags=mbp.PROJECT_RHS)
    plan.close()
    assert info.status == 0 and info.rel_residual <= RTOL
    out = p.cpu().numpy()
    del p
    return out, info


def _single(torch, mbp, prob, seed, dist, ref_fn):
    f = W.rhs(prob, seed, dist)
    fd = torch.from_numpy(f).cuda()
    sols = {}
    for precision in ("fp64", "mixed"):
        print(f"full-size {prob.name} {precision}: solving on the GPU", flush=True)
        sols[precision], info = _solve_one(torch, mbp, prob, fd, precision)
        print(f"  {info}", flush=True)
    # the comparison solver (3D multigrid without z synthesis) reaches the same solution
    print(f"full-size {prob.name} 3D multigrid: solving on the GPU", flush=True)
    sols["mg3d"], info = _solve_mg3d(torch, mbp, prob, fd)
    print(f"  {info}", flush=True)
    del fd
    torch.cuda.empty_cache()
    print(f"full-size {prob.name}: oracle", flush=True)
    ref = ref_fn(prob, f)
    for precision, got in sols.items():
        _compare(prob, f, got, ref, precision)


def test_full_field_lshape(torch_cuda, mbp):
    """3 x 256^2 x 512 L-shape: Algorithm 1 in the oracle, per-shift LUs in a process pool."""
    _single(torch_cuda, mbp, W.config2(), W.CONFIG_SEEDS[2], W.CONFIG_DIST[2],
            lambda prob, f: oracle.solve_alg1(prob, f, workers=_workers()))


def test_full_field_box(torch_cuda, mbp):
    """512 x 512 x 1024 box: separable eigen-decomposition in the oracle."""
    _single(torch_cuda, mbp, W.config3(), W.CONFIG_SEEDS[3], W.CONFIG_DIST[3], oracle.solve_separable)


def test_full_field_obstacle8(torch_cuda, mbp):
    """Eight blocks around a square obstacle, 64 cells per side, 576 periodic z
    cells: Algorithm 1 in the oracle with per-shift LUs in a process pool."""
    _single(torch_cuda, mbp, W.obstacle8(64, 576), 6, "normal",
            lambda prob, f: oracle.solve_alg1(prob, f, workers=_workers()))


BATCH_SEED0 = 4000  # rhs seed of batch problem i is BATCH_SEED0 + i


def test_full_field_batch64(torch_cuda, mbp):
    """All 64 batch problems, batched mixed form and batched FP64 form."""
    torch = torch_cuda
    probs = W.config4()
    print(f"full-size batch of {len(probs)}: {sum(p.ncells for p in probs)} cells", flush=True)
    fs = [W.rhs(p, BATCH_SEED0 + i, "uniform") for i, p in enumerate(probs)]
    sols = {}
    for precision in ("mixed", "fp64"):
        rhs = [torch.from_numpy(f).cuda() for f in fs]
        outs = [torch.zeros_like(r) for r in rhs]
        plans = [mbp.Plan(p, precision=precision) for p in probs]
        infos = mbp.solve_batch(plans, rhs, outs, rtol=RTOL, flags=mbp.PROJECT_RHS)
        assert all(i.status == 0 and i.rel_residual <= RTOL for i in infos)
        sols[precision] = [o.cpu().numpy() for o in outs]
        for pl in plans:
            pl.close()
        del rhs, outs
        torch.cuda.empty_cache()
    worst = {k: [0.0, 0.0, 0.0] for k in sols}
    for i, (prob, f) in enumerate(zip(probs, fs)):
        ref = oracle.solve_separable(prob, f)
        for precision in sols:
            r = _compare(prob, f, sols[precision][i], ref, f"batch {precision}")
            worst[precision] = [max(a, b) for a, b in zip(worst[precision], r)]
    print(f"  batch worst (residual, error_l2, error_max): {worst}", flush=True)


def _serve_sample():
    reqs = W.config5(count=200)
    sample = reqs[:16]
    largest = max(reqs, key=lambda r: r.problem.ncells)
    if largest not in sample:
        sample.append(largest)
    return sample


def test_full_field_serve_sample(torch_cuda, mbp):
    """Requests of the served stream (its first 16 and the largest of its first
    200), served concurrently in the mixed form and solved alone in FP64."""
    torch = torch_cuda
    sample = _serve_sample()
    print(f"served sample: {len(sample)} requests, {sum(r.problem.ncells for r in sample)} cells", flush=True)
    fs = [W.rhs(r.problem, r.seed, "uniform") for r in sample]
    rhs = [torch.from_numpy(f).cuda() for f in fs]
    outs = [torch.zeros_like(x) for x in rhs]
    torch.cuda.synchronize()
    srv = mbp.Server(hbm_budget=64 << 30, slots=8, precision="mixed")
    tickets = [srv.submit(r.problem, x, o, rtol=RTOL, flags=mbp.PROJECT_RHS) for r, x, o in zip(sample, rhs, outs)]
    for t in tickets:
        st, info, _ = srv.wait(t)
        assert st == 0 and info.rel_residual <= RTOL
    srv.close()
    served = [o.cpu().numpy() for o in outs]
    alone = []
    for r, x in zip(sample, rhs):
        got, _ = _solve_one(torch, mbp, r.problem, x, "fp64")
        alone.append(got)
    del rhs, outs
    torch.cuda.empty_cache()
    for r, f, a, b in zip(sample, fs, served, alone):
        ref = oracle.solve_separable(r.problem, f)
        _compare(r.problem, f, a, ref, "served-mixed")
        _compare(r.problem, f, b, ref, "alone-fp64")
