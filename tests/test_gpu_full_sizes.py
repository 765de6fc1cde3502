"""Full-size checks of the batched and served forms, on the workloads bench.py
times: the 64-problem batch (boxes 64..384 x 64..384 x 64..256, every
condition pair) and a sample of the Poisson request stream (sizes
log-uniform 32..512 per axis, stretched walls).

Every problem is checked through the residual of its full 3D operator
(every cell, on the device); a few modes of a few problems are checked
against the oracle's plane-by-plane solves of the same modal rhs (Eq. (9),
sparse LU).  The rhs are seeded uniform [-1, 1) draws made on the device, as
in the throughput runs; only the sampled problems come back to the host.
"""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def mbp():
    import paper_2106_03583_amd as m
    return m


def _device_rhs(torch, n, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(int(seed))
    return torch.rand(n, generator=g, dtype=torch.float64, device="cuda") * 2.0 - 1.0


def _residual3d(torch, mbp, prob, f, p, removed_mean):
    """||f - mean - L_h p|| / ||f - mean|| with an FP64 plan's operator."""
    plan = mbp.Plan(prob, precision="fp64")
    Ap = torch.empty_like(p)
    plan.apply(p, Ap)
    plan.close()
    fp = f - removed_mean
    return float(torch.linalg.vector_norm(fp - Ap) / torch.linalg.vector_norm(fp))


def _mode_errors(torch, mbp, prob, f_dev, p_dev, modes):
    """Relative errors of the sampled modes of p against the oracle's solves."""
    plan = mbp.Plan(prob, precision="fp64")
    ph = torch.empty_like(p_dev)
    plan.forward(p_dev, ph)
    plan.close()
    ph = ph.cpu().numpy().reshape(prob.nz, -1)
    f = f_dev.cpu().numpy()
    fproj = oracle.project_compatible(prob, f) if oracle.is_singular(prob) else f
    fh = oracle.modal_rhs(prob, fproj, modes)
    errs = []
    for i, q in enumerate(modes):
        ref = oracle.solve_mode(prob, fh[i], q)
        errs.append(float(np.linalg.norm(ph[q] - ref) / np.linalg.norm(ref)))
    return errs


def test_full_size_batch64(torch_cuda, mbp):
    torch = torch_cuda
    probs = W.config4()
    print(f"full-size batch of {len(probs)}: {sum(p.ncells for p in probs)} cells", flush=True)
    rhs = [_device_rhs(torch, p.ncells, 4000 + i) for i, p in enumerate(probs)]
    plans = [mbp.Plan(p, precision="mixed") for p in probs]
    outs = [torch.zeros_like(r) for r in rhs]
    infos = mbp.solve_batch(plans, rhs, outs, rtol=1e-10, flags=mbp.PROJECT_RHS | mbp.AUTOTUNE)
    for pl in plans:
        pl.close()
    worst = 0.0
    for prob, r, o, inf in zip(probs, rhs, outs, infos):
        assert inf.status == 0 and inf.rel_residual <= 1e-10, (prob.name, inf)
        worst = max(worst, _residual3d(torch, mbp, prob, r, o, inf.removed_mean))
    print(f"  worst 3D residual over the batch {worst:.2e}", flush=True)
    assert worst <= 1e-10
    # sampled problems: the smallest, the largest and one in between; the
    # first, a middle and the last mode of each
    order = sorted(range(len(probs)), key=lambda i: probs[i].ncells)
    for i in (order[0], order[len(order) // 2], order[-1]):
        prob = probs[i]
        modes = [0, prob.nz // 2, prob.nz - 1]
        errs = _mode_errors(torch, mbp, prob, rhs[i], outs[i], modes)
        print(f"  {prob.name} ({prob.ncells} cells): mode errors {[f'{e:.1e}' for e in errs]}", flush=True)
        assert max(errs) <= 1e-9


def test_full_size_serve_sample(torch_cuda, mbp):
    torch = torch_cuda
    reqs = W.config5(count=12, rate_per_s=1.0)
    print(f"full-size request sample: {[r.problem.ncells for r in reqs]} cells", flush=True)
    rhs = [_device_rhs(torch, r.problem.ncells, r.seed) for r in reqs]
    outs = [torch.zeros_like(x) for x in rhs]
    srv = mbp.Server(hbm_budget=96 << 30, slots=8, precision="mixed")
    tickets = [srv.submit(r.problem, x, o, rtol=1e-10, flags=mbp.PROJECT_RHS) for r, x, o in zip(reqs, rhs, outs)]
    results = [srv.wait(t) for t in tickets]
    srv.close()
    worst = 0.0
    for r, x, o, (st, inf, _lat) in zip(reqs, rhs, outs, results):
        assert st == 0 and inf.status == 0 and inf.rel_residual <= 1e-10, (r.problem.name, st, inf)
        worst = max(worst, _residual3d(torch, mbp, r.problem, x, o, inf.removed_mean))
    print(f"  worst 3D residual over the sample {worst:.2e}", flush=True)
    assert worst <= 1e-10
    order = sorted(range(len(reqs)), key=lambda i: reqs[i].problem.ncells)
    for i in (order[0], order[len(order) // 2]):
        prob = reqs[i].problem
        modes = [0, prob.nz - 1]
        errs = _mode_errors(torch, mbp, prob, rhs[i], outs[i], modes)
        print(f"  {prob.name} ({prob.ncells} cells): mode errors {[f'{e:.1e}' for e in errs]}", flush=True)
        assert max(errs) <= 1e-9
