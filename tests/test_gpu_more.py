"""More HIP-path checks through the C ABI: block-split invariance, warm starts,
and the two batched forms (grouped stage launches and per-problem graphs).

Block split: the same grid cut into two joined blocks must give the same
solution as one block (the multi-block halos are exact), to 1e-9 relative;
this is the GPU side of the oracle's block-split pin (Sec. 3.1).
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


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def _split_pair(nx=96, ny=64, nz=8):
    """One nx x ny block and the same grid as two joined nx/2 x ny blocks."""
    xf = W.faces(nx, 0.0, 1.5)
    yf = W.faces(ny, 0.0, 1.0, 0, 1.4)
    one = W.Problem([W.Block((1, 1), (nx, ny), xf, yf, (W.DIRICHLET, W.NEUMANN, W.NEUMANN, W.NEUMANN))],
                    nz, 0.5, W.PAIRS["ND"], name="split_one")
    h = nx // 2
    A = W.Block((1, 1), (h, ny), xf[:h + 1].copy(), yf.copy(), (W.DIRICHLET, W.CONNECT, W.NEUMANN, W.NEUMANN))
    B = W.Block((h + 1, 1), (nx, ny), xf[h:].copy(), yf.copy(), (W.CONNECT, W.NEUMANN, W.NEUMANN, W.NEUMANN))
    two = W.Problem([A, B], nz, 0.5, W.PAIRS["ND"], name="split_two")
    return one, two


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_block_split_invariance(torch_cuda, mbp, precision):
    torch = torch_cuda
    one, two = _split_pair()
    nx, ny, nz, h = 96, 64, 8, 48
    f3 = np.random.default_rng(11).uniform(-1.0, 1.0, (nz, ny, nx))
    f_one = f3.reshape(-1)
    f_two = np.concatenate([f3[:, :, :h].reshape(-1), f3[:, :, h:].reshape(-1)])
    out = []
    for prob, f in ((one, f_one), (two, f_two)):
        plan = mbp.Plan(prob, precision=precision)
        p = torch.zeros(plan.ncells, dtype=torch.float64, device="cuda")
        info = plan.solve(dev(torch, f), p, rtol=1e-10, flags=mbp.RETIRE)
        assert info.status == 0 and info.rel_residual <= 1e-10
        out.append(host(p))
        plan.close()
    p3 = out[0].reshape(nz, ny, nx)
    p_one_as_two = np.concatenate([p3[:, :, :h].reshape(-1), p3[:, :, h:].reshape(-1)])
    diff = np.linalg.norm(out[1] - p_one_as_two) / np.linalg.norm(p_one_as_two)
    print(f"split {precision}: rel diff {diff:.2e}", flush=True)
    assert diff <= 1e-9
    # and both are the discrete solution
    assert oracle.rel_residual(two, out[1], f_two) <= 1e-10


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_warm_start(torch_cuda, mbp, precision):
    torch = torch_cuda
    prob = W.box(80, 72, 12, 80 / 128, 72 / 128, 12 / 128, "DD", "NN", "PP", yfactor=1.3, name="warm")
    f = W.rhs(prob, 3)
    ref = oracle.solve(prob, f)
    plan = mbp.Plan(prob, precision=precision)
    fd = dev(torch, f)
    p = torch.zeros(plan.ncells, dtype=torch.float64, device="cuda")
    cold = plan.solve(fd, p, rtol=1e-10, flags=mbp.RETIRE)
    # restart from the converged answer: no cycle is needed, p is kept
    again = p.clone()
    warm = plan.solve(fd, again, rtol=1e-10, flags=mbp.RETIRE | mbp.WARM_START)
    assert warm.status == 0 and warm.cycles == 0, warm
    assert float(torch.linalg.vector_norm(again - p) / torch.linalg.vector_norm(p)) <= 1e-14
    # restart from a perturbed answer: fewer cycles than from zero, same solution
    pert = p + 1e-6 * torch.linalg.vector_norm(p) / plan.ncells ** 0.5 * torch.sin(
        torch.arange(plan.ncells, device="cuda", dtype=torch.float64))
    warm2 = plan.solve(fd, pert, rtol=1e-10, flags=mbp.RETIRE | mbp.WARM_START)
    assert warm2.status == 0 and warm2.cycles < cold.cycles, (warm2, cold)
    assert oracle.rel_error(host(pert), ref) <= 1e-9
    plan.close()


def _grouped_set():
    """Mixed-precision problems whose strip levels all take the grouped form."""
    return [
        W.box(128, 96, 8, 1.0, 0.75, 0.0625, "DD", "NN", "PP", yfactor=1.5, name="g128x96"),
        W.box(160, 128, 6, 1.25, 1.0, 0.05, "NN", "DD", "NN", xfactor=1.2, name="g160x128"),
        W.lshape(32, 8, 1.5, 2.0),
    ]


def _run_batch(torch, mbp, probs, seed0):
    fs = [W.rhs(p, seed0 + i) for i, p in enumerate(probs)]
    plans = [mbp.Plan(p, precision="mixed") for p in probs]
    rhs = [dev(torch, f) for f in fs]
    outs = [torch.zeros(pl.ncells, dtype=torch.float64, device="cuda") for pl in plans]
    infos = mbp.solve_batch(plans, rhs, outs, rtol=1e-10, flags=mbp.PROJECT_RHS | mbp.AUTOTUNE)
    sched = mbp.batch_schedule(plans)
    singles = []
    for pl, r in zip(plans, rhs):
        p = torch.zeros(pl.ncells, dtype=torch.float64, device="cuda")
        pl.solve(r, p, rtol=1e-10, flags=mbp.PROJECT_RHS | mbp.RETIRE)
        singles.append(host(p))
    for pl in plans:
        pl.close()
    return fs, [host(o) for o in outs], singles, infos, sched


def _check_all(probs, fs, got, singles, infos):
    for prob, f, g, s1, info in zip(probs, fs, got, singles, infos):
        ref = oracle.solve(prob, f)
        fproj = oracle.project_compatible(prob, f) if oracle.is_singular(prob) else f
        res = oracle.rel_residual(prob, g, fproj)
        err = oracle.rel_error(g, ref)
        same = np.linalg.norm(g - s1) / np.linalg.norm(s1)
        print(f"  {prob.name}: residual={res:.2e} error={err:.2e} vs single {same:.2e}", flush=True)
        assert info.status == 0
        assert res <= 1e-10 and err <= 1e-9 and same <= 1e-9


def test_batch_grouped_form(torch_cuda, mbp):
    probs = _grouped_set()
    fs, got, singles, infos, sched = _run_batch(torch_cuda, mbp, probs, 700)
    assert sched is not None and sched[0] == 0, sched  # grouped stage launches
    _check_all(probs, fs, got, singles, infos)


def test_batch_per_problem_form(torch_cuda, mbp):
    # an odd periodic ring on the second strip level (302 -> 151 cells) keeps
    # that level off the strip kernels, so the batch runs per-problem graphs
    odd = W.box(302, 256, 4, 302 / 128, 2.0, 4 / 128, "PP", "NN", "DD", name="odd302")
    probs = _grouped_set() + [odd]
    fs, got, singles, infos, sched = _run_batch(torch_cuda, mbp, probs, 800)
    assert sched is not None and sched[0] > 0, sched
    _check_all(probs, fs, got, singles, infos)


# Modes that pass the test before the first V-cycle are never relaxed; their
# modal solution must be zero even when the plan's buffers still hold a
# previous solve (the retiring FP64 solve does not zero the whole modal field
# up front, only these planes at the end).  A zero right-hand side makes every
# mode pass at once; the solve after it must be unaffected.
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_unrelaxed_modes_zero(torch_cuda, mbp, precision):
    torch = torch_cuda
    prob = W.box(128, 96, 16, 1.0, 0.75, 0.5, "DD", "NN", "NN", name="box128x96_DD_NN_NN")
    plan = mbp.Plan(prob, precision=precision)
    p = torch.zeros(plan.ncells, dtype=torch.float64, device="cuda")
    f1 = W.rhs(prob, 81)
    assert plan.solve(dev(torch, f1), p, rtol=1e-10, flags=mbp.RETIRE).status == 0
    p.fill_(7.0)
    info0 = plan.solve(dev(torch, np.zeros_like(f1)), p, rtol=1e-10, flags=mbp.RETIRE)
    assert info0.status == 0 and info0.cycles == 0, info0
    assert float(p.abs().max()) == 0.0
    f2 = W.rhs(prob, 82)
    p.fill_(7.0)
    info2 = plan.solve(dev(torch, f2), p, rtol=1e-10, flags=mbp.RETIRE)
    got = host(p)
    res = oracle.rel_residual(prob, got, f2)
    err = oracle.rel_error(got, oracle.solve(prob, f2))
    print(f"  {precision}: {info2} residual={res:.2e} error={err:.2e}", flush=True)
    assert info2.status == 0 and res <= 1e-10 and err <= 1e-9
    plan.close()


# The batched form over the seeded random layouts (mixed precision, every
# problem its own shape, many of them off the grouped form): each result
# against the oracle and against the same plan's single solve.
def test_batch_random_layouts(torch_cuda, mbp):
    probs = [W.random_layout(seed) for seed in range(40)]
    fs, got, singles, infos, sched = _run_batch(torch_cuda, mbp, probs, 900)
    _check_all(probs, fs, got, singles, infos)


# The package imported before torch (a fresh process, so nothing has loaded
# a HIP runtime yet) must still find the device and solve: the package loads
# torch's runtime ahead of its library.
def test_import_before_torch(torch_cuda):
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import paper_2106_03583_amd as m\n"
        "import torch, numpy as np, workloads as W\n"
        "prob = W.box(48, 40, 8, 1.0, 0.8, 0.5, 'DD', 'NN', 'PP', name='order')\n"
        "f = W.rhs(prob, 3)\n"
        "plan = m.Plan(prob)\n"
        "p = torch.zeros(plan.ncells, dtype=torch.float64, device='cuda')\n"
        "info = plan.solve(torch.from_numpy(f).cuda(), p, rtol=1e-10, flags=m.RETIRE)\n"
        "print('status', info.status, 'residual', info.rel_residual, flush=True)\n"
        "sys.exit(0 if info.status == 0 and info.rel_residual <= 1e-10 else 1)\n" % root)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=240, cwd=root)
    print(r.stdout, r.stderr[-2000:], flush=True)
    assert r.returncode == 0, r.stdout + r.stderr[-2000:]
