"""3D multigrid without the z synthesis (the paper's comparison solver,
Sec. 3.3.1 and Sec. 4.2) through the C ABI, against the oracle.

The 3D MG reaches the same discrete solution of Eq. (8) as the
FFT-accelerated path by a different route, so the bar is the same: relative
residual <= 1e-10 with the oracle's operator and relative error <= 1e-9
against the oracle's direct solution (dense LU on tiny grids, Algorithm 1 or
the separable route on small ones).  Cases: every z pair, stretched and
joined blocks (L-shape, four blocks meeting at a point), periodic x-y,
singular problems (projection and gauge) and the Helmholtz term.
"""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

KINDS = ["PP", "NN", "DD", "ND", "DN"]


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


def _run(torch, mbp, prob, f, ref, alpha=0.0, rtol=1e-10, warm=None):
    plan = mbp.Plan3D(prob, helmholtz=alpha)
    p = torch.zeros(prob.ncells, dtype=torch.float64, device="cuda") if warm is None else dev(torch, warm)
    flags = mbp.PROJECT_RHS | (mbp.WARM_START if warm is not None else 0)
    info = plan.solve(dev(torch, f), p, rtol=rtol, flags=flags)
    got = host(p)
    fp = oracle.project_compatible(prob, f) if oracle.is_singular(prob, alpha) else f
    res = oracle.rel_residual(prob, got, fp, alpha)
    err = oracle.rel_error(got, ref)
    print(f"  mg3d {prob.name} alpha={alpha}: levels={plan.nlevels} nz={plan.nz_per_level} {info} "
          f"residual={res:.2e} error={err:.2e}", flush=True)
    plan.close()
    assert info.status == 0
    assert info.rel_residual <= rtol
    assert res <= rtol
    assert err <= 1e-9
    return info


def _tiny():
    out = []
    for zk in KINDS:
        out.append(W.box(6, 4, 4, 1.0, 0.7, 0.5, "DD", "NN", zk, name=f"tiny_{zk}"))
    out.append(W.box(6, 4, 4, 1.2, 1.0, 1.0, "ND", "DN", "PP", xfactor=1.5, yfactor=2.0, name="tiny_stretch"))
    out.append(W.box(4, 6, 4, 1.0, 1.0, 1.0, "PP", "PP", "NN", name="tiny_periodic_xy"))
    out.append(W.box(4, 4, 6, 1.0, 1.0, 1.0, "NN", "NN", "PP", name="tiny_singular"))
    out.append(W.lshape(4, 4, 1.5, 1.0))
    return out


@pytest.mark.parametrize("prob", _tiny(), ids=lambda p: p.name)
def test_mg3d_tiny_dense(torch_cuda, mbp, prob):
    print(f"mg3d tiny {prob.name}", flush=True)
    f = W.rhs(prob, 61)
    _run(torch_cuda, mbp, prob, f, oracle.solve_dense(prob, f))


def four_block(n=32, nz=8):
    """Four blocks meeting at a point, stretched in both directions."""
    C, N, D = W.CONNECT, W.NEUMANN, W.DIRICHLET
    x0 = W.faces(n, 0.0, 1.0, 0, 1.2)
    x1 = W.faces(n, 1.0, 2.0, 0, 1.2)
    y0 = W.faces(n, 0.0, 1.0, 0, 0.9)
    y1 = W.faces(n, 1.0, 2.0, 0, 0.9)
    blocks = [W.Block((1, 1), (n, n), x0, y0, (D, C, N, C)),
              W.Block((n + 1, 1), (2 * n, n), x1, y0.copy(), (C, N, N, C)),
              W.Block((1, n + 1), (n, 2 * n), x0.copy(), y1, (D, C, C, N)),
              W.Block((n + 1, n + 1), (2 * n, 2 * n), x1.copy(), y1.copy(), (C, N, C, N))]
    return W.Problem(blocks, nz, 0.5, W.PAIRS["PP"], name=f"four_block_{n}")


def _small():
    out = [W.lshape(32, 16, 1.5, 1.0), four_block(), W.obstacle8(8, 12)]
    for i, zk in enumerate(KINDS):
        xp, yp = KINDS[(i + 2) % 5], KINDS[(i + 4) % 5]
        out.append(W.box(40, 36, 12, 40 / 64, 36 / 64, 12 / 64, xp, yp, zk, xfactor=1.3, yfactor=1.1,
                         name=f"box40x36x12_{xp}{yp}{zk}"))
    out.append(W.box(70, 52, 10, 70 / 64, 52 / 64, 10 / 64, "NN", "PP", "NN", name="box70x52x10_odd"))
    out.append(W.box(15, 12, 8, 15 / 16, 12 / 16, 0.5, "PP", "NN", "PP", name="box15x12_oddring_x"))
    return out


@pytest.mark.parametrize("prob", _small(), ids=lambda p: p.name)
def test_mg3d_small(torch_cuda, mbp, prob):
    print(f"mg3d small {prob.name}", flush=True)
    f = W.rhs(prob, 62)
    _run(torch_cuda, mbp, prob, f, oracle.solve(prob, f))


@pytest.mark.parametrize("zk", KINDS)
def test_mg3d_z_marching_transfers(torch_cuda, mbp, zk):
    """Isotropic boxes (x-y and z coarsen together over several levels, with
    32 and 64 z cells) run the z-marching prolongation; every z pair."""
    prob = W.box(64, 48, 32, 1.0, 0.75, 0.5, "DN", "PP", zk, xfactor=1.2, name=f"box64x48x32_{zk}")
    print(f"mg3d z-march {prob.name}", flush=True)
    f = W.rhs(prob, 66)
    _run(torch_cuda, mbp, prob, f, oracle.solve(prob, f))


@pytest.mark.parametrize("alpha", [3.0, 500.0])
def test_mg3d_helmholtz(torch_cuda, mbp, alpha):
    prob = W.lshape(24, 8, 1.5, 1.0)
    print(f"mg3d helmholtz {prob.name} alpha={alpha}", flush=True)
    f = W.rhs(prob, 63)
    _run(torch_cuda, mbp, prob, f, oracle.solve(prob, f, alpha=alpha), alpha=alpha)


def test_mg3d_warm_start_and_same_answer_as_fft_path(torch_cuda, mbp):
    """A warm start from the FFT path's answer converges at once; both
    solvers agree to the error bar."""
    torch = torch_cuda
    prob = W.lshape(48, 16, 1.5, 1.0)
    f = W.rhs(prob, 64)
    ref = oracle.solve(prob, f)
    plan = mbp.Plan(prob)
    p = torch.zeros(prob.ncells, dtype=torch.float64, device="cuda")
    plan.solve(dev(torch, f), p, rtol=1e-10, flags=mbp.PROJECT_RHS | mbp.RETIRE)
    plan.close()
    p2 = host(p)
    info = _run(torch, mbp, prob, f, ref, warm=p2)
    assert info.cycles <= 2


def test_mg3d_errors(torch_cuda, mbp):
    torch = torch_cuda
    prob = W.box(16, 16, 8, 1.0, 1.0, 0.5, "NN", "NN", "NN", name="incompatible")
    f = W.rhs(prob, 65) + 1.0  # non-zero mean: incompatible without projection
    plan = mbp.Plan3D(prob)
    p = torch.zeros(prob.ncells, dtype=torch.float64, device="cuda")
    info = plan.solve(dev(torch, f), p, rtol=1e-10, flags=0, raise_on_error=False)
    assert info.status == mbp.ERR_INCOMPATIBLE
    f2 = f.copy()
    f2[5] = np.nan
    info = plan.solve(dev(torch, f2), p, rtol=1e-10, flags=mbp.PROJECT_RHS, raise_on_error=False)
    assert info.status == mbp.ERR_NONFINITE
    plan.close()
    with pytest.raises(mbp.MBPError):
        mbp.Plan3D(prob, nu1=0)


# The 3D multigrid on the seeded random layouts of the FFT path's sweep (the
# same x-y hierarchy rule: uniform steps unless they leave more than 256
# coarsest cells).
@pytest.mark.parametrize("seed", range(0, 40, 2))
def test_mg3d_random_layouts(torch_cuda, mbp, seed):
    prob = W.random_layout(seed)
    print(f"mg3d random {prob.name} {[(b.nx, b.ny) for b in prob.blocks]} nz={prob.nz}", flush=True)
    f = W.rhs(prob, 300 + seed)
    _run(torch_cuda, mbp, prob, f, oracle.solve(prob, f))
