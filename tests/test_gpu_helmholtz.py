"""Helmholtz form (L_h - alpha) p = f through the C ABI, against the oracle.

The paper solves the implicit-diffusion systems of each Runge-Kutta substep
"with the same numerical method" as the pressure equation (Sec. 2), the
matrix diagonal changing every substep (footnote of Sec. 3.3.1).  Here the
term alpha enters every modal shift, sigma_q = lambda_q / dz^2 - alpha; with
alpha > 0 no problem is singular (no projection, no gauge).  Bar: relative
residual <= 1e-10 (oracle operator) and relative error <= 1e-9 against the
oracle's direct solution with the same alpha.
"""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

RK3_GAMMA = (8.0 / 15.0, 2.0 / 15.0, 1.0 / 3.0)  # gamma = alpha + beta of the paper's RK3


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


def _problems():
    return [
        W.lshape(48, 8, 1.5, 1.0),                                                   # singular at alpha = 0
        W.box(70, 52, 10, 70 / 128, 52 / 128, 10 / 128, "NN", "PP", "NN", yfactor=0.0, name="box_NN_PP_NN"),
        W.box(64, 40, 6, 0.5, 40 / 128, 6 / 128, "DD", "ND", "DN", xfactor=1.6, name="box_DD_ND_DN"),
    ]


def _check(torch, mbp, plan, prob, f, alpha, precision):
    p = torch.zeros(plan.ncells, dtype=torch.float64, device="cuda")
    info = plan.solve(dev(torch, f), p, rtol=1e-10, flags=mbp.PROJECT_RHS | mbp.RETIRE)
    got = host(p)
    ref = oracle.solve(prob, f, alpha=alpha)
    res = oracle.rel_residual(prob, got, f, alpha)
    err = oracle.rel_error(got, ref)
    print(f"  {prob.name} alpha={alpha:g} {precision}: {info} residual={res:.2e} error={err:.2e}", flush=True)
    assert info.status == 0
    assert info.removed_mean == 0.0  # nothing is projected once alpha > 0
    assert res <= 1e-10 and err <= 1e-9


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("alpha", [0.75, 40.0, 2.0e4])
@pytest.mark.parametrize("prob", _problems(), ids=lambda p: p.name)
def test_helmholtz_parity(torch_cuda, mbp, prob, alpha, precision):
    torch = torch_cuda
    print(f"helmholtz {prob.name} alpha={alpha} {precision}", flush=True)
    f = W.rhs(prob, 41)
    plan = mbp.Plan(prob, precision=precision, helmholtz=alpha)
    assert not plan.singular
    _check(torch, mbp, plan, prob, f, alpha, precision)
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_helmholtz_per_substep(torch_cuda, mbp, precision):
    """One plan, the term changed before each RK3 substep, then back to the
    singular pressure equation (alpha = 0: projection and gauge return)."""
    torch = torch_cuda
    prob = _problems()[0]
    print(f"helmholtz substeps {prob.name} {precision}", flush=True)
    f = W.rhs(prob, 42)
    plan = mbp.Plan(prob, precision=precision)
    assert plan.singular
    nu, dt = 2.0e-3, 5.0e-3
    for g in RK3_GAMMA:
        alpha = 1.0 / (nu * g * dt)
        plan.set_helmholtz(alpha)
        assert not plan.singular
        _check(torch, mbp, plan, prob, f, alpha, precision)
    plan.set_helmholtz(0.0)
    assert plan.singular
    p = torch.zeros(plan.ncells, dtype=torch.float64, device="cuda")
    info = plan.solve(dev(torch, f), p, rtol=1e-10, flags=mbp.PROJECT_RHS | mbp.RETIRE)
    fp = oracle.project_compatible(prob, f)
    assert info.status == 0
    assert oracle.rel_residual(prob, host(p), fp) <= 1e-10
    assert oracle.rel_error(host(p), oracle.solve(prob, f)) <= 1e-9
    plan.close()


def test_helmholtz_apply_operator(torch_cuda, mbp):
    torch = torch_cuda
    prob = _problems()[0]
    alpha = 12.5
    plan = mbp.Plan(prob, helmholtz=alpha)
    x = np.random.default_rng(43).standard_normal(prob.ncells)
    out = torch.empty(plan.ncells, dtype=torch.float64, device="cuda")
    plan.apply(dev(torch, x), out)
    ref = oracle.apply_3d(oracle.Geometry(prob), x, alpha)
    assert np.allclose(host(out), ref, rtol=1e-12, atol=1e-10 * np.abs(ref).max())
    shifts = plan.modal_shift()
    lam = oracle.eigenvalues(oracle.Geometry(prob).zkind, prob.nz)
    dz = prob.lz / prob.nz
    assert np.allclose(shifts, lam / dz**2 - alpha, rtol=1e-13, atol=1e-12)
    plan.close()
