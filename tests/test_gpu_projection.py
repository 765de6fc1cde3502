"""Pressure projection (Eqs. (3)-(6)) through the C ABI, against the oracle.

mbp_divergence must match the oracle's face divergence cell by cell; one
mbp_project step must reproduce the oracle's projection (rhs = D u* / gamma
dt, direct solve, u = u* - gamma dt G Phi) to the solver's error, and leave a
velocity whose divergence is at the solver's tolerance relative to D u*
(the divergence-free check of Sec. 4.1).  Cases: joined blocks around an
obstacle (Dirichlet outflow), the singular L-shape with walls that let no
flow through, boxes with Dirichlet ends along z (nz + 1 z faces), and seeded
random multi-block layouts.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import projection as PJ

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


def _faces(prob, seed, closed_walls=False):
    nu, nv, nw = PJ.face_sizes(prob)
    rng = np.random.default_rng(seed)
    u, v, w = PJ.make_consistent(prob, rng.standard_normal(nu), rng.standard_normal(nv), rng.standard_normal(nw))
    if closed_walls:  # no flow through Neumann walls: the singular problem stays compatible
        g = oracle.Geometry(prob)
        us, vs, ws = PJ.split_faces(prob, u, v, w)
        for b in range(g.nb):
            if g.bc[b][0] == W.NEUMANN:
                us[b][:, :, 0] = 0.0
            if g.bc[b][1] == W.NEUMANN:
                us[b][:, :, -1] = 0.0
            if g.bc[b][2] == W.NEUMANN:
                vs[b][:, 0, :] = 0.0
            if g.bc[b][3] == W.NEUMANN:
                vs[b][:, -1, :] = 0.0
            if g.zkind[0] == "N" and len(ws[b]) == g.nz + 1:
                ws[b][0] = 0.0
            if g.zkind[1] == "N" and len(ws[b]) == g.nz + 1:
                ws[b][-1] = 0.0
    return u, v, w


def _cases():
    return [
        (W.obstacle8(16, 12), False),
        (W.lshape(24, 8, 1.5, 1.0), True),
        (W.box(48, 40, 10, 0.75, 0.625, 0.15, "DD", "NN", "DD", xfactor=1.2, name="box_DD_NN_DDz"), True),
        (W.box(40, 36, 8, 0.6, 0.5, 0.12, "PP", "ND", "NN", yfactor=1.4, name="box_PP_ND_NNz"), True),
    ] + [(W.random_layout(seed), True) for seed in (3, 11, 100, 102)]  # seeded layouts, two periodic rings


@pytest.mark.parametrize("prob,closed", _cases(), ids=lambda c: getattr(c, "name", str(c)))
def test_divergence_matches_oracle(torch_cuda, mbp, prob, closed):
    torch = torch_cuda
    u, v, w = _faces(prob, 101)
    plan = mbp.Plan(prob)
    assert plan.velocity_sizes() == PJ.face_sizes(prob)
    out = torch.empty(plan.ncells, dtype=torch.float64, device="cuda")
    plan.divergence(dev(torch, u), dev(torch, v), dev(torch, w), out, scale=0.5)
    ref = 0.5 * PJ.divergence(prob, u, v, w)
    got = host(out)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("prob,closed", _cases(), ids=lambda c: getattr(c, "name", str(c)))
def test_project_matches_oracle(torch_cuda, mbp, prob, closed, precision):
    torch = torch_cuda
    print(f"projection {prob.name} {precision}", flush=True)
    u, v, w = _faces(prob, 102, closed_walls=closed)
    gdt = 0.05
    ur, vr, wr, phir = PJ.project(prob, u, v, w, gdt)
    plan = mbp.Plan(prob, precision=precision)
    ud, vd, wd = dev(torch, u), dev(torch, v), dev(torch, w)
    phi = torch.zeros(plan.ncells, dtype=torch.float64, device="cuda")
    work = torch.empty_like(phi)
    info = plan.project(ud, vd, wd, gdt, phi, work, rtol=1e-10, flags=mbp.RETIRE)
    ug, vg, wg = host(ud), host(vd), host(wd)
    corr = np.linalg.norm(np.concatenate([u - ur, v - vr, w - wr]))
    diff = np.linalg.norm(np.concatenate([ug - ur, vg - vr, wg - wr]))
    d0 = np.linalg.norm(PJ.divergence(prob, u, v, w))
    d1 = np.linalg.norm(PJ.divergence(prob, ug, vg, wg))
    print(f"  {info} |u - u_oracle| / |correction| = {diff / corr:.2e}, |D u| / |D u*| = {d1 / d0:.2e}",
          flush=True)
    assert info.status == 0
    assert diff <= 1e-8 * corr
    assert d1 <= 2e-10 * d0
    # a second projection of the projected field finds (almost) nothing to do
    phi2 = torch.zeros_like(phi)
    plan.project(ud, vd, wd, gdt, phi2, work, rtol=1e-10, flags=mbp.RETIRE)
    assert float(phi2.abs().max()) <= 1e-8 * float(phi.abs().max())
    plan.close()
