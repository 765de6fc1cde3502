"""Host-side checks of the C ABI (no GPU needed).

The library must load and export every function include/mbp.h declares;
plan validation (mbp_plan_check runs on the host only) must accept the
paper's layouts and reject the malformed ones with MBP_ERR_INVALID; the grid
helper must reproduce the tanh face mapping the workload generator uses.
"""
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def mbp():
    import paper_2106_03583_amd as m
    return m


def _declared():
    src = open(os.path.join(ROOT, "include", "mbp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mbp3?_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol(mbp):
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(mbp.lib, n), n
    assert set(names) == set(mbp.EXPORTED)


def test_version_and_status_strings(mbp):
    assert mbp.lib.mbp_version() >= 100
    for st in [mbp.OK, mbp.PENDING, mbp.ERR_INVALID, mbp.ERR_NOMEM, mbp.ERR_HIP, mbp.ERR_NOT_CONVERGED,
               mbp.ERR_NONFINITE, mbp.ERR_INCOMPATIBLE, mbp.ERR_BUSY, mbp.ERR_TOO_LARGE, mbp.ERR_NO_DEVICE]:
        assert len(mbp.status_string(st)) >= 2 and mbp.status_string(st) != "unknown status"
    assert mbp.status_string(12345) == "unknown status"


@pytest.mark.parametrize("gtype,factor", [(0, 0.0), (0, 1.5), (-1, 1.2), (1, 2.0)])
def test_grid_tanh_matches_generator(mbp, gtype, factor):
    a = mbp.grid_tanh(37, 0.25, 1.75, gtype, factor)
    b = W.faces(37, 0.25, 1.75, gtype, factor)
    assert np.allclose(a, b, rtol=0, atol=1e-14)
    assert a[0] == 0.25 and a[-1] == 1.75 and np.all(np.diff(a) > 0)


# Properties the stretched-grid mapping must have whatever its exact form
# (the paper names tanh clustering but prints no formula): exact end faces,
# strictly increasing faces, the two-sided form symmetric about the middle and
# finest at both walls, the one-sided forms mirror images of each other and
# finest at their own wall, and the uniform grid as the stretching goes to 0
# (the deviation falls like the square of the factor).
@pytest.mark.parametrize("factor", [0.5, 1.5, 3.0])
def test_grid_tanh_properties(mbp, factor):
    n = 48
    for gen in (lambda g, a: W.faces(n, 0.0, 1.0, g, a), lambda g, a: mbp.grid_tanh(n, 0.0, 1.0, g, a)):
        two, lo, hi = gen(0, factor), gen(-1, factor), gen(1, factor)
        for x in (two, lo, hi):
            assert x[0] == 0.0 and x[-1] == 1.0 and np.all(np.diff(x) > 0)
        d = np.diff(two)
        assert np.allclose(two + two[::-1], 1.0, rtol=0, atol=1e-14)
        assert d[0] < d[n // 2] and d[-1] < d[n // 2] and np.argmax(d) in (n // 2 - 1, n // 2)
        assert np.allclose(lo, 1.0 - hi[::-1], rtol=0, atol=1e-14)
        assert np.all(np.diff(np.diff(lo)) > 0) and np.all(np.diff(np.diff(hi)) < 0)
        uni = np.linspace(0.0, 1.0, n + 1)
        e1 = np.abs(gen(0, 1e-2) - uni).max()
        e2 = np.abs(gen(0, 5e-3) - uni).max()
        assert e1 < 1e-4 and 3.5 < e1 / e2 < 4.5


def test_plan_check_layouts(mbp):
    s = mbp.plan_check(W.config2())
    assert s["ncells"] == 3 * 256 * 256 * 512
    assert s["nblocks"] == 3 and s["singular"]
    # Table 2 of the paper: A joined to B (x) and C (y)
    assert s["nbr"][0] == [-1, 1, -1, 2]
    assert s["nbr"][1] == [0, -1, -1, -1]
    assert s["nbr"][2] == [-1, -1, 0, -1]
    s3 = mbp.plan_check(W.config3())
    assert s3["ncells"] == 512 * 512 * 1024 and not s3["singular"]
    assert s3["nlevels"] >= 7
    # about 32 B/pt of workspace plus the hierarchy: well under the 288 GB card
    assert s3["workspace_bytes"] < 100 * s3["ncells"]


def _with(prob, **kw):
    blocks = [W.Block(b.lo, b.hi, b.xf, b.yf, b.bc) for b in prob.blocks]
    p = W.Problem(blocks, prob.nz, prob.lz, prob.zbc, prob.name)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_plan_check_rejects(mbp):
    base = W.box(16, 12, 8, 1.0, 0.75, 0.5, "DD", "NN", "PP")
    assert mbp.plan_check_status(base) == mbp.OK
    assert mbp.plan_check_status(_with(base, nz=7)) == mbp.ERR_INVALID      # odd nz
    assert mbp.plan_check_status(_with(base, nz=0)) == mbp.ERR_INVALID
    assert mbp.plan_check_status(_with(base, zbc=(W.PERIODIC, W.NEUMANN))) == mbp.ERR_INVALID
    assert mbp.plan_check_status(_with(base, zbc=(W.CONNECT, W.CONNECT))) == mbp.ERR_INVALID
    assert mbp.plan_check_status(_with(base, lz=-1.0)) == mbp.ERR_INVALID
    # faces not increasing
    b = base.blocks[0]
    bad = W.Problem([W.Block(b.lo, b.hi, b.xf[::-1].copy(), b.yf, b.bc)], 8, 0.5, base.zbc)
    assert mbp.plan_check_status(bad) == mbp.ERR_INVALID
    # a joined face with no partner
    lone = W.Problem([W.Block(b.lo, b.hi, b.xf, b.yf, (W.CONNECT, W.DIRICHLET, W.NEUMANN, W.NEUMANN))], 8, 0.5,
                     base.zbc)
    assert mbp.plan_check_status(lone) == mbp.ERR_INVALID
    # an odd cell count around a periodic wrap is accepted (its last column
    # is relaxed in two extra colours on every level)
    odd = W.box(15, 12, 8, 1.0, 0.75, 0.5, "PP", "NN", "PP")
    assert mbp.plan_check_status(odd) == mbp.OK
    # any even nz: a half length with a prime factor above 31 (37, 509) plans
    assert mbp.plan_check_status(_with(base, nz=74)) == mbp.OK
    assert mbp.plan_check_status(_with(base, nz=1018)) == mbp.OK


def test_plan_check_rejects_overlap_and_nonconforming(mbp):
    xf, yf = W.faces(8, 0.0, 1.0), W.faces(8, 0.0, 1.0)
    A = W.Block((1, 1), (8, 8), xf, yf, (W.DIRICHLET, W.CONNECT, W.NEUMANN, W.NEUMANN))
    B = W.Block((5, 1), (12, 8), W.faces(8, 0.5, 1.5), yf.copy(), (W.CONNECT, W.NEUMANN, W.NEUMANN, W.NEUMANN))
    assert mbp.plan_check_status(W.Problem([A, B], 4, 1.0, W.PAIRS["PP"])) == mbp.ERR_INVALID  # overlap
    C = W.Block((9, 1), (16, 8), W.faces(8, 1.0, 2.0), W.faces(8, 0.0, 1.0, 0, 1.5),
                (W.CONNECT, W.NEUMANN, W.NEUMANN, W.NEUMANN))
    # faces of the joined edge do not coincide (stretched vs uniform y)
    assert mbp.plan_check_status(W.Problem([A, C], 4, 1.0, W.PAIRS["PP"])) == mbp.ERR_INVALID
    D = W.Block((9, 1), (16, 8), W.faces(8, 1.0, 2.0), yf.copy(), (W.CONNECT, W.NEUMANN, W.NEUMANN, W.NEUMANN))
    assert mbp.plan_check_status(W.Problem([A, D], 4, 1.0, W.PAIRS["PP"])) == mbp.OK


@pytest.mark.parametrize("kind", ["thin_wide", "stacked", "sandwich", "large", "sliver1", "sliver2"])
def test_plan_check_disparate_blocks(mbp, kind):
    """A block too thin to follow its neighbours down the hierarchy stops
    coarsening on its own (its class of blocks sharing cells across joined
    faces) where uniform steps would leave more than 256 coarsest cells, and
    the others go on down to at most 256, so such planes are not refused."""
    s = mbp.plan_check(W.disparate(kind))
    assert s["coarse_cells"] <= 256
    assert s["nlevels"] >= 3


def test_plan_check_random_layouts(mbp):
    """Every seeded random layout of the GPU sweep plans (its coarsest plane
    within the 2048 cells of the exact solve)."""
    for seed in range(40):
        s = mbp.plan_check(W.random_layout(seed))
        assert s["coarse_cells"] <= 2048, seed


def test_plan_check_singular_flag(mbp):
    assert mbp.plan_check(W.box(8, 8, 4, 1, 1, 1, "NN", "NN", "PP"))["singular"]
    assert mbp.plan_check(W.box(8, 8, 4, 1, 1, 1, "PP", "PP", "NN"))["singular"]
    assert not mbp.plan_check(W.box(8, 8, 4, 1, 1, 1, "NN", "NN", "DN"))["singular"]
    assert not mbp.plan_check(W.box(8, 8, 4, 1, 1, 1, "ND", "PP", "PP"))["singular"]


def test_helmholtz_and_smoother_options(mbp):
    """The Helmholtz term (Sec. 2, implicit diffusion) removes the singular
    null space; negative or non-finite terms and unknown smoothers are refused."""
    prob = W.box(8, 8, 4, 1, 1, 1, "NN", "NN", "PP")
    assert mbp.plan_check(prob)["singular"]
    assert not mbp.plan_check(prob, helmholtz=2.0)["singular"]
    assert mbp.plan_check_status(prob, helmholtz=-1.0) == mbp.ERR_INVALID
    assert mbp.plan_check_status(prob, helmholtz=float("nan")) == mbp.ERR_INVALID
    assert mbp.plan_check_status(prob, helmholtz=float("inf")) == mbp.ERR_INVALID
    assert mbp.plan_check_status(prob, smoother=7) == mbp.ERR_INVALID
    assert mbp.lib.mbp_plan_set_helmholtz(None, 1.0) == mbp.ERR_INVALID


def test_workload_generators():
    c4 = W.config4()
    assert len(c4) == 64
    sizes = [p.ncells for p in c4]
    assert min(sizes) >= 64 * 64 * 64 and max(sizes) <= 384 * 384 * 256
    assert {tuple(p.zbc) for p in c4} == set(W.PAIRS.values())
    c5 = W.config5(count=50, rate_per_s=100.0)
    assert len(c5) == 50
    t = [r.arrival_s for r in c5]
    assert all(b >= a for a, b in zip(t, t[1:]))
