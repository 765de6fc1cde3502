"""HIP path vs the CPU oracle, element by element, on small seeded problems.

Sizes are chosen so the oracle finishes in seconds while the GPU kernels see
several tiles, ragged tile tails, odd-size coarsening (three-cell merges),
odd periodic wraps (extra smoothing colours), joined blocks and stretched
faces.  Tolerances: transforms and the operator to ~1e-12 (FP64 rounding);
solves to the stated bar, relative residual <= 1e-10 (checked with the
oracle's own operator) and relative solution error <= 1e-9.
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


def two_block(nz, zpair, nx1=12, nx2=7, ny=9):
    """Two joined blocks side by side, stretched y, ragged x sizes."""
    yf = W.faces(ny, 0.0, 1.0, 0, 1.3)
    A = W.Block((1, 1), (nx1, ny), W.faces(nx1, 0.0, 1.0), yf, (W.DIRICHLET, W.CONNECT, W.NEUMANN, W.NEUMANN))
    B = W.Block((nx1 + 1, 1), (nx1 + nx2, ny), W.faces(nx2, 1.0, 1.6, 0, 0.8), yf.copy(),
                (W.CONNECT, W.NEUMANN, W.NEUMANN, W.DIRICHLET))
    return W.Problem([A, B], nz, 1.3, W.PAIRS[zpair], name=f"two_block_{zpair}_{nz}")


# nz covers every radix (2..31 through n/2 = 1..31, and the any-radix stage
# for the primes 37, 83 and 509 of n/2 = 37, 74, 83, 509), and the workgroup shapes
# of the power-of-two lengths: 64-column tiles of the per-tile kernel (32, 64),
# the streaming kernel's 64-, 32- and 16-column tiles (256, 512, 1024), and
# 4 columns with eight radix-2 butterflies per thread (2048).
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("nz", [2, 4, 6, 8, 10, 14, 22, 26, 32, 48, 62, 64, 96, 160, 256, 512, 1024, 2048,
                                74, 148, 166, 1018])
def test_transforms(torch_cuda, mbp, kind, nz):
    torch = torch_cuda
    prob = two_block(nz, kind)
    print(f"transform {kind} nz={nz}", flush=True)
    plan = mbp.Plan(prob)
    f = W.rhs(prob, 11 + nz)
    fh = torch.empty(plan.ncells, dtype=torch.float64, device="cuda")
    plan.forward(dev(torch, f), fh)
    ref = oracle.modal_rhs(prob, f, range(nz))  # (nz, plane)
    got = host(fh).reshape(nz, -1)
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() <= 1e-12 * scale * max(1.0, np.sqrt(nz))
    # inverse of random modal data
    ph = np.random.default_rng(nz).standard_normal(plan.ncells)
    p = torch.empty(plan.ncells, dtype=torch.float64, device="cuda")
    plan.inverse(dev(torch, ph), p)
    T = oracle.basis(kind, nz)
    g = oracle.Geometry(prob)
    phm = ph.reshape(nz, -1)
    expect = np.concatenate([(T @ phm[:, g.off2[i]:g.off2[i + 1]]).ravel() for i in range(g.nb)])
    assert np.abs(host(p) - expect).max() <= 1e-12 * np.abs(expect).max() * max(1.0, np.sqrt(nz))
    plan.close()


# The streaming kernel's workgroups loop over tiles: planes of 25,344 columns
# give 396 to 1,584 tiles (several per workgroup), ragged at both blocks' ends;
# a 64 x 192 box at nz = 256 gives 192 tiles, one per workgroup (each
# workgroup's first tile reads the tables it has just staged in LDS).
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("nz", [256, 512, 1024, "box256"])
def test_transforms_streaming(torch_cuda, mbp, kind, nz):
    torch = torch_cuda
    if nz == "box256":
        prob = W.box(64, 192, 256, 0.5, 1.5, 2.0, "DD", "DN", kind, name=f"box64x192x256_{kind}")
        nz = 256
    else:
        prob = two_block(nz, kind, 161, 95, 99)
    print(f"transform (streaming) {kind} nz={nz}", flush=True)
    plan = mbp.Plan(prob)
    g = oracle.Geometry(prob)
    T = oracle.basis(kind, nz)
    f = W.rhs(prob, 7 + nz)
    fh = torch.empty(plan.ncells, dtype=torch.float64, device="cuda")
    plan.forward(dev(torch, f), fh)
    got = host(fh).reshape(nz, -1)
    ref = oracle.modal_rhs(prob, f, range(nz))
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max() * np.sqrt(nz)
    ph = np.random.default_rng(nz).standard_normal(plan.ncells)
    p = torch.empty(plan.ncells, dtype=torch.float64, device="cuda")
    plan.inverse(dev(torch, ph), p)
    phm = ph.reshape(nz, -1)
    expect = np.concatenate([(T @ phm[:, g.off2[i]:g.off2[i + 1]]).ravel() for i in range(g.nb)])
    assert np.abs(host(p) - expect).max() <= 1e-12 * np.abs(expect).max() * np.sqrt(nz)
    plan.close()


@pytest.mark.parametrize("kind", KINDS)
def test_apply_operator(torch_cuda, mbp, kind):
    torch = torch_cuda
    prob = W.lshape(12, 6, 1.5, 1.0)
    prob.zbc = W.PAIRS[kind]
    plan = mbp.Plan(prob)
    p = np.random.default_rng(3).standard_normal(plan.ncells)
    out = torch.empty(plan.ncells, dtype=torch.float64, device="cuda")
    plan.apply(dev(torch, p), out)
    ref = oracle.apply_3d(oracle.Geometry(prob), p)
    assert np.abs(host(out) - ref).max() <= 1e-12 * np.abs(ref).max()
    plan.close()


def _problems():
    out = [
        W.config1(),
        W.lshape(32, 16, 1.5, 2.0),
        W.box(96, 80, 12, 0.75, 0.625, 0.1, "DN", "NN", "ND", xfactor=1.7, yfactor=1.2, name="box96x80_DN_NN_ND"),
        W.box(40, 36, 10, 40 / 128, 36 / 128, 10 / 128, "PP", "DD", "DD", name="box40x36_oddwrap"),
        W.box(70, 130, 8, 70 / 128, 130 / 128, 8 / 128, "ND", "PP", "NN", xfactor=2.0, name="box70x130_ragged"),
        two_block(6, "PP", 100, 36, 44),
    ]
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("prob", _problems(), ids=lambda p: p.name)
def test_solve_parity(torch_cuda, mbp, prob, precision):
    torch = torch_cuda
    print(f"solve {prob.name} {precision}", flush=True)
    f = W.rhs(prob, 21)
    ref = oracle.solve(prob, f)  # projects f when singular, gauge-fixed
    fproj = oracle.project_compatible(prob, f) if oracle.is_singular(prob) else f
    plan = mbp.Plan(prob, precision=precision)
    p = torch.zeros(plan.ncells, dtype=torch.float64, device="cuda")
    info = plan.solve(dev(torch, f), p, rtol=1e-10, flags=mbp.PROJECT_RHS)
    got = host(p)
    res = oracle.rel_residual(prob, got, fproj)
    err = oracle.rel_error(got, ref)
    print(f"  {info} residual={res:.2e} error={err:.2e}", flush=True)
    assert info.status == 0
    assert info.rel_residual <= 1e-10
    assert res <= 1e-10
    assert err <= 1e-9
    plan.close()


@pytest.mark.parametrize("retire", [False, True])
def test_retirement_same_answer(torch_cuda, mbp, retire):
    torch = torch_cuda
    prob = W.lshape(32, 16, 1.5, 2.0)
    f = W.rhs(prob, 5, "normal")
    ref = oracle.solve(prob, f)
    plan = mbp.Plan(prob)
    p = torch.zeros(plan.ncells, dtype=torch.float64, device="cuda")
    flags = mbp.PROJECT_RHS | (mbp.RETIRE if retire else 0)
    info = plan.solve(dev(torch, f), p, rtol=1e-10, flags=flags)
    assert oracle.rel_error(host(p), ref) <= 1e-9
    cpm = info.cycles_per_mode
    if retire:
        # the slowest modes are the small-|lambda| ones (Appendix B trend)
        assert cpm.max() > cpm.min()
        assert cpm[0] == cpm.max()
    plan.close()


def test_status_codes(torch_cuda, mbp):
    torch = torch_cuda
    prob = W.lshape(8, 4, 1.5, 1.0)  # singular
    plan = mbp.Plan(prob, max_cycles=60)
    f = W.rhs(prob, 1)
    p = torch.zeros(plan.ncells, dtype=torch.float64, device="cuda")
    info = plan.solve(dev(torch, f), p, flags=0, raise_on_error=False)
    assert info.status == mbp.ERR_INCOMPATIBLE
    bad = f.copy()
    bad[17] = np.nan
    info = plan.solve(dev(torch, bad), p, flags=mbp.PROJECT_RHS, raise_on_error=False)
    assert info.status == mbp.ERR_NONFINITE
    plan.close()
    plan = mbp.Plan(W.box(64, 64, 4, 1, 1, 1, "NN", "DD", "NN"), max_cycles=1)
    f = W.rhs(plan.problem, 2)
    p = torch.zeros(plan.ncells, dtype=torch.float64, device="cuda")
    info = plan.solve(dev(torch, f), p, raise_on_error=False)
    assert info.status == mbp.ERR_NOT_CONVERGED
    with pytest.raises(ValueError):
        plan.solve(dev(torch, f[:-1]), p)
    plan.close()


def four_block(n=64, nz=4):
    """2 x 2 blocks meeting at one point (joined on all inner faces)."""
    C_, N_, D_ = W.CONNECT, W.NEUMANN, W.DIRICHLET
    xl, xr = W.faces(n, 0.0, 1.0, 0, 1.2), W.faces(n, 1.0, 2.0)
    yb, yt = W.faces(n, 0.0, 1.0), W.faces(n, 1.0, 2.0, 0, 1.4)
    blocks = [
        W.Block((1, 1), (n, n), xl, yb, (D_, C_, N_, C_)),
        W.Block((n + 1, 1), (2 * n, n), xr, yb.copy(), (C_, N_, D_, C_)),
        W.Block((1, n + 1), (n, 2 * n), xl.copy(), yt, (N_, C_, C_, N_)),
        W.Block((n + 1, n + 1), (2 * n, 2 * n), xr.copy(), yt.copy(), (C_, D_, C_, N_)),
    ]
    return W.Problem(blocks, nz, 0.5, W.PAIRS["DN"], name=f"four_block_{n}")


def _global_problems():
    return [
        W.lshape(96, 6, 1.5, 1.0),
        four_block(64, 4),
        W.box(256, 192, 4, 1.0, 0.75, 0.1, "DD", "NN", "PP", xfactor=1.3, yfactor=1.8, name="box256x192"),
        W.box(250, 130, 4, 250 / 128, 130 / 128, 4 / 128, "PP", "ND", "NN", name="box250x130_oddwrap"),
        W.box(200, 300, 6, 200 / 128, 300 / 128, 6 / 128, "DN", "PP", "DD", xfactor=2.0, name="box200x300"),
    ]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("prob", _global_problems(), ids=lambda p: p.name)
def test_solve_parity_global_levels(torch_cuda, mbp, prob, precision):
    torch = torch_cuda
    print(f"solve {prob.name} {precision}", flush=True)
    f = W.rhs(prob, 31)
    ref = oracle.solve(prob, f)
    fproj = oracle.project_compatible(prob, f) if oracle.is_singular(prob) else f
    plan = mbp.Plan(prob, precision=precision)
    p = torch.zeros(plan.ncells, dtype=torch.float64, device="cuda")
    info = plan.solve(dev(torch, f), p, rtol=1e-10, flags=mbp.PROJECT_RHS)
    got = host(p)
    res = oracle.rel_residual(prob, got, fproj)
    err = oracle.rel_error(got, ref)
    print(f"  {info} residual={res:.2e} error={err:.2e}", flush=True)
    assert info.status == 0 and res <= 1e-10 and err <= 1e-9
    plan.close()


@pytest.mark.parametrize("nu", [(1, 1), (2, 2), (2, 1), (1, 3)])
def test_smoothing_counts(torch_cuda, mbp, nu):
    torch = torch_cuda
    prob = W.lshape(96, 4, 1.5, 1.0)
    f = W.rhs(prob, 41, "normal")
    ref = oracle.solve(prob, f)
    plan = mbp.Plan(prob, nu1=nu[0], nu2=nu[1])
    p = torch.zeros(plan.ncells, dtype=torch.float64, device="cuda")
    info = plan.solve(dev(torch, f), p, rtol=1e-10, flags=mbp.PROJECT_RHS)
    assert info.status == 0
    assert oracle.rel_error(host(p), ref) <= 1e-9
    plan.close()


def test_deterministic(torch_cuda, mbp):
    """Two solves of the same input are bitwise equal (no races in the sweeps)."""
    torch = torch_cuda
    prob = four_block(64, 4)
    f = dev(torch, W.rhs(prob, 3))
    plan = mbp.Plan(prob)
    p1 = torch.zeros(plan.ncells, dtype=torch.float64, device="cuda")
    p2 = torch.zeros_like(p1)
    plan.solve(f, p1, rtol=1e-10)
    plan.solve(f, p2, rtol=1e-10)
    assert torch.equal(p1, p2)
    plan.close()


# ---------------------------------------------------------------------------
# Schedules: the register-march pre-smoothing form and the plan autotuner must
# leave the answer unchanged.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("prob", _global_problems(), ids=lambda p: p.name)
def test_register_march_form(torch_cuda, mbp, prob, precision):
    torch = torch_cuda
    print(f"register march {prob.name} {precision}", flush=True)
    f = W.rhs(prob, 33)
    ref = oracle.solve(prob, f)
    fproj = oracle.project_compatible(prob, f) if oracle.is_singular(prob) else f
    plan = mbp.Plan(prob, precision=precision, march=1)
    p = torch.zeros(plan.ncells, dtype=torch.float64, device="cuda")
    info = plan.solve(dev(torch, f), p, rtol=1e-10, flags=mbp.PROJECT_RHS | mbp.RETIRE)
    got = host(p)
    res = oracle.rel_residual(prob, got, fproj)
    err = oracle.rel_error(got, ref)
    print(f"  {info} residual={res:.2e} error={err:.2e}", flush=True)
    assert info.status == 0 and res <= 1e-10 and err <= 1e-9
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("prob", [W.lshape(96, 6, 1.5, 1.0), _global_problems()[2]], ids=lambda p: p.name)
def test_plan_autotune(torch_cuda, mbp, prob, precision):
    torch = torch_cuda
    f = W.rhs(prob, 35)
    fd = dev(torch, f)
    plan = mbp.Plan(prob, precision=precision)
    t = plan.autotune(fd)
    print(f"  tuning {prob.name}: {t}", flush=True)
    assert t["ms_tuned"] <= t["ms_default"] + 1e-9
    assert t["wg_target"] > 0 and all(x in (0, 1) for x in t["form"])
    p = torch.zeros_like(fd)
    info = plan.solve(fd, p, rtol=1e-10, flags=mbp.PROJECT_RHS | mbp.RETIRE)
    ref = oracle.solve(prob, f)
    assert info.status == 0
    assert oracle.rel_error(host(p), ref) <= 1e-9
    plan.close()


# ---------------------------------------------------------------------------
# Final check (mbp_residual_norm): the 3D residual norm of any field, against
# the oracle's operator, with the rhs shift of a projected singular solve and
# the Helmholtz term.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("alpha", [0.0, 7.5])
@pytest.mark.parametrize("prob", [W.lshape(40, 12, 1.5, 1.0), two_block(10, "DN"),
                                  W.box(70, 33, 8, 1.0, 0.5, 0.25, "PP", "ND", "PP", yfactor=1.2, name="box70x33")],
                         ids=lambda p: p.name)
def test_residual_norm(torch_cuda, mbp, prob, alpha):
    torch = torch_cuda
    rng = np.random.default_rng(71)
    p = rng.standard_normal(prob.ncells)
    f = rng.standard_normal(prob.ncells)
    shift = 0.125
    plan = mbp.Plan(prob, helmholtz=alpha)
    out = host(plan.residual_norm(dev(torch, f), dev(torch, p), shift))
    g = oracle.Geometry(prob)
    r = f - shift - oracle.apply_3d(g, p, alpha)
    print(f"  {prob.name} alpha={alpha}: {out} vs {np.linalg.norm(r)}, {np.linalg.norm(f - shift)}", flush=True)
    assert abs(out[0] - np.linalg.norm(r)) <= 1e-12 * np.linalg.norm(r)
    assert abs(out[1] - np.linalg.norm(f - shift)) <= 1e-12 * np.linalg.norm(f - shift)
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_obstacle8_small(torch_cuda, mbp, precision):
    """Eight blocks around a square obstacle (Sec. 4.2): joined faces on all
    sides of the obstacle, Neumann inflow and walls, Dirichlet outflow."""
    torch = torch_cuda
    prob = W.obstacle8(16, 12)
    f = W.rhs(prob, 91, "normal")
    ref = oracle.solve(prob, f)
    plan = mbp.Plan(prob, precision=precision)
    p = torch.zeros(plan.ncells, dtype=torch.float64, device="cuda")
    info = plan.solve(dev(torch, f), p, rtol=1e-10, flags=mbp.PROJECT_RHS | mbp.RETIRE)
    got = host(p)
    res = oracle.rel_residual(prob, got, f)
    err = oracle.rel_error(got, ref)
    print(f"  obstacle8 {precision}: {info} residual={res:.2e} error={err:.2e}", flush=True)
    assert info.status == 0 and res <= 1e-10 and err <= 1e-9
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("prob", [W.box(15, 12, 8, 15 / 16, 12 / 16, 0.5, "PP", "NN", "PP", name="box15x12_oddring_x"),
                                  W.box(40, 27, 6, 40 / 32, 27 / 32, 0.25, "DN", "PP", "NN", xfactor=1.3,
                                        name="box40x27_oddring_y")],
                         ids=lambda p: p.name)
def test_odd_periodic_finest_ring(torch_cuda, mbp, prob, precision):
    """An odd number of cells around a periodic wrap on the finest grid: the
    last column (row) takes the two extra smoothing colours."""
    torch = torch_cuda
    f = W.rhs(prob, 92)
    ref = oracle.solve(prob, f)
    fproj = oracle.project_compatible(prob, f) if oracle.is_singular(prob) else f
    plan = mbp.Plan(prob, precision=precision)
    p = torch.zeros(plan.ncells, dtype=torch.float64, device="cuda")
    info = plan.solve(dev(torch, f), p, rtol=1e-10, flags=mbp.PROJECT_RHS | mbp.RETIRE)
    got = host(p)
    res = oracle.rel_residual(prob, got, fproj)
    err = oracle.rel_error(got, ref)
    print(f"  {prob.name} {precision}: {info} residual={res:.2e} error={err:.2e}", flush=True)
    assert info.status == 0 and res <= 1e-10 and err <= 1e-9
    plan.close()


@pytest.mark.parametrize("zk", ["PP", "NN", "DD", "ND", "DN"])
def test_solve_prime_half_length(torch_cuda, mbp, zk):
    """nz = 74: the half-length FFT of 37 points runs the any-radix stage."""
    torch = torch_cuda
    prob = two_block(74, zk)
    f = W.rhs(prob, 93)
    ref = oracle.solve(prob, f)
    fproj = oracle.project_compatible(prob, f) if oracle.is_singular(prob) else f
    plan = mbp.Plan(prob)
    p = torch.zeros(plan.ncells, dtype=torch.float64, device="cuda")
    info = plan.solve(dev(torch, f), p, rtol=1e-10, flags=mbp.PROJECT_RHS | mbp.RETIRE)
    got = host(p)
    res = oracle.rel_residual(prob, got, fproj)
    err = oracle.rel_error(got, ref)
    print(f"  {prob.name}: {info} residual={res:.2e} error={err:.2e}", flush=True)
    assert info.status == 0 and res <= 1e-10 and err <= 1e-9
    plan.close()


def _aniso_problems():
    D, N, C = W.DIRICHLET, W.NEUMANN, W.CONNECT
    # two joined blocks of 1 x 4 cells (dx = 1/128, dy = 1/32)
    A = W.Block((1, 1), (128, 32), W.faces(128, 0.0, 1.0), W.faces(32, 0.0, 1.0), (D, C, N, N))
    B = W.Block((129, 1), (192, 32), W.faces(64, 1.0, 1.5), W.faces(32, 0.0, 1.0), (C, N, N, D))
    joined = W.Problem([A, B], 8, 0.5, W.PAIRS["DN"], name="two_block_aspect4")
    return [
        W.box(256, 64, 8, 1.0, 1.0, 0.25, "DD", "NN", "PP", name="box256x64_aspect4"),
        W.box(64, 256, 6, 1.0, 0.25, 0.1, "NN", "DD", "NN", yfactor=1.2, name="box64x256_aspect16"),
        W.box(64, 128, 8, 0.125, 1.0, 0.5, "PP", "ND", "DD", name="box64x128_aspect4_periodic"),
        joined,
        two_block(6, "PP", 100, 36, 44),
    ]


# Blocks of disparate sizes (a 4- or 6-cell-wide block beside a 256- or
# 512-cell one, a 4-cell block of half-width cells between two wide ones, an
# 8 x 8 block below an 8 x 200 one, a 1- or 2-cell sliver between two 64 x 64
# blocks on the finest grid).  Where uniform steps would leave more than 256
# coarsest cells, each class of blocks that share cells across joined faces
# coarsens on its own, so the wide blocks go on coarsening after the thin one
# has stopped (down to 256 coarsest cells), and the thin one merges its last
# cells into one where that keeps its cells near square.  Five of these
# planes were refused before (coarsest plane above 2048 cells).
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("kind,zpair", [("thin_wide", "PP"), ("stacked", "NN"), ("sandwich", "DN"),
                                        ("large", "DD"), ("sliver1", "NN"), ("sliver2", "ND")])
def test_disparate_blocks(torch_cuda, mbp, kind, zpair, precision):
    torch = torch_cuda
    prob = W.disparate(kind, 8, zpair)
    print(f"disparate {prob.name} {precision}", flush=True)
    f = W.rhs(prob, 37)
    ref = oracle.solve(prob, f)
    fproj = oracle.project_compatible(prob, f) if oracle.is_singular(prob) else f
    plan = mbp.Plan(prob, precision=precision)
    p = torch.zeros(plan.ncells, dtype=torch.float64, device="cuda")
    info = plan.solve(dev(torch, f), p, rtol=1e-10, flags=mbp.PROJECT_RHS | mbp.RETIRE)
    got = host(p)
    res = oracle.rel_residual(prob, got, fproj)
    err = oracle.rel_error(got, ref)
    print(f"  {info} residual={res:.2e} error={err:.2e}", flush=True)
    assert info.status == 0
    assert res <= 1e-10
    assert err <= 1e-9
    assert info.cycles <= 30
    plan.close()


# Anisotropic cells: the hierarchy halves only the direction of the smaller
# mean width (PFMG's semicoarsening rule) until the cells are near square;
# point red-black smoothing then keeps its rate (cycles stay <= 30).  The
# last layout mixes a uniform block of 0.01-wide cells with a stretched one
# (cell aspect 1.3 to 2.9 across the plane); it needed 48 cycles with full
# coarsening and takes about 24 with semicoarsening.
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("prob", _aniso_problems(), ids=lambda p: p.name)
def test_anisotropic_semicoarsening(torch_cuda, mbp, prob, precision):
    torch = torch_cuda
    print(f"anisotropic {prob.name} {precision}", flush=True)
    f = W.rhs(prob, 31)
    ref = oracle.solve(prob, f)
    fproj = oracle.project_compatible(prob, f) if oracle.is_singular(prob) else f
    plan = mbp.Plan(prob, precision=precision)
    p = torch.zeros(plan.ncells, dtype=torch.float64, device="cuda")
    info = plan.solve(dev(torch, f), p, rtol=1e-10, flags=mbp.PROJECT_RHS | mbp.RETIRE)
    got = host(p)
    res = oracle.rel_residual(prob, got, fproj)
    err = oracle.rel_error(got, ref)
    print(f"  {info} residual={res:.2e} error={err:.2e}", flush=True)
    assert info.status == 0
    assert res <= 1e-10
    assert err <= 1e-9
    assert info.cycles <= 30
    plan.close()


# The fused correcting sweep sums the squared residual of the red cells only
# (the black cells were relaxed last, so their residual is zero up to
# rounding).  Pin that shortcut on mid-cycle iterates: stop a lockstep FP64
# solve after k V-cycles and compare the reported largest ratio
# ||rhat_q|| / ||fhat_q|| with the same ratio taken by the oracle over every
# cell of every mode of the returned field (Eq. (9) per mode, unweighted sums
# over the plane as the solver's test uses).
@pytest.mark.parametrize("prob", [W.box(192, 160, 16, 1.2, 1.0, 0.5, "DD", "NN", "NN", name="box192x160_DD_NN_NN"),
                                  W.lshape(64, 16, 1.5, 1.0)], ids=lambda p: p.name)
@pytest.mark.parametrize("k", [1, 2, 4])
def test_fused_norm_mid_cycle(torch_cuda, mbp, prob, k):
    import scipy.sparse as sp
    from oracle.solve import _geom
    from oracle.operator import assemble_2d
    from oracle.transforms import eigenvalues
    torch = torch_cuda
    print(f"fused norm {prob.name} k={k}", flush=True)
    f = W.rhs(prob, 71)
    singular = oracle.is_singular(prob)
    fproj = oracle.project_compatible(prob, f) if singular else f
    plan = mbp.Plan(prob, max_cycles=k)
    p = torch.zeros(plan.ncells, dtype=torch.float64, device="cuda")
    info = plan.solve(dev(torch, f), p, rtol=1e-14, flags=mbp.PROJECT_RHS if singular else 0,
                      raise_on_error=False)
    assert info.status == mbp.ERR_NOT_CONVERGED and info.cycles == k, info
    plan.close()
    g = _geom(prob)
    qs = range(prob.nz)
    ph = oracle.modal_rhs(prob, host(p), qs)  # the same contraction applied to the field
    fh = oracle.modal_rhs(prob, fproj, qs)
    A2 = assemble_2d(g)
    lam = eigenvalues(g.zkind, g.nz) / (g.dz * g.dz)
    ratios = []
    for q in qs:
        r = fh[q] - (A2 @ ph[q] + lam[q] * ph[q])
        ratios.append(np.linalg.norm(r) / np.linalg.norm(fh[q]))
    worst = max(ratios)
    print(f"  {info} oracle max ratio {worst:.6e}", flush=True)
    assert worst > 1e-8  # a genuine mid-cycle iterate
    assert abs(info.rel_residual - worst) <= 1e-6 * worst


# The smallest problems: two z cells (every Table 1 pair), planes of 2 x 2 to
# 8 x 6 cells (one multigrid level, or a hierarchy that ends after one step,
# so the whole solve runs in one workgroup's LDS), singular ones included.
def _tiny_problems():
    out = []
    for i, zk in enumerate(KINDS):
        xp, yp = KINDS[(i + 1) % 5], KINDS[(i + 3) % 5]
        out.append(W.box(8, 6, 2, 1.0, 0.75, 0.25, xp, yp, zk, name=f"box8x6x2_{xp}_{yp}_{zk}"))
    out.append(W.box(2, 2, 2, 1.0, 1.0, 1.0, "NN", "NN", "PP", name="box2x2x2_NN_NN_PP"))
    out.append(W.box(3, 5, 4, 0.3, 0.5, 0.4, "DD", "PP", "NN", name="box3x5x4_DD_PP_NN"))
    out.append(W.box(4, 4, 2, 1.0, 1.0, 0.5, "NN", "NN", "NN", name="box4x4x2_NN_NN_NN"))
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("prob", _tiny_problems(), ids=lambda p: p.name)
def test_tiny_problems(torch_cuda, mbp, prob, precision):
    torch = torch_cuda
    print(f"tiny {prob.name} {precision}", flush=True)
    f = W.rhs(prob, 91)
    ref = oracle.solve(prob, f)
    fproj = oracle.project_compatible(prob, f) if oracle.is_singular(prob) else f
    plan = mbp.Plan(prob, precision=precision)
    p = torch.zeros(plan.ncells, dtype=torch.float64, device="cuda")
    info = plan.solve(dev(torch, f), p, rtol=1e-10, flags=mbp.PROJECT_RHS | mbp.RETIRE)
    got = host(p)
    res = oracle.rel_residual(prob, got, fproj)
    err = oracle.rel_error(got, ref)
    print(f"  {info} residual={res:.2e} error={err:.2e}", flush=True)
    assert info.status == 0 and res <= 1e-10 and err <= 1e-9
    plan.close()


# Seeded random layouts (rows, columns, L shapes and 2 x 2 grids of blocks 1
# to 40 cells wide, mildly stretched, random walls and z pairs; from seed 100
# on, rows and columns may close into periodic rings of any length) against
# the oracle: the hierarchy, merges, halos across joined faces, colour
# parities and the coarsest operator on layouts nobody picked by hand, with
# the default cycle cap.
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("seed", list(range(40)) + list(range(100, 140)))
def test_random_layouts(torch_cuda, mbp, seed, precision):
    torch = torch_cuda
    prob = W.random_layout(seed)
    print(f"random {prob.name} {[(b.nx, b.ny) for b in prob.blocks]} nz={prob.nz} {precision}", flush=True)
    f = W.rhs(prob, 100 + seed)
    ref = oracle.solve(prob, f)
    fproj = oracle.project_compatible(prob, f) if oracle.is_singular(prob) else f
    plan = mbp.Plan(prob, precision=precision)
    p = torch.zeros(plan.ncells, dtype=torch.float64, device="cuda")
    info = plan.solve(dev(torch, f), p, rtol=1e-10, flags=mbp.PROJECT_RHS | mbp.RETIRE)
    got = host(p)
    res = oracle.rel_residual(prob, got, fproj)
    err = oracle.rel_error(got, ref)
    print(f"  {info} residual={res:.2e} error={err:.2e}", flush=True)
    assert info.status == 0 and res <= 1e-10 and err <= 1e-9
    plan.close()


# The Helmholtz form (L_h - alpha) p = f on random layouts: alpha shifts every
# plane away from singularity, including the all-Neumann ones.
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("seed", range(1, 40, 4))
def test_random_layouts_helmholtz(torch_cuda, mbp, seed, precision):
    torch = torch_cuda
    prob = W.random_layout(seed)
    alpha = 40.0 + 10.0 * (seed % 3)
    print(f"random helmholtz {prob.name} alpha={alpha} {precision}", flush=True)
    f = W.rhs(prob, 200 + seed)
    ref = oracle.solve(prob, f, alpha=alpha)
    plan = mbp.Plan(prob, precision=precision, helmholtz=alpha)
    p = torch.zeros(plan.ncells, dtype=torch.float64, device="cuda")
    info = plan.solve(dev(torch, f), p, rtol=1e-10, flags=mbp.RETIRE)
    got = host(p)
    res = oracle.rel_residual(prob, got, f, alpha)
    err = oracle.rel_error(got, ref)
    print(f"  {info} residual={res:.2e} error={err:.2e}", flush=True)
    assert info.status == 0 and res <= 1e-10 and err <= 1e-9
    plan.close()


# The same layouts with the wide blocks four times larger (planes of up to
# about 60,000 cells, so the fused strip kernels, their halos across joined
# faces and block corners run on them), against the oracle.  Some planes of
# mode 0 are near-singular (a large all-Neumann block reached from a small
# Dirichlet wall through a thin arm): rediscretised coarse operators miss
# their smallest eigenvalue by a margin, and such modes need 50-70
# V-cycles, within the default cap of 100.
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("seed", list(range(40)) + list(range(100, 120)))
def test_random_layouts_large(torch_cuda, mbp, seed, precision):
    torch = torch_cuda
    prob = W.random_layout(seed, 4)
    print(f"random {prob.name} {[(b.nx, b.ny) for b in prob.blocks]} nz={prob.nz} {precision}", flush=True)
    f = W.rhs(prob, 400 + seed)
    ref = oracle.solve(prob, f)
    fproj = oracle.project_compatible(prob, f) if oracle.is_singular(prob) else f
    plan = mbp.Plan(prob, precision=precision)
    p = torch.zeros(plan.ncells, dtype=torch.float64, device="cuda")
    info = plan.solve(dev(torch, f), p, rtol=1e-10, flags=mbp.PROJECT_RHS | mbp.RETIRE)
    got = host(p)
    res = oracle.rel_residual(prob, got, fproj)
    err = oracle.rel_error(got, ref)
    print(f"  {info} residual={res:.2e} error={err:.2e}", flush=True)
    assert info.status == 0 and res <= 1e-10 and err <= 1e-9
    plan.close()


# The other solve forms on random layouts: lockstep modes (no retirement)
# and a warm start from a perturbed answer, in both precisions.
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("seed", list(range(0, 40, 5)) + [101, 106, 112])
def test_random_layouts_lockstep_warm(torch_cuda, mbp, seed, precision):
    torch = torch_cuda
    prob = W.random_layout(seed)
    print(f"random forms {prob.name} {precision}", flush=True)
    f = W.rhs(prob, 600 + seed)
    ref = oracle.solve(prob, f)
    fproj = oracle.project_compatible(prob, f) if oracle.is_singular(prob) else f
    plan = mbp.Plan(prob, precision=precision)
    p = torch.zeros(plan.ncells, dtype=torch.float64, device="cuda")
    info = plan.solve(dev(torch, f), p, rtol=1e-10, flags=mbp.PROJECT_RHS)
    got = host(p)
    res, err = oracle.rel_residual(prob, got, fproj), oracle.rel_error(got, ref)
    print(f"  lockstep {info} residual={res:.2e} error={err:.2e}", flush=True)
    assert info.status == 0 and res <= 1e-10 and err <= 1e-9
    guess = ref + 1e-3 * np.random.default_rng(seed).standard_normal(ref.size) * np.abs(ref).max()
    p = dev(torch, guess)
    info = plan.solve(dev(torch, f), p, rtol=1e-10, flags=mbp.PROJECT_RHS | mbp.RETIRE | mbp.WARM_START)
    got = host(p)
    res, err = oracle.rel_residual(prob, got, fproj), oracle.rel_error(got, ref)
    print(f"  warm {info} residual={res:.2e} error={err:.2e}", flush=True)
    assert info.status == 0 and res <= 1e-10 and err <= 1e-9
    plan.close()
