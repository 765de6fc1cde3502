"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every check here compares the oracle with something other than itself:
library transforms (scipy / numpy FFT), brute-force eigen-decompositions,
closed-form discrete eigenfunctions, the printed tables (tests/golden), an
independent loop-by-loop assembly of the 3D matrix, and invariants (self-
adjointness, conservation, block-split independence, Sec. 4.1).
"""
import os

import numpy as np
import pytest
import scipy.fft as sfft

import oracle
import workloads as W
from oracle.grid import Geometry
from oracle.operator import apply_3d, assemble_2d, assemble_3d_dense, second_difference_1d
from oracle.transforms import basis, eigenvalues, table1_unnormalised

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
NS = [2, 4, 6, 8, 16, 64]
KINDS = ["PP", "NN", "DD", "ND", "DN"]


# ---------------------------------------------------------------------------
# Transforms and eigenvalues (Table 1)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n", NS)
def test_basis_orthonormal(kind, n):
    T = basis(kind, n)
    assert np.allclose(T.T @ T, np.eye(n), atol=1e-13)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n", NS)
def test_basis_diagonalises_ghost_second_difference(kind, n):
    """D_bc T = T diag(lambda): staggered ghost rules N: g=p0, D: g=-p0, P: wrap."""
    D = second_difference_1d(kind, n)
    T = basis(kind, n)
    lam = eigenvalues(kind, n)
    assert np.allclose(D @ T, T * lam[None, :], atol=1e-12)
    # brute force: the same spectrum as a symmetric eigen-solver finds
    assert np.allclose(np.sort(lam), np.linalg.eigvalsh(D), atol=1e-12)


@pytest.mark.parametrize("n", NS)
def test_library_transforms(n):
    rng = np.random.default_rng(n)
    f = rng.standard_normal(n)
    assert np.allclose(basis("NN", n).T @ f, sfft.dct(f, type=2, norm="ortho"), atol=1e-13)
    assert np.allclose(basis("DD", n).T @ f, sfft.dst(f, type=2, norm="ortho"), atol=1e-13)
    assert np.allclose(basis("ND", n).T @ f, sfft.dct(f, type=4, norm="ortho"), atol=1e-13)
    assert np.allclose(basis("DN", n).T @ f, sfft.dst(f, type=4, norm="ortho"), atol=1e-13)
    F = np.fft.fft(f)
    assert np.allclose(basis("PP", n).T @ f, (F.real - F.imag) / np.sqrt(n), atol=1e-13)
    # inverses: DCT-III / DST-III, self-inverse IV kinds and Hartley
    assert np.allclose(basis("NN", n) @ f, sfft.idct(f, type=2, norm="ortho"), atol=1e-13)
    assert np.allclose(basis("DD", n) @ f, sfft.idst(f, type=2, norm="ortho"), atol=1e-13)


def _table1_rows():
    rows = []
    with open(os.path.join(GOLDEN, "table1.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            pair, kexpr, fwd, bwd, theta = line.split()
            rows.append((pair, kexpr, fwd, bwd, theta))
    return rows


@pytest.mark.parametrize("row", _table1_rows(), ids=lambda r: r[0])
@pytest.mark.parametrize("n", [4, 8, 16])
def test_table1_golden(row, n):
    pair, kexpr, fwd, bwd, theta = row
    q = np.arange(n, dtype=np.float64)
    k = eval(kexpr, {"q": q})  # expressions are the printed kappa_q / (2 pi / l)
    lam = 2.0 * (np.cos(2.0 * np.pi * k / n) - 1.0)  # kappa dl = 2 pi k / n
    assert np.allclose(eigenvalues(pair, n), lam, atol=1e-14)
    F, B, th = table1_unnormalised(pair, n)
    assert th == eval(theta, {"n": n})
    assert np.allclose(B @ F, th * np.eye(n), atol=1e-10)
    # the unnormalised forward transform spans the same eigen-space mode by mode
    T = basis(pair, n)
    if pair != "PP":
        scale = np.diag(F @ T)
        assert np.allclose(F @ T, np.diag(scale), atol=1e-10)


def test_dirichlet_neumann_row():
    """The DN pair (not printed) has the ND eigenvalues and a DST-IV basis."""
    for n in (4, 8, 16):
        assert np.allclose(eigenvalues("DN", n), eigenvalues("ND", n))
        D = second_difference_1d("DN", n)
        assert np.allclose(np.sort(eigenvalues("DN", n)), np.linalg.eigvalsh(D), atol=1e-12)


# ---------------------------------------------------------------------------
# Geometry
# ---------------------------------------------------------------------------

def _table2_problem():
    blocks = []
    with open(os.path.join(GOLDEN, "table2_blocks.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            v = line.split()
            lo = (int(v[1]), int(v[2]))
            hi = (int(v[4]), int(v[5]))
            lmin = (float(v[7]), float(v[8]))
            lmax = (float(v[10]), float(v[11]))
            nx, ny = hi[0] - lo[0] + 1, hi[1] - lo[1] + 1
            blocks.append(W.Block(lo, hi, W.faces(nx, lmin[0], lmax[0]), W.faces(ny, lmin[1], lmax[1]),
                                  [0, 0, 0, 0]))
    # faces touching another block in index space are joined, the rest are walls
    for i, b in enumerate(blocks):
        bc = []
        for f, (axis, side) in enumerate([(0, -1), (0, 1), (1, -1), (1, 1)]):
            t = 1 - axis
            touch = any(
                (c.lo[t], c.hi[t]) == (b.lo[t], b.hi[t]) and
                ((side < 0 and c.hi[axis] + 1 == b.lo[axis]) or (side > 0 and b.hi[axis] + 1 == c.lo[axis]))
                for c in blocks if c is not b)
            bc.append(W.CONNECT if touch else W.NEUMANN)
        b.bc = tuple(bc)
    return W.Problem(blocks, nz=2, lz=0.1, zbc=W.PAIRS["NN"])


def test_table2_connectivity():
    g = Geometry(_table2_problem())
    XM, XP, YM, YP = 0, 1, 2, 3
    assert g.nbr[0][XP] == 1 and g.nbr[1][XM] == 0
    assert g.nbr[1][XP] == 2 and g.nbr[2][XM] == 1
    assert g.nbr[1][YP] == 3 and g.nbr[3][YM] == 1
    assert g.nbr[0][YP] == -1 and g.nbr[3][XP] == -1
    assert [g.nx[i] for i in range(4)] == [20, 10, 10, 10]


def test_nonconforming_face_rejected():
    ya = W.faces(8, 0.0, 1.0)
    yb = W.faces(8, 0.0, 1.0, 0, 1.5)
    A = W.Block((1, 1), (8, 8), W.faces(8, 0, 1), ya, (W.NEUMANN, W.CONNECT, W.NEUMANN, W.NEUMANN))
    B = W.Block((9, 1), (16, 8), W.faces(8, 1, 2), yb, (W.CONNECT, W.NEUMANN, W.NEUMANN, W.NEUMANN))
    with pytest.raises(ValueError):
        Geometry(W.Problem([A, B], 4, 1.0, W.PAIRS["NN"]))


# ---------------------------------------------------------------------------
# Operator
# ---------------------------------------------------------------------------

def _tiny_problems():
    out = []
    for zk in KINDS:
        out.append(W.box(6, 4, 4, 1.0, 0.7, 0.5, "DD", "NN", zk, name=f"u_{zk}"))
    out.append(W.box(6, 4, 4, 1.2, 1.0, 1.0, "ND", "DN", "PP", xfactor=1.5, yfactor=2.0, name="stretch"))
    out.append(W.box(4, 6, 4, 1.0, 1.0, 1.0, "PP", "PP", "NN", name="periodic_xy"))
    out.append(W.box(4, 4, 6, 1.0, 1.0, 1.0, "NN", "NN", "PP", name="singular_box"))
    out.append(W.lshape(4, 4, 1.5, 1.0))
    return out


@pytest.mark.parametrize("prob", _tiny_problems(), ids=lambda p: p.name)
def test_apply_matches_loop_assembly(prob):
    g = Geometry(prob)
    A = assemble_3d_dense(g)
    p = np.random.default_rng(0).standard_normal(g.ncell3)
    assert np.allclose(apply_3d(g, p), A @ p, rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("prob", _tiny_problems(), ids=lambda p: p.name)
def test_operator_self_adjoint_in_volume_inner_product(prob):
    g = Geometry(prob)
    rng = np.random.default_rng(1)
    u, v = rng.standard_normal((2, g.ncell3))
    V = g.volumes()
    lhs = np.dot(V * u, apply_3d(g, v))
    rhs = np.dot(V * apply_3d(g, u), v)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.linalg.norm(u) * np.linalg.norm(v))


def test_singular_null_space_and_conservation():
    for prob in (W.box(4, 4, 6, 1.0, 1.0, 1.0, "NN", "NN", "PP"), W.lshape(4, 4, 1.5, 1.0)):
        g = Geometry(prob)
        assert np.allclose(apply_3d(g, np.ones(g.ncell3)), 0.0, atol=1e-10)
        p = np.random.default_rng(2).standard_normal(g.ncell3)
        assert abs(np.dot(g.volumes(), apply_3d(g, p))) < 1e-9


def test_uniform_box_is_eq8():
    """On a uniform box the FV operator is the 7-point stencil of Eq. (8)."""
    nx, ny, nz = 6, 5, 4
    dx, dy, dz = 1.0 / nx, 1.0 / ny, 2.0 / nz
    prob = W.box(nx, ny, nz, 1.0, 1.0, 2.0, "PP", "PP", "PP")
    g = Geometry(prob)
    p = np.random.default_rng(3).standard_normal((nz, ny, nx))
    L = ((np.roll(p, 1, 2) - 2 * p + np.roll(p, -1, 2)) / dx**2 +
         (np.roll(p, 1, 1) - 2 * p + np.roll(p, -1, 1)) / dy**2 +
         (np.roll(p, 1, 0) - 2 * p + np.roll(p, -1, 0)) / dz**2)
    assert np.allclose(apply_3d(g, p.ravel()), L.ravel(), rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("pairs", [("DD", "NN", "PP"), ("ND", "DN", "DD"), ("PP", "DD", "ND"),
                                   ("NN", "PP", "DN"), ("DN", "ND", "NN")])
def test_closed_form_eigenfunctions(pairs):
    """Products of Table-1 eigenvectors are eigenfunctions of the 3D operator."""
    xp, yp, zp = pairs
    nx, ny, nz = 8, 6, 4
    lx, ly, lz = 1.0, 0.75, 0.5
    prob = W.box(nx, ny, nz, lx, ly, lz, xp, yp, zp)
    g = Geometry(prob)
    a, b, c = 3, 2, 1
    X = basis(xp, nx)[:, a]
    Y = basis(yp, ny)[:, b]
    Z = basis(zp, nz)[:, c]
    p = np.einsum("k,j,i->kji", Z, Y, X).ravel()
    mu = (eigenvalues(xp, nx)[a] / (lx / nx) ** 2 + eigenvalues(yp, ny)[b] / (ly / ny) ** 2 +
          eigenvalues(zp, nz)[c] / (lz / nz) ** 2)
    assert np.allclose(apply_3d(g, p), mu * p, atol=1e-9 * abs(mu))
    # ... and the direct solvers invert it exactly
    for solver in (oracle.solve_alg1, oracle.solve_separable):
        assert np.allclose(solver(prob, mu * p, project=False), p, atol=1e-12)


@pytest.mark.parametrize("pairs", [("DD", "NN", "PP"), ("NN", "NN", "NN"), ("PP", "PP", "PP"),
                                   ("ND", "PP", "DN")])
@pytest.mark.parametrize("alpha", [0.5, 37.0])
def test_helmholtz_closed_form(pairs, alpha):
    """Helmholtz form (L_h - alpha) of the implicit-diffusion systems (Sec. 2):
    a product of Table-1 eigenvectors with 3D eigenvalue mu solves it with
    rhs (mu - alpha) p.  All-Neumann / all-periodic boxes are no longer
    singular once alpha > 0, so the constant mode (a = b = c = 0) is included."""
    xp, yp, zp = pairs
    nx, ny, nz = 8, 6, 4
    lx, ly, lz = 1.0, 0.75, 0.5
    prob = W.box(nx, ny, nz, lx, ly, lz, xp, yp, zp)
    g = Geometry(prob)
    for a, b, c in ((0, 0, 0), (3, 2, 1)):
        X = basis(xp, nx)[:, a]
        Y = basis(yp, ny)[:, b]
        Z = basis(zp, nz)[:, c]
        p = np.einsum("k,j,i->kji", Z, Y, X).ravel()
        mu = (eigenvalues(xp, nx)[a] / (lx / nx) ** 2 + eigenvalues(yp, ny)[b] / (ly / ny) ** 2 +
              eigenvalues(zp, nz)[c] / (lz / nz) ** 2)
        assert np.allclose(apply_3d(g, p, alpha), (mu - alpha) * p, atol=1e-9 * (abs(mu) + alpha))
        assert not oracle.is_singular(prob, alpha)
        for solver in (oracle.solve_alg1, oracle.solve_separable, oracle.solve_dense):
            got = solver(prob, (mu - alpha) * p, project=False, alpha=alpha)
            assert np.allclose(got, p, atol=1e-12), solver.__name__


def test_helmholtz_dense_matches_apply_on_lshape():
    """Loop-assembled dense (L_h - alpha) equals the vectorised apply, and the
    three routes agree on a multi-block stretched grid."""
    prob = W.lshape(4, 4, 1.5, 1.0)
    g = Geometry(prob)
    alpha = 3.25
    A = assemble_3d_dense(g, alpha)
    p = np.random.default_rng(11).standard_normal(g.ncell3)
    assert np.allclose(A @ p, apply_3d(g, p, alpha), rtol=1e-12, atol=1e-9)
    # the shift only moves the diagonal
    assert np.allclose(A + alpha * np.eye(g.ncell3), assemble_3d_dense(g), atol=1e-12)
    f = W.rhs(prob, 12)
    a = oracle.solve_alg1(prob, f, alpha=alpha)
    b = oracle.solve_dense(prob, f, alpha=alpha)
    assert oracle.rel_error(a, b) < 1e-12
    assert oracle.rel_residual(prob, a, f, alpha) < 1e-13


def test_alg1_process_pool_same_result():
    """Per-shift solves in worker processes give the serial result bit for bit
    (Algorithm 1: the modes are independent)."""
    prob = W.lshape(6, 8, 1.5, 1.0)
    f = W.rhs(prob, 13, "normal")
    a = oracle.solve_alg1(prob, f)
    b = oracle.solve_alg1(prob, f, workers=2)
    assert np.array_equal(a, b)


def test_reduced_equation_eq9():
    """A z-eigenvector times a plane field maps to (A_2D + lambda_q/dz^2) on the plane."""
    prob = W.lshape(4, 6, 1.5, 1.0)
    g = Geometry(prob)
    A2 = assemble_2d(g)
    P2 = np.random.default_rng(4).standard_normal(g.ncell2)
    for q in range(g.nz):
        Z = basis(g.zkind, g.nz)[:, q]
        blocks = [np.einsum("k,yx->kyx", Z, b) for b in g.split2(P2)]
        p = np.concatenate([b.ravel() for b in blocks])
        Lp = g.split3(apply_3d(g, p))
        expect = A2 @ P2 + eigenvalues(g.zkind, g.nz)[q] / g.dz**2 * P2
        got = np.concatenate([(np.tensordot(Z, b, axes=(0, 0))).ravel() for b in Lp])
        assert np.allclose(got, expect, rtol=1e-11, atol=1e-8)


# ---------------------------------------------------------------------------
# Solves
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prob", _tiny_problems(), ids=lambda p: p.name)
def test_manufactured_solution_all_routes(prob):
    g = Geometry(prob)
    p = np.random.default_rng(5).standard_normal(g.ncell3)
    if oracle.is_singular(prob):
        p = oracle.remove_mean(prob, p)
    f = apply_3d(g, p)
    routes = [oracle.solve_alg1, oracle.solve_dense]
    if g.nb == 1:
        routes.append(oracle.solve_separable)
    for solve in routes:
        got = solve(prob, f)
        assert oracle.rel_error(got, p) < 1e-11, solve.__name__
        assert oracle.rel_residual(prob, got, f) < 1e-12


def test_routes_agree_on_random_rhs():
    prob = W.box(12, 10, 8, 1.0, 1.0, 1.0, "DN", "PP", "ND", xfactor=1.7)
    f = W.rhs(prob, 7)
    a = oracle.solve_alg1(prob, f)
    b = oracle.solve_separable(prob, f)
    assert oracle.rel_error(a, b) < 1e-12


def test_singular_gauge_and_projection():
    prob = W.lshape(6, 4, 1.5, 1.0)
    g = Geometry(prob)
    f = W.rhs(prob, 8)  # raw samples: not compatible
    p = oracle.solve_alg1(prob, f)
    V = g.volumes()
    assert abs(np.dot(V, p)) < 1e-12 * np.linalg.norm(p)
    fc = oracle.project_compatible(prob, f)
    assert abs(np.dot(V, fc)) < 1e-12 * np.linalg.norm(f)
    assert oracle.rel_residual(prob, p, fc) < 1e-12
    # a constant shift leaves the residual unchanged
    assert oracle.rel_residual(prob, p + 3.0, fc) < 1e-11
    # same answer as the dense bordered route
    assert oracle.rel_error(oracle.solve_dense(prob, f), p) < 1e-11


def test_block_split_invariance():
    """The same assembled grid cut into two blocks gives the same solution (Sec. 4.1)."""
    n, nz = 8, 4
    xf = W.faces(2 * n, 0.0, 2.0, 0, 1.2)
    yf = W.faces(n, 0.0, 1.0, 0, 1.5)
    one = W.Problem([W.Block((1, 1), (2 * n, n), xf, yf, (W.DIRICHLET, W.NEUMANN, W.NEUMANN, W.DIRICHLET))],
                    nz, 1.0, W.PAIRS["DD"])
    A = W.Block((1, 1), (n, n), xf[:n + 1], yf, (W.DIRICHLET, W.CONNECT, W.NEUMANN, W.DIRICHLET))
    B = W.Block((n + 1, 1), (2 * n, n), xf[n:], yf.copy(), (W.CONNECT, W.NEUMANN, W.NEUMANN, W.DIRICHLET))
    two = W.Problem([A, B], nz, 1.0, W.PAIRS["DD"])
    f = W.rhs(one, 9).reshape(nz, n, 2 * n)
    f2 = np.concatenate([f[:, :, :n].ravel(), f[:, :, n:].ravel()])
    p1 = oracle.solve(one, f.ravel()).reshape(nz, n, 2 * n)
    p2 = oracle.solve_alg1(two, f2)
    g2 = Geometry(two)
    pa, pb = g2.split3(p2)
    assert np.allclose(np.concatenate([pa, pb], axis=2), p1, atol=1e-12 * np.abs(p1).max())


def test_mode_solver_matches_full_solution():
    prob = W.lshape(8, 8, 1.5, 1.0)
    f = oracle.project_compatible(prob, W.rhs(prob, 10, "normal"))
    p = oracle.solve_alg1(prob, f)
    qs = [0, 1, 5]
    fh = oracle.modal_rhs(prob, f, qs)
    ph = oracle.modal_rhs(prob, p, qs)
    for i, q in enumerate(qs):
        got = oracle.solve_mode(prob, fh[i], q)
        if q == 0:  # singular plane: compare up to the area-weighted gauge
            a = Geometry(prob).areas()
            got = got - np.dot(a, got) / a.sum()
            ref = ph[i] - np.dot(a, ph[i]) / a.sum()
        else:
            ref = ph[i]
        assert np.allclose(got, ref, atol=1e-12 * np.abs(ref).max())


def test_workload_shapes():
    c1 = W.config1()
    assert c1.ncells == 32**3
    c2 = W.config2()
    assert c2.ncells == 3 * 256 * 256 * 512
    Geometry(c2)  # connectivity of the L-shape resolves
    c3 = W.config3()
    assert c3.ncells == 512 * 512 * 1024
    c4 = W.config4()
    assert len(c4) == 64
    assert all(p.nz % 2 == 0 for p in c4)
    kinds = {Geometry(p).zkind for p in c4}
    assert kinds == set(KINDS)
    c5 = W.config5(50)
    assert all(32 <= b.nx <= 512 and b.nx % 16 == 0 for r in c5 for b in r.problem.blocks)


def test_obstacle8_layout_and_routes():
    """Eight blocks around a square obstacle (Sec. 4.2): every block is joined
    to its neighbours in the 3 x 3 arrangement except across the obstacle,
    whose four sides are walls; Algorithm 1 and the dense route agree."""
    prob = W.obstacle8(4, 6)
    g = Geometry(prob)
    assert g.nb == 8
    # rows bottom (0, 1, 2), middle (3: left, 4: right), top (5, 6, 7)
    assert g.nbr == [[-1, 1, -1, 3], [0, 2, -1, -1], [1, -1, -1, 4], [-1, -1, 0, 5],
                     [-1, -1, 2, 7], [-1, 6, 3, -1], [5, 7, -1, -1], [6, -1, 4, -1]]
    assert prob.blocks[1].bc[3] == W.NEUMANN and prob.blocks[6].bc[2] == W.NEUMANN  # obstacle walls
    assert prob.blocks[3].bc[1] == W.NEUMANN and prob.blocks[4].bc[0] == W.NEUMANN
    assert prob.blocks[0].bc[0] == W.NEUMANN and prob.blocks[2].bc[1] == W.DIRICHLET  # inflow / outflow
    f = W.rhs(prob, 14, "normal")
    a = oracle.solve_alg1(prob, f)
    b = oracle.solve_dense(prob, f)
    assert oracle.rel_error(a, b) < 1e-12
    assert oracle.rel_residual(prob, a, f) < 1e-12


# ---------------------------------------------------------------------------
# Projection (Eqs. (3)-(6)): divergence and face gradient of the staggered grid
# ---------------------------------------------------------------------------

from oracle import projection as PJ  # noqa: E402


def _random_faces(prob, seed):
    nu, nv, nw = PJ.face_sizes(prob)
    rng = np.random.default_rng(seed)
    return PJ.make_consistent(prob, rng.standard_normal(nu), rng.standard_normal(nv), rng.standard_normal(nw))


@pytest.mark.parametrize("prob", _tiny_problems() + [W.obstacle8(4, 4)], ids=lambda p: p.name)
def test_divergence_of_gradient_is_the_operator(prob):
    """D G = L_h: the face gradient and divergence, written on their own,
    compose to the (independently pinned) finite-volume operator."""
    g = Geometry(prob)
    phi = np.random.default_rng(15).standard_normal(g.ncell3)
    gu, gv, gw = PJ.gradient(prob, phi)
    assert np.allclose(PJ.divergence(prob, gu, gv, gw), apply_3d(g, phi), rtol=1e-12, atol=1e-8)


@pytest.mark.parametrize("pairs", [("DD", "NN", "PP"), ("PP", "PP", "NN"), ("ND", "DN", "DD")])
def test_divergence_of_discrete_curl_vanishes(pairs):
    """u = d psi / dy, v = -d psi / dx from corner values of a stream function
    psi (constant in z, w = 0) is discretely divergence free on any spacing."""
    xp, yp, zp = pairs
    prob = W.box(9, 7, 4, 1.0, 0.8, 0.5, xp, yp, zp, xfactor=1.3 if xp != "PP" else 0.0,
                 yfactor=1.6 if yp != "PP" else 0.0)
    g = Geometry(prob)
    nx, ny, nz = 9, 7, 4
    psi = np.random.default_rng(16).standard_normal((ny + 1, nx + 1))
    if xp == "PP":
        psi[:, -1] = psi[:, 0]
    if yp == "PP":
        psi[-1, :] = psi[0, :]
    u = np.broadcast_to(np.diff(psi, axis=0)[None, :, :] / g.dcy[0][None, :, None], (nz, ny, nx + 1))
    v = np.broadcast_to(-np.diff(psi, axis=1)[None, :, :] / g.dcx[0][None, None, :], (nz, ny + 1, nx))
    nwz = nz if zp == "PP" else nz + 1
    div = PJ.divergence(prob, u.ravel(), v.ravel(), np.zeros(nwz * ny * nx))
    assert np.abs(div).max() < 1e-12 * (np.abs(u).max() / g.dcx[0].min())


def test_divergence_theorem_and_projection():
    """Gauss: sum V D u equals the net outflow through the walls; after the
    projection D u vanishes, the velocity changes by -gamma dt G Phi only, and
    a field that is already divergence free is left as it is."""
    prob = W.obstacle8(4, 6)
    g = Geometry(prob)
    u, v, w = _random_faces(prob, 17)
    us, vs, ws = PJ.split_faces(prob, u, v, w)
    flux = 0.0
    for b in range(g.nb):
        if g.nbr[b][1] < 0:
            flux += (us[b][:, :, -1] * g.dcy[b][None, :] * g.dz).sum()
        if g.nbr[b][0] < 0:
            flux -= (us[b][:, :, 0] * g.dcy[b][None, :] * g.dz).sum()
        if g.nbr[b][3] < 0:
            flux += (vs[b][:, -1, :] * g.dcx[b][None, :] * g.dz).sum()
        if g.nbr[b][2] < 0:
            flux -= (vs[b][:, 0, :] * g.dcx[b][None, :] * g.dz).sum()
    div = PJ.divergence(prob, u, v, w)
    assert abs(np.dot(g.volumes(), div) - flux) < 1e-10 * np.abs(div).sum() * g.volumes().max()
    gdt = 0.37
    u2, v2, w2, phi = PJ.project(prob, u, v, w, gdt)
    d2 = PJ.divergence(prob, u2, v2, w2)
    assert np.linalg.norm(d2) < 1e-11 * np.linalg.norm(div)
    gu, gv, gw = PJ.gradient(prob, phi)
    assert np.allclose(u2, u - gdt * gu) and np.allclose(w2, w - gdt * gw)
    u3, v3, w3, phi3 = PJ.project(prob, u2, v2, w2, gdt)
    assert np.abs(phi3).max() < 1e-9 * np.abs(phi).max()
    assert np.allclose(u3, u2, atol=1e-9 * np.abs(u2).max())
