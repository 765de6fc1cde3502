"""Direct FP64 solutions of L_h p = f (test infrastructure only).

``solve_alg1`` follows Algorithm 1: transform the rhs along the homogeneous
direction with the eigenfunctions of Table 1, solve the decoupled 2D systems
of Eq. (9),

    (A_2D + lambda_q / dz^2) phat_q = fhat_q,   q = 0..nz-1,

one per mode (here by sparse LU instead of multigrid: the method's result is
the exact discrete solution, so a direct solve is its plain definition), then
transform back.  ``solve_separable`` diagonalises all three 1D operators of a
single box (the direct matrix-decomposition route the paper describes for
simple boxes, Sec. 2).  ``solve_dense`` assembles the whole 3D matrix.

Every route also takes the Helmholtz shift ``alpha`` >= 0 and then solves
(L_h - alpha) p = f, the implicit-diffusion systems of Sec. 2 (same method;
in Eq. (9) the shift of mode q becomes lambda_q / dz^2 - alpha).  With
alpha > 0 no problem is singular.

Singular problems (no Dirichlet condition anywhere, alpha = 0): the rhs must be
compatible, sum(V f) = 0 with V the cell volumes (``project_compatible``
enforces it), and the solution is returned with zero volume-weighted mean.
In Eq. (9) this affects only a mode with lambda_q = 0 on an x-y plane without
Dirichlet faces; it is solved with the area-bordered system
[[A, a], [a^T, 0]], which pins sum(a phat) = 0.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .grid import Geometry, DIRICHLET, NEUMANN, PERIODIC, XM, XP, YM, YP
from .operator import apply_3d, assemble_2d, assemble_3d_dense, fv_1d
from .transforms import basis, eigenvalues


def _geom(problem):
    return problem if isinstance(problem, Geometry) else Geometry(problem)


def is_singular(problem, alpha: float = 0.0) -> bool:
    return alpha == 0.0 and not _geom(problem).has_dirichlet()


def project_compatible(problem, f: np.ndarray) -> np.ndarray:
    """f minus its volume-weighted mean (the range condition of L_h)."""
    g = _geom(problem)
    V = g.volumes()
    return f - np.dot(V, f) / V.sum()


def remove_mean(problem, p: np.ndarray) -> np.ndarray:
    g = _geom(problem)
    V = g.volumes()
    return p - np.dot(V, p) / V.sum()


def residual(problem, p, f, alpha: float = 0.0):
    return f - apply_3d(_geom(problem), p, alpha)


def rel_residual(problem, p, f, alpha: float = 0.0) -> float:
    return float(np.linalg.norm(residual(problem, p, f, alpha)) / np.linalg.norm(f))


def rel_error(p, p_ref) -> float:
    return float(np.linalg.norm(p - p_ref) / np.linalg.norm(p_ref))


# ---------------------------------------------------------------------------
# Algorithm 1
# ---------------------------------------------------------------------------

def _to_modes(g, f_flat, T):
    """fhat[q, plane] = sum_k T[k, q] f[k, plane] for every block."""
    parts = []
    for fb in g.split3(f_flat):
        parts.append((T.T @ fb.reshape(g.nz, -1)))
    return np.concatenate(parts, axis=1)


def _from_modes(g, phat, T):
    parts = []
    for i in range(g.nb):
        blk = phat[:, g.off2[i]:g.off2[i + 1]]
        parts.append((T @ blk).ravel())
    return np.concatenate(parts)


def modal_rhs(problem, f: np.ndarray, qs) -> np.ndarray:
    """fhat_q for the listed modes only (rows), packed plane layout."""
    g = _geom(problem)
    T = basis(g.zkind, g.nz)[:, list(qs)]
    return _to_modes(g, f, T)


def modal_values(problem, p: np.ndarray, qs) -> np.ndarray:
    """Same contraction for a solution field (to compare in mode space)."""
    return modal_rhs(problem, p, qs)


def _plane_factor(g, A2, sigma, singular2d):
    M = g.ncell2
    A = (A2 + sigma * sp.identity(M, format="csr")).tocsc()
    if not singular2d:
        return spla.splu(A), False
    a = g.areas()
    Ab = sp.bmat([[A, sp.csc_matrix(a[:, None])], [sp.csr_matrix(a[None, :]), None]]).tocsc()
    return spla.splu(Ab), True


def _plane_solve(lu_b, rhs):
    lu, bordered = lu_b
    if bordered:
        x = lu.solve(np.concatenate([rhs, [0.0]]))
        return x[:-1]
    return lu.solve(rhs)


def solve_mode(problem, fhat_q: np.ndarray, q: int, A2=None, alpha: float = 0.0) -> np.ndarray:
    """Solve Eq. (9) for one mode q (sparse LU)."""
    g = _geom(problem)
    lam = eigenvalues(g.zkind, g.nz)[q]
    if A2 is None:
        A2 = assemble_2d(g)
    sing = (lam == 0.0) and alpha == 0.0 and not g.has_dirichlet_xy()
    fac = _plane_factor(g, A2, lam / (g.dz * g.dz) - alpha, sing)
    rhs = fhat_q
    if sing:
        a = g.areas()
        rhs = fhat_q - np.dot(a, fhat_q) / a.sum()
    return _plane_solve(fac, rhs)


def _pool_job(args):
    """Worker: factor one shifted plane and solve its modes (runs in a child
    process; the problem description is rebuilt there)."""
    problem, sigma, sing, rows = args
    g = _geom(problem)
    fac = _plane_factor(g, assemble_2d(g), sigma, sing)
    return np.stack([_plane_solve(fac, r) for r in rows])


def _one_thread_per_worker():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:  # pragma: no cover - threadpoolctl missing
        pass


def _solve_groups_in_pool(problem, g, fhat, phat, jobs, workers):
    import concurrent.futures as cf
    import multiprocessing as mp
    ctx = mp.get_context("spawn")  # fresh interpreters: no state of the parent is inherited
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=ctx,
                                initializer=_one_thread_per_worker) as ex:
        futs = {ex.submit(_pool_job, (problem, sigma, sing, fhat[qs])): qs for qs, sigma, sing in jobs}
        for fu in cf.as_completed(futs):
            qs = futs[fu]
            phat[qs] = fu.result()


def solve_alg1(problem, f: np.ndarray, project: bool = True, alpha: float = 0.0,
               workers: int = 1) -> np.ndarray:
    """Algorithm 1 with a sparse direct solve per mode.  ``workers`` > 1 runs
    the independent per-shift solves in that many processes (the modes are
    decoupled, so the result is the same; only the wall time changes)."""
    g = _geom(problem)
    f = np.asarray(f, dtype=np.float64)
    singular = alpha == 0.0 and not g.has_dirichlet()
    if singular and project:
        f = project_compatible(g, f)
    T = basis(g.zkind, g.nz)
    lam = eigenvalues(g.zkind, g.nz)
    fhat = _to_modes(g, f, T)                      # forward transform
    sing_xy = alpha == 0.0 and not g.has_dirichlet_xy()
    # modes sharing one shift (the periodic pairs q, n - q) share one factor
    groups = {}
    for q in range(g.nz):
        key = (float(np.round(lam[q], 12)), bool((lam[q] == 0.0) and sing_xy))
        groups.setdefault(key, []).append(q)
    phat = np.empty_like(fhat)
    jobs = [(qs, lam[qs[0]] / (g.dz * g.dz) - alpha, sing) for (_, sing), qs in groups.items()]
    if workers <= 1:
        A2 = assemble_2d(g)
        for qs, sigma, sing in jobs:               # one 2D solve per mode
            fac = _plane_factor(g, A2, sigma, sing)
            for q in qs:
                phat[q] = _plane_solve(fac, fhat[q])
    else:
        _solve_groups_in_pool(problem, g, fhat, phat, jobs, workers)
    p = _from_modes(g, phat, T)                    # inverse transform
    if singular:
        p = remove_mean(g, p)
    return p


# ---------------------------------------------------------------------------
# Separable direct solve (single box, any spacing)
# ---------------------------------------------------------------------------

def _axis_pair(bc_lo, bc_hi):
    names = {DIRICHLET: "D", NEUMANN: "N", PERIODIC: "P"}
    return names[bc_lo], names[bc_hi]


def _eig_axis(faces, lo, hi):
    A, K, dc = fv_1d(faces, lo, hi)
    s = np.sqrt(dc)
    S = K / s[:, None] / s[None, :]
    S = 0.5 * (S + S.T)
    mu, V = np.linalg.eigh(S)
    W = V / s[:, None]          # columns: eigenvectors of A
    Winv = V.T * s[None, :]     # W^{-1}
    return mu, W, Winv


def solve_separable(problem, f: np.ndarray, project: bool = True, alpha: float = 0.0) -> np.ndarray:
    g = _geom(problem)
    if g.nb != 1:
        raise ValueError("separable route needs a single box")
    b = g.blocks[0]
    f = np.asarray(f, dtype=np.float64)
    singular = alpha == 0.0 and not g.has_dirichlet()
    if singular and project:
        f = project_compatible(g, f)
    mux, Wx, Wix = _eig_axis(g.xf[0], *_axis_pair(b.bc[XM], b.bc[XP]))
    muy, Wy, Wiy = _eig_axis(g.yf[0], *_axis_pair(b.bc[YM], b.bc[YP]))
    zf = np.linspace(0.0, g.lz, g.nz + 1)
    muz, Wz, Wiz = _eig_axis(zf, g.zkind[0], g.zkind[1])
    F = f.reshape(g.nz, g.ny[0], g.nx[0])
    C = F @ Wix.T                                        # x
    C = np.einsum("jy,kyx->kjx", Wiy, C, optimize=True)  # y
    C = (Wiz @ C.reshape(g.nz, -1)).reshape(C.shape)     # z
    den = muz[:, None, None] + muy[None, :, None] + mux[None, None, :] - alpha
    if singular:
        k0, j0, i0 = int(np.argmax(muz)), int(np.argmax(muy)), int(np.argmax(mux))
        den[k0, j0, i0] = 1.0
        C[k0, j0, i0] = 0.0
    C = C / den
    P = (Wz @ C.reshape(g.nz, -1)).reshape(C.shape)
    P = np.einsum("yj,kjx->kyx", Wy, P, optimize=True)
    P = P @ Wx.T
    p = P.ravel()
    if singular:
        p = remove_mean(g, p)
    return p


# ---------------------------------------------------------------------------
# Dense 3D solve (tiny grids)
# ---------------------------------------------------------------------------

def solve_dense(problem, f: np.ndarray, project: bool = True, alpha: float = 0.0) -> np.ndarray:
    g = _geom(problem)
    f = np.asarray(f, dtype=np.float64)
    A = assemble_3d_dense(g, alpha)
    singular = alpha == 0.0 and not g.has_dirichlet()
    if not singular:
        return sla.solve(A, f)
    if project:
        f = project_compatible(g, f)
    V = g.volumes()
    N = len(f)
    Ab = np.zeros((N + 1, N + 1))
    Ab[:N, :N] = A
    Ab[:N, N] = V
    Ab[N, :N] = V
    x = sla.solve(Ab, np.concatenate([f, [0.0]]))
    return x[:N]


def solve(problem, f: np.ndarray, project: bool = True, alpha: float = 0.0, workers: int = 1) -> np.ndarray:
    """Direct solution by the cheapest applicable route."""
    g = _geom(problem)
    if g.nb == 1:
        return solve_separable(g, f, project, alpha)
    return solve_alg1(problem, f, project, alpha, workers)
