"""The discrete operator L_h of Eq. (8), written three independent ways.

Finite-volume form on a cell-centred grid (Sec. 2: second-order finite
differences / finite volumes, spacing free to vary off the synthesis
direction):

    (L_h p)_c = sum over axes of  ( F_{c+1/2} - F_{c-1/2} ) / dc_c,
    F_{c+1/2} = ( p_{c+1} - p_c ) / df_{c+1/2},

dc = cell width (face difference), df = distance between the two cell centres
on either side of the face.  On a uniform grid this is exactly Eq. (8).
Homogeneous staggered conditions use a mirrored ghost cell one cell width
away: Neumann g = p_0 (no flux), Dirichlet g = -p_0 (zero on the face).
Across a joined or periodic face df is half the sum of the two cell widths.
z is uniform with spacing dz = lz / nz.

The Helmholtz form (L_h - alpha) p, alpha >= 0, is the operator of the
implicit-diffusion systems the paper solves "with the same numerical method"
as the pressure equation (Sec. 2; the diagonal changes every Runge-Kutta
substep, footnote of Sec. 3.3.1).  ``alpha`` defaults to 0 (Eq. (8) itself).

  * ``apply_3d``          vectorised apply on the packed multi-block field;
  * ``assemble_2d``       sparse x-y operator of one plane (for Eq. (9));
  * ``assemble_3d_dense`` dense 3D matrix built cell by cell with loops.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .grid import CONNECT, DIRICHLET, NEUMANN, PERIODIC, XM, XP, YM, YP


def second_difference_1d(kind: str, n: int) -> np.ndarray:
    """Unit-spacing 1D second difference with the ghost rules of ``kind``."""
    D = np.zeros((n, n))
    for j in range(n):
        D[j, j] = -2.0
        if j > 0:
            D[j, j - 1] = 1.0
        if j < n - 1:
            D[j, j + 1] = 1.0
    lo, hi = kind[0], kind[1]
    if lo == "P":
        D[0, n - 1] += 1.0
        D[n - 1, 0] += 1.0
        return D
    D[0, 0] += 1.0 if lo == "N" else -1.0
    D[n - 1, n - 1] += 1.0 if hi == "N" else -1.0
    return D


def fv_1d(faces: np.ndarray, lo: str, hi: str):
    """Dense 1D FV operator A (n x n) = diag(1/dc) K with K symmetric.

    Returns (A, K, dc).  ``lo``/``hi`` in {"D","N","P"}.
    """
    faces = np.asarray(faces, dtype=np.float64)
    n = len(faces) - 1
    dc = np.diff(faces)
    xc = 0.5 * (faces[1:] + faces[:-1])
    K = np.zeros((n, n))
    for c in range(n - 1):  # interior faces c+1/2
        w = 1.0 / (xc[c + 1] - xc[c])
        K[c, c] -= w
        K[c, c + 1] += w
        K[c + 1, c + 1] -= w
        K[c + 1, c] += w
    if lo == "P":
        w = 1.0 / (0.5 * (dc[0] + dc[-1]))
        K[0, 0] -= w
        K[0, n - 1] += w
        K[n - 1, n - 1] -= w
        K[n - 1, 0] += w
    else:
        if lo == "D":
            K[0, 0] -= 2.0 / dc[0]
        if hi == "D":
            K[n - 1, n - 1] -= 2.0 / dc[-1]
    A = K / dc[:, None]
    return A, K, dc


def _ghost_x(g, i, P, side):
    """Ghost column beyond face ``side`` of block i and the centre distance."""
    bc = g.bc[i][side]
    dc = g.dcx[i]
    first = 0 if side == XM else -1
    if bc in (CONNECT, PERIODIC):
        k = g.nbr[i][side]
        Pk = P[k]
        col = Pk[:, :, -1] if side == XM else Pk[:, :, 0]
        dk = g.dcx[k][-1] if side == XM else g.dcx[k][0]
        return col, 0.5 * (dc[first] + dk)
    sgn = 1.0 if bc == NEUMANN else -1.0
    return sgn * P[i][:, :, first], dc[first]


def _ghost_y(g, i, P, side):
    bc = g.bc[i][side]
    dc = g.dcy[i]
    first = 0 if side == YM else -1
    if bc in (CONNECT, PERIODIC):
        k = g.nbr[i][side]
        Pk = P[k]
        row = Pk[:, -1, :] if side == YM else Pk[:, 0, :]
        dk = g.dcy[k][-1] if side == YM else g.dcy[k][0]
        return row, 0.5 * (dc[first] + dk)
    sgn = 1.0 if bc == NEUMANN else -1.0
    return sgn * P[i][:, first, :], dc[first]


def apply_3d(g, p_flat: np.ndarray, alpha: float = 0.0) -> np.ndarray:
    """(L_h - alpha) p on the packed field (block after block, each (nz, ny, nx))."""
    P = g.split3(np.asarray(p_flat, dtype=np.float64))
    out = []
    kz = g.zkind
    for i in range(g.nb):
        Pi = P[i]
        # x fluxes
        gl, dl = _ghost_x(g, i, P, XM)
        gr, dr = _ghost_x(g, i, P, XP)
        Q = np.concatenate([gl[:, :, None], Pi, gr[:, :, None]], axis=2)
        df = np.concatenate([[dl], np.diff(g.xc[i]), [dr]])
        Fx = np.diff(Q, axis=2) / df
        Lx = np.diff(Fx, axis=2) / g.dcx[i]
        # y fluxes
        gl, dl = _ghost_y(g, i, P, YM)
        gr, dr = _ghost_y(g, i, P, YP)
        Q = np.concatenate([gl[:, None, :], Pi, gr[:, None, :]], axis=1)
        df = np.concatenate([[dl], np.diff(g.yc[i]), [dr]])
        Fy = np.diff(Q, axis=1) / df[:, None]
        Ly = np.diff(Fy, axis=1) / g.dcy[i][:, None]
        # z second difference, uniform spacing
        if kz[0] == "P":
            zl, zr = Pi[-1:], Pi[:1]
        else:
            zl = Pi[:1] * (1.0 if kz[0] == "N" else -1.0)
            zr = Pi[-1:] * (1.0 if kz[1] == "N" else -1.0)
        Q = np.concatenate([zl, Pi, zr], axis=0)
        Lz = (Q[2:] - 2.0 * Q[1:-1] + Q[:-2]) / (g.dz * g.dz)
        out.append((Lx + Ly + Lz - alpha * Pi).ravel())
    return np.concatenate(out)


def assemble_2d(g) -> sp.csr_matrix:
    """Sparse x-y FV operator A_2D on the packed plane (no z term)."""
    rows, cols, vals = [], [], []
    for i in range(g.nb):
        nx, ny = g.nx[i], g.ny[i]
        base = g.off2[i]
        J, R = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        gid = base + J * nx + R
        dcx = g.dcx[i][R]
        dcy = g.dcy[i][J]
        diag = np.zeros((ny, nx))

        def couple(mask, nb_gid, df, dcc):
            w = 1.0 / (dcc[mask] * df[mask])
            rows.append(gid[mask])
            cols.append(nb_gid[mask])
            vals.append(w)
            diag[mask] -= w

        # interior x couplings
        dfx = np.zeros((ny, nx))
        dfx[:, 1:] = np.diff(g.xc[i])[None, :]
        m = R > 0
        couple(m, gid - 1, dfx, dcx)
        dfx2 = np.zeros((ny, nx))
        dfx2[:, :-1] = np.diff(g.xc[i])[None, :]
        m = R < nx - 1
        couple(m, gid + 1, dfx2, dcx)
        dfy = np.zeros((ny, nx))
        dfy[1:, :] = np.diff(g.yc[i])[:, None]
        m = J > 0
        couple(m, gid - nx, dfy, dcy)
        dfy2 = np.zeros((ny, nx))
        dfy2[:-1, :] = np.diff(g.yc[i])[:, None]
        m = J < ny - 1
        couple(m, gid + nx, dfy2, dcy)
        # faces of the block
        for side in (XM, XP, YM, YP):
            bc = g.bc[i][side]
            if side in (XM, XP):
                c = 0 if side == XM else nx - 1
                sl = (slice(None), c)
                dc0 = g.dcx[i][c]
            else:
                c = 0 if side == YM else ny - 1
                sl = (c, slice(None))
                dc0 = g.dcy[i][c]
            if bc == NEUMANN:
                continue
            if bc == DIRICHLET:
                diag[sl] -= 2.0 / (dc0 * dc0)
                continue
            k = g.nbr[i][side]
            if side == XM:
                nb = g.off2[k] + np.arange(ny) * g.nx[k] + (g.nx[k] - 1)
                dk = g.dcx[k][-1]
            elif side == XP:
                nb = g.off2[k] + np.arange(ny) * g.nx[k]
                dk = g.dcx[k][0]
            elif side == YM:
                nb = g.off2[k] + (g.ny[k] - 1) * g.nx[k] + np.arange(nx)
                dk = g.dcy[k][-1]
            else:
                nb = g.off2[k] + np.arange(nx)
                dk = g.dcy[k][0]
            w = 1.0 / (dc0 * 0.5 * (dc0 + dk))
            rows.append(gid[sl].ravel())
            cols.append(nb)
            vals.append(np.full(nb.shape, w))
            diag[sl] -= w
        rows.append(gid.ravel())
        cols.append(gid.ravel())
        vals.append(diag.ravel())
    r = np.concatenate([np.ravel(a) for a in rows])
    c = np.concatenate([np.ravel(a) for a in cols])
    v = np.concatenate([np.ravel(a) for a in vals])
    M = g.ncell2
    return sp.coo_matrix((v, (r, c)), shape=(M, M)).tocsr()


def assemble_3d_dense(g, alpha: float = 0.0) -> np.ndarray:
    """Full 3D matrix of L_h - alpha, one cell at a time (tiny grids only)."""
    N = g.ncell3
    if N > 6000:
        raise ValueError("dense assembly is for tiny grids")
    A = np.zeros((N, N))

    def gidx(b, k, j, r):
        return g.off3[b] + (k * g.ny[b] + j) * g.nx[b] + r

    nz, dz = g.nz, g.dz
    zlo, zhi = g.zkind[0], g.zkind[1]
    for b in range(g.nb):
        nx, ny = g.nx[b], g.ny[b]
        for k in range(nz):
            for j in range(ny):
                for r in range(nx):
                    row = gidx(b, k, j, r)
                    # x direction
                    for side, step in ((XM, -1), (XP, +1)):
                        dc = g.dcx[b][r]
                        rr = r + step
                        if 0 <= rr < nx:
                            df = abs(g.xc[b][rr] - g.xc[b][r])
                            w = 1.0 / (dc * df)
                            A[row, gidx(b, k, j, rr)] += w
                            A[row, row] -= w
                        else:
                            bc = g.bc[b][side]
                            if bc == NEUMANN:
                                pass
                            elif bc == DIRICHLET:
                                A[row, row] -= 2.0 / (dc * dc)
                            else:
                                o = g.nbr[b][side]
                                ro = g.nx[o] - 1 if step < 0 else 0
                                df = 0.5 * (dc + g.dcx[o][ro])
                                w = 1.0 / (dc * df)
                                A[row, gidx(o, k, j, ro)] += w
                                A[row, row] -= w
                    # y direction
                    for side, step in ((YM, -1), (YP, +1)):
                        dc = g.dcy[b][j]
                        jj = j + step
                        if 0 <= jj < ny:
                            df = abs(g.yc[b][jj] - g.yc[b][j])
                            w = 1.0 / (dc * df)
                            A[row, gidx(b, k, jj, r)] += w
                            A[row, row] -= w
                        else:
                            bc = g.bc[b][side]
                            if bc == NEUMANN:
                                pass
                            elif bc == DIRICHLET:
                                A[row, row] -= 2.0 / (dc * dc)
                            else:
                                o = g.nbr[b][side]
                                jo = g.ny[o] - 1 if step < 0 else 0
                                df = 0.5 * (dc + g.dcy[o][jo])
                                w = 1.0 / (dc * df)
                                A[row, gidx(o, k, jo, r)] += w
                                A[row, row] -= w
                    A[row, row] -= alpha
                    # z direction (uniform)
                    w = 1.0 / (dz * dz)
                    for step, end in ((-1, zlo), (+1, zhi)):
                        kk = k + step
                        if 0 <= kk < nz:
                            A[row, gidx(b, kk, j, r)] += w
                            A[row, row] -= w
                        elif end == "P":
                            A[row, gidx(b, kk % nz, j, r)] += w
                            A[row, row] -= w
                        elif end == "D":
                            A[row, row] -= 2.0 * w
    return A
