"""Pressure projection around the Poisson solve (test infrastructure only).

The fractional step of Eqs. (3)-(6): from a predicted velocity u* on the
staggered grid (Sec. 2: staggered flow variables, velocities on cell
faces),

    rhs = D u* / (gamma dt),   L_h Phi = rhs,   u = u* - gamma dt G Phi,

after which D u = 0 up to the solver's tolerance, the check the paper uses
to verify its Poisson solver and projection (Sec. 4.1).  D is the
finite-volume divergence (face fluxes over the cell width) and G the face
gradient (centre difference over the centre distance), so that D G = L_h
with the conditions of Sec. 3.1: a Neumann face (prescribed normal velocity)
has G Phi = 0 and keeps its velocity; a Dirichlet face (prescribed
pressure) has the mirrored ghost Phi_g = -Phi_0; a joined or periodic face
uses the partner's cell at half the sum of the two widths.

Face fields are packed like cell fields, block after block:
  u (x faces)  (nz, ny, nx + 1)
  v (y faces)  (nz, ny + 1, nx)
  w (z faces)  (nz, ny, nx) when z is periodic (face k - 1/2, cyclic),
               (nz + 1, ny, nx) otherwise.
A face shared by two joined blocks appears in both; ``make_consistent``
copies the lower block's value into its partner's slot.
"""
from __future__ import annotations

import numpy as np

from .grid import DIRICHLET, NEUMANN, XM, XP, YM, YP
from .solve import _geom, solve


def _nzw(g) -> int:
    return g.nz if g.zkind == "PP" else g.nz + 1


def face_sizes(problem):
    """Element counts of the packed u, v, w fields."""
    g = _geom(problem)
    nu = sum(g.nz * g.ny[b] * (g.nx[b] + 1) for b in range(g.nb))
    nv = sum(g.nz * (g.ny[b] + 1) * g.nx[b] for b in range(g.nb))
    nw = sum(_nzw(g) * g.ny[b] * g.nx[b] for b in range(g.nb))
    return nu, nv, nw


def split_faces(problem, u, v, w):
    """Per-block views (nz, ny, nx+1), (nz, ny+1, nx), (nzw, ny, nx)."""
    g = _geom(problem)
    us, vs, ws = [], [], []
    ou = ov = ow = 0
    for b in range(g.nb):
        nx, ny = g.nx[b], g.ny[b]
        n = g.nz * ny * (nx + 1)
        us.append(u[ou:ou + n].reshape(g.nz, ny, nx + 1))
        ou += n
        n = g.nz * (ny + 1) * nx
        vs.append(v[ov:ov + n].reshape(g.nz, ny + 1, nx))
        ov += n
        n = _nzw(g) * ny * nx
        ws.append(w[ow:ow + n].reshape(_nzw(g), ny, nx))
        ow += n
    return us, vs, ws


def make_consistent(problem, u, v, w):
    """Copies of (u, v, w) in which every face shared by two blocks (or by a
    periodic block with itself) holds one value: the partner across a +x / +y
    face receives the value of the block below or left of it."""
    g = _geom(problem)
    u, v, w = u.copy(), v.copy(), w.copy()
    us, vs, ws = split_faces(problem, u, v, w)
    for b in range(g.nb):
        k = g.nbr[b][XP]
        if k >= 0:
            us[k][:, :, 0] = us[b][:, :, -1]
        k = g.nbr[b][YP]
        if k >= 0:
            vs[k][:, 0, :] = vs[b][:, -1, :]
    return u, v, w


def divergence(problem, u, v, w) -> np.ndarray:
    """D u: packed cell field of (flux differences) / (cell widths)."""
    g = _geom(problem)
    us, vs, ws = split_faces(problem, u, v, w)
    out = []
    for b in range(g.nb):
        d = (np.diff(us[b], axis=2) / g.dcx[b][None, None, :] +
             np.diff(vs[b], axis=1) / g.dcy[b][None, :, None])
        wb = ws[b]
        if g.zkind == "PP":
            wb = np.concatenate([wb, wb[:1]], axis=0)  # face nz - 1/2 is face -1/2
        d = d + np.diff(wb, axis=0) / g.dz
        out.append(d.ravel())
    return np.concatenate(out)


def gradient(problem, phi):
    """G Phi on the faces (packed u, v, w shapes)."""
    g = _geom(problem)
    P = g.split3(np.asarray(phi, dtype=np.float64))
    gu, gv, gw = [], [], []
    for b in range(g.nb):
        p = P[b]
        nz, ny, nx = p.shape
        # x faces
        x = np.zeros((nz, ny, nx + 1))
        x[:, :, 1:nx] = np.diff(p, axis=2) / np.diff(g.xc[b])[None, None, :]
        for side, col in ((XM, 0), (XP, nx)):
            bc = g.bc[b][side]
            first = p[:, :, 0] if side == XM else p[:, :, -1]
            dc = g.dcx[b][0] if side == XM else g.dcx[b][-1]
            if bc == NEUMANN:
                x[:, :, col] = 0.0
            elif bc == DIRICHLET:
                x[:, :, col] = (2.0 * first / dc) if side == XM else (-2.0 * first / dc)
            else:
                k = g.nbr[b][side]
                q = P[k]
                if side == XM:
                    x[:, :, col] = (p[:, :, 0] - q[:, :, -1]) / (0.5 * (dc + g.dcx[k][-1]))
                else:
                    x[:, :, col] = (q[:, :, 0] - p[:, :, -1]) / (0.5 * (dc + g.dcx[k][0]))
        # y faces
        y = np.zeros((nz, ny + 1, nx))
        y[:, 1:ny, :] = np.diff(p, axis=1) / np.diff(g.yc[b])[None, :, None]
        for side, row in ((YM, 0), (YP, ny)):
            bc = g.bc[b][side]
            first = p[:, 0, :] if side == YM else p[:, -1, :]
            dc = g.dcy[b][0] if side == YM else g.dcy[b][-1]
            if bc == NEUMANN:
                y[:, row, :] = 0.0
            elif bc == DIRICHLET:
                y[:, row, :] = (2.0 * first / dc) if side == YM else (-2.0 * first / dc)
            else:
                k = g.nbr[b][side]
                q = P[k]
                if side == YM:
                    y[:, row, :] = (p[:, 0, :] - q[:, -1, :]) / (0.5 * (dc + g.dcy[k][-1]))
                else:
                    y[:, row, :] = (q[:, 0, :] - p[:, -1, :]) / (0.5 * (dc + g.dcy[k][0]))
        # z faces (uniform)
        if g.zkind == "PP":
            z = (p - np.roll(p, 1, axis=0)) / g.dz
        else:
            z = np.zeros((nz + 1, ny, nx))
            z[1:nz] = np.diff(p, axis=0) / g.dz
            lo, hi = g.zkind[0], g.zkind[1]
            z[0] = 0.0 if lo == "N" else 2.0 * p[0] / g.dz
            z[nz] = 0.0 if hi == "N" else -2.0 * p[-1] / g.dz
        gu.append(x.ravel())
        gv.append(y.ravel())
        gw.append(z.ravel())
    return np.concatenate(gu), np.concatenate(gv), np.concatenate(gw)


def project(problem, u, v, w, gamma_dt: float):
    """One projection step: returns (u, v, w, Phi) after the correction."""
    rhs = divergence(problem, u, v, w) / gamma_dt
    phi = solve(problem, rhs)  # singular problems: rhs made compatible, Phi gauged
    gu, gv, gw = gradient(problem, phi)
    return u - gamma_dt * gu, v - gamma_dt * gv, w - gamma_dt * gw, phi
