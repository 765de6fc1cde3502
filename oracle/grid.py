"""Multi-block geometry as the oracle reads it (Sec. 3.1, Table 2).

Blocks are given in index space by inclusive corners lo/hi; a face marked
CONNECT is joined to the block whose opposite face touches it in index space
over exactly the same tangential range (every face has at most one
neighbour, Sec. 3.1).  A PERIODIC face on the lower side of a block is joined
to the PERIODIC upper face of the block with the same tangential range
(cyclic connectivity, Sec. 3.1); on a single block it wraps onto itself.

Cell centres are face midpoints; a cell's width is its face difference.
"""
from __future__ import annotations

import numpy as np

DIRICHLET, NEUMANN, CONNECT, PERIODIC = 1, 2, 3, 4
XM, XP, YM, YP = 0, 1, 2, 3


def pair_kind(lo: int, hi: int) -> str:
    names = {DIRICHLET: "D", NEUMANN: "N", PERIODIC: "P"}
    k = names[lo] + names[hi]
    if k not in ("PP", "NN", "DD", "ND", "DN"):
        raise ValueError(f"invalid z condition pair {k}")
    return k


class Geometry:
    def __init__(self, problem):
        self.blocks = list(problem.blocks)
        self.nb = len(self.blocks)
        self.nz = int(problem.nz)
        self.lz = float(problem.lz)
        self.dz = self.lz / self.nz
        self.zkind = pair_kind(*problem.zbc)
        self.nx = [b.hi[0] - b.lo[0] + 1 for b in self.blocks]
        self.ny = [b.hi[1] - b.lo[1] + 1 for b in self.blocks]
        self.xf = [np.asarray(b.xf, dtype=np.float64) for b in self.blocks]
        self.yf = [np.asarray(b.yf, dtype=np.float64) for b in self.blocks]
        for i, b in enumerate(self.blocks):
            if len(self.xf[i]) != self.nx[i] + 1 or len(self.yf[i]) != self.ny[i] + 1:
                raise ValueError("face arrays must hold n+1 coordinates")
        self.dcx = [np.diff(x) for x in self.xf]
        self.dcy = [np.diff(y) for y in self.yf]
        self.xc = [0.5 * (x[1:] + x[:-1]) for x in self.xf]
        self.yc = [0.5 * (y[1:] + y[:-1]) for y in self.yf]
        self.bc = [tuple(b.bc) for b in self.blocks]
        self.nbr = [[-1] * 4 for _ in range(self.nb)]
        self._connect()
        # offsets of each block in a packed 2D plane and in a packed 3D field
        self.off2 = [0]
        for i in range(self.nb):
            self.off2.append(self.off2[-1] + self.nx[i] * self.ny[i])
        self.ncell2 = self.off2[-1]
        self.off3 = [self.nz * o for o in self.off2]
        self.ncell3 = self.off3[-1]

    def _connect(self):
        B = self.blocks
        for i, b in enumerate(B):
            for f in range(4):
                kind = b.bc[f]
                if kind in (DIRICHLET, NEUMANN):
                    continue
                axis = 0 if f in (XM, XP) else 1
                t = 1 - axis
                cands = []
                for k, c in enumerate(B):
                    if (c.lo[t], c.hi[t]) != (b.lo[t], b.hi[t]):
                        continue
                    opp = f ^ 1
                    if c.bc[opp] != kind:
                        continue
                    if kind == CONNECT:
                        if f in (XM, YM) and c.hi[axis] + 1 == b.lo[axis]:
                            cands.append(k)
                        if f in (XP, YP) and b.hi[axis] + 1 == c.lo[axis]:
                            cands.append(k)
                    else:
                        cands.append(k)
                if len(cands) != 1:
                    raise ValueError(f"block {i} face {f}: {len(cands)} neighbours")
                self.nbr[i][f] = cands[0]
        for i in range(self.nb):
            for f in range(4):
                k = self.nbr[i][f]
                if k >= 0 and self.nbr[k][f ^ 1] != i:
                    raise ValueError("connectivity is not symmetric")
        # congruence: tangential faces of joined blocks must coincide (Sec. 3.1)
        for i in range(self.nb):
            for f in range(4):
                k = self.nbr[i][f]
                if k < 0:
                    continue
                a = self.yf[i] if f in (XM, XP) else self.xf[i]
                c = self.yf[k] if f in (XM, XP) else self.xf[k]
                if len(a) != len(c):
                    raise ValueError("joined faces differ in cell count")
                if self.bc[i][f] == CONNECT and not np.allclose(a, c, rtol=1e-12, atol=1e-12):
                    raise ValueError("joined faces are not congruent")

    # --- helpers -----------------------------------------------------------
    def has_dirichlet(self) -> bool:
        if "D" in self.zkind:
            return True
        return any(DIRICHLET in bc for bc in self.bc)

    def has_dirichlet_xy(self) -> bool:
        return any(DIRICHLET in bc for bc in self.bc)

    def areas(self) -> np.ndarray:
        """Cell areas of the packed 2D plane."""
        return np.concatenate([np.outer(self.dcy[i], self.dcx[i]).ravel() for i in range(self.nb)])

    def volumes(self) -> np.ndarray:
        """Cell volumes of the packed 3D field (uniform dz)."""
        parts = []
        for i in range(self.nb):
            a = np.outer(self.dcy[i], self.dcx[i]) * self.dz
            parts.append(np.broadcast_to(a, (self.nz,) + a.shape).ravel())
        return np.concatenate(parts)

    def split3(self, flat):
        return [flat[self.off3[i]:self.off3[i + 1]].reshape(self.nz, self.ny[i], self.nx[i])
                for i in range(self.nb)]

    def split2(self, flat):
        return [flat[..., self.off2[i]:self.off2[i + 1]].reshape(flat.shape[:-1] + (self.ny[i], self.nx[i]))
                for i in range(self.nb)]
