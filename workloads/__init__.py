"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module describes problems (block layout, face coordinates, boundary
conditions, the homogeneous z direction) and draws right-hand sides.  It holds
none of the solver's arithmetic: no operator, transform, projection or solve.
Both the oracle and the HIP path receive exactly the arrays built here.

Problem model (the paper's problem statement, Sec. 3.1 and Table 2):
  * the x-y cross-section is a set of logically rectangular blocks given in
    index space by inclusive corners ``lo``/``hi`` (cells = hi - lo + 1), with
    physical face coordinates ``xf`` (nx+1) and ``yf`` (ny+1) per block;
  * every block face is Dirichlet, Neumann, connected to the block that touches
    it in index space, or periodic (cyclic connection);
  * z is uniform with ``nz`` cells on ``[0, lz)`` and a boundary-condition pair
    at its two ends (Table 1 rows, plus Dirichlet-Neumann).
Unknowns are cell-centred; the packed field stores block after block, each in
C order ``(nz, ny, nx)`` (x fastest).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np

# Face / end conditions.  Values are part of the C ABI as well.
DIRICHLET = 1
NEUMANN = 2
CONNECT = 3
PERIODIC = 4

BC_NAMES = {DIRICHLET: "D", NEUMANN: "N", CONNECT: "C", PERIODIC: "P"}

# The five valid conditions pairs along a direction (lower end, upper end).
PAIRS = {
    "PP": (PERIODIC, PERIODIC),
    "NN": (NEUMANN, NEUMANN),
    "DD": (DIRICHLET, DIRICHLET),
    "ND": (NEUMANN, DIRICHLET),
    "DN": (DIRICHLET, NEUMANN),
}
PAIR_CYCLE = ["PP", "NN", "DD", "ND", "DN"]


@dataclasses.dataclass
class Block:
    lo: Tuple[int, int]
    hi: Tuple[int, int]
    xf: np.ndarray
    yf: np.ndarray
    bc: Tuple[int, int, int, int]  # (-x, +x, -y, +y)

    @property
    def nx(self) -> int:
        return self.hi[0] - self.lo[0] + 1

    @property
    def ny(self) -> int:
        return self.hi[1] - self.lo[1] + 1


@dataclasses.dataclass
class Problem:
    blocks: List[Block]
    nz: int
    lz: float
    zbc: Tuple[int, int]
    name: str = ""

    @property
    def ncells(self) -> int:
        return self.nz * sum(b.nx * b.ny for b in self.blocks)

    def block_offsets(self) -> List[int]:
        off = [0]
        for b in self.blocks:
            off.append(off[-1] + self.nz * b.nx * b.ny)
        return off

    def split(self, flat: np.ndarray) -> List[np.ndarray]:
        """Views of a packed field as one (nz, ny, nx) array per block."""
        off = self.block_offsets()
        return [flat[off[i]:off[i + 1]].reshape(self.nz, b.ny, b.nx)
                for i, b in enumerate(self.blocks)]


# ---------------------------------------------------------------------------
# Face coordinates.  Hyperbolic-tangent clustering (Sec. 3.1, Table 2 caption:
# type 0 clusters at both ends, -1 / +1 at the lower / upper end, factor 0 is
# uniform).  The paper does not print the mapping; the profile used here is
# x(s) = (1 + tanh(a (s - 1/2)) / tanh(a / 2)) / 2 for two-sided clustering.
# ---------------------------------------------------------------------------

def faces(n: int, lmin: float, lmax: float, gtype: int = 0, factor: float = 0.0) -> np.ndarray:
    s = np.arange(n + 1, dtype=np.float64) / n
    a = float(factor)
    if a == 0.0:
        x = s
    elif gtype == 0:
        x = 0.5 * (1.0 + np.tanh(a * (s - 0.5)) / math.tanh(0.5 * a))
    elif gtype == -1:
        x = 1.0 + np.tanh(a * (s - 1.0)) / math.tanh(a)
    elif gtype == 1:
        x = np.tanh(a * s) / math.tanh(a)
    else:
        raise ValueError("grid type must be 0, -1 or +1")
    x[0], x[-1] = 0.0, 1.0
    return lmin + (lmax - lmin) * x


def box(nx: int, ny: int, nz: int, lx: float, ly: float, lz: float,
        xpair: str, ypair: str, zpair: str,
        xfactor: float = 0.0, yfactor: float = 0.0, name: str = "") -> Problem:
    """One block on [0,lx] x [0,ly] x [0,lz) with the given condition pairs."""
    bx, by = PAIRS[xpair], PAIRS[ypair]
    blk = Block(lo=(1, 1), hi=(nx, ny),
                xf=faces(nx, 0.0, lx, 0, xfactor if xpair != "PP" else 0.0),
                yf=faces(ny, 0.0, ly, 0, yfactor if ypair != "PP" else 0.0),
                bc=(bx[0], bx[1], by[0], by[1]))
    return Problem(blocks=[blk], nz=nz, lz=lz, zbc=PAIRS[zpair], name=name)


# ---------------------------------------------------------------------------
# Workloads.  Shapes follow the paper's cases: the single-box cavity (Sec. 4),
# the three-block L-shaped duct (Sec. 4.2) and batches / streams of boxes.
# ---------------------------------------------------------------------------

def config1() -> Problem:
    """32^3 box on [0,1]^3: Dirichlet x, Neumann y, periodic z."""
    return box(32, 32, 32, 1.0, 1.0, 1.0, "DD", "NN", "PP", name="box32_DD_NN_PP")


def lshape(n: int = 256, nz: int = 512, factor: float = 1.5, lz: float = 2.0) -> Problem:
    """Three-block L-shaped cross-section: A=[0,1]^2, B=[1,2]x[0,1], C=[0,1]x[1,2].

    n x n cells per block, y clustered two-sided (tanh) toward the walls of
    each block, x uniform, Neumann on every outer wall, periodic z.
    """
    N, C = NEUMANN, CONNECT
    xa = faces(n, 0.0, 1.0)
    xb = faces(n, 1.0, 2.0)
    ya = faces(n, 0.0, 1.0, 0, factor)
    yc = faces(n, 1.0, 2.0, 0, factor)
    A = Block((1, 1), (n, n), xa, ya, (N, C, N, C))
    B = Block((n + 1, 1), (2 * n, n), xb, ya.copy(), (C, N, N, N))
    Cb = Block((1, n + 1), (n, 2 * n), xa.copy(), yc, (N, N, C, N))
    return Problem(blocks=[A, B, Cb], nz=nz, lz=lz, zbc=PAIRS["PP"],
                   name=f"lshape3x{n}^2x{nz}_stretch{factor}")


def obstacle8(n: int = 64, nz: int = 576, lz_per_h: float = 9.0) -> Problem:
    """Eight blocks around a square obstacle of side H = 1 (Sec. 4.2, the flow
    around a square cylinder): a 3 x 3 arrangement of blocks with the centre
    one removed.  Widths along x: 2H upstream, H, 2H downstream; heights H
    below, H, H above (the performance setup shrinks the top, bottom and
    downstream blocks by 3 from a 3H / 6H layout).  n cells per H, uniform
    spacing; z periodic with nz cells on [0, lz_per_h * H * nz / 576) so that
    dz = H / 64 at nz = 576.  Pressure-correction conditions: Neumann at the
    inflow (x = 0) and on the obstacle walls, Dirichlet (zero pressure) at the
    outflow, top and bottom."""
    D, N, C = DIRICHLET, NEUMANN, CONNECT
    widths, heights = [2, 1, 2], [1, 1, 1]  # in units of H
    x0 = [0, 2, 3, 5]
    y0 = [0, 1, 2, 3]
    blocks = []
    for row in range(3):
        for col in range(3):
            if row == 1 and col == 1:
                continue
            nx, ny = widths[col] * n, heights[row] * n
            lo = (x0[col] * n + 1, y0[row] * n + 1)
            hi = (lo[0] + nx - 1, lo[1] + ny - 1)
            bxm = N if col == 0 else (N if (row == 1 and col == 2) else C)
            bxp = D if col == 2 else (N if (row == 1 and col == 0) else C)
            bym = D if row == 0 else (N if (col == 1 and row == 2) else C)
            byp = D if row == 2 else (N if (col == 1 and row == 0) else C)
            blocks.append(Block(lo, hi, faces(nx, float(x0[col]), float(x0[col + 1])),
                                faces(ny, float(y0[row]), float(y0[row + 1])), (bxm, bxp, bym, byp)))
    lz = lz_per_h * nz / 576.0
    return Problem(blocks=blocks, nz=nz, lz=lz, zbc=PAIRS["PP"], name=f"obstacle8_{n}perH_nz{nz}")


def disparate(kind: str, nz: int = 8, zpair: str = "PP") -> Problem:
    """Blocks of very different sizes joined along whole faces, square cells
    of width 1/64 unless stated.  These are the layouts where one thin block
    cannot follow its neighbours down the multigrid hierarchy.
      "thin_wide":   a 4 x 64 block left of a 256 x 64 block (x faces joined);
      "stacked":     an 8 x 8 block below an 8 x 200 block (y faces joined);
      "sandwich":    128 x 96, 4 x 96 and 64 x 96 blocks side by side, the
                     middle one with cells half as wide;
      "large":       a 6 x 128 block left of a 512 x 128 block;
      "sliver1", "sliver2": a 1- or 2-cell-wide block between two 64 x 64
                     blocks (x faces joined)."""
    D, N, C = DIRICHLET, NEUMANN, CONNECT
    h = 1.0 / 64.0
    if kind == "thin_wide":
        blocks = [Block((1, 1), (4, 64), faces(4, 0.0, 4 * h), faces(64, 0.0, 1.0), (D, C, N, N)),
                  Block((5, 1), (260, 64), faces(256, 4 * h, 260 * h), faces(64, 0.0, 1.0), (C, N, N, D))]
    elif kind == "stacked":
        blocks = [Block((1, 1), (8, 8), faces(8, 0.0, 8 * h), faces(8, 0.0, 8 * h), (D, N, N, C)),
                  Block((1, 9), (8, 208), faces(8, 0.0, 8 * h), faces(200, 8 * h, 208 * h), (N, N, C, N))]
    elif kind == "sandwich":
        blocks = [Block((1, 1), (128, 96), faces(128, 0.0, 2.0), faces(96, 0.0, 1.5), (D, C, N, N)),
                  Block((129, 1), (132, 96), faces(4, 2.0, 2.0 + 2 * h), faces(96, 0.0, 1.5), (C, C, N, N)),
                  Block((133, 1), (196, 96), faces(64, 2.0 + 2 * h, 3.0 + 2 * h), faces(96, 0.0, 1.5),
                        (C, N, D, N))]
    elif kind == "large":
        blocks = [Block((1, 1), (6, 128), faces(6, 0.0, 6 * h), faces(128, 0.0, 2.0), (N, C, N, N)),
                  Block((7, 1), (518, 128), faces(512, 6 * h, 518 * h), faces(128, 0.0, 2.0), (C, D, N, N))]
    elif kind in ("sliver1", "sliver2"):
        w = 1 if kind == "sliver1" else 2
        blocks = [Block((1, 1), (64, 64), faces(64, 0.0, 1.0), faces(64, 0.0, 1.0), (D, C, N, N)),
                  Block((65, 1), (64 + w, 64), faces(w, 1.0, 1.0 + w * h), faces(64, 0.0, 1.0), (C, C, N, N)),
                  Block((65 + w, 1), (128 + w, 64), faces(64, 1.0 + w * h, 2.0 + w * h), faces(64, 0.0, 1.0),
                        (C, N, N, D))]
    else:
        raise ValueError(kind)
    return Problem(blocks=blocks, nz=nz, lz=0.5, zbc=PAIRS[zpair], name=f"disparate_{kind}_{zpair}_{nz}")


def random_layout(seed: int, scale: int = 1) -> Problem:
    """A seeded multi-block layout for sweeps of the hierarchy and halo code:
    a row of 2-4 blocks joined across x faces, a column of 2-4 joined across
    y faces, an L of three blocks or a 2 x 2 grid of four.  Block widths are
    1..40 cells of width 1/32 (thin blocks included), the shared faces of a
    row or column are mildly tanh-stretched (factor up to 0.8), outer faces
    are Dirichlet or Neumann at random, and z takes a random pair and an even
    count up to 16.  Seeds from 100 on close half of the rows and columns into
    periodic rings (the two end faces joined cyclically; ring lengths may be
    odd).  scale > 1 multiplies the wide blocks' cell counts (not the thin
    ones') and divides the cell width, so the fused strip kernels see the
    same kinds of layouts on planes of tens of thousands of cells."""
    rng = np.random.default_rng(np.random.SeedSequence([7, seed]))
    ring = seed >= 100 and rng.random() < 0.5
    D, N, C, P = DIRICHLET, NEUMANN, CONNECT, PERIODIC
    h = 1.0 / (32.0 * scale)
    kind = int(rng.integers(0, 4))
    wall = lambda: D if rng.random() < 0.5 else N  # noqa: E731

    def stretched(n, lo):
        return faces(n, lo, lo + n * h, 0, float(rng.uniform(0.0, 0.8)))

    def widths(k):
        return [int(rng.choice([1, 2, 3, 4, 5])) if rng.random() < 0.3 else scale * int(rng.integers(6, 41))
                for _ in range(k)]
    blocks = []
    if kind == 0:  # row: x faces joined, shared y faces
        k = int(rng.integers(2, 5))
        nxs, ny = widths(k), scale * int(rng.integers(4, 41))
        yf = stretched(ny, 0.0)
        x0, i0 = 0.0, 1
        for b, nx in enumerate(nxs):
            bc = (P if ring else wall()) if b == 0 else C, (P if ring else wall()) if b == k - 1 else C
            bc = (bc[0], bc[1], wall(), wall())
            blocks.append(Block((i0, 1), (i0 + nx - 1, ny), faces(nx, x0, x0 + nx * h), yf.copy(), bc))
            x0 += nx * h
            i0 += nx
    elif kind == 1:  # column: y faces joined, shared x faces
        k = int(rng.integers(2, 5))
        nys, nx = widths(k), scale * int(rng.integers(4, 41))
        xf = stretched(nx, 0.0)
        y0, j0 = 0.0, 1
        for b, ny in enumerate(nys):
            bc = (wall(), wall(), (P if ring else wall()) if b == 0 else C,
                  (P if ring else wall()) if b == k - 1 else C)
            blocks.append(Block((1, j0), (nx, j0 + ny - 1), xf.copy(), faces(ny, y0, y0 + ny * h), bc))
            y0 += ny * h
            j0 += ny
    else:
        na, nb = widths(2)
        ma, mb = scale * int(rng.integers(4, 41)), scale * int(rng.integers(4, 41))
        xa, xb = stretched(na, 0.0), faces(nb, na * h, (na + nb) * h)
        ya, yb = stretched(ma, 0.0), faces(mb, ma * h, (ma + mb) * h)
        if kind == 2:  # L: A, B right of A, C above A
            blocks = [Block((1, 1), (na, ma), xa, ya, (wall(), C, wall(), C)),
                      Block((na + 1, 1), (na + nb, ma), xb, ya.copy(), (C, wall(), wall(), wall())),
                      Block((1, ma + 1), (na, ma + mb), xa.copy(), yb, (wall(), wall(), C, wall()))]
        else:  # 2 x 2 grid
            blocks = [Block((1, 1), (na, ma), xa, ya, (wall(), C, wall(), C)),
                      Block((na + 1, 1), (na + nb, ma), xb, ya.copy(), (C, wall(), wall(), C)),
                      Block((1, ma + 1), (na, ma + mb), xa.copy(), yb, (wall(), C, C, wall())),
                      Block((na + 1, ma + 1), (na + nb, ma + mb), xb.copy(), yb.copy(), (C, wall(), C, wall()))]
    zk = ["PP", "NN", "DD", "ND", "DN"][int(rng.integers(0, 5))]
    nz = int(rng.choice([2, 4, 6, 8, 12, 16]))
    sc = "" if scale == 1 else f"x{scale}"
    return Problem(blocks=blocks, nz=nz, lz=nz * h, zbc=PAIRS[zk],
                   name=f"random{seed}{sc}_{['row', 'col', 'L', 'grid'][kind]}_{zk}")


def config2() -> Problem:
    return lshape(256, 512, 1.5, 2.0)


def config3() -> Problem:
    """512 x 512 x 1024 box on [0,1]x[0,1]x[0,2]: Dirichlet x, Neumann y, Neumann z."""
    return box(512, 512, 1024, 1.0, 1.0, 2.0, "DD", "NN", "NN", name="box512x512x1024_DD_NN_NN")


H_ISO = 1.0 / 128.0  # isotropic base spacing of the batched and served boxes


def config4(count: int = 64) -> List[Problem]:
    """Batch of boxes of uneven size with the condition pairs cycled per axis."""
    seeds = np.random.SeedSequence(4).spawn(count)
    out = []
    xy_choices = np.arange(64, 385, 32)
    z_choices = np.arange(64, 257, 32)
    for i, ss in enumerate(seeds):
        rng = np.random.default_rng(ss)
        nx = int(rng.choice(xy_choices))
        ny = int(rng.choice(xy_choices))
        nz = int(rng.choice(z_choices))
        zp = PAIR_CYCLE[i % 5]
        xp = PAIR_CYCLE[(i // 5) % 5]
        yp = PAIR_CYCLE[(i // 25 + i) % 5]
        out.append(box(nx, ny, nz, nx * H_ISO, ny * H_ISO, nz * H_ISO, xp, yp, zp,
                       name=f"batch{i}_{nx}x{ny}x{nz}_{xp}{yp}{zp}"))
    return out


def _log_uniform16(rng, lo=32, hi=512) -> int:
    v = math.exp(rng.uniform(math.log(lo), math.log(hi)))
    return int(min(hi, max(lo, 16 * round(v / 16))))


@dataclasses.dataclass
class Request:
    problem: Problem
    arrival_s: float
    seed: int


def config5(count: int = 1000, rate_per_s: float = 100.0, seed: int = 5,
            max_cells: int | None = None) -> List[Request]:
    """Poisson-process stream of solve requests (exponential gaps at ``rate_per_s``).

    Each of nx, ny, nz is log-uniform in [32, 512] rounded to a multiple of 16,
    every axis draws its condition pair uniformly from the five kinds, and
    non-periodic x / y axes are clustered two-sided with a factor in [1, 2].
    ``max_cells`` (optional) redraws requests larger than that many cells.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    i = 0
    while len(out) < count:
        t += rng.exponential(1.0 / rate_per_s)
        nx, ny, nz = (_log_uniform16(rng) for _ in range(3))
        xp, yp, zp = (PAIR_CYCLE[int(rng.integers(5))] for _ in range(3))
        a = float(rng.uniform(1.0, 2.0))
        b = float(rng.uniform(1.0, 2.0))
        req_seed = int(rng.integers(2**31 - 1))
        if max_cells is not None and nx * ny * nz > max_cells:
            continue
        p = box(nx, ny, nz, nx * H_ISO, ny * H_ISO, nz * H_ISO, xp, yp, zp,
                xfactor=a, yfactor=b, name=f"req{i}_{nx}x{ny}x{nz}_{xp}{yp}{zp}")
        out.append(Request(problem=p, arrival_s=t, seed=req_seed))
        i += 1
    return out


# ---------------------------------------------------------------------------
# Right-hand sides: raw samples only (no compatibility projection here).
# ---------------------------------------------------------------------------

def rhs(problem: Problem, seed: int, dist: str = "uniform") -> np.ndarray:
    """Packed float64 rhs, block after block in block order, each (nz, ny, nx)."""
    rng = np.random.default_rng(seed)
    parts = []
    for b in problem.blocks:
        shape = (problem.nz, b.ny, b.nx)
        if dist == "uniform":
            parts.append(rng.uniform(-1.0, 1.0, size=shape).ravel())
        elif dist == "normal":
            parts.append(rng.standard_normal(size=shape).ravel())
        else:
            raise ValueError(dist)
    return np.concatenate(parts)


CONFIG_SEEDS = {1: 1, 2: 2, 3: 3, 4: 4, 5: 5}
CONFIG_DIST = {1: "uniform", 2: "normal", 3: "uniform", 4: "uniform", 5: "uniform"}
