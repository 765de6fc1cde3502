// Fused one-pass smoothing kernels for the global-memory multigrid levels.
//
// One wave owns a strip of up to 58 output columns of one block and marches
// down its rows, keeping a five-row register window.  Each step loads one
// row, relaxes the red cells of the row above it and the black cells of the
// row above that, so a whole red-black Gauss-Seidel sweep costs one read of
// p and f and one write of p.  Lanes 0-2 and 61-63 (and three rows above and
// below the strip) are halo: they are relaxed too, from the same old values
// the owning strip sees, so every strip reproduces the sweep exactly.  The
// sweep is out of place (old -> new buffer), which keeps the halo reads free
// of races between strips.  Optional fusions:
//   PRO  add the bilinear coarse-grid correction to every row as it loads
//        (prolongation + correction before the post-smoothing sweep);
//   RES  residual of the smoothed rows, area-weighted, summed into the coarse
//        rhs of the next level (pre-smoothing sweep + restriction);
//   NRM  per-strip sum of the squared residual (convergence test).
#include <type_traits>

#include "internal.h"

namespace mbp {

// One strip of the fused sweep, with the geometry of every block its halo
// meets, so a workgroup needs a single descriptor load before its bulk loads.
// Region indices: row region 0 below / 1 inside / 2 above the block, column
// region 0 left halo / 1 the block / 2 right halo.
struct MTile {
    int b, x0, w, y0, y1, bnx, bny, pad;
    int blk[3][3], off[3][3], nx[3][3], ny[3][3], cx[3][3], cy[3][3], par[3][3];
};

__device__ __forceinline__ int pick3(int i, int a, int b, int c) { return i == 0 ? a : (i == 1 ? b : c); }

template <typename T>
struct MArgs {
    const DBlock* B;   // this level
    const DBlock* Bc;  // next coarser level (PRO / RES)
    const double* dp;
    const int* ip;
    const MTile* tiles;
    int ntiles;
    const T* pold;
    T* pnew;
    const T* f;
    long long plane;
    const T* ec;       // PRO: coarse correction
    T* fc;             // RES: coarse rhs out
    T* pc;             // RES: coarse initial guess out (zeroed)
    long long plane_c;
    const double* shift;
    const int* act;
    const int* nact;
    double* part;      // NRM: per (mode, tile) partial sums
};

__device__ __forceinline__ int xcd_remap_m(int g, int n) {
    int x = g & 7, l = g >> 3;
    int per = n >> 3, rem = n & 7;
    return x * per + min(x, rem) + l;
}

template <typename T>
__device__ __forceinline__ T shfl_up1(T v) { return __shfl_up(v, 1); }
template <typename T>
__device__ __forceinline__ T shfl_dn1(T v) { return __shfl_down(v, 1); }

// Geometry of one of the (up to three) blocks a lane's column visits.
struct ColBlk {
    int id, off, nx, ny, par, cx, cy;
};

__device__ __forceinline__ ColBlk colblk(const DBlock* __restrict__ B, int id) {
    ColBlk c{};
    c.id = id;
    if (id >= 0) {
        const DBlock& d = B[id];
        c.off = d.off; c.nx = d.nx; c.ny = d.ny; c.par = d.par; c.cx = d.cx; c.cy = d.cy;
    }
    return c;
}

// Coarse correction at fine cell (ci, cj) of block `fb` (prolong_at, inlined
// here with the coarse block table of the next level).
template <typename T>
__device__ __forceinline__ T coarse_at(const T* __restrict__ pl, const DBlock* __restrict__ B, int b,
                                       int I, int J) {
    T s = T(1);
    const DBlock* bb = &B[b];
    if (J < 0) {
        if (bb->nbr[YM] >= 0) { bb = &B[bb->nbr[YM]]; J = bb->ny - 1; }
        else { if (bb->bc[YM] == MBP_DIRICHLET) s = -s; J = 0; }
    } else if (J >= bb->ny) {
        if (bb->nbr[YP] >= 0) { bb = &B[bb->nbr[YP]]; J = 0; }
        else { if (bb->bc[YP] == MBP_DIRICHLET) s = -s; J = bb->ny - 1; }
    }
    if (I < 0) {
        if (bb->nbr[XM] >= 0) { bb = &B[bb->nbr[XM]]; I = bb->nx - 1; }
        else { if (bb->bc[XM] == MBP_DIRICHLET) s = -s; I = 0; }
    } else if (I >= bb->nx) {
        if (bb->nbr[XP] >= 0) { bb = &B[bb->nbr[XP]]; I = 0; }
        else { if (bb->bc[XP] == MBP_DIRICHLET) s = -s; I = bb->nx - 1; }
    }
    return s * pl[bb->off + J * bb->nx + I];
}

template <typename T>
__device__ __forceinline__ T correction(const DBlock* __restrict__ B, const DBlock* __restrict__ Bc,
                                       const int* __restrict__ ip, const double* __restrict__ dp,
                                       const T* __restrict__ ecq, int fb, int ci, int cj) {
    const DBlock& d = B[fb];
    const int cx = ip[d.pcx + ci], cy = ip[d.pcy + cj];
    const T wx = T(dp[d.pwx + ci]), wy = T(dp[d.pwy + cj]);
    const T e00 = coarse_at(ecq, Bc, fb, cx, cy), e10 = coarse_at(ecq, Bc, fb, cx + 1, cy);
    const T e01 = coarse_at(ecq, Bc, fb, cx, cy + 1), e11 = coarse_at(ecq, Bc, fb, cx + 1, cy + 1);
    return wy * (wx * e00 + (T(1) - wx) * e10) + (T(1) - wy) * (wx * e01 + (T(1) - wx) * e11);
}

// Compile-time loop: the body gets a constant index, so per-thread arrays
// indexed by it stay in registers.
template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// ------------------------- LDS tile form of the sweep -------------------------
// Same sweep, same strips, but a workgroup loads its whole strip (rows y0-3 ..
// y1+2, 64 columns) into LDS in one burst, then relaxes red, black, computes
// the residual and restricts it with barriers between the phases.  Bulk loads
// keep many requests in flight, which the row march cannot do in float64.
constexpr int kTileRows = 30;               // output rows per strip (host cuts at this)
constexpr int kLdsRows = kTileRows + 6;

// Block met at (column region cr, virtual row k) of a strip of block tb:
// column region 0 = left halo, 1 = the block, 2 = right halo.  Beyond a
// corner: the y neighbour's x neighbour, else the x neighbour's y neighbour
// (the host rejects levels where both exist and differ).
__device__ __forceinline__ int block_at(const DBlock* __restrict__ B, int tb, int cr, int k, int bny) {
    const int colb = cr == 1 ? tb : B[tb].nbr[cr == 0 ? XM : XP];
    if (k >= 0 && k < bny) return colb;
    const int fy = k < 0 ? YM : YP;
    const int M = B[tb].nbr[fy];
    if (cr == 1) return M;
    const int fx = cr == 0 ? XM : XP;
    if (M >= 0 && B[M].nbr[fx] >= 0) return B[M].nbr[fx];
    if (colb >= 0 && B[colb].nbr[fy] >= 0) return B[colb].nbr[fy];
    return -1;
}

template <typename T>
__device__ __forceinline__ T xcoef(const DBlock* __restrict__ B, const double* __restrict__ dp, int blk,
                                   int cc, int which) {
    return blk >= 0 ? T(dp[B[blk].cx + which * B[blk].nx + cc]) : T(0);
}

template <typename T, bool PRO, bool RES, bool NRM>
__global__ void __launch_bounds__(256) k_tile(const MArgs<T> args) {
    // argument fields as scalars (no reference to the argument block survives)
    const DBlock* __restrict__ aB = args.B;
    const DBlock* __restrict__ aBc = args.Bc;
    const int* __restrict__ aip = args.ip;
    const double* __restrict__ dp = args.dp;
    const int ntiles = args.ntiles;
    const long long plane = args.plane, plane_c = args.plane_c;

    __shared__ T sp[kLdsRows][64];
    __shared__ T sf[kLdsRows][64];
    __shared__ double sy[kLdsRows][3][3];  // per row and column region: wm, wp, dy
    __shared__ int scol[kLdsRows][3];      // (row index + parity) & 1, or -1: no cell
    __shared__ double sred[4][2];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tix = xcd_remap_m(blockIdx.x, ntiles);
    const int item = blockIdx.y;
    if (item >= *args.nact) return;
    const int q = args.act[item];
    const MTile& t = args.tiles[tix];
    const int tb = t.b, tx0 = t.x0, tw = t.w, ty0 = t.y0, ty1 = t.y1;
    const int bnx = t.bnx, bny = t.bny;
    const int nrow = ty1 - ty0 + 6;
    const T sig = T(args.shift[q]);
    const T* __restrict__ po = args.pold + q * plane;
    T* __restrict__ pn = args.pnew + q * plane;
    const T* __restrict__ fq = args.f + q * plane;
    const T* __restrict__ ecq = PRO ? args.ec + q * plane_c : nullptr;

    // ---- phase 0: per-row coefficient table ----
    for (int e = threadIdx.x; e < 3 * nrow; e += blockDim.x) {
        const int r = e / 3, cr = e - 3 * r;
        const int k = ty0 - 3 + r;
        const int rr = k < 0 ? 0 : (k >= bny ? 2 : 1);
        const int blk = pick3(rr, pick3(cr, t.blk[0][0], t.blk[0][1], t.blk[0][2]),
                              pick3(cr, t.blk[1][0], t.blk[1][1], t.blk[1][2]),
                              pick3(cr, t.blk[2][0], t.blk[2][1], t.blk[2][2]));
        if (blk < 0) {
            scol[r][cr] = -1;
            sy[r][cr][0] = sy[r][cr][1] = 0.0;
            sy[r][cr][2] = 1.0;
            continue;
        }
        const int ny = pick3(rr, pick3(cr, t.ny[0][0], t.ny[0][1], t.ny[0][2]),
                             pick3(cr, t.ny[1][0], t.ny[1][1], t.ny[1][2]),
                             pick3(cr, t.ny[2][0], t.ny[2][1], t.ny[2][2]));
        const int cy = pick3(rr, pick3(cr, t.cy[0][0], t.cy[0][1], t.cy[0][2]),
                             pick3(cr, t.cy[1][0], t.cy[1][1], t.cy[1][2]),
                             pick3(cr, t.cy[2][0], t.cy[2][1], t.cy[2][2]));
        const int par = pick3(rr, pick3(cr, t.par[0][0], t.par[0][1], t.par[0][2]),
                              pick3(cr, t.par[1][0], t.par[1][1], t.par[1][2]),
                              pick3(cr, t.par[2][0], t.par[2][1], t.par[2][2]));
        const int cj = k < 0 ? ny + k : (k >= bny ? k - bny : k);
        sy[r][cr][0] = dp[cy + cj];
        sy[r][cr][1] = dp[cy + ny + cj];
        sy[r][cr][2] = dp[cy + 2 * ny + cj];
        scol[r][cr] = (cj + par) & 1;
    }

    // ---- the lane's column: region, per-row-region block and column index ----
    const int c = tx0 - 3 + lane;
    const bool live = lane < tw + 6;
    const int cr = c < 0 ? 0 : (c < bnx ? 1 : 2);
    const int b0 = live ? pick3(cr, t.blk[1][0], t.blk[1][1], t.blk[1][2]) : -1;
    const int bm = live ? pick3(cr, t.blk[0][0], t.blk[0][1], t.blk[0][2]) : -1;
    const int bp = live ? pick3(cr, t.blk[2][0], t.blk[2][1], t.blk[2][2]) : -1;
    const int nx0 = pick3(cr, t.nx[1][0], t.nx[1][1], t.nx[1][2]);
    const int nxm = pick3(cr, t.nx[0][0], t.nx[0][1], t.nx[0][2]);
    const int nxp = pick3(cr, t.nx[2][0], t.nx[2][1], t.nx[2][2]);
    const int nym = pick3(cr, t.ny[0][0], t.ny[0][1], t.ny[0][2]);
    // column index inside the region's block
    const int ci = cr == 0 ? nx0 + c : (cr == 2 ? c - bnx : c);
    const int cim = cr == 0 ? nxm + c : (cr == 2 ? c - bnx : c);
    const int cip = cr == 0 ? nxp + c : (cr == 2 ? c - bnx : c);
    const int off0 = b0 >= 0 ? pick3(cr, t.off[1][0], t.off[1][1], t.off[1][2]) + ci : 0;
    const int offm = bm >= 0 ? pick3(cr, t.off[0][0], t.off[0][1], t.off[0][2]) + cim : 0;
    const int offp = bp >= 0 ? pick3(cr, t.off[2][0], t.off[2][1], t.off[2][2]) + cip : 0;
    const int cx0 = pick3(cr, t.cx[1][0], t.cx[1][1], t.cx[1][2]);
    const int cxm = pick3(cr, t.cx[0][0], t.cx[0][1], t.cx[0][2]);
    const int cxp = pick3(cr, t.cx[2][0], t.cx[2][1], t.cx[2][2]);
    // x coefficients per row region (lane constants)
    const T xwm0 = b0 >= 0 ? T(dp[cx0 + ci]) : T(0), xwp0 = b0 >= 0 ? T(dp[cx0 + nx0 + ci]) : T(0);
    const T xd0 = b0 >= 0 ? T(dp[cx0 + 2 * nx0 + ci]) : T(0);
    const T xwmm = bm >= 0 ? T(dp[cxm + cim]) : T(0), xwpm = bm >= 0 ? T(dp[cxm + nxm + cim]) : T(0);
    const T xdm = bm >= 0 ? T(dp[cxm + 2 * nxm + cim]) : T(0);
    const T xwmp = bp >= 0 ? T(dp[cxp + cip]) : T(0), xwpp = bp >= 0 ? T(dp[cxp + nxp + cip]) : T(0);
    const T xdp = bp >= 0 ? T(dp[cxp + 2 * nxp + cip]) : T(0);

    // coarse columns of the correction for inside rows (resolved per lane)
    int cbaseA = 0, cbaseB = 0, cstrA = 0, cstrB = 0, ncyc = 0, bpcy = 0, bpwy = 0;
    T csA = T(0), csB = T(0), cwx = T(0);
    if (PRO) {
        ncyc = aBc[tb].ny;
        bpcy = aB[tb].pcy;
        bpwy = aB[tb].pwy;
        if (b0 >= 0) {
            const int cx = aip[aB[b0].pcx + ci];
            cwx = T(dp[aB[b0].pwx + ci]);
            int I = cx;
            for (int s = 0; s < 2; ++s, ++I) {
                int cb = b0, II = I;
                T sg = T(1);
                if (II < 0) {
                    if (aBc[cb].nbr[XM] >= 0) { cb = aBc[cb].nbr[XM]; II = aBc[cb].nx - 1; }
                    else { if (aBc[cb].bc[XM] == MBP_DIRICHLET) sg = T(-1); II = 0; }
                } else if (II >= aBc[cb].nx) {
                    if (aBc[cb].nbr[XP] >= 0) { cb = aBc[cb].nbr[XP]; II = 0; }
                    else { if (aBc[cb].bc[XP] == MBP_DIRICHLET) sg = T(-1); II = aBc[cb].nx - 1; }
                }
                if (s == 0) { cbaseA = aBc[cb].off + II; cstrA = aBc[cb].nx; csA = sg; }
                else { cbaseB = aBc[cb].off + II; cstrB = aBc[cb].nx; csB = sg; }
            }
        }
    }

    // ---- phase 1: load p and f of every held row.  All loads of the strip
    //      are issued first (constant trip count, values in registers), then
    //      written to LDS, so they overlap in flight. ----
    constexpr int NR = (kLdsRows + 3) / 4;
    T lp[NR], lf[NR];
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) {
        const int r = wave + 4 * rr;
        const int k = ty0 - 3 + r;
        lp[rr] = T(0);
        lf[rr] = T(0);
        if (r >= nrow) continue;
        const bool below = k < 0, above = k >= bny;
        const bool alive = below ? bm >= 0 : (above ? bp >= 0 : b0 >= 0);
        if (!alive) continue;
        const int o = below ? offm + (nym + k) * nxm : (above ? offp + (k - bny) * nxp : off0 + k * nx0);
        lp[rr] = po[o];
        lf[rr] = fq[o];
    }
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) {
        const int r = wave + 4 * rr;
        if (r >= nrow) continue;
        sp[r][lane] = lp[rr];
        sf[r][lane] = lf[rr];
    }
    // coarse-grid correction of the held rows (bilinear, physical weights)
    if (PRO) {
#pragma unroll 3
        for (int rr = 0; rr < NR; ++rr) {
            const int r = wave + 4 * rr;
            if (r >= nrow) continue;
            const int k = ty0 - 3 + r;
            const bool below = k < 0, above = k >= bny;
            const bool alive = below ? bm >= 0 : (above ? bp >= 0 : b0 >= 0);
            if (!alive) continue;
            T corr;
            const int cy = (!below && !above) ? aip[bpcy + k] : -1;
            if (!below && !above && cy >= 0 && cy + 1 < ncyc) {
                const T wy = T(dp[bpwy + k]);
                corr = wy * (cwx * csA * ecq[cbaseA + cy * cstrA] + (T(1) - cwx) * csB * ecq[cbaseB + cy * cstrB]) +
                       (T(1) - wy) * (cwx * csA * ecq[cbaseA + (cy + 1) * cstrA] +
                                      (T(1) - cwx) * csB * ecq[cbaseB + (cy + 1) * cstrB]);
            } else if (below) {
                corr = correction(aB, aBc, aip, dp, ecq, bm, cim, nym + k);
            } else if (above) {
                corr = correction(aB, aBc, aip, dp, ecq, bp, cip, k - bny);
            } else {
                corr = correction(aB, aBc, aip, dp, ecq, b0, ci, k);
            }
            sp[r][lane] += corr;
        }
    }
    __syncthreads();

    // ---- phases 2 and 3: red on rows 1 .. nrow-2 / lanes 1 .. 62, then black
    //      on rows 2 .. nrow-3 / lanes 2 .. 61 (the valid region shrinks) ----
    for (int colour = 0; colour < 2; ++colour) {
        if (lane >= 1 + colour && lane <= 62 - colour) {
            for (int r = wave; r < nrow; r += 4) {
                if (r < 1 + colour || r > nrow - 2 - colour) continue;
                const int k = ty0 - 3 + r;
                const int sc = scol[r][cr];
                const bool below = k < 0, above = k >= bny;
                const bool alive = below ? bm >= 0 : (above ? bp >= 0 : b0 >= 0);
                if (sc < 0 || !alive) continue;
                const int cc = below ? cim : (above ? cip : ci);
                if (((cc + sc) & 1) != colour) continue;
                const T wm = below ? xwmm : (above ? xwmp : xwm0);
                const T wp = below ? xwpm : (above ? xwpp : xwp0);
                const T xd = below ? xdm : (above ? xdp : xd0);
                const T d = xd + T(sy[r][cr][2]) + sig;
                const T off = wm * sp[r][lane - 1] + wp * sp[r][lane + 1] + T(sy[r][cr][0]) * sp[r - 1][lane] +
                              T(sy[r][cr][1]) * sp[r + 1][lane];
                sp[r][lane] = (sf[r][lane] - off) / d;
            }
        }
        __syncthreads();
    }
    // ---- phase 4: store, residual (weighted residual kept in sf for the restriction) ----
    const bool out_lane = lane >= 3 && lane < 3 + tw;
    const T wrx = (RES && out_lane) ? T(dp[aB[tb].rwx + c]) : T(0);
    const int rwy = aB[tb].rwy;
    double nrm = 0.0, pnr = 0.0;
    for (int r = wave; r < nrow; r += 4) {
        const int k = ty0 - 3 + r;
        const bool own = r >= 3 && k < ty1 && out_lane;
        if (own) {
            const T pc = sp[r][lane];
            pn[off0 + k * nx0] = pc;
            if (RES || NRM) {
                const T d = xd0 + T(sy[r][1][2]) + sig;
                const T res = sf[r][lane] - (xwm0 * sp[r][lane - 1] + xwp0 * sp[r][lane + 1] +
                                             T(sy[r][1][0]) * sp[r - 1][lane] + T(sy[r][1][1]) * sp[r + 1][lane] + d * pc);
                if (NRM) {
                    nrm += double(res) * double(res);
                    pnr += double(pc) * double(pc);
                }
                if (RES) sf[r][lane] = res * wrx * T(dp[rwy + k]);
            }
        } else if (RES) {
            sf[r][lane] = T(0);
        }
    }
    if (RES) {
        __syncthreads();
        // leaders: first fine column / row of each coarse cell inside the strip
        const int ncx = aBc[tb].nx, ncy = aBc[tb].ny, bcoff = aBc[tb].off;
        if (out_lane && c == 2 * min(c >> 1, ncx - 1)) {
            const int I = min(c >> 1, ncx - 1);
            const int i1 = (I == ncx - 1) ? bnx : 2 * I + 2;  // exclusive fine end
            for (int r = wave; r < nrow; r += 4) {
                const int k = ty0 - 3 + r;
                if (r < 3 || k >= ty1) continue;
                const int J = min(k >> 1, ncy - 1);
                if (k != 2 * J) continue;
                const int j1 = (J == ncy - 1) ? bny : 2 * J + 2;
                T s = T(0);
                for (int kk = k; kk < j1; ++kk)
                    for (int x = c; x < i1; ++x) s += sf[r + (kk - k)][lane + (x - c)];
                const long long o = q * plane_c + bcoff + (long long)J * ncx + I;
                args.fc[o] = s;
                args.pc[o] = T(0);
            }
        }
    }
    if (NRM) {
        for (int o = 32; o > 0; o >>= 1) {
            nrm += __shfl_xor(nrm, o);
            pnr += __shfl_xor(pnr, o);
        }
        if (lane == 0) { sred[wave][0] = nrm; sred[wave][1] = pnr; }
        __syncthreads();
        if (threadIdx.x == 0) {
            args.part[2 * ((long long)q * ntiles + tix)] = sred[0][0] + sred[1][0] + sred[2][0] + sred[3][0];
            args.part[2 * ((long long)q * ntiles + tix) + 1] = sred[0][1] + sred[1][1] + sred[2][1] + sred[3][1];
        }
    }
}

// ------------------------------- host side -------------------------------

// Strips of one level: x ranges of at most 58 columns and y ranges of at most
// `seg` rows, both cut at coarse-cell boundaries of the next level so that a
// strip owns whole coarse cells (the last coarse cell of an odd count spans
// three fine cells).
void march_build_tiles(const mbp_plan* P, int l, int seg, std::vector<MTile>& out) {
    const Level& L = P->levels[l];
    const bool has_coarse = l + 1 < P->nlev;
    for (int b = 0; b < L.nb; ++b) {
        auto cuts = [&](int n, int nc, int maxw) __attribute__((always_inline)) {
            std::vector<int> edges{0};
            int start = 0;
            for (int I = 0; I < (has_coarse ? nc : n); ++I) {
                const int lo = has_coarse ? 2 * I : I;
                const int hi = has_coarse ? (I == nc - 1 ? n : 2 * I + 2) : I + 1;
                if (hi - start > maxw) {
                    edges.push_back(lo);
                    start = lo;
                }
            }
            edges.push_back(n);
            return edges;
        };
        const int ncx = has_coarse ? P->levels[l + 1].nx[b] : 0;
        const int ncy = has_coarse ? P->levels[l + 1].ny[b] : 0;
        std::vector<int> ex = cuts(L.nx[b], ncx, 58);
        std::vector<int> ey = cuts(L.ny[b], ncy, seg);
        // block met at (row region rr, column region cr), same rule as the halo lanes
        const Geometry& g = P->g;
        auto at = [&](int rr, int cr) {
            const int colb = cr == 1 ? b : g.nbr[b][cr == 0 ? XM : XP];
            if (rr == 1) return colb;
            const int fy = rr == 0 ? YM : YP;
            const int M = g.nbr[b][fy];
            if (cr == 1) return M;
            const int fx = cr == 0 ? XM : XP;
            if (M >= 0 && g.nbr[M][fx] >= 0) return g.nbr[M][fx];
            if (colb >= 0 && g.nbr[colb][fy] >= 0) return g.nbr[colb][fy];
            return -1;
        };
        MTile base{};
        base.b = b;
        base.bnx = L.nx[b];
        base.bny = L.ny[b];
        for (int rr = 0; rr < 3; ++rr)
            for (int cr = 0; cr < 3; ++cr) {
                const int k = at(rr, cr);
                base.blk[rr][cr] = k;
                if (k < 0) continue;
                const DBlock& d = P->hblk[L.blk_off + k];
                base.off[rr][cr] = d.off;
                base.nx[rr][cr] = d.nx;
                base.ny[rr][cr] = d.ny;
                base.cx[rr][cr] = d.cx;
                base.cy[rr][cr] = d.cy;
                base.par[rr][cr] = d.par;
            }
        for (size_t yi = 0; yi + 1 < ey.size(); ++yi)
            for (size_t xi = 0; xi + 1 < ex.size(); ++xi) {
                MTile t = base;
                t.x0 = ex[xi];
                t.w = ex[xi + 1] - ex[xi];
                t.y0 = ey[yi];
                t.y1 = ey[yi + 1];
                out.push_back(t);
            }
    }
}

void march_build_tiles_bytes(const mbp_plan* P, int l, int seg, std::vector<unsigned char>& out, int* count) {
    std::vector<MTile> t;
    march_build_tiles(P, l, seg, t);
    *count = int(t.size());
    out.assign(reinterpret_cast<unsigned char*>(t.data()),
               reinterpret_cast<unsigned char*>(t.data()) + t.size() * sizeof(MTile));
}

// The march needs every block at the level to be at least four cells wide
// in both directions (halo lanes and rows stay inside partner blocks), no odd
// periodic wrap, and unambiguous corners: the cell diagonally beyond a block
// corner, reached through the y neighbour's x neighbour or through the x
// neighbour's y neighbour, must be the same block whenever both routes exist.
bool march_level_ok(const mbp_plan* P, int l) {
    const Level& L = P->levels[l];
    const Geometry& g = P->g;
    for (int b = 0; b < L.nb; ++b) {
        if (L.nx[b] < 4 || L.ny[b] < 4) return false;
        if (P->hblk[L.blk_off + b].oddwrap) return false;
        for (int fy : {int(YM), int(YP)})
            for (int fx : {int(XM), int(XP)}) {
                const int M = g.nbr[b][fy], N = g.nbr[b][fx];
                const int a1 = (M >= 0) ? g.nbr[M][fx] : -1;
                const int a2 = (N >= 0) ? g.nbr[N][fy] : -1;
                if (a1 >= 0 && a2 >= 0 && a1 != a2) return false;
            }
    }
    return true;
}

template <typename T>
static MArgs<T> margs(const mbp_plan* P, int l, const T* pold, T* pnew, const T* f, const T* ec, T* fc,
                      T* pc, const int* act, const int* nact) {
    MArgs<T> a{};
    a.B = P->d_blk + P->levels[l].blk_off;
    a.Bc = l + 1 < P->nlev ? P->d_blk + P->levels[l + 1].blk_off : nullptr;
    a.dp = P->d_dbl;
    a.ip = P->d_int;
    a.tiles = reinterpret_cast<const MTile*>(P->d_mtiles) + P->mtile_off[l];
    a.ntiles = P->mtile_cnt[l];
    a.pold = pold;
    a.pnew = pnew;
    a.f = f;
    a.plane = P->levels[l].plane;
    a.ec = ec;
    a.fc = fc;
    a.pc = pc;
    a.plane_c = l + 1 < P->nlev ? P->levels[l + 1].plane : 0;
    a.shift = P->d_shift;
    a.act = act;
    a.nact = nact;
    a.part = P->d_part;
    return a;
}

template <typename T, bool PRO, bool RES, bool NRM>
static void launch_march(const MArgs<T>& a, int nitems, hipStream_t s) {
    hipLaunchKernelGGL((k_tile<T, PRO, RES, NRM>), dim3(a.ntiles, nitems), dim3(256), 0, s, a);
}

// Pre-smoothing sweep of level l (old -> new) fused with the residual
// restriction into level l+1 (rhs fc, initial guess pc = 0).
template <typename T>
void march_pre(const mbp_plan* P, int l, const T* pold, T* pnew, const T* f, T* fc, T* pc,
               const int* act, const int* nact, int nitems, hipStream_t s) {
    MArgs<T> a = margs<T>(P, l, pold, pnew, f, nullptr, fc, pc, act, nact);
    launch_march<T, false, true, false>(a, nitems, s);
}

// Plain sweep (extra smoothing steps).
template <typename T>
void march_sweep(const mbp_plan* P, int l, const T* pold, T* pnew, const T* f, const int* act,
                 const int* nact, int nitems, hipStream_t s) {
    MArgs<T> a = margs<T>(P, l, pold, pnew, f, nullptr, nullptr, nullptr, act, nact);
    launch_march<T, false, false, false>(a, nitems, s);
}

// Coarse-grid correction from level l+1 (ec) fused with a post-smoothing
// sweep; with norm, per-strip squared residuals go to the partial buffer.
template <typename T>
void march_post(const mbp_plan* P, int l, const T* pold, T* pnew, const T* f, const T* ec, bool norm,
                const int* act, const int* nact, int nitems, hipStream_t s) {
    MArgs<T> a = margs<T>(P, l, pold, pnew, f, ec, nullptr, nullptr, act, nact);
    if (norm) launch_march<T, true, false, true>(a, nitems, s);
    else launch_march<T, true, false, false>(a, nitems, s);
}

template void march_pre<double>(const mbp_plan*, int, const double*, double*, const double*, double*,
                                double*, const int*, const int*, int, hipStream_t);
template void march_pre<float>(const mbp_plan*, int, const float*, float*, const float*, float*, float*,
                               const int*, const int*, int, hipStream_t);
template void march_sweep<double>(const mbp_plan*, int, const double*, double*, const double*,
                                  const int*, const int*, int, hipStream_t);
template void march_sweep<float>(const mbp_plan*, int, const float*, float*, const float*, const int*,
                                 const int*, int, hipStream_t);
template void march_post<double>(const mbp_plan*, int, const double*, double*, const double*,
                                 const double*, bool, const int*, const int*, int, hipStream_t);
template void march_post<float>(const mbp_plan*, int, const float*, float*, const float*, const float*,
                                bool, const int*, const int*, int, hipStream_t);

}  // namespace mbp
