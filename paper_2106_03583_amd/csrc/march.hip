// Fused one-pass smoothing kernels for the global-memory multigrid levels.
//
// A workgroup owns a strip of one block: up to 58 output columns and 26
// output rows, held in LDS with three halo columns and rows on every side
// (rows and columns of neighbouring blocks across joined faces).  One
// launch runs a whole red-black Gauss-Seidel sweep out of place (old -> new
// buffer), so a sweep costs one read of p and f and one write of p; the halo
// cells are relaxed too, from the same old values the owning strip sees, so
// every strip reproduces the global sweep exactly.  Optional fusions:
//   PRO  add the bilinear coarse-grid correction before the sweep
//        (prolongation + correction + post-smoothing);
//   RES  residual of the smoothed cells, area-weighted and summed into the
//        coarse rhs of the next level (pre-smoothing + restriction);
//   NRM  per-wave sums of the squared residual and solution (convergence).
// A workgroup runs several modes of its strip in turn, issuing the loads of
// the next mode before relaxing the current one.
#include <algorithm>
#include <map>
#include <mutex>
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
    int per;           // modes per workgroup (consecutive active items)
    int zero_in;       // the old iterate is zero: pold is not read
    int wg_target;     // host: workgroups a launch aims at (modes per workgroup follow)
};

constexpr int kMaxModes = 16;  // most modes one workgroup runs in turn

__device__ __forceinline__ int xcd_remap_m(int g, int n) {
    int x = g & 7, l = g >> 3;
    int per = n >> 3, rem = n & 7;
    return x * per + min(x, rem) + l;
}

// ------------------------- LDS tile form of the sweep -------------------------
// A workgroup owns one strip (rows y0-3 .. y1+2, 64 columns) and runs the
// sweep for up to kMaxModes modes of it in turn.  The strip geometry (row
// and lane tables) is set up once; the loads of the next mode (p, f and the
// coarse correction rows) are issued before the current mode is relaxed, so
// they are in flight during its compute.  p and f are staged in LDS.  Phases per mode: stage p (+ correction), red, black, store with the
// residual, restriction / norm.
constexpr int kTileRows = 26;               // output rows per strip (host cuts at this)
constexpr int kLdsRows = kTileRows + 6;
constexpr int kRowsPerWave = kLdsRows / 4;  // contiguous rows per wave
constexpr int kWaveCoarse = 6;              // coarse rows of the correction staged per wave
static_assert(kLdsRows % 4 == 0, "four waves share the strip rows");
static_assert(2 * (kWaveCoarse - 2) + 1 >= kRowsPerWave, "a wave's rows fit its coarse rows");

// Sum over the 64 lanes of a wave with DPP moves (no LDS round trips);
// lane 63 ends up with the total.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// a / d by a hardware reciprocal refined with Newton-Raphson steps and one
// residual correction of the quotient (d is a nonzero diagonal of moderate
// magnitude here; within an ulp or two of the rounded quotient).
__device__ __forceinline__ double div_nr(double a, double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    const double q = a * r;
    return fma(fma(-d, q, a), r, q);
}
__device__ __forceinline__ float div_nr(float a, float d) {
    float r = __builtin_amdgcn_rcpf(d);
    r = fmaf(r, fmaf(-d, r, 1.0f), r);
    const float q = a * r;
    return fmaf(fmaf(-d, q, a), r, q);
}

__device__ __forceinline__ double wave_sum63(double v) {
    v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]: every lane holds its quad's sum
    v += dpp_move<0x114>(v);  // row_shr:4
    v += dpp_move<0x118>(v);  // row_shr:8: lane 15 of each row holds the row's sum
    v += dpp_move<0x142>(v);  // row_bcast:15
    v += dpp_move<0x143>(v);  // row_bcast:31
    return v;
}
constexpr int kNoRow = -1000000;            // row table: not a row of the strip's own block

// Offset and sign of coarse value (I, J) of block b, one cell beyond a face
// allowed: y first (neighbour or mirror), then x, as the prolongation
// resolves a coarse value beyond a face.
template <typename T>
__device__ __forceinline__ int coarse_addr(const DBlock* __restrict__ B, int b, int I, int J, T& sign) {
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
    sign = s;
    return bb->off + J * bb->nx + I;
}

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

template <typename T, bool PRO, bool RES, bool NRM>
__device__ __forceinline__ void tile_sweep(const MArgs<T> args, int bx, int by) {
    // argument fields as scalars (no reference to the argument block survives)
    const DBlock* __restrict__ aB = args.B;
    const DBlock* __restrict__ aBc = args.Bc;
    const int* __restrict__ aip = args.ip;
    const double* __restrict__ dp = args.dp;
    const int ntiles = args.ntiles;
    const int per = args.per;
    const long long plane = args.plane, plane_c = args.plane_c;
    const T* __restrict__ pold = args.pold;
    T* __restrict__ pnew = args.pnew;
    const T* __restrict__ fsrc = args.f;
    const T* __restrict__ ec = args.ec;

    __shared__ T sp[kLdsRows][64];
    __shared__ T sf[kLdsRows][64];
    __shared__ T sE[PRO ? 4 : 1][PRO ? kWaveCoarse : 1][64];  // per wave: x-interpolated coarse rows
    __shared__ double sy[kLdsRows][3][3];        // per row and column region: wm, wp, dy
    __shared__ int scol[kLdsRows][3];            // (row index + parity) & 1, or -1: no cell
    __shared__ int scy[kLdsRows];                // PRO: coarse lower row of inside rows, kNoRow else
    __shared__ double swy[kLdsRows];             // PRO: weight of that row; RES: row restriction weight
    __shared__ int sgo[PRO ? 6 : 1][64];         // PRO: coarse column A, B offsets: ghost row below,
    __shared__ T sgw[PRO ? 6 : 1][64];           //      ghost row above, inside rows; weights with signs
    __shared__ T sxc[2][3][64];                  // x coefficients of the halo rows below / above
    __shared__ int shA[PRO ? 2 : 1][3][4][64];   // PRO: halo rows of other blocks below / above:
    __shared__ T shW[PRO ? 2 : 1][3][4][64];     //      coarse offsets and signed weights per corner
    __shared__ int sq[kMaxModes];
    __shared__ double ssig[kMaxModes];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tix = xcd_remap_m(bx, ntiles);
    const int nact = *args.nact;
    const int i0 = by * per;
    const int i1 = min(i0 + per, nact);
    if (i0 >= i1) return;
    const MTile& t = args.tiles[tix];
    const int tb = t.b, tx0 = t.x0, tw = t.w, ty0 = t.y0, ty1 = t.y1;
    const int bnx = t.bnx, bny = t.bny;
    const int nrow = ty1 - ty0 + 6;

    // ---- strip tables (once per workgroup) ----
    if (threadIdx.x < i1 - i0) {
        const int q = args.act[i0 + threadIdx.x];
        sq[threadIdx.x] = q;
        ssig[threadIdx.x] = args.shift[q];
    }
    int ncyc = 0, bpcy = 0, bpwy = 0;
    if (PRO) {
        ncyc = aBc[tb].ny;
        bpcy = aB[tb].pcy;
        bpwy = aB[tb].pwy;
    }
    const int rwy = RES ? aB[tb].rwy : 0;
    for (int e = threadIdx.x; e < 3 * nrow; e += blockDim.x) {
        const int r = e / 3, cr = e - 3 * r;
        const int k = ty0 - 3 + r;
        const int rr = k < 0 ? 0 : (k >= bny ? 2 : 1);
        if (cr == 1) {
            if (PRO) {
                scy[r] = rr == 1 ? aip[bpcy + k] : kNoRow;
                swy[r] = rr == 1 ? dp[bpwy + k] : 0.0;
            } else if (RES) {
                swy[r] = rr == 1 ? dp[rwy + k] : 0.0;
            }
        }
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
    if (wave == 0) {
        sxc[0][0][lane] = bm >= 0 ? T(dp[cxm + cim]) : T(0);
        sxc[0][1][lane] = bm >= 0 ? T(dp[cxm + nxm + cim]) : T(0);
        sxc[0][2][lane] = bm >= 0 ? T(dp[cxm + 2 * nxm + cim]) : T(0);
        sxc[1][0][lane] = bp >= 0 ? T(dp[cxp + cip]) : T(0);
        sxc[1][1][lane] = bp >= 0 ? T(dp[cxp + nxp + cip]) : T(0);
        sxc[1][2][lane] = bp >= 0 ? T(dp[cxp + 2 * nxp + cip]) : T(0);
    }

    // the wave's rows: offsets inside the plane and which of them hold a cell
    const int rbase = wave * kRowsPerWave;
    int roff[kRowsPerWave];
    unsigned amask = 0;
#pragma unroll
    for (int m = 0; m < kRowsPerWave; ++m) {
        const int r = rbase + m;
        const int k = ty0 - 3 + r;
        const bool below = k < 0, above = k >= bny;
        const bool alive = r < nrow && (below ? bm >= 0 : (above ? bp >= 0 : b0 >= 0));
        roff[m] = !alive ? 0 : (below ? offm + (nym + k) * nxm : (above ? offp + (k - bny) * nxp : off0 + k * nx0));
        amask |= alive ? (1u << m) : 0u;
    }

    // coarse columns of the correction for inside rows (resolved per lane)
    int cstrA = 0, cstrB = 0;
    if (PRO && b0 >= 0) {
        const int cx = aip[aB[b0].pcx + ci];
        const T cwx = T(dp[aB[b0].pwx + ci]);
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
            if (s == 0) { cstrA = aBc[cb].nx; }
            else { cstrB = aBc[cb].nx; }
            if (wave == 2) {
                sgo[4 + s][lane] = aBc[cb].off + II;
                sgw[4 + s][lane] = sg * (s == 0 ? cwx : T(1) - cwx);
            }
        }
        // ghost coarse rows below (J = -1) and above (J = ncyc), resolved from
        // this lane's block the same way as the cell-by-cell correction
        if (wave < 2) {
            const int J = wave == 0 ? -1 : ncyc;
            T sa, sb;
            const int oa = coarse_addr(aBc, b0, cx, J, sa);
            const int ob = coarse_addr(aBc, b0, cx + 1, J, sb);
            sgo[2 * wave][lane] = oa;
            sgo[2 * wave + 1][lane] = ob;
            sgw[2 * wave][lane] = sa * cwx;
            sgw[2 * wave + 1][lane] = sb * (T(1) - cwx);
        }
    } else if (PRO && wave < 3) {
        sgo[2 * wave][lane] = sgo[2 * wave + 1][lane] = 0;
        sgw[2 * wave][lane] = sgw[2 * wave + 1][lane] = T(0);
    }
    // correction of the halo rows that lie in other blocks: the four coarse
    // offsets and signed bilinear weights of every such cell, resolved once
    // (the same rules as the cell-by-cell correction)
    if (PRO) {
        for (int e = threadIdx.x; e < 2 * 3 * 64; e += blockDim.x) {
            const int side = e / 192, j = (e / 64) % 3, ln = e % 64;
            const int r = side == 0 ? j : nrow - 3 + j;
            const int k = ty0 - 3 + r;
            const int cl = tx0 - 3 + ln;
            const int crl = cl < 0 ? 0 : (cl < bnx ? 1 : 2);
            int fb = -1, fi = 0, fj = 0;
            if (ln < tw + 6 && (side == 0 ? k < 0 : k >= bny)) {
                const int rr = side == 0 ? 0 : 2;
                fb = pick3(crl, t.blk[rr][0], t.blk[rr][1], t.blk[rr][2]);
                const int fnx = pick3(crl, t.nx[rr][0], t.nx[rr][1], t.nx[rr][2]);
                const int fny = pick3(crl, t.ny[rr][0], t.ny[rr][1], t.ny[rr][2]);
                fi = crl == 0 ? fnx + cl : (crl == 2 ? cl - bnx : cl);
                fj = side == 0 ? fny + k : k - bny;
            }
            if (fb >= 0) {
                const DBlock& d = aB[fb];
                const int cx = aip[d.pcx + fi], cy = aip[d.pcy + fj];
                const T wx = T(dp[d.pwx + fi]), wy = T(dp[d.pwy + fj]);
                for (int c = 0; c < 4; ++c) {
                    const int dx = c & 1, dy = c >> 1;
                    T sg;
                    shA[side][j][c][ln] = coarse_addr(aBc, fb, cx + dx, cy + dy, sg);
                    shW[side][j][c][ln] = sg * (dx ? T(1) - wx : wx) * (dy ? T(1) - wy : wy);
                }
            } else {
                for (int c = 0; c < 4; ++c) {
                    shA[side][j][c][ln] = 0;
                    shW[side][j][c][ln] = T(0);
                }
            }
        }
    }
    const bool out_lane = lane >= 3 && lane < 3 + tw;
    const T wrx = (RES && out_lane) ? T(dp[aB[tb].rwx + c]) : T(0);

    // ---- loads of one mode: p and f of the wave's rows, coarse rows ----
    T lp[kRowsPerWave], lf[kRowsPerWave];
    T leA[kWaveCoarse], leB[kWaveCoarse];
    const bool zin = args.zero_in != 0;
    auto issue_pf = [&](int q) __attribute__((always_inline)) {
        const T* __restrict__ fq = fsrc + q * plane;
#pragma unroll
        for (int m = 0; m < kRowsPerWave; ++m) {
            lp[m] = T(0);
            lf[m] = T(0);
            if ((amask >> m) & 1u) {
                if (!zin) lp[m] = pold[q * plane + roff[m]];
                lf[m] = fq[roff[m]];
            }
        }
    };
    auto issue_e = [&](int q, int cyb) __attribute__((always_inline)) {
        const T* __restrict__ ecq = ec + q * plane_c;
#pragma unroll
        for (int m = 0; m < kWaveCoarse; ++m) {
            const int J = cyb + m;
            leA[m] = T(0);
            leB[m] = T(0);
            if (b0 >= 0 && J >= 0 && J < ncyc) {
                leA[m] = ecq[sgo[4][lane] + J * cstrA];
                leB[m] = ecq[sgo[5][lane] + J * cstrB];
            } else if (b0 >= 0 && (J == -1 || J == ncyc)) {
                const int g = J < 0 ? 0 : 2;
                leA[m] = ecq[sgo[g][lane]];
                leB[m] = ecq[sgo[g + 1][lane]];
            }
        }
    };

    issue_pf(args.act[i0]);
    __syncthreads();  // strip tables ready
    // Rows go in pairs (m, m + 1): colours alternate down a column (the block
    // parities keep the checkerboard across joined faces), so of a pair each
    // lane relaxes at most one row per colour.  relax: pairs with a cell of
    // the colour; pick: that cell is in the second row.  Red covers rows
    // 1 .. nrow-2 / lanes 1 .. 62, black rows 2 .. nrow-3 / lanes 2 .. 61
    // (the valid region shrinks).
    constexpr int kPairs = (kRowsPerWave + 1) / 2;
    unsigned relax[2] = {0u, 0u}, pick[2] = {0u, 0u};
#pragma unroll
    for (int colour = 0; colour < 2; ++colour) {
        if (lane < 1 + colour || lane > 62 - colour) continue;
#pragma unroll
        for (int m = 0; m < kRowsPerWave; ++m) {
            const int r = rbase + m;
            if (!((amask >> m) & 1u) || r < 1 + colour || r > nrow - 2 - colour) continue;
            const int k = ty0 - 3 + r;
            const int sc = scol[r][cr];
            const int cc = k < 0 ? cim : (k >= bny ? cip : ci);
            if (sc >= 0 && ((cc + sc) & 1) == colour && !((relax[colour] >> (m >> 1)) & 1u)) {
                relax[colour] |= 1u << (m >> 1);
                if (m & 1) pick[colour] |= 1u << (m >> 1);
            }
        }
    }
    // pairs whose red cell is an output cell of this lane
    unsigned red_out = 0u;
    if (PRO && NRM && lane >= 3 && lane < 3 + tw) {
#pragma unroll
        for (int pi = 0; pi < kPairs; ++pi) {
            const int r = rbase + 2 * pi + int((pick[0] >> pi) & 1u);
            if (((relax[0] >> pi) & 1u) && r >= 3 && ty0 - 3 + r < ty1) red_out |= 1u << pi;
        }
    }
    int cyb = kNoRow;  // first coarse row the wave stages for its own rows
    // per row of the wave (mode-invariant): fmask, the correction comes from
    // the staged coarse rows, crow (3 bits a row) the first of its two;
    // hmask, the correction is summed cell by cell (halo rows of other blocks)
    unsigned fmask = 0u, hmask = 0u, crow = 0u;
    if (PRO) {
        for (int m = 0; m < kRowsPerWave; ++m) {
            const int r = rbase + m;
            if (r < nrow && scy[r] != kNoRow) { cyb = scy[r]; break; }
        }
        for (int m = 0; m < kRowsPerWave; ++m) {
            const int r = rbase + m;
            if (r >= nrow || !((amask >> m) & 1u)) continue;
            const int cy = scy[r];
            if (cy != kNoRow && cy - cyb + 1 < kWaveCoarse) {
                fmask |= 1u << m;
                crow |= unsigned(cy - cyb) << (3 * m);
            } else {
                hmask |= 1u << m;
            }
        }
        issue_e(sq[0], cyb);
    }

    for (int it = i0; it < i1; ++it) {
        const int q = sq[it - i0];
        const T sig = T(ssig[it - i0]);
        // stage this mode; rows inside the block take the coarse-grid
        // correction (bilinear, physical weights) from the wave's own staged
        // coarse rows on the way in
        if (PRO) {
#pragma unroll
            for (int m = 0; m < kWaveCoarse; ++m) {
                const int J = cyb + m;
                const int g = J == -1 ? 0 : (J == ncyc ? 2 : 4);
                sE[wave][m][lane] = sgw[g][lane] * leA[m] + sgw[g + 1][lane] * leB[m];
            }
        }
        // an opaque zero (correcting sweep): its per-row table reads (swy, sy)
        // stay inside the mode loop instead of being hoisted into registers
        int zr = 0;
        if (PRO) asm volatile("v_mov_b32 %0, 0" : "=v"(zr));
#pragma unroll
        for (int m = 0; m < kRowsPerWave; ++m) {
            const int r = rbase + m;
            if (r < nrow) {
                T v = lp[m];
                if (PRO && ((fmask >> m) & 1u)) {
                    const int c0 = int((crow >> (3 * m)) & 7u);
                    const T wy = T(swy[r + zr]);
                    v += wy * sE[wave][c0][lane] + (T(1) - wy) * sE[wave][c0 + 1][lane];
                }
                sp[r][lane] = v;
                sf[r][lane] = lf[m];
            }
        }
        // halo rows of other blocks: four corners each from the offset table
        // (all loads of a wave's rows issued together)
        if (PRO && hmask) {
            const T* __restrict__ ecq = ec + q * plane_c;
#pragma unroll
            for (int m = 0; m < kRowsPerWave; ++m) {
                if (!((hmask >> m) & 1u)) continue;
                const int r = rbase + m;
                const int k = ty0 - 3 + r;
                const int side = k < 0 ? 0 : 1;
                const int j = min(max(side == 0 ? r : r - (nrow - 3), 0), 2);
                T corr = T(0);
#pragma unroll
                for (int c = 0; c < 4; ++c) corr += shW[side][j][c][lane] * ecq[shA[side][j][c][lane]];
                sp[r][lane] += corr;
            }
        }
        __syncthreads();
        // the next mode's loads fly during this mode's compute
        if (it + 1 < i1) {
            issue_pf(sq[it + 1 - i0]);
            if (PRO) issue_e(sq[it + 1 - i0], cyb);
        }

        // One red-black sweep over the pairs chosen above.  Cells of one
        // colour never neighbour each other, so the reads of the next row
        // pair are issued before the current pair's value is written and LDS
        // latency overlaps the arithmetic of the previous pair.  The FP64
        // restricting sweep runs one pair at a time: two pairs in flight do
        // not fit its register budget (four waves per SIMD) next to the next
        // mode's prefetched loads.
#define MBP_PAIR_LOAD(P, pi)                                                                       \
    {                                                                                              \
        const int rr_ = max(min(rbase + 2 * (pi) + int((pick[colour] >> (pi)) & 1u), kLdsRows - 2), 1) + zc; \
        const int k_ = ty0 - 3 + rr_;                                                              \
        P.wm = xwm0;                                                                               \
        P.wp = xwp0;                                                                               \
        T xd_ = xd0;                                                                               \
        if (k_ < 0 || k_ >= bny) {                                                                 \
            const int hh_ = k_ < 0 ? 0 : 1;                                                        \
            P.wm = sxc[hh_][0][la];                                                                \
            P.wp = sxc[hh_][1][la];                                                                \
            xd_ = sxc[hh_][2][la];                                                                 \
        }                                                                                          \
        P.d = xd_ + T(sy[rr_][cr][2]) + sig;                                                       \
        P.y0 = T(sy[rr_][cr][0]);                                                                  \
        P.y1 = T(sy[rr_][cr][1]);                                                                  \
        P.pl = sp[rr_][la - 1];                                                                    \
        P.pr = sp[rr_][la + 1];                                                                    \
        P.pd = sp[rr_ - 1][la];                                                                    \
        P.pu = sp[rr_ + 1][la];                                                                    \
        P.f = sf[rr_][la];                                                                         \
    }
#define MBP_PAIR_DONE(P, pi)                                                                       \
    {                                                                                              \
        const T off_ = P.wm * P.pl + P.wp * P.pr + P.y0 * P.pd + P.y1 * P.pu;                     \
        const T v_ = div_nr(P.f - off_, P.d);                                                      \
        if ((relax[colour] >> (pi)) & 1u) sp[rbase + 2 * (pi) + int((pick[colour] >> (pi)) & 1u)][lane] = v_; \
    }
#pragma unroll
        for (int colour = 0; colour < 2; ++colour) {
            const int la = min(max(lane, 1), 62);
            // the same for the coefficient reads of every pair
            int zc;
            asm volatile("v_mov_b32 %0, 0" : "=v"(zc));
            if constexpr (sizeof(T) == 4 || PRO) {
                // two slots: pair pi loads into slot pi & 1 while pair pi - 1
                // finishes from the other
                struct { T wm, wp, d, y0, y1, pl, pr, pd, pu, f; } A, B;
                MBP_PAIR_LOAD(A, 0)
#pragma unroll
                for (int pi = 1; pi <= kPairs; ++pi) {
                    if (pi < kPairs) {
                        if (pi & 1) MBP_PAIR_LOAD(B, pi)
                        else MBP_PAIR_LOAD(A, pi)
                    }
                    if ((pi - 1) & 1) MBP_PAIR_DONE(B, pi - 1)
                    else MBP_PAIR_DONE(A, pi - 1)
                }
            } else {
#pragma unroll
                for (int pi = 0; pi < kPairs; ++pi) {
                    if (!((relax[colour] >> pi) & 1u)) continue;
                    struct { T wm, wp, d, y0, y1, pl, pr, pd, pu, f; } A;
                    MBP_PAIR_LOAD(A, pi)
                    MBP_PAIR_DONE(A, pi)
                }
            }
            __syncthreads();
        }
#undef MBP_PAIR_LOAD
#undef MBP_PAIR_DONE

        // store, residual (weighted for the restriction, squared for the
        // norm).  The black cells were relaxed last, each solving its own
        // equation with the final red neighbours, so their residual is zero up
        // to rounding: the correcting sweep's norm evaluates only the red cell
        // of each row pair.  (The restricting sweep evaluates every cell: its
        // register budget has no room for the pair bookkeeping.)
        double nrm = 0.0, pnr = 0.0;
        T wres[kRowsPerWave];
#pragma unroll
        for (int m = 0; m < kRowsPerWave; ++m) {
            const int r = rbase + m;
            const int k = ty0 - 3 + r;
            wres[m] = T(0);
            if (r >= 3 && k < ty1 && out_lane) {
                const T pc = sp[r][lane];
                pnew[q * plane + roff[m]] = pc;
                if (NRM) pnr += double(pc) * double(pc);
                if (!PRO && (RES || NRM)) {
                    const T d = xd0 + T(sy[r][1][2]) + sig;
                    const T res = sf[r][lane] - (xwm0 * sp[r][lane - 1] + xwp0 * sp[r][lane + 1] +
                                                 T(sy[r][1][0]) * sp[r - 1][lane] + T(sy[r][1][1]) * sp[r + 1][lane] +
                                                 d * pc);
                    if (NRM) nrm += double(res) * double(res);
                    if (RES) wres[m] = res * wrx * T(swy[r]);
                }
            }
        }
        if (PRO && NRM) {
#pragma unroll
            for (int pi = 0; pi < kPairs; ++pi) {
                if (!((red_out >> pi) & 1u)) continue;
                const int r = rbase + 2 * pi + int((pick[0] >> pi) & 1u) + zr;
                const T pc = sp[r][lane];
                const T d = xd0 + T(sy[r][1][2]) + sig;
                const T res = sf[r][lane] - (xwm0 * sp[r][lane - 1] + xwp0 * sp[r][lane + 1] +
                                             T(sy[r][1][0]) * sp[r - 1][lane] + T(sy[r][1][1]) * sp[r + 1][lane] +
                                             d * pc);
                nrm += double(res) * double(res);
            }
        }
        if (NRM) {
            // one partial pair per wave: no barrier on the way out
            nrm = wave_sum63(nrm);
            pnr = wave_sum63(pnr);
            if (lane == 63) {
                const long long o = 2 * (((long long)q * ntiles + tix) * 4 + wave);
                args.part[o] = nrm;
                args.part[o + 1] = pnr;
            }
        }
        if (RES) {
            __syncthreads();  // every residual has read its neighbours
#pragma unroll
            for (int m = 0; m < kRowsPerWave; ++m)
                if (rbase + m < nrow) sp[rbase + m][lane] = wres[m];
            __syncthreads();
            // one thread per coarse cell of the strip (the strip owns whole
            // coarse cells; the last cell of an odd count spans three)
            const int ncx = aBc[tb].nx, ncy = aBc[tb].ny, bcoff = aBc[tb].off;
            const int I0 = tx0 >> 1, J0 = ty0 >> 1;
            const int I1 = (tx0 + tw == bnx) ? ncx : (tx0 + tw) >> 1;
            const int J1 = (ty1 == bny) ? ncy : ty1 >> 1;
            const int nI = I1 - I0, ncell = nI * (J1 - J0);
            for (int e = threadIdx.x; e < ncell; e += blockDim.x) {
                const int J = J0 + e / nI, I = I0 + e % nI;
                const int x1 = (I == ncx - 1) ? bnx : 2 * I + 2;
                const int y1 = (J == ncy - 1) ? bny : 2 * J + 2;
                const int lx = 2 * I - tx0 + 3, ry = 2 * J - ty0 + 3;
                T sum = sp[ry][lx] + sp[ry][lx + 1] + sp[ry + 1][lx] + sp[ry + 1][lx + 1];
                if (x1 - 2 * I == 3) sum += sp[ry][lx + 2] + sp[ry + 1][lx + 2];
                if (y1 - 2 * J == 3) {
                    sum += sp[ry + 2][lx] + sp[ry + 2][lx + 1];
                    if (x1 - 2 * I == 3) sum += sp[ry + 2][lx + 2];
                }
                const long long o = q * plane_c + bcoff + (long long)J * ncx + I;
                args.fc[o] = sum;
                if (args.pc) args.pc[o] = T(0);
            }
        }
        __syncthreads();  // LDS is restaged by the next mode
    }
}

// Sweep kernels.  The correction form holds more state per lane; it is
// capped at three waves per SIMD in FP32 and two in FP64 (which then needs
// no spills), the others at four.
template <typename T, bool RES, bool NRM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_tile(const MArgs<T> args) {
    tile_sweep<T, false, RES, NRM>(args, blockIdx.x, blockIdx.y);
}

template <typename T, bool NRM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 2 : 3)))
k_tile_corr(const MArgs<T> args) {
    tile_sweep<T, true, false, NRM>(args, blockIdx.x, blockIdx.y);
}

// The FP32 pre- (restricting) or post- (correcting) sweep of one level for
// many problems in one launch.
template <bool PRO>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PRO ? 3 : 4)))
k_tile_group(const GEnt* __restrict__ e, int n, const MArgs<float>* __restrict__ jobs) {
    int bx, by;
    const int j = group_locate(e, n, bx, by);
    tile_sweep<float, PRO, !PRO, false>(jobs[j], bx, by);
}

// ------------------------- register march form of the sweep -------------------------
// One wave owns a tall strip (58 output columns, up to 128 rows) and marches
// down it with a five-row register window: each step takes row k, relaxes the
// red cells of row k-1, the black cells of row k-2, stores row k-2 and forms
// the residual of row k-3.  x neighbours come from DPP lane shifts, so there
// is no LDS and no barrier; the loads of the next kRing rows are always in
// flight.  The vertical halo is read once per strip instead of once per
// short tile.  Rows of the strip's own block take the block's y coefficients
// for every lane (joined blocks are congruent along their common faces).
constexpr int kRing = 8;

template <int CTRL>
__device__ __forceinline__ double dpp_shift(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_shift(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
// value of lane - 1 (0 at lane 0) and of lane + 1 (0 at lane 63)
template <typename T>
__device__ __forceinline__ T from_left(T v) { return dpp_shift<0x138>(v); }
template <typename T>
__device__ __forceinline__ T from_right(T v) { return dpp_shift<0x130>(v); }

template <typename T, bool RES, bool NRM>
__global__ void __launch_bounds__(256) k_rmarch(const MArgs<T> args, const double* __restrict__ dp) {
    // dp: the coefficient pool, passed on its own so that uniform row
    // coefficients are read through the scalar cache
    const DBlock* __restrict__ aB = args.B;
    const DBlock* __restrict__ aBc = args.Bc;
    const int ntiles = args.ntiles;
    const long long plane = args.plane, plane_c = args.plane_c;
    const int lane = threadIdx.x & 63;
    // the wave index is uniform per wave: say so, so that everything derived
    // from the strip descriptor lives in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nact = *args.nact;
    const long long item = (long long)xcd_remap_m(blockIdx.x, gridDim.x) * 4 + wave;
    if (item >= (long long)ntiles * nact) return;
    const int mi = int(item / ntiles), tix = int(item - (long long)mi * ntiles);
    const int q = __builtin_amdgcn_readfirstlane(args.act[mi]);
    const MTile& t = args.tiles[tix];
    const int tb = t.b, tx0 = t.x0, tw = t.w, ty0 = t.y0, ty1 = t.y1;
    const int bnx = t.bnx, bny = t.bny;
    const T sig = T(args.shift[q]);

    // ---- the lane's column (as in the strip form) ----
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
    const int ci = cr == 0 ? nx0 + c : (cr == 2 ? c - bnx : c);
    const int cim = cr == 0 ? nxm + c : (cr == 2 ? c - bnx : c);
    const int cip = cr == 0 ? nxp + c : (cr == 2 ? c - bnx : c);
    const int off0 = b0 >= 0 ? pick3(cr, t.off[1][0], t.off[1][1], t.off[1][2]) + ci : 0;
    const int offm = bm >= 0 ? pick3(cr, t.off[0][0], t.off[0][1], t.off[0][2]) + cim : 0;
    const int offp = bp >= 0 ? pick3(cr, t.off[2][0], t.off[2][1], t.off[2][2]) + cip : 0;
    const int cx0 = pick3(cr, t.cx[1][0], t.cx[1][1], t.cx[1][2]);
    const int cxm = pick3(cr, t.cx[0][0], t.cx[0][1], t.cx[0][2]);
    const int cxp = pick3(cr, t.cx[2][0], t.cx[2][1], t.cx[2][2]);
    const int par0 = pick3(cr, t.par[1][0], t.par[1][1], t.par[1][2]);
    const int parm = pick3(cr, t.par[0][0], t.par[0][1], t.par[0][2]);
    const int parp = pick3(cr, t.par[2][0], t.par[2][1], t.par[2][2]);
    const T xwm0 = b0 >= 0 ? T(dp[cx0 + ci]) : T(0), xwp0 = b0 >= 0 ? T(dp[cx0 + nx0 + ci]) : T(0);
    const T xd0 = b0 >= 0 ? T(dp[cx0 + 2 * nx0 + ci]) : T(0);
    const T xwmm = bm >= 0 ? T(dp[cxm + cim]) : T(0), xwpm = bm >= 0 ? T(dp[cxm + nxm + cim]) : T(0);
    const T xdm = bm >= 0 ? T(dp[cxm + 2 * nxm + cim]) : T(0);
    const T xwmp = bp >= 0 ? T(dp[cxp + cip]) : T(0), xwpp = bp >= 0 ? T(dp[cxp + nxp + cip]) : T(0);
    const T xdp = bp >= 0 ? T(dp[cxp + 2 * nxp + cip]) : T(0);
    // y coefficients per row region (one table per region, shared by its lanes)
    const int ybm = t.blk[0][1] >= 0 ? 1 : (t.blk[0][0] >= 0 ? 0 : 2);
    const int ybp = t.blk[2][1] >= 0 ? 1 : (t.blk[2][0] >= 0 ? 0 : 2);
    const int ycy0 = t.cy[1][1], yny0 = bny;
    const int ycym = t.cy[0][ybm], ynym = t.ny[0][ybm];
    const int ycyp = t.cy[2][ybp], ynyp = t.ny[2][ybp];
    const bool out_lane = lane >= 3 && lane < 3 + tw;
    // y coefficients per column region of the rows near the block's edges:
    // slots 0..3 hold rows y0-3 .. y0 (the rows up to the first one when the
    // strip starts near it), slots 4..7 rows bny-1 .. bny+2
    __shared__ T sY[4][8][3][3];
    if (lane < 8 * 3) {
        const int slot = lane / 3, j = lane - 3 * slot;
        const int k = slot < 4 ? ty0 - 3 + slot : bny - 1 + (slot - 4);
        const bool used = k >= ty0 - 3 && k <= ty1 + 2;  // rows the strip touches
        const int rr = k < 0 ? 0 : (k >= bny ? 2 : 1);
        const int jb = pick3(rr, t.blk[0][j], t.blk[1][j], t.blk[2][j]);
        const int jcy = pick3(rr, t.cy[0][j], t.cy[1][j], t.cy[2][j]);
        const int jny = pick3(rr, t.ny[0][j], t.ny[1][j], t.ny[2][j]);
        const int lj = k < 0 ? jny + k : (k >= bny ? k - bny : k);
        const bool ok = used && jb >= 0;
        sY[wave][slot][j][0] = ok ? T(dp[jcy + lj]) : T(0);
        sY[wave][slot][j][1] = ok ? T(dp[jcy + jny + lj]) : T(0);
        sY[wave][slot][j][2] = ok ? T(dp[jcy + 2 * jny + lj]) : T(1);
    }

    const T* __restrict__ po = args.pold + q * plane;
    const T* __restrict__ fq = args.f + q * plane;
    T* __restrict__ pn = args.pnew + q * plane;
    const bool zin = args.zero_in != 0;

    // restriction bookkeeping (output lanes lie in the strip's block)
    int ncx = 0, ncy = 0, bcoff = 0, I = 0, rwy = 0;
    bool leader = false, three = false;
    T wrx = T(0);
    if (RES) {
        ncx = aBc[tb].nx;
        ncy = aBc[tb].ny;
        bcoff = aBc[tb].off;
        rwy = aB[tb].rwy;
        if (out_lane) {
            I = min(c >> 1, ncx - 1);
            leader = c == 2 * I;
            three = leader && (I == ncx - 1) && (bnx - 2 * I == 3);
            wrx = T(dp[aB[tb].rwx + c]);
        }
    }

    T rp[kRing], rf[kRing];
    const int kbeg = ty0 - 3, kend = ty1 + 2;
    // row k: its lane offset, or -1 where the lane's region has no block
#define MBP_RM_OFF(k)                                                                               \
    ((k) < 0 ? (bm >= 0 ? offm + (nym + (k)) * nxm : -1)                                             \
             : ((k) >= bny ? (bp >= 0 ? offp + ((k) - bny) * nxp : -1) : (b0 >= 0 ? off0 + (k) * nx0 : -1)))
    // loads are unconditional (a dead lane reads cell 0 of the plane) so that
    // no branch joins on a value in flight; dead cells are masked at use
#pragma unroll
    for (int u = 0; u < kRing; ++u) {
        const int k = kbeg + u;
        const int o = k <= kend ? MBP_RM_OFF(k) : -1;
        rp[u] = po[o >= 0 ? o : 0];
        rf[u] = fq[o >= 0 ? o : 0];
    }
    T w4 = T(0), w3 = T(0), w2 = T(0), w1 = T(0);  // p of rows k-4 .. k-1
    T g3 = T(0), g2 = T(0), g1 = T(0);             // f of rows k-3 .. k-1
    double nrm = 0.0, pnr = 0.0;
    T acc = T(0);
    for (int k0 = kbeg; k0 <= kend; k0 += kRing) {
#pragma unroll
        for (int u = 0; u < kRing; ++u) {
            // steps past the last row only relax rows that are never stored;
            // keeping every step (and every load) unconditional leaves no
            // branch joining on a value in flight
            const int k = k0 + u;
            {
                const bool here = k <= kend && MBP_RM_OFF(k) >= 0;
                const T p0 = (here && !zin) ? rp[u] : T(0), f0 = here ? rf[u] : T(0);
                {
                    const int kn = min(k + kRing, kend);
                    const int o = MBP_RM_OFF(kn);
                    rp[u] = po[o >= 0 ? o : 0];
                    rf[u] = fq[o >= 0 ? o : 0];
                }
                // red cells of row k-1 (old black neighbours), then black cells of row k-2
#pragma unroll
                for (int colour = 0; colour < 2; ++colour) {
                    const int kk = k - 1 - colour;
                    if (kk < ty0 - 2 + colour) continue;
                    const T v = colour == 0 ? w1 : w2;
                    const T dn = colour == 0 ? w2 : w3;
                    const T up = colour == 0 ? p0 : w1;
                    const T fv = colour == 0 ? g1 : g2;
                    const bool below = kk < 0, above = kk >= bny;
                    const int cj = below ? ynym + kk : (above ? kk - bny : kk);
                    // interior rows: one (scalar) table for the whole row; first
                    // and last rows and halo rows: the lane's own block (faces
                    // beyond may differ between joined blocks) from the wave's
                    // table of the edge rows.  Both are read and the values
                    // selected, so that no load goes through a generic pointer.
                    const bool interior = kk > 0 && kk < bny - 1;
                    const int ki = min(max(kk, 0), bny - 1);
                    const int slot = min(max(kk <= 0 ? kk - kbeg : 4 + kk - (bny - 1), 0), 7);
                    const T ys0 = T(dp[ycy0 + ki]), ys1 = T(dp[ycy0 + yny0 + ki]), ys2 = T(dp[ycy0 + 2 * yny0 + ki]);
                    const T yl0 = sY[wave][slot][cr][0], yl1 = sY[wave][slot][cr][1], yl2 = sY[wave][slot][cr][2];
                    const T ym = interior ? ys0 : yl0;
                    const T yp = interior ? ys1 : yl1;
                    const T yd = interior ? ys2 : yl2;
                    T wm = xwm0, wp = xwp0, xd = xd0;
                    int cc = ci, par = par0;
                    bool alive = b0 >= 0;
                    if (below) {
                        wm = xwmm; wp = xwpm; xd = xdm; cc = cim; par = parm; alive = bm >= 0;
                    } else if (above) {
                        wm = xwmp; wp = xwpp; xd = xdp; cc = cip; par = parp; alive = bp >= 0;
                    }
                    const T xm = from_left(v), xp = from_right(v);
                    const T nv = (fv - (wm * xm + wp * xp + ym * dn + yp * up)) / (xd + yd + sig);
                    const bool mine = alive && ((cc + cj + par) & 1) == colour && lane >= 1 + colour &&
                                      lane <= 62 - colour;
                    if (colour == 0) w1 = mine ? nv : v;
                    else w2 = mine ? nv : v;
                }
                // row k-2 is final
                if (k - 2 >= ty0 && k - 2 < ty1 && out_lane) pn[off0 + (k - 2) * nx0] = w2;
                // residual of row k-3 (rows k-4 .. k-2 are final)
                const int kr = k - 3;
                if ((RES || NRM) && kr >= ty0 && kr < ty1) {
                    const T xm = from_left(w3), xp = from_right(w3);
                    const T d = xd0 + T(dp[ycy0 + 2 * yny0 + kr]) + sig;
                    T r = g3 - (xwm0 * xm + xwp0 * xp + T(dp[ycy0 + kr]) * w4 + T(dp[ycy0 + yny0 + kr]) * w2 +
                                d * w3);
                    if (!out_lane) r = T(0);
                    if (NRM) {
                        nrm += double(r) * double(r);
                        pnr += out_lane ? double(w3) * double(w3) : 0.0;
                    }
                    if (RES) {
                        const T rw = r * wrx * T(dp[rwy + kr]);
                        const T r1 = from_right(rw);
                        T sx = rw + r1;
                        if (three) sx += from_right(r1);
                        acc += sx;
                        const int J = min(kr >> 1, ncy - 1);
                        const int Jn = kr + 1 < ty1 ? min((kr + 1) >> 1, ncy - 1) : -1;
                        if (Jn != J) {
                            if (leader) {
                                const long long o = q * plane_c + bcoff + (long long)J * ncx + I;
                                args.fc[o] = acc;
                                if (args.pc) args.pc[o] = T(0);
                            }
                            acc = T(0);
                        }
                    }
                }
                w4 = w3;
                w3 = w2;
                w2 = w1;
                w1 = p0;
                g3 = g2;
                g2 = g1;
                g1 = f0;
            }
        }
    }
#undef MBP_RM_OFF
    if (NRM) {
        nrm = wave_sum63(nrm);
        pnr = wave_sum63(pnr);
        if (lane == 63) {
            args.part[2 * ((long long)q * ntiles + tix)] = nrm;
            args.part[2 * ((long long)q * ntiles + tix) + 1] = pnr;
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
    a.wg_target = P->wg_target;
    return a;
}

// Modes per workgroup: enough workgroups to fill the chip several times
// over, each reusing its strip set-up for as many modes as that allows.
static int modes_per_wg(int ntiles, int nitems, int target) {
    long long per = (long long)ntiles * nitems / std::max(1, target);
    return int(std::max(1LL, std::min<long long>(kMaxModes, per)));
}

// Workgroups of a strip kernel resident on the chip at once (occupancy x CUs,
// taken once per kernel on the current device).
static int chip_slots(const void* kernel) {
    static std::mutex mu;
    static std::map<std::pair<int, const void*>, int> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find({dev, kernel});
    if (it != cache.end()) return it->second;
    int per_cu = 0, ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        per_cu = 1;
        ncu = 256;
    }
    const int slots = std::max(1, per_cu) * std::max(1, ncu);
    cache[{dev, kernel}] = slots;
    return slots;
}

// Modes per workgroup of a single-problem launch: the count for which the
// rounds of workgroups the chip runs (the last one often nearly empty) times
// the time of one workgroup (per modes plus its strip set-up, about two
// modes' worth) is smallest; ties go to the count the workgroup target gives
// or, failing that, to the larger count.
static int modes_per_wg_balanced(int ntiles, int nitems, int target, int slots) {
    const int pref = modes_per_wg(ntiles, nitems, target);
    int best = pref;
    long long best_cost = -1;
    for (int per = 1; per <= kMaxModes; ++per) {
        if (per > nitems) break;
        const long long wgs = (long long)ntiles * ((nitems + per - 1) / per);
        const long long rounds = (wgs + slots - 1) / slots;
        const long long cost = rounds * (per + 2);
        if (best_cost < 0 || cost < best_cost || (cost == best_cost && best != pref && (per == pref || per > best))) {
            best_cost = cost;
            best = per;
        }
    }
    return best;
}

template <typename T, bool PRO, bool RES, bool NRM>
static void launch_march(MArgs<T> a, int nitems, hipStream_t s) {
    const void* fn = PRO ? reinterpret_cast<const void*>(k_tile_corr<T, NRM>)
                         : reinterpret_cast<const void*>(k_tile<T, RES, NRM>);
    a.per = modes_per_wg_balanced(a.ntiles, nitems, a.wg_target, chip_slots(fn));
    const int groups = (nitems + a.per - 1) / a.per;
    if constexpr (PRO)
        hipLaunchKernelGGL((k_tile_corr<T, NRM>), dim3(a.ntiles, groups), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_tile<T, RES, NRM>), dim3(a.ntiles, groups), dim3(256), 0, s, a);
}

template <typename T, bool RES>
static void launch_rmarch(const mbp_plan* P, int l, MArgs<T> a, int nitems, hipStream_t s) {
    a.tiles = reinterpret_cast<const MTile*>(P->d_mtiles) + P->rtile_off[l];
    a.ntiles = P->rtile_cnt[l];
    const long long work = (long long)a.ntiles * nitems;
    const int groups = int((work + 3) / 4);
    hipLaunchKernelGGL((k_rmarch<T, RES, false>), dim3(groups), dim3(256), 0, s, a, a.dp);
}

// Pre-smoothing sweep of level l (old -> new) fused with the residual
// restriction into level l+1 (rhs fc; pc, if given, set to the zero initial
// guess).  zero_in: the old iterate is zero and is not read.
template <typename T>
void march_pre(const mbp_plan* P, int l, const T* pold, T* pnew, const T* f, T* fc, T* pc,
               const int* act, const int* nact, int nitems, bool zero_in, hipStream_t s) {
    MArgs<T> a = margs<T>(P, l, pold, pnew, f, nullptr, fc, pc, act, nact);
    a.zero_in = zero_in ? 1 : 0;
    if (P->use_rmarch[l]) launch_rmarch<T, true>(P, l, a, nitems, s);
    else launch_march<T, false, true, false>(a, nitems, s);
}

// Plain sweep (extra smoothing steps).
template <typename T>
void march_sweep(const mbp_plan* P, int l, const T* pold, T* pnew, const T* f, const int* act,
                 const int* nact, int nitems, bool zero_in, hipStream_t s) {
    MArgs<T> a = margs<T>(P, l, pold, pnew, f, nullptr, nullptr, nullptr, act, nact);
    a.zero_in = zero_in ? 1 : 0;
    if (P->use_rmarch[l]) launch_rmarch<T, false>(P, l, a, nitems, s);
    else launch_march<T, false, false, false>(a, nitems, s);
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
                                double*, const int*, const int*, int, bool, hipStream_t);
template void march_pre<float>(const mbp_plan*, int, const float*, float*, const float*, float*, float*,
                               const int*, const int*, int, bool, hipStream_t);
template void march_sweep<double>(const mbp_plan*, int, const double*, double*, const double*,
                                  const int*, const int*, int, bool, hipStream_t);
template void march_sweep<float>(const mbp_plan*, int, const float*, float*, const float*, const int*,
                                 const int*, int, bool, hipStream_t);
template void march_post<double>(const mbp_plan*, int, const double*, double*, const double*,
                                 const double*, bool, const int*, const int*, int, hipStream_t);
template void march_post<float>(const mbp_plan*, int, const float*, float*, const float*, const float*,
                                bool, const int*, const int*, int, hipStream_t);

bool group_ok(const SolveCtx& c) {
    const mbp_plan* P = c.P;
    if (!c.mixed || c.full_lds || P->opt.nu1 != 1 || P->opt.nu2 != 1) return false;
    for (int l = 0; l < P->lds_level32; ++l)
        if (!P->march_ok[l] || P->use_rmarch[l] || P->p32B[l] == nullptr) return false;
    return true;
}

// Level `level` of every problem that has it above its LDS-resident levels:
// pre-sweep A -> B with the restriction into level + 1, or correction from
// level + 1 with the post-sweep B -> A (the buffers of the strip V-cycle).
GStage group_march32(GroupBlob& gb, const std::vector<SolveCtx*>& cs, int level, bool post, bool zero0) {
    std::vector<MArgs<float>> jobs;
    std::vector<int> gx, gy;
    // the launch's workgroup target is shared by its problems in proportion
    // to their work (strips x modes): every problem's workgroups share the
    // chip, so each can reuse its strip set-up for more modes than alone
    double total = 0.0;
    for (const SolveCtx* c : cs)
        if (level < c->P->lds_level32) total += double(c->P->mtile_cnt[level]) * c->nitems;
    for (const SolveCtx* c : cs) {
        const mbp_plan* P = c->P;
        if (level >= P->lds_level32) continue;
        const int l = level;
        MArgs<float> a = post ? margs<float>(P, l, P->p32B[l], P->p32[l], P->f32[l], P->p32[l + 1], nullptr,
                                             nullptr, P->d_act, P->d_nact)
                              : margs<float>(P, l, P->p32[l], P->p32B[l], P->f32[l], nullptr, P->f32[l + 1],
                                             nullptr, P->d_act, P->d_nact);
        a.zero_in = post ? 0 : ((l == 0 ? zero0 : true) ? 1 : 0);
        const double share = total > 0.0 ? double(a.ntiles) * c->nitems / total : 1.0;
        a.per = modes_per_wg(a.ntiles, c->nitems, std::max(1, int(a.wg_target * share + 0.5)));
        jobs.push_back(a);
        gx.push_back(a.ntiles);
        gy.push_back((c->nitems + a.per - 1) / a.per);
    }
    return group_build(gb, post ? G_POST32 : G_PRE32, jobs, gx, gy);
}

void group_launch_march(const GStage& st, const unsigned char* dev, hipStream_t s) {
    if (st.wgs <= 0) return;
    const GEnt* e = reinterpret_cast<const GEnt*>(dev + st.ent_off);
    const MArgs<float>* j = reinterpret_cast<const MArgs<float>*>(dev + st.job_off);
    if (st.kind == G_POST32)
        hipLaunchKernelGGL(k_tile_group<true>, dim3(st.wgs), dim3(256), 0, s, e, st.nent, j);
    else if (st.kind == G_PRE32)
        hipLaunchKernelGGL(k_tile_group<false>, dim3(st.wgs), dim3(256), 0, s, e, st.nent, j);
}

}  // namespace mbp
