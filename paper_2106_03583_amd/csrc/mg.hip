// Geometric multigrid for the shifted 2D systems of Eq. (9),
//     (A_2D + sigma_q) phat_q = fhat_q,   sigma_q = lambda_q / dz^2,
// one system per z mode, on a multi-block x-y plane with possibly stretched
// spacing.  A_2D is the cell-centred finite-volume Laplacian; joined faces
// couple blocks directly (the halo is read from the neighbour block), walls
// enter through the coefficients (Neumann: no coupling, Dirichlet: a mirrored
// ghost folded into the diagonal).
//
// Components: red-black Gauss-Seidel smoothing, residual + area-weighted
// restriction (fused), bilinear prolongation in physical coordinates +
// correction (fused), and an exact coarsest solve from a precomputed
// eigen-decomposition.  Fine levels stream through HBM with tiled kernels;
// the levels whose hierarchy fits in LDS run inside one workgroup per mode.
#include <map>
#include <mutex>
#include <utility>

#include "internal.h"

namespace mbp {

__device__ __forceinline__ int xcd_remap_mg(int g, int n) {
    int x = g & 7, l = g >> 3;
    int per = n >> 3, rem = n & 7;
    return x * per + min(x, rem) + l;
}

// Values of the four stencil neighbours of cell (i, j) of block b.  A
// neighbour beyond a joined face comes from the partner block (same
// tangential index); beyond a wall the coefficient is zero and 0 is returned.
template <typename T>
__device__ __forceinline__ void neighbours(const T* __restrict__ pl, const DBlock* __restrict__ B,
                                           const DBlock& b, int i, int j, T& xm, T& xp, T& ym,
                                           T& yp) {
    const T* row = pl + b.off + j * b.nx;
    if (i > 0) xm = row[i - 1];
    else if (b.nbr[XM] >= 0) { const DBlock& k = B[b.nbr[XM]]; xm = pl[k.off + j * k.nx + k.nx - 1]; }
    else xm = T(0);
    if (i < b.nx - 1) xp = row[i + 1];
    else if (b.nbr[XP] >= 0) { const DBlock& k = B[b.nbr[XP]]; xp = pl[k.off + j * k.nx]; }
    else xp = T(0);
    if (j > 0) ym = row[i - b.nx];
    else if (b.nbr[YM] >= 0) { const DBlock& k = B[b.nbr[YM]]; ym = pl[k.off + (k.ny - 1) * k.nx + i]; }
    else ym = T(0);
    if (j < b.ny - 1) yp = row[i + b.nx];
    else if (b.nbr[YP] >= 0) { const DBlock& k = B[b.nbr[YP]]; yp = pl[k.off + i]; }
    else yp = T(0);
}

// (A_2D + sigma) p at cell (i, j).
template <typename T>
__device__ __forceinline__ T apply_at(const T* __restrict__ pl, const DBlock* __restrict__ B,
                                      const DBlock& b, const double* __restrict__ dp, int i, int j,
                                      T sig) {
    T xm, xp, ym, yp;
    neighbours(pl, B, b, i, j, xm, xp, ym, yp);
    const T c = pl[b.off + j * b.nx + i];
    const T d = T(dp[b.cx + 2 * b.nx + i]) + T(dp[b.cy + 2 * b.ny + j]) + sig;
    return T(dp[b.cx + i]) * xm + T(dp[b.cx + b.nx + i]) * xp + T(dp[b.cy + j]) * ym +
           T(dp[b.cy + b.ny + j]) * yp + d * c;
}

// Smoothing colour of cell (i, j): red / black by index parity (0 / 1); on an
// odd periodic wrap the last column / row gets colours 2 / 3 so that no two
// neighbours are ever relaxed in the same pass.
__device__ __forceinline__ int colour_of(const DBlock& b, int i, int j) {
    int c = (i + j + b.par) & 1;
    if (((b.oddwrap & 1) && i == b.nx - 1) || ((b.oddwrap & 2) && j == b.ny - 1)) c += 2;
    return c;
}

// Red-black Gauss-Seidel update of one cell: solve its own equation with the
// current neighbour values.
template <typename T>
__device__ __forceinline__ T gs_value(const T* __restrict__ pl, const T* __restrict__ fl,
                                      const DBlock* __restrict__ B, const DBlock& b,
                                      const double* __restrict__ dp, int i, int j, T sig) {
    T xm, xp, ym, yp;
    neighbours(pl, B, b, i, j, xm, xp, ym, yp);
    const T d = T(dp[b.cx + 2 * b.nx + i]) + T(dp[b.cy + 2 * b.ny + j]) + sig;
    const T off = T(dp[b.cx + i]) * xm + T(dp[b.cx + b.nx + i]) * xp + T(dp[b.cy + j]) * ym +
                  T(dp[b.cy + b.ny + j]) * yp;
    return (fl[b.off + j * b.nx + i] - off) / d;
}

// Coarse value at (I, J) of block b, I in [-1, nx], J in [-1, ny]: beyond a
// joined face it is the partner's cell, beyond a wall the mirror image
// (Neumann +, Dirichlet -).  A corner is reached through the y face first.
template <typename T>
__device__ __forceinline__ T coarse_value(const T* __restrict__ pl, const DBlock* __restrict__ B,
                                          int b, int I, int J) {
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

// Area-weighted restriction of the residual for coarse cell (I, J).
template <typename T>
__device__ __forceinline__ T restrict_at(const T* __restrict__ pf, const T* __restrict__ ff,
                                         const DBlock* __restrict__ Bf, const DBlock& bf,
                                         const double* __restrict__ dp, const int* __restrict__ ip,
                                         int I, int J, T sig) {
    const int i0 = ip[bf.rsx + I], i1 = ip[bf.rsx + I + 1];
    const int j0 = ip[bf.rsy + J], j1 = ip[bf.rsy + J + 1];
    T acc = T(0);
    for (int j = j0; j < j1; ++j) {
        const T wy = T(dp[bf.rwy + j]);
        T row = T(0);
        for (int i = i0; i < i1; ++i) {
            const T r = ff[bf.off + j * bf.nx + i] - apply_at(pf, Bf, bf, dp, i, j, sig);
            row += T(dp[bf.rwx + i]) * r;
        }
        acc += wy * row;
    }
    return acc;
}

// Bilinear interpolation (physical-coordinate weights) of the coarse
// correction at fine cell (i, j).
template <typename T>
__device__ __forceinline__ T prolong_at(const T* __restrict__ pc, const DBlock* __restrict__ Bc,
                                        const DBlock& bf, int b, const double* __restrict__ dp,
                                        const int* __restrict__ ip, int i, int j) {
    const int cx = ip[bf.pcx + i], cy = ip[bf.pcy + j];
    const T wx = T(dp[bf.pwx + i]), wy = T(dp[bf.pwy + j]);
    const T e00 = coarse_value(pc, Bc, b, cx, cy), e10 = coarse_value(pc, Bc, b, cx + 1, cy);
    const T e01 = coarse_value(pc, Bc, b, cx, cy + 1), e11 = coarse_value(pc, Bc, b, cx + 1, cy + 1);
    return wy * (wx * e00 + (T(1) - wx) * e10) + (T(1) - wy) * (wx * e01 + (T(1) - wx) * e11);
}

// =========================== global-memory kernels ===========================

template <typename T>
__global__ void __launch_bounds__(256)
k_rbgs(const DBlock* __restrict__ B, const int4* __restrict__ tiles, int ntiles,
       const double* __restrict__ dp, T* __restrict__ p, const T* __restrict__ f, long long plane,
       const double* __restrict__ shift, const int* __restrict__ act, const int* __restrict__ nact,
       int colour) {
    const int item = blockIdx.y;
    if (item >= *nact) return;
    const int q = act[item];
    const int4 t = tiles[xcd_remap_mg(blockIdx.x, ntiles)];
    const DBlock b = B[t.x];
    T* pq = p + q * plane;
    const T* fq = f + q * plane;
    const T sig = T(shift[q]);
    const int i = t.y + threadIdx.x;
    if (i >= b.nx) return;
    for (int r = threadIdx.y; r < kTileY; r += kRowsPerPass) {
        const int j = t.z + r;
        if (j >= b.ny) break;
        if (colour_of(b, i, j) != colour) continue;
        pq[b.off + j * b.nx + i] = gs_value(pq, fq, B, b, dp, i, j, sig);
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_restrict(const DBlock* __restrict__ Bf, const DBlock* __restrict__ Bc,
           const int4* __restrict__ tiles_c, int ntiles_c, const double* __restrict__ dp,
           const int* __restrict__ ip, const T* __restrict__ pf, const T* __restrict__ ff,
           T* __restrict__ fc, T* __restrict__ pc, long long plane_f, long long plane_c,
           const double* __restrict__ shift, const int* __restrict__ act,
           const int* __restrict__ nact) {
    const int item = blockIdx.y;
    if (item >= *nact) return;
    const int q = act[item];
    const int4 t = tiles_c[xcd_remap_mg(blockIdx.x, ntiles_c)];
    const DBlock bc = Bc[t.x];
    const DBlock bf = Bf[t.x];
    const T* pq = pf + q * plane_f;
    const T* fq = ff + q * plane_f;
    const T sig = T(shift[q]);
    const int I = t.y + threadIdx.x;
    if (I >= bc.nx) return;
    for (int r = threadIdx.y; r < kTileY; r += kRowsPerPass) {
        const int J = t.z + r;
        if (J >= bc.ny) break;
        const long long o = q * plane_c + bc.off + J * bc.nx + I;
        fc[o] = restrict_at(pq, fq, Bf, bf, dp, ip, I, J, sig);
        pc[o] = T(0);
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_prolong(const DBlock* __restrict__ Bf, const DBlock* __restrict__ Bc,
          const int4* __restrict__ tiles_f, int ntiles_f, const double* __restrict__ dp,
          const int* __restrict__ ip, const T* __restrict__ pc, T* __restrict__ pf,
          long long plane_f, long long plane_c, const int* __restrict__ act,
          const int* __restrict__ nact) {
    const int item = blockIdx.y;
    if (item >= *nact) return;
    const int q = act[item];
    const int4 t = tiles_f[xcd_remap_mg(blockIdx.x, ntiles_f)];
    const DBlock bf = Bf[t.x];
    const T* cq = pc + q * plane_c;
    T* fq = pf + q * plane_f;
    const int i = t.y + threadIdx.x;
    if (i >= bf.nx) return;
    for (int r = threadIdx.y; r < kTileY; r += kRowsPerPass) {
        const int j = t.z + r;
        if (j >= bf.ny) break;
        fq[bf.off + j * bf.nx + i] += prolong_at(cq, Bc, bf, t.x, dp, ip, i, j);
    }
}

// Wave + workgroup sum of a double; the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* scratch) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int lane = threadIdx.x + threadIdx.y * blockDim.x;
    const int wid = lane >> 6, nw = (blockDim.x * blockDim.y + 63) >> 6;
    __syncthreads();
    if ((lane & 63) == 0) scratch[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (lane == 0)
        for (int w = 0; w < nw; ++w) s += scratch[w];
    return s;
}

// Per-tile partial sums of the squared finest-level residual of each mode;
// mode == 1 also writes r as float32 (the refinement rhs) and, if given, zeroes e32.
constexpr int kResModes = 8;  // most items one residual workgroup runs in turn

struct ResJob {
    const DBlock* B;
    const int4* tiles;
    int ntiles;
    const double* dp;
    const double* p;
    const double* f;
    long long plane;
    const double* shift;
    const int* act;
    const int* nact;
    double* part;
    float* r32;
    float* e32;
    int per;             // items per workgroup
    int pzero;           // p is zero (first refinement step): r = f, p is not read
};

// Items per residual workgroup: enough workgroups to fill the chip several
// times over, the rest of the items run in turn.
static int res_per(int ntiles, int nitems, double share = 1.0) {
    const long long per = (long long)(double(ntiles) * nitems / std::max(1.0, 2048.0 * share));
    return int(std::max(1LL, std::min<long long>(kResModes, per)));
}

constexpr int kResRows = kTileY / kRowsPerPass;  // consecutive rows per thread
static_assert(kTileY % kRowsPerPass == 0, "whole row groups per tile");

template <int MODE>
__device__ __forceinline__ void residual_body(const ResJob& J, int bx, int by) {
    // a workgroup runs one tile for `per` consecutive active items; per-wave
    // sums wait in LDS and one barrier at the end publishes every item's pair
    __shared__ double red[kResModes][kRowsPerPass][2];
    const int n = *J.nact;
    const int i0 = by * J.per, i1 = min(i0 + J.per, n);
    if (i0 >= i1) return;
    const DBlock* __restrict__ B = J.B;
    const double* __restrict__ dp = J.dp;
    const int ntiles = J.ntiles;
    const int tix = xcd_remap_mg(bx, ntiles);
    const int4 t = wave_uniform(J.tiles[tix]);
    const DBlock b = wave_uniform(B[t.x]);
    // each thread owns kResRows consecutive rows of one column; its loads use
    // indices clamped into the block, so all of them can be in flight at once
    // (lanes past the block's edge compute values that are never used)
    const int i = t.y + threadIdx.x;
    // a wave is one row group (blockDim.x = 64): its rows and their
    // coefficients are wave-uniform and live in scalar registers
    const int j0 = t.z + __builtin_amdgcn_readfirstlane(threadIdx.y) * kResRows;
    const int ic = min(i, b.nx - 1);
    const int im = max(ic - 1, 0), ip = min(ic + 1, b.nx - 1);
    const double cxm = dp[b.cx + ic], cxp = dp[b.cx + b.nx + ic], dx = dp[b.cx + 2 * b.nx + ic];
    int jr[kResRows + 2];
    double cym[kResRows], cyp[kResRows], dy[kResRows];
#pragma unroll
    for (int k = 0; k < kResRows + 2; ++k) jr[k] = min(max(j0 - 1 + k, 0), b.ny - 1) * b.nx;
#pragma unroll
    for (int k = 0; k < kResRows; ++k) {
        const int j = min(j0 + k, b.ny - 1);
        cym[k] = dp[b.cy + j];
        cyp[k] = dp[b.cy + b.ny + j];
        dy[k] = dp[b.cy + 2 * b.ny + j];
    }
    for (int it = i0; it < i1; ++it) {
        const int q = J.act[it];
        const double* __restrict__ pl = J.p + q * J.plane;
        const double* __restrict__ pq = pl + b.off;
        const double* __restrict__ fq = J.f + q * J.plane + b.off;
        const double sig = J.shift[q];
        double pc[kResRows + 2], xm[kResRows], xp[kResRows], fv[kResRows];
        const bool pz = J.pzero != 0;
#pragma unroll
        for (int k = 0; k < kResRows + 2; ++k) pc[k] = pz ? 0.0 : pq[jr[k] + ic];
#pragma unroll
        for (int k = 0; k < kResRows; ++k) {
            xm[k] = pz ? 0.0 : pq[jr[k + 1] + im];
            xp[k] = pz ? 0.0 : pq[jr[k + 1] + ip];
            fv[k] = fq[jr[k + 1] + ic];
        }
        double acc = 0.0, pacc = 0.0;
#pragma unroll
        for (int k = 0; k < kResRows; ++k) {
            const int j = j0 + k;
            if (i >= b.nx || j >= b.ny) continue;
            double vxm = xm[k], vxp = xp[k], vym = pc[k], vyp = pc[k + 2];
            // cells on a joined or periodic face take their neighbours by the
            // face rules; on a wall the face coefficient is zero, so the
            // clamped (finite) value already contributes nothing
            if (!pz && ((i == 0 && b.nbr[XM] >= 0) || (i == b.nx - 1 && b.nbr[XP] >= 0) ||
                        (j == 0 && b.nbr[YM] >= 0) || (j == b.ny - 1 && b.nbr[YP] >= 0)))
                neighbours(pl, B, b, i, j, vxm, vxp, vym, vyp);
            const double c = pc[k + 1];
            const double d = dx + dy[k] + sig;
            const double res = fv[k] - (cxm * vxm + cxp * vxp + cym[k] * vym + cyp[k] * vyp + d * c);
            acc += res * res;
            pacc += c * c;
            if (MODE == 1) {
                const long long o = q * J.plane + b.off + j * b.nx + i;
                J.r32[o] = float(res);
                if (J.e32) J.e32[o] = 0.0f;
            }
        }
        for (int o = 32; o > 0; o >>= 1) {  // one wave is one row group (blockDim.x = 64)
            acc += __shfl_xor(acc, o);
            pacc += __shfl_xor(pacc, o);
        }
        if (threadIdx.x == 0) {
            red[it - i0][threadIdx.y][0] = acc;
            red[it - i0][threadIdx.y][1] = pacc;
        }
    }
    __syncthreads();
    const int lane = threadIdx.x + threadIdx.y * blockDim.x;
    if (lane < i1 - i0) {
        double s = 0.0, sp = 0.0;
        for (int w = 0; w < kRowsPerPass; ++w) {
            s += red[lane][w][0];
            sp += red[lane][w][1];
        }
        const int q = J.act[i0 + lane];
        J.part[2 * ((long long)q * ntiles + tix)] = s;
        J.part[2 * ((long long)q * ntiles + tix) + 1] = sp;
    }
}

template <int MODE>
__global__ void __launch_bounds__(256) k_residual(const ResJob J) {
    residual_body<MODE>(J, blockIdx.x, blockIdx.y);
}

// Per-tile partial sums of fhat_q^2.
__global__ void __launch_bounds__(256)
k_sumsq(const DBlock* __restrict__ B, const int4* __restrict__ tiles, int ntiles,
        const double* __restrict__ f, long long plane, double* __restrict__ part) {
    __shared__ double scratch[8];
    const int q = blockIdx.y;
    const int tix = xcd_remap_mg(blockIdx.x, ntiles);
    const int4 t = tiles[tix];
    const DBlock b = B[t.x];
    const double* fq = f + q * plane;
    const int i = t.y + threadIdx.x;
    double acc = 0.0;
    if (i < b.nx)
        for (int r = threadIdx.y; r < kTileY; r += kRowsPerPass) {
            const int j = t.z + r;
            if (j >= b.ny) break;
            const double v = fq[b.off + j * b.nx + i];
            acc += v * v;
        }
    const double s = block_sum(acc, scratch);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        part[2 * ((long long)q * ntiles + tix)] = s;
        part[2 * ((long long)q * ntiles + tix) + 1] = 0.0;
    }
}

// Deterministic per-mode reduction of the tile partial pairs (one workgroup
// per item): out[q] = sum of first entries, out2[q] (optional) of seconds.
struct FinJob {
    const double* part;
    int ntiles;
    const int* act;
    const int* nact;
    double* out;
    double* out2;
};

__device__ __forceinline__ void finish_body(const FinJob& J, int item) {
    __shared__ double scratch[8];
    if (J.act && item >= *J.nact) return;
    const int q = J.act ? J.act[item] : item;
    const int ntiles = J.ntiles;
    double acc = 0.0, acc2 = 0.0;
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x) {
        acc += J.part[2 * ((long long)q * ntiles + t)];
        acc2 += J.part[2 * ((long long)q * ntiles + t) + 1];
    }
    const double s = block_sum(acc, scratch);
    const double s2 = block_sum(acc2, scratch);
    if (threadIdx.x == 0) {
        J.out[q] = s;
        if (J.out2) J.out2[q] = s2;
    }
}

__global__ void __launch_bounds__(256) k_finish(const FinJob J) { finish_body(J, blockIdx.x); }

// p += e on the whole plane of every active mode: an elementwise pass, so a
// workgroup takes a contiguous chunk of one mode's plane (coalesced, no tiles).
constexpr int kAddChunk = 2048;  // plane cells per workgroup (8 per thread)

struct AddJob {
    double* p;
    const float* e;
    long long plane;
    const int* act;
    const int* nact;
    int first;  // p is zero before the add: write e, do not read p
};

__device__ __forceinline__ void addcorr_body(const AddJob& J, int chunk, int item) {
    if (item >= *J.nact) return;
    const long long base = (long long)J.act[item] * J.plane;
    const long long c0 = (long long)chunk * kAddChunk + threadIdx.x;
#pragma unroll
    for (int k = 0; k < kAddChunk / 256; ++k) {
        const long long c = c0 + k * 256;
        if (c < J.plane) J.p[base + c] = (J.first ? 0.0 : J.p[base + c]) + double(J.e[base + c]);
    }
}

__global__ void __launch_bounds__(256) k_addcorr(const AddJob J) { addcorr_body(J, blockIdx.x, blockIdx.y); }

static int add_chunks(long long plane) { return int((plane + kAddChunk - 1) / kAddChunk); }

// Convergence bookkeeping after a residual evaluation (single workgroup):
// ratio_q = ||r_q||^2 / ||f_q||^2.  scal[0] = max ratio over the active list.
// With retirement, converged modes record the cycle count and leave the list.
struct UpdJob {
    int nz;
    const double* rnorm;
    const double* fnorm;
    const double* pnorm;
    const double* sabs;
    double rtol2, etol2;
    int retire, maxc;
    int* act;
    int* nact;
    int* cyc;
    double* scal;
    int* state;
    double* out;  // optional (host-visible): scal[0..1], state[0..3], nact after the update
};

__device__ __forceinline__ void update_body(const UpdJob& J) {
    const double* __restrict__ rnorm = J.rnorm;
    const double* __restrict__ fnorm = J.fnorm;
    const double* __restrict__ pnorm = J.pnorm;
    const double* __restrict__ sabs = J.sabs;
    const double rtol2 = J.rtol2, etol2 = J.etol2;
    const int retire = J.retire, maxc = J.maxc;
    int* __restrict__ act = J.act;
    int* __restrict__ nact = J.nact;
    int* __restrict__ cyc = J.cyc;
    double* __restrict__ scal = J.scal;
    int* __restrict__ state = J.state;
    // state[0]: non-finite rhs, state[1]: cycle counter, state[2]: max cycles reached
    __shared__ int keep[4096];
    __shared__ double mx[16];
    const int n = *nact;
    const int cycle = state[1];
    const bool stop = cycle >= maxc;
    double m = 0.0;
    for (int it = threadIdx.x; it < n; it += blockDim.x) {
        const int q = act[it];
        const double fn = fnorm[q];
        const double ratio = fn > 0.0 ? rnorm[q] / fn : (rnorm[q] > 0.0 ? 1e300 : 0.0);
        m = fmax(m, ratio);
        // estimated error ||r|| / (mu0 + |sigma|), doubled, against etol ||p||
        const bool err_ok = etol2 < 0.0 || 4.0 * rnorm[q] <= etol2 * sabs[q] * sabs[q] * pnorm[q];
        const bool done = ratio <= rtol2 && err_ok;
        keep[it] = done ? -1 : q;
        if (done || !retire || stop) cyc[q] = cycle;
    }
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) mx[threadIdx.x >> 6] = m;
    // modes still to run, in list order: a ballot prefix per wave, the wave
    // totals in LDS (retiring form: compacted into act, which every thread
    // has finished reading at the barrier below)
    __shared__ int wsum[16];
    __shared__ int kept;
    if (threadIdx.x == 0) kept = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = int(blockDim.x >> 6);
    for (int r0 = 0; r0 < n; r0 += blockDim.x) {
        const int it = r0 + threadIdx.x;
        const bool k = it < n && keep[it] >= 0;
        const unsigned long long mask = __ballot(k);
        if (lane == 0) wsum[wv] = __popcll(mask);
        __syncthreads();
        int off = kept;
        for (int v = 0; v < wv; ++v) off += wsum[v];
        if (k && retire) act[off + __popcll(mask & ((1ull << lane) - 1))] = keep[it];
        __syncthreads();
        if (threadIdx.x == 0)
            for (int v = 0; v < nw; ++v) kept += wsum[v];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double g = 0.0;
        for (int w = 0; w < nw; ++w) g = fmax(g, mx[w]);
        scal[0] = g;
        int c = kept;
        if (!retire) {  // lockstep: done when every mode passes both tests
            scal[1] = double(c);
        } else {
            if (stop && c > 0) {
                state[2] = 1;
                c = 0;
            }
            *nact = c;
        }
        if (stop && !retire && c > 0) state[2] = 1;
        state[1] = cycle + 1;
        if (J.out) {
            J.out[0] = scal[0];
            J.out[1] = scal[1];
            int* oi = reinterpret_cast<int*>(J.out + 2);
            for (int i = 0; i < 4; ++i) oi[i] = state[i];
            oi[4] = *nact;
        }
    }
}

__global__ void __launch_bounds__(1024) k_update(const UpdJob J) { update_body(J); }

__global__ void k_zero64(double* p, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

__global__ void k_fill_int(int* p, int n, int v) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = v;
}

__global__ void k_iota(int* act, int n, int* nact, int* cyc) {
    for (int i = threadIdx.x + blockIdx.x * blockDim.x; i < n; i += blockDim.x * gridDim.x) {
        act[i] = i;
        cyc[i] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *nact = n;
}

// Zero the planes of the modes that no V-cycle relaxed (cyc[q] == 0: they
// passed the test before the first cycle); the others were all written.
__global__ void k_zero_unrelaxed(double* __restrict__ p, long long plane, const int* __restrict__ cyc) {
    const int q = blockIdx.y;
    if (cyc[q] != 0) return;
    double* pq = p + q * plane;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < plane;
         i += (long long)gridDim.x * blockDim.x)
        pq[i] = 0.0;
}

// sum(a x) over one plane (single workgroup, fixed order).
__global__ void __launch_bounds__(1024)
k_area_dot(const double* __restrict__ x, const double* __restrict__ a, long long n,
           double* __restrict__ out) {
    __shared__ double scratch[16];
    constexpr int kBatch = 8;  // elements per thread whose loads go out together
    double acc = 0.0;
    for (long long i0 = threadIdx.x; i0 < n; i0 += kBatch * (long long)blockDim.x) {
        double av[kBatch], xv[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const long long i = min(i0 + k * (long long)blockDim.x, n - 1);  // in bounds, no branch
            av[k] = a[i];
            xv[k] = x[i];
        }
#pragma unroll
        for (int k = 0; k < kBatch; ++k)
            acc += i0 + k * (long long)blockDim.x < n ? av[k] * xv[k] : 0.0;
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < int(blockDim.x >> 6); ++w) s += scratch[w];
        out[0] = s;
    }
}

__global__ void k_sub(double* __restrict__ x, long long n, const double* __restrict__ num, double den) {
    const double m = num[0] / den;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        x[i] -= m;
}

// (L_h - alpha) p at cell c = (b, k, j, i) of the packed 3D field: x-y part
// from the level-0 tables, z part with the ghost rules of the pair (N: g =
// p0, D: g = -p0, P: wrap), alpha the Helmholtz term (0 for the pressure
// equation).
__device__ __forceinline__ double apply3d_value(const DBlock* __restrict__ B, const DBlock& b,
                                                const double* __restrict__ dp, const double* __restrict__ p,
                                                int nz, double idz2, int zkind, double alpha, int i, int j, int k,
                                                long long c) {
    const long long cols = (long long)b.nx * b.ny;
    const double v = p[c];
    // x-y neighbours (other blocks addressed through their own base)
    auto at = [&](const DBlock& bb, int ii, int jj) __attribute__((always_inline)) {
        return p[(long long)bb.off * nz + k * (long long)bb.nx * bb.ny + jj * bb.nx + ii];
    };
    double xm = 0, xp = 0, ym = 0, yp = 0;
    if (i > 0) xm = p[c - 1];
    else if (b.nbr[XM] >= 0) { const DBlock& kk = B[b.nbr[XM]]; xm = at(kk, kk.nx - 1, j); }
    if (i < b.nx - 1) xp = p[c + 1];
    else if (b.nbr[XP] >= 0) { const DBlock& kk = B[b.nbr[XP]]; xp = at(kk, 0, j); }
    if (j > 0) ym = p[c - b.nx];
    else if (b.nbr[YM] >= 0) { const DBlock& kk = B[b.nbr[YM]]; ym = at(kk, i, kk.ny - 1); }
    if (j < b.ny - 1) yp = p[c + b.nx];
    else if (b.nbr[YP] >= 0) { const DBlock& kk = B[b.nbr[YP]]; yp = at(kk, i, 0); }
    double zm, zp;
    if (k > 0) zm = p[c - cols];
    else zm = zkind == Z_PP ? p[c + (nz - 1) * cols] : ((zkind == Z_NN || zkind == Z_ND) ? v : -v);
    if (k < nz - 1) zp = p[c + cols];
    else zp = zkind == Z_PP ? p[c - (nz - 1) * cols] : ((zkind == Z_NN || zkind == Z_DN) ? v : -v);
    const double d = dp[b.cx + 2 * b.nx + i] + dp[b.cy + 2 * b.ny + j] - alpha;
    return dp[b.cx + i] * xm + dp[b.cx + b.nx + i] * xp + dp[b.cy + j] * ym + dp[b.cy + b.ny + j] * yp +
           d * v + (zm - 2.0 * v + zp) * idz2;
}

__global__ void __launch_bounds__(256)
k_apply3d(const DBlock* __restrict__ B, const int4* __restrict__ tiles, int ntiles,
          const double* __restrict__ dp, const double* __restrict__ p, double* __restrict__ out,
          int nz, double idz2, int zkind, double alpha) {
    const int k = blockIdx.y;
    const int4 t = tiles[xcd_remap_mg(blockIdx.x, ntiles)];
    const DBlock b = B[t.x];
    const long long base = (long long)b.off * nz;  // block start in the packed field
    const int i = t.y + threadIdx.x;
    if (i >= b.nx) return;
    for (int r = threadIdx.y; r < kTileY; r += kRowsPerPass) {
        const int j = t.z + r;
        if (j >= b.ny) break;
        const long long c = base + k * (long long)b.nx * b.ny + j * b.nx + i;
        out[c] = apply3d_value(B, b, dp, p, nz, idz2, zkind, alpha, i, j, k, c);
    }
}

// Final check of a solve (every cell of the packed field): per-workgroup
// partial sums of (f - shift - (L_h - alpha) p)^2 into part[w] and of
// (f - shift)^2 into part[nw + w], nw = workgroups of the launch.
__global__ void __launch_bounds__(256)
k_resnorm3d(const DBlock* __restrict__ B, const int4* __restrict__ tiles, int ntiles,
            const double* __restrict__ dp, const double* __restrict__ p, const double* __restrict__ f,
            double shift, int nz, double idz2, int zkind, double alpha, double* __restrict__ part) {
    const int k = blockIdx.y;
    const int4 t = tiles[xcd_remap_mg(blockIdx.x, ntiles)];
    const DBlock b = B[t.x];
    const long long base = (long long)b.off * nz;
    const int i = t.y + threadIdx.x;
    double rr = 0.0, ff = 0.0;
    if (i < b.nx)
        for (int r = threadIdx.y; r < kTileY; r += kRowsPerPass) {
            const int j = t.z + r;
            if (j >= b.ny) break;
            const long long c = base + k * (long long)b.nx * b.ny + j * b.nx + i;
            const double fv = f[c] - shift;
            const double res = fv - apply3d_value(B, b, dp, p, nz, idz2, zkind, alpha, i, j, k, c);
            rr += res * res;
            ff += fv * fv;
        }
    __shared__ double red[8];
    const long long w = (long long)blockIdx.y * gridDim.x + blockIdx.x;
    const long long nw = (long long)gridDim.y * gridDim.x;
    const double sr = block_sum(rr, red);
    if (threadIdx.x == 0 && threadIdx.y == 0) part[w] = sr;
    const double sf = block_sum(ff, red);
    if (threadIdx.x == 0 && threadIdx.y == 0) part[nw + w] = sf;
}

// out[0] = sqrt(sum part[0, n)), out[1] = sqrt(sum part[n, 2n)).
__global__ void __launch_bounds__(1024) k_resnorm_finish(const double* __restrict__ part, long long n,
                                                         double* __restrict__ out) {
    __shared__ double red[16];
    for (int h = 0; h < 2; ++h) {
        double acc = 0.0;
        for (long long e = threadIdx.x; e < n; e += blockDim.x) acc += part[h * n + e];
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
        __syncthreads();
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s2 = 0.0;
            for (int w = 0; w < int(blockDim.x >> 6); ++w) s2 += red[w];
            out[h] = sqrt(s2);
        }
    }
}

// ============================ LDS-resident levels ============================

struct LdsArgs {
    const DBlock* Ball;  // every level's blocks
    const double* dp;
    const int* ip;
    int lvinfo;          // int-pool offset of {plane, blk_off, tile_off, ntiles} per level
    int nlev, L, nb;
    int nu1, nu2;
    const double* cwl;   // coarsest eigen tables
    const double* cwr;
    const double* cmu;
    double cmumax;       // max |cmu| (host)
    int nc;
    int dpb, dpn, ipb, ipn;  // pool ranges of the tables of levels L.. (copied into LDS)
    int fglob;           // level L's rhs is read from device memory, not copied into LDS
    const double* cdp;   // in the kernel: the copies, indexed like the pools
    const int* cip;
    int nthr;            // in the kernel: threads of the workgroup, held in a register
                         // (blockDim.x is a memory load that each loop would repeat)
};

template <typename T>
struct LdsView {
    T* base;             // LDS image: per level l >= L: p (plane) then f (plane; not
                         // for level L when its rhs stays in device memory)
    T* fL;               // level L's rhs (LDS or device memory)
    double* ctmp;        // coarse temp (nc doubles)
    double* red;         // reduction scratch (16 doubles)
    double* tdp;         // copy of the levels' coefficient / transfer tables
    int* tip;            //   and index tables
    DBlock* tblk;        //   and block descriptors
};

template <typename T>
__device__ __forceinline__ T* lds_p(const LdsArgs& a, const LdsView<T>& v, int l) {
    long long o = 0;
    for (int k = a.L; k < l; ++k) o += (k == a.L && a.fglob ? 1LL : 2LL) * a.ip[a.lvinfo + 4 * k];
    return v.base + o;
}

// On the small levels (at most two cells per thread) the three phases below
// spread the cells of all blocks over the workgroup at once (cell h of the
// level's list is found by a scan of the per-block counts): a block's cells
// then do not wait for the previous block's, which would put one latency
// chain per block in every phase.  Larger levels go block by block, with the
// block's descriptor in scalar registers.

// Cells of one colour in block b (red-black blocks only).
__device__ __forceinline__ int colour_cells(const DBlock& b) { return ((b.nx + 1) >> 1) * b.ny; }

template <typename T>
__device__ void lds_smooth(const LdsArgs& a, T* p, const T* f, const DBlock* B, T sig, int colour) {
    bool any_odd = false;
    int total = 0;
    for (int bi = 0; bi < a.nb; ++bi) {
        any_odd |= B[bi].oddwrap != 0;
        if (B[bi].oddwrap == 0) total += colour_cells(B[bi]);
    }
    if (total > 2 * a.nthr) {
        for (int bi = 0; bi < a.nb; ++bi) {
            const DBlock b = wave_uniform(B[bi]);
            if (b.oddwrap != 0) continue;
            const int hx = (b.nx + 1) >> 1;
            const int cnt = hx * b.ny;
            for (int h = threadIdx.x; h < cnt; h += a.nthr) {
                const int j = h / hx;
                const int i = 2 * (h - j * hx) + ((colour + j + b.par) & 1);
                if (i < b.nx) p[b.off + j * b.nx + i] = gs_value(p, f, B, b, a.cdp, i, j, sig);
            }
        }
    } else {
        for (int h = threadIdx.x; h < total; h += a.nthr) {
            int bi = 0, r = h;
            for (;; ++bi) {
                if (B[bi].oddwrap != 0) continue;
                const int c = colour_cells(B[bi]);
                if (r < c) break;
                r -= c;
            }
            const DBlock& b = B[bi];
            const int hx = (b.nx + 1) >> 1;
            const int j = r / hx;
            const int i = 2 * (r - j * hx) + ((colour + j + b.par) & 1);
            if (i < b.nx) p[b.off + j * b.nx + i] = gs_value(p, f, B, b, a.cdp, i, j, sig);
        }
    }
    if (any_odd) {  // blocks with an odd periodic wrap: per block, by colour
        for (int bi = 0; bi < a.nb; ++bi) {
            const DBlock b = wave_uniform(B[bi]);
            if (b.oddwrap == 0) continue;
            const int cnt = b.nx * b.ny;
            for (int c = threadIdx.x; c < cnt; c += a.nthr) {
                const int j = c / b.nx, i = c - j * b.nx;
                if (colour_of(b, i, j) != colour) continue;
                p[b.off + c] = gs_value(p, f, B, b, a.cdp, i, j, sig);
            }
        }
    }
    // cells of one colour are never neighbours, also across blocks
    __syncthreads();
    if (any_odd && colour == 1) {  // the two extra colours of odd periodic wraps
        for (int extra = 2; extra < 4; ++extra) {
            for (int bi = 0; bi < a.nb; ++bi) {
                const DBlock b = wave_uniform(B[bi]);
                if (b.oddwrap == 0) continue;
                const int cnt = b.nx * b.ny;
                for (int c = threadIdx.x; c < cnt; c += a.nthr) {
                    const int j = c / b.nx, i = c - j * b.nx;
                    if (colour_of(b, i, j) != extra) continue;
                    p[b.off + c] = gs_value(p, f, B, b, a.cdp, i, j, sig);
                }
            }
            __syncthreads();
        }
    }
}

// Cell h of the concatenated cells of the level's blocks: block index and
// index inside the block (the block offsets are the packed plane offsets).
__device__ __forceinline__ int block_of(const DBlock* B, int nb, int h) {
    int bi = 0;
    while (bi + 1 < nb && h >= B[bi + 1].off) ++bi;
    return bi;
}

template <typename T>
__device__ void lds_restrict(const LdsArgs& a, const T* pf, const T* ff, T* pc, T* fc,
                             const DBlock* Bf, const DBlock* Bc, T sig) {
    const int total = Bc[a.nb - 1].off + Bc[a.nb - 1].nx * Bc[a.nb - 1].ny;
    if (total > 2 * a.nthr) {
        for (int bi = 0; bi < a.nb; ++bi) {
            const DBlock bc = wave_uniform(Bc[bi]);
            const DBlock bf = wave_uniform(Bf[bi]);
            const int cnt = bc.nx * bc.ny;
            for (int c = threadIdx.x; c < cnt; c += a.nthr) {
                const int J = c / bc.nx, I = c - J * bc.nx;
                fc[bc.off + c] = restrict_at(pf, ff, Bf, bf, a.cdp, a.cip, I, J, sig);
                pc[bc.off + c] = T(0);
            }
        }
    } else {
        for (int h = threadIdx.x; h < total; h += a.nthr) {
            const int bi = block_of(Bc, a.nb, h);
            const DBlock& bc = Bc[bi];
            const int c = h - bc.off;
            const int J = c / bc.nx, I = c - J * bc.nx;
            fc[h] = restrict_at(pf, ff, Bf, Bf[bi], a.cdp, a.cip, I, J, sig);
            pc[h] = T(0);
        }
    }
    __syncthreads();
}

template <typename T>
__device__ void lds_prolong(const LdsArgs& a, const T* pc, T* pf, const DBlock* Bf, const DBlock* Bc) {
    const int total = Bf[a.nb - 1].off + Bf[a.nb - 1].nx * Bf[a.nb - 1].ny;
    if (total > 2 * a.nthr) {
        for (int bi = 0; bi < a.nb; ++bi) {
            const DBlock bf = wave_uniform(Bf[bi]);
            const int cnt = bf.nx * bf.ny;
            for (int c = threadIdx.x; c < cnt; c += a.nthr) {
                const int j = c / bf.nx, i = c - j * bf.nx;
                pf[bf.off + c] += prolong_at(pc, Bc, bf, bi, a.cdp, a.cip, i, j);
            }
        }
    } else {
        for (int h = threadIdx.x; h < total; h += a.nthr) {
            const int bi = block_of(Bf, a.nb, h);
            const DBlock& bf = Bf[bi];
            const int c = h - bf.off;
            const int j = c / bf.nx, i = c - j * bf.nx;
            pf[h] += prolong_at(pc, Bc, bf, bi, a.cdp, a.cip, i, j);
        }
    }
    __syncthreads();
}

// Exact coarsest solve in float64: x = Wl diag(1/(mu + sigma)) Wr b, with the
// null mode (mu + sigma = 0, singular plane) dropped.
// Both products run kCoarseLanes lanes per row, each summing a strided part
// of it, so a lane has only nc / kCoarseLanes dependent loads of the
// (device-memory) eigenvector tables in its chain.
constexpr int kCoarseLanes = 8;

template <typename T>
__device__ void lds_coarse(const LdsArgs& a, const LdsView<T>& v, T* p, const T* f, double sig) {
    const int nc = a.nc;
    const double mumax = a.cmumax;
    const int g = threadIdx.x & (kCoarseLanes - 1);
    const int rows = a.nthr / kCoarseLanes;
    for (int k0 = 0; k0 < nc; k0 += rows) {
        const int k = k0 + threadIdx.x / kCoarseLanes;
        double acc = 0.0;
        if (k < nc) {
            const double* row = a.cwr + (long long)k * nc;
#pragma unroll 4
            for (int j = g; j < nc; j += kCoarseLanes) acc += row[j] * double(f[j]);
        }
        for (int o = 1; o < kCoarseLanes; o <<= 1) acc += __shfl_xor(acc, o);
        if (k < nc && g == 0) {
            const double d = a.cmu[k] + sig;
            v.ctmp[k] = fabs(d) > 1e-11 * (mumax + fabs(sig)) ? acc / d : 0.0;
        }
    }
    __syncthreads();
    for (int i0 = 0; i0 < nc; i0 += rows) {
        const int i = i0 + threadIdx.x / kCoarseLanes;
        double acc = 0.0;
        if (i < nc) {
            const double* row = a.cwl + (long long)i * nc;
#pragma unroll 4
            for (int k = g; k < nc; k += kCoarseLanes) acc += row[k] * v.ctmp[k];
        }
        for (int o = 1; o < kCoarseLanes; o <<= 1) acc += __shfl_xor(acc, o);
        if (i < nc && g == 0) p[i] = T(acc);
    }
    __syncthreads();
}

template <typename T>
__device__ void lds_vcycle(const LdsArgs& a, const LdsView<T>& v, double sigd) {
    const T sig = T(sigd);
    for (int l = a.L; l < a.nlev - 1; ++l) {
        const DBlock* Bf = a.Ball + a.ip[a.lvinfo + 4 * l + 1];
        const DBlock* Bc = a.Ball + a.ip[a.lvinfo + 4 * (l + 1) + 1];
        T* pf = lds_p(a, v, l);
        T* ff = l == a.L ? v.fL : pf + a.ip[a.lvinfo + 4 * l];
        T* pc = lds_p(a, v, l + 1);
        T* fc = pc + a.ip[a.lvinfo + 4 * (l + 1)];
        for (int s = 0; s < a.nu1; ++s) {
            lds_smooth(a, pf, ff, Bf, sig, 0);
            lds_smooth(a, pf, ff, Bf, sig, 1);
        }
        lds_restrict(a, pf, ff, pc, fc, Bf, Bc, sig);
    }
    {
        T* pc = lds_p(a, v, a.nlev - 1);
        T* fc = pc + a.ip[a.lvinfo + 4 * (a.nlev - 1)];
        lds_coarse(a, v, pc, fc, sigd);
    }
    for (int l = a.nlev - 2; l >= a.L; --l) {
        const DBlock* Bf = a.Ball + a.ip[a.lvinfo + 4 * l + 1];
        const DBlock* Bc = a.Ball + a.ip[a.lvinfo + 4 * (l + 1) + 1];
        T* pf = lds_p(a, v, l);
        T* ff = l == a.L ? v.fL : pf + a.ip[a.lvinfo + 4 * l];
        const T* pc = lds_p(a, v, l + 1);
        lds_prolong(a, pc, pf, Bf, Bc);
        for (int s = 0; s < a.nu2; ++s) {
            lds_smooth(a, pf, ff, Bf, sig, 0);
            lds_smooth(a, pf, ff, Bf, sig, 1);
        }
    }
}

template <typename T>
__device__ LdsView<T> lds_view(const LdsArgs& a, unsigned char* raw) {
    LdsView<T> v;
    v.base = reinterpret_cast<T*>(raw);
    long long e = 0;
    for (int l = a.L; l < a.nlev; ++l) e += (l == a.L && a.fglob ? 1LL : 2LL) * a.ip[a.lvinfo + 4 * l];
    long long bytes = (e * (long long)sizeof(T) + 15) & ~15LL;
    v.ctmp = reinterpret_cast<double*>(raw + bytes);
    v.red = v.ctmp + ((a.nc + 1) & ~1);
    v.tdp = v.red + 16;
    v.tip = reinterpret_cast<int*>(v.tdp + a.dpn);
    v.tblk = reinterpret_cast<DBlock*>(v.tip + a.ipn);
    v.fL = v.base + a.ip[a.lvinfo + 4 * a.L];  // after level L's p (unless fglob)
    return v;
}

// Copy the level tables and block descriptors into LDS and point the stencil
// routines at the copies (the pointers are rebased so that pool offsets and
// block indices index them directly): a neighbour lookup across a joined
// face then costs an LDS read, not a dependent device-memory load.
template <typename T>
__device__ __forceinline__ void lds_tables(LdsArgs& a, const LdsView<T>& v) {
    a.nthr = __builtin_amdgcn_readfirstlane(int(blockDim.x));
    for (int t = threadIdx.x; t < a.dpn; t += a.nthr) v.tdp[t] = a.dp[a.dpb + t];
    for (int t = threadIdx.x; t < a.ipn; t += a.nthr) v.tip[t] = a.ip[a.ipb + t];
    const int blk0 = a.ip[a.lvinfo + 4 * a.L + 1];
    constexpr int kWords = int(sizeof(DBlock) / sizeof(int));
    const int words = (a.nlev - a.L) * a.nb * kWords;
    const int* src = reinterpret_cast<const int*>(a.Ball + blk0);
    int* dst = reinterpret_cast<int*>(v.tblk);
    for (int t = threadIdx.x; t < words; t += a.nthr) dst[t] = src[t];
    a.cdp = v.tdp - a.dpb;
    a.cip = v.tip - a.ipb;
    a.Ball = v.tblk - blk0;
}

// One V-cycle on levels L.. of every active mode: f_L in, p_L out (from 0).
template <typename T>
struct LdsJob {
    LdsArgs a;
    T* pL;
    const T* fL;
    long long planeL;
    const double* shift;
    const int* act;
    const int* nact;
};

template <typename T>
__device__ __forceinline__ void lds_vcycle_body(const LdsJob<T>& J, int item) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    if (item >= *J.nact) return;
    LdsArgs a = J.a;
    const long long planeL = J.planeL;
    const int q = J.act[item];
    LdsView<T> v = lds_view<T>(a, lds_raw);
    lds_tables(a, v);
    T* p = lds_p(a, v, a.L);
    if (a.fglob) {
        // the rhs is only read; the sweeps and the restriction take it from
        // device memory (just written by the level above, so cached)
        v.fL = const_cast<T*>(J.fL + q * planeL);
        for (long long c = threadIdx.x; c < planeL; c += a.nthr) p[c] = T(0);
    } else {
        T* f = v.fL;
        for (long long c = threadIdx.x; c < planeL; c += a.nthr) {
            f[c] = J.fL[q * planeL + c];
            p[c] = T(0);
        }
    }
    __syncthreads();
    lds_vcycle(a, v, J.shift[q]);
    for (long long c = threadIdx.x; c < planeL; c += a.nthr) J.pL[q * planeL + c] = p[c];
}

template <typename T>
__global__ void __launch_bounds__(1024) k_lds_vcycle(const LdsJob<T> J) {
    lds_vcycle_body<T>(J, blockIdx.x);
}

__device__ double lds_block_sum(double x, double* red, int nthr) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < (nthr >> 6); ++w) s += red[w];
    __syncthreads();
    return s;  // every thread holds the same sum
}

// Whole solve of one mode in LDS (the plane's full hierarchy fits): iterate
// V-cycles until ||r_q||^2 <= rtol2 ||f_q||^2 or maxc cycles; each mode stops
// on its own (early retirement).
__global__ void __launch_bounds__(1024)
k_lds_full(LdsArgs a, double* __restrict__ p0, const double* __restrict__ f0, long long plane,
           const double* __restrict__ shift, const double* __restrict__ sabs,
           const int* __restrict__ act, const int* __restrict__ nact, int maxc, double rtol2,
           double etol2, int* __restrict__ cyc, double* __restrict__ rnorm,
           double* __restrict__ fnorm) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int item = blockIdx.x;
    if (item >= *nact) return;
    const int q = act[item];
    LdsView<double> v = lds_view<double>(a, lds_raw);
    lds_tables(a, v);
    double* p = v.base;
    double* f = p + plane;
    const DBlock* B = a.Ball + a.ip[a.lvinfo + 1];
    double fs = 0.0;
    for (long long c = threadIdx.x; c < plane; c += a.nthr) {
        const double x = f0[q * plane + c];
        f[c] = x;
        p[c] = p0[q * plane + c];
        fs += x * x;
    }
    const double fn = lds_block_sum(fs, v.red, a.nthr);
    const double sig = shift[q];
    int c = 0;
    double rn = 0.0;
    const double sa = sabs[q];
    for (;; ++c) {
        double rs = 0.0, ps = 0.0;
        for (int bi = 0; bi < a.nb; ++bi) {
            const DBlock b = B[bi];
            const int cnt = b.nx * b.ny;
            for (int k = threadIdx.x; k < cnt; k += a.nthr) {
                const int j = k / b.nx, i = k - j * b.nx;
                const double r = f[b.off + k] - apply_at(p, B, b, a.cdp, i, j, sig);
                rs += r * r;
                ps += p[b.off + k] * p[b.off + k];
            }
        }
        rn = lds_block_sum(rs, v.red, a.nthr);
        const double pn = lds_block_sum(ps, v.red, a.nthr);
        const bool err_ok = etol2 < 0.0 || 4.0 * rn <= etol2 * sa * sa * pn;
        if ((rn <= rtol2 * fn && err_ok) || c >= maxc) break;
        lds_vcycle(a, v, sig);
    }
    for (long long k = threadIdx.x; k < plane; k += a.nthr) p0[q * plane + k] = p[k];
    if (threadIdx.x == 0) {
        cyc[q] = c;
        rnorm[q] = rn;
        fnorm[q] = fn;
    }
}

// ================================ launchers ================================

// Threads of an LDS-resident workgroup: one workgroup holds a whole CU's LDS,
// so it brings its own waves to hide the latency of its sweeps.
static int lds_threads(int64_t plane) { return plane >= 4096 ? 1024 : plane >= 1024 ? 512 : 256; }

static LdsArgs lds_args(const mbp_plan* P, int L) {
    LdsArgs a{};
    a.Ball = P->d_blk;
    a.dp = P->d_dbl;
    a.ip = P->d_int;
    a.lvinfo = P->lvinfo;
    a.nlev = P->nlev;
    a.L = L;
    a.nb = P->g.nb;
    a.nu1 = P->opt.nu1;
    a.nu2 = P->opt.nu2;
    a.cwl = P->d_cwl;
    a.cwr = P->d_cwr;
    a.cmu = P->d_cmu;
    a.cmumax = 0.0;
    for (double mu : P->coarse_mu) a.cmumax = std::max(a.cmumax, std::fabs(mu));
    a.nc = P->coarse_n;
    a.dpb = P->levels[L].dp_begin;
    a.dpn = P->dp_levels_end - a.dpb;
    a.ipb = P->levels[L].ip_begin;
    a.ipn = P->ip_levels_end - a.ipb;
    return a;
}

template <typename T>
static T* level_p(const mbp_plan* P, int l);
template <>
double* level_p<double>(const mbp_plan* P, int l) { return P->p64[l]; }
template <>
float* level_p<float>(const mbp_plan* P, int l) { return P->p32[l]; }
template <typename T>
static T* level_f(const mbp_plan* P, int l);
template <>
double* level_f<double>(const mbp_plan* P, int l) { return P->f64[l]; }
template <>
float* level_f<float>(const mbp_plan* P, int l) { return P->f32[l]; }

// Raise a kernel's dynamic LDS limit once per device and size, so that
// launches recorded into a graph later never need the call.
static void set_lds(const void* fn, size_t bytes) {
    if (bytes <= 64 * 1024) return;
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, size_t> done;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(mu);
    size_t& have = done[{fn, dev}];
    if (have >= bytes) return;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes)) == hipSuccess) have = bytes;
}

template <typename T>
static T* level_pB(const mbp_plan* P, int l);
template <>
double* level_pB<double>(const mbp_plan* P, int l) { return P->p64B[l]; }
template <>
float* level_pB<float>(const mbp_plan* P, int l) { return P->p32B[l]; }

template <typename T>
int launch_vcycle(const mbp_plan* P, T* p0, T* p0B, T* f0, const int* act, const int* nact, int nitems,
                  bool norm0, bool zero0, hipStream_t s) {
    const bool is32 = sizeof(T) == 4;
    const int L = is32 ? P->lds_level32 : P->lds_level;
    const dim3 blk(kTileX, kRowsPerPass);
    const int nu1 = P->opt.nu1, nu2 = P->opt.nu2;
    const bool fused_ok = ((nu1 + nu2) % 2 == 0) && nu1 >= 1 && nu2 >= 1;
    auto P_ = [&](int l) -> T* { return l == 0 ? p0 : level_p<T>(P, l); };
    auto PB_ = [&](int l) -> T* { return l == 0 ? p0B : level_pB<T>(P, l); };
    auto F_ = [&](int l) -> T* { return l == 0 ? f0 : level_f<T>(P, l); };
    auto use_march = [&](int l) __attribute__((always_inline)) { return fused_ok && P->march_ok[l] && PB_(l) != nullptr; };
    auto rbgs = [&](int l) __attribute__((always_inline)) {
        const Level& Lf = P->levels[l];
        for (int colour = 0; colour < (Lf.oddwrap ? 4 : 2); ++colour)
            hipLaunchKernelGGL(k_rbgs<T>, dim3(Lf.ntiles, nitems), blk, 0, s, P->d_blk + Lf.blk_off,
                               P->d_tiles + Lf.tile_off, Lf.ntiles, P->d_dbl, P_(l), F_(l),
                               (long long)Lf.plane, P->d_shift, act, nact, colour);
    };
    for (int l = 0; l < L; ++l) {
        const Level& Lf = P->levels[l];
        const Level& Lc = P->levels[l + 1];
        if (use_march(l)) {
            // sweeps alternate A -> B -> A ...; the restricting sweep ends in B.
            // Coarse levels start from zero, so their first sweep reads no p;
            // the next level needs zeros written only if it reads its guess.
            bool zin = l == 0 ? zero0 : true;
            T* a = P_(l);
            T* b = PB_(l);
            for (int it = 0; it + 1 < nu1; ++it) {
                march_sweep<T>(P, l, a, b, F_(l), act, nact, nitems, zin, s);
                zin = false;
                std::swap(a, b);
            }
            T* pc = (l + 1 < L && !use_march(l + 1)) ? P_(l + 1) : nullptr;
            if (l == 0) prof_begin(P, 0, s, double(Lf.plane) * nitems);
            march_pre<T>(P, l, a, b, F_(l), F_(l + 1), pc, act, nact, nitems, zin, s);
            if (l == 0) prof_end(P, 0, s);
        } else {
            for (int it = 0; it < nu1; ++it) rbgs(l);
            hipLaunchKernelGGL(k_restrict<T>, dim3(Lc.ntiles, nitems), blk, 0, s, P->d_blk + Lf.blk_off,
                               P->d_blk + Lc.blk_off, P->d_tiles + Lc.tile_off, Lc.ntiles, P->d_dbl,
                               P->d_int, P_(l), F_(l), F_(l + 1), P_(l + 1), (long long)Lf.plane,
                               (long long)Lc.plane, P->d_shift, act, nact);
        }
    }
    {
        LdsArgs a = lds_args(P, L);
        a.fglob = is32 ? 0 : P->lds_fglob64;
        const size_t bytes = size_t(is32 ? P->lds_bytes32 : P->lds_bytes64);
        set_lds(reinterpret_cast<const void*>(k_lds_vcycle<T>), bytes);
        const LdsJob<T> J{a, P_(L), F_(L), (long long)P->levels[L].plane, P->d_shift, act, nact};
        hipLaunchKernelGGL(k_lds_vcycle<T>, dim3(nitems), dim3(lds_threads(P->levels[L].plane)), bytes, s, J);
    }
    int nparts = 0;
    for (int l = L - 1; l >= 0; --l) {
        const Level& Lf = P->levels[l];
        const Level& Lc = P->levels[l + 1];
        if (use_march(l)) {
            // the current iterate sits in A after nu1 - 1 swaps and one more sweep: B if nu1 odd
            T* a = P_(l);
            T* b = PB_(l);
            T* cur = (nu1 % 2 == 1) ? b : a;
            T* oth = (cur == a) ? b : a;
            const bool nrm = norm0 && l == 0 && nu2 == 1;
            if (l == 0) prof_begin(P, 1, s, double(Lf.plane) * nitems);
            march_post<T>(P, l, cur, oth, F_(l), P_(l + 1), nrm, act, nact, nitems, s);
            if (l == 0) prof_end(P, 1, s);
            std::swap(cur, oth);
            for (int it = 1; it < nu2; ++it) {
                const bool last = it == nu2 - 1;
                if (norm0 && l == 0 && last) {
                    // extra sweeps do not carry the norm; the caller evaluates it
                }
                march_sweep<T>(P, l, cur, oth, F_(l), act, nact, nitems, false, s);
                std::swap(cur, oth);
            }
            if (nrm) nparts = 4 * P->mtile_cnt[0];  // one partial pair per wave of each strip
        } else {
            hipLaunchKernelGGL(k_prolong<T>, dim3(Lf.ntiles, nitems), blk, 0, s, P->d_blk + Lf.blk_off,
                               P->d_blk + Lc.blk_off, P->d_tiles + Lf.tile_off, Lf.ntiles, P->d_dbl,
                               P->d_int, P_(l + 1), P_(l), (long long)Lf.plane, (long long)Lc.plane, act,
                               nact);
            for (int it = 0; it < nu2; ++it) rbgs(l);
        }
    }
    return nparts;
}

template int launch_vcycle<double>(const mbp_plan*, double*, double*, double*, const int*, const int*,
                                   int, bool, bool, hipStream_t);
template int launch_vcycle<float>(const mbp_plan*, float*, float*, float*, const int*, const int*, int,
                                  bool, bool, hipStream_t);

__global__ void k_norm_from_rhs(const double* __restrict__ fnorm, double* __restrict__ rnorm,
                                double* __restrict__ pnorm, const int* __restrict__ act,
                                const int* __restrict__ nact) {
    const int item = blockIdx.x * blockDim.x + threadIdx.x;
    if (item >= *nact) return;
    const int q = act[item];
    rnorm[q] = fnorm[q];
    pnorm[q] = 0.0;
}

void launch_norm_from_rhs(const mbp_plan* P, int nitems, hipStream_t s) {
    hipLaunchKernelGGL(k_norm_from_rhs, dim3((nitems + 255) / 256), dim3(256), 0, s, P->d_fnorm, P->d_rnorm,
                       P->d_pnorm, P->d_act, P->d_nact);
}

void launch_finish(const mbp_plan* P, int nparts, double* out, const int* act, const int* nact,
                   int nitems, hipStream_t s) {
    const FinJob F{P->d_part, nparts, act, nact, out, P->d_pnorm};
    hipLaunchKernelGGL(k_finish, dim3(nitems), dim3(256), 0, s, F);
}

void launch_lds_full(const mbp_plan* P, double* p, const double* f, const int* act, const int* nact,
                     int nitems, int maxc, double rtol2, double etol2, int* cyc, double* rnorm,
                     double* fnorm, hipStream_t s) {
    LdsArgs a = lds_args(P, 0);
    const size_t bytes = size_t(P->lds_bytes64);
    set_lds(reinterpret_cast<const void*>(k_lds_full), bytes);
    hipLaunchKernelGGL(k_lds_full, dim3(nitems), dim3(lds_threads(P->plane0)), bytes, s, a, p, f,
                       (long long)P->plane0, P->d_shift, P->d_sabs, act, nact, maxc, rtol2, etol2, cyc,
                       rnorm, fnorm);
}

void launch_residual_norm(const mbp_plan* P, const double* p, const double* f, double* rnorm,
                          const int* act, const int* nact, int nitems, hipStream_t s) {
    const Level& L = P->levels[0];
    const int per = res_per(L.ntiles, nitems);
    const ResJob J{P->d_blk + L.blk_off, P->d_tiles + L.tile_off, L.ntiles, P->d_dbl, p, f,
                   (long long)L.plane, P->d_shift, act, nact, P->d_part, nullptr, nullptr, per};
    hipLaunchKernelGGL(k_residual<0>, dim3(L.ntiles, (nitems + per - 1) / per), dim3(kTileX, kRowsPerPass), 0, s, J);
    const FinJob F{P->d_part, L.ntiles, act, nact, rnorm, P->d_pnorm};
    hipLaunchKernelGGL(k_finish, dim3(nitems), dim3(256), 0, s, F);
}

void launch_residual_to32(const mbp_plan* P, const double* p, const double* f, float* r32, float* e32,
                          double* rnorm, const int* act, const int* nact, int nitems, hipStream_t s,
                          bool pzero) {
    const Level& L = P->levels[0];
    const int per = res_per(L.ntiles, nitems);
    const ResJob J{P->d_blk + L.blk_off, P->d_tiles + L.tile_off, L.ntiles, P->d_dbl, p, f,
                   (long long)L.plane, P->d_shift, act, nact, P->d_part, r32, e32, per, pzero ? 1 : 0};
    hipLaunchKernelGGL(k_residual<1>, dim3(L.ntiles, (nitems + per - 1) / per), dim3(kTileX, kRowsPerPass), 0, s, J);
    const FinJob F{P->d_part, L.ntiles, act, nact, rnorm, P->d_pnorm};
    hipLaunchKernelGGL(k_finish, dim3(nitems), dim3(256), 0, s, F);
}

void launch_add_correction(const mbp_plan* P, double* p, const float* e32, const int* act,
                           const int* nact, int nitems, hipStream_t s, bool first) {
    const Level& L = P->levels[0];
    const AddJob J{p, e32, (long long)L.plane, act, nact, first ? 1 : 0};
    hipLaunchKernelGGL(k_addcorr, dim3(add_chunks(L.plane), nitems), dim3(256), 0, s, J);
}

void launch_plane_norm(const mbp_plan* P, const double* f, double* out, hipStream_t s) {
    const Level& L = P->levels[0];
    hipLaunchKernelGGL(k_sumsq, dim3(L.ntiles, P->g.nz), dim3(kTileX, kRowsPerPass), 0, s,
                       P->d_blk + L.blk_off, P->d_tiles + L.tile_off, L.ntiles, f, (long long)L.plane,
                       P->d_part);
    const FinJob F{P->d_part, L.ntiles, nullptr, nullptr, out, nullptr};
    hipLaunchKernelGGL(k_finish, dim3(P->g.nz), dim3(256), 0, s, F);
}

void launch_update_active(const mbp_plan* P, double rtol2, double etol2, int retire, int maxc,
                          hipStream_t s, double* out) {
    const UpdJob J{P->g.nz, P->d_rnorm, P->d_fnorm, P->d_pnorm, P->d_sabs, rtol2, etol2,
                   retire, maxc, P->d_act, P->d_nact, P->d_cyc, P->d_scal, P->d_flag, out};
    hipLaunchKernelGGL(k_update, dim3(1), dim3(1024), 0, s, J);
}

void launch_reset_active(const mbp_plan* P, hipStream_t s) {
    hipLaunchKernelGGL(k_iota, dim3(1), dim3(1024), 0, s, P->d_act, P->g.nz, P->d_nact, P->d_cyc);
}

void launch_zero_unrelaxed(const mbp_plan* P, double* p, hipStream_t s) {
    const int chunks = int(std::min<long long>(64, (P->plane0 + 1023) / 1024));
    hipLaunchKernelGGL(k_zero_unrelaxed, dim3(chunks, P->g.nz), dim3(256), 0, s, p, (long long)P->plane0,
                       P->d_cyc);
}

// The first V-cycle from a zero iterate reads no finest-level p: its first
// sweep is a fused strip sweep that takes the old iterate as zero (the
// residual test before it uses f itself).  The V-cycle then writes p of
// every active mode.
bool vcycle_zero_start_reads_none(const mbp_plan* P) {
    const int nu1 = P->opt.nu1, nu2 = P->opt.nu2;
    const bool fused_ok = ((nu1 + nu2) % 2 == 0) && nu1 >= 1 && nu2 >= 1;
    return P->lds_level > 0 && fused_ok && !P->march_ok.empty() && P->march_ok[0] && P->phatB != nullptr;
}

void launch_fill_int(int* p, int n, int v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(256), 0, s, p, n, v);
}

void launch_zero(double* p, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_zero64, dim3(1024), dim3(256), 0, s, p, (long long)n);
}

// Remove the area-weighted mean of one plane; the removed sum(a x) goes to out.
void launch_singular_fix(const mbp_plan* P, double* plane, double* out_sum, hipStream_t s) {
    hipLaunchKernelGGL(k_area_dot, dim3(1), dim3(1024), 0, s, plane, P->d_area0, (long long)P->plane0,
                       out_sum);
    hipLaunchKernelGGL(k_sub, dim3(256), dim3(256), 0, s, plane, (long long)P->plane0, out_sum,
                       P->area_sum);
}

void launch_area_dot(const mbp_plan* P, const double* plane, double* out_sum, hipStream_t s) {
    hipLaunchKernelGGL(k_area_dot, dim3(1), dim3(1024), 0, s, plane, P->d_area0, (long long)P->plane0,
                       out_sum);
}

size_t resnorm_scratch_doubles(const mbp_plan* P) {
    return 2 * size_t(P->levels[0].ntiles) * size_t(P->g.nz);
}

void launch_resnorm3d(const mbp_plan* P, const double* f, const double* p, double shift, double* part,
                      double* out, hipStream_t s) {
    const Level& L = P->levels[0];
    hipLaunchKernelGGL(k_resnorm3d, dim3(L.ntiles, P->g.nz), dim3(kTileX, kRowsPerPass), 0, s,
                       P->d_blk + L.blk_off, P->d_tiles + L.tile_off, L.ntiles, P->d_dbl, p, f, shift, P->g.nz,
                       1.0 / (P->g.dz * P->g.dz), int(P->g.zkind), P->opt.helmholtz, part);
    hipLaunchKernelGGL(k_resnorm_finish, dim3(1), dim3(1024), 0, s, part, (long long)L.ntiles * P->g.nz, out);
}

void launch_apply3d(const mbp_plan* P, const double* p, double* out, hipStream_t s) {
    const Level& L = P->levels[0];
    hipLaunchKernelGGL(k_apply3d, dim3(L.ntiles, P->g.nz), dim3(kTileX, kRowsPerPass), 0, s,
                       P->d_blk + L.blk_off, P->d_tiles + L.tile_off, L.ntiles, P->d_dbl, p, out,
                       P->g.nz, 1.0 / (P->g.dz * P->g.dz), int(P->g.zkind), P->opt.helmholtz);
}

// ============================ grouped launches ============================
// The same stage for many problems in one launch: each workgroup finds its
// job in the entry table and runs the single-problem body with its own
// (bx, by).  Jobs sit in device memory, uploaded before the launches are
// recorded.

__global__ void __launch_bounds__(256) k_residual32_group(const GEnt* __restrict__ e, int n,
                                                          const ResJob* __restrict__ jobs) {
    int bx, by;
    const int j = group_locate(e, n, bx, by);
    residual_body<1>(jobs[j], bx, by);
}

__global__ void __launch_bounds__(256) k_finish_group(const GEnt* __restrict__ e, int n,
                                                      const FinJob* __restrict__ jobs) {
    int bx, by;
    const int j = group_locate(e, n, bx, by);
    finish_body(jobs[j], bx);
}

__global__ void __launch_bounds__(1024) k_update_group(const GEnt* __restrict__ e, int n,
                                                       const UpdJob* __restrict__ jobs) {
    int bx, by;
    const int j = group_locate(e, n, bx, by);
    update_body(jobs[j]);
}

__global__ void __launch_bounds__(256) k_addcorr_group(const GEnt* __restrict__ e, int n,
                                                       const AddJob* __restrict__ jobs) {
    int bx, by;
    const int j = group_locate(e, n, bx, by);
    addcorr_body(jobs[j], bx, by);
}

__global__ void __launch_bounds__(1024) k_lds_vcycle_group(const GEnt* __restrict__ e, int n,
                                                           const LdsJob<float>* __restrict__ jobs) {
    int bx, by;
    const int j = group_locate(e, n, bx, by);
    lds_vcycle_body<float>(jobs[j], bx);
}

// The FP32 V-cycle reads its finest initial guess only on the generic
// (non-strip) finest level: the strip sweeps and the LDS-resident kernel start
// from zero without reading it.  Only then must the guess be zeroed.
float* fp32_guess_to_zero(const mbp_plan* P) {
    const int nu1 = P->opt.nu1, nu2 = P->opt.nu2;
    const bool fused_ok = ((nu1 + nu2) % 2 == 0) && nu1 >= 1 && nu2 >= 1;
    const bool strip0 = fused_ok && P->march_ok[0] && P->p32B[0] != nullptr;
    return (P->lds_level32 == 0 || strip0) ? nullptr : P->p32[0];
}

GStage group_res32(GroupBlob& gb, const std::vector<SolveCtx*>& cs) {
    std::vector<ResJob> jobs;
    std::vector<int> gx, gy;
    // one launch for all problems: the workgroup target is shared in
    // proportion to each problem's tiles x modes
    double total = 0.0;
    for (const SolveCtx* c : cs) total += double(c->P->levels[0].ntiles) * c->nitems;
    for (const SolveCtx* c : cs) {
        const mbp_plan* P = c->P;
        const Level& L = P->levels[0];
        const double share = total > 0.0 ? double(L.ntiles) * c->nitems / total : 1.0;
        const int per = res_per(L.ntiles, c->nitems, share);
        jobs.push_back(ResJob{P->d_blk + L.blk_off, P->d_tiles + L.tile_off, L.ntiles, P->d_dbl, P->phat,
                              P->fhat, (long long)L.plane, P->d_shift, P->d_act, P->d_nact, P->d_part,
                              P->f32[0], fp32_guess_to_zero(P), per});
        gx.push_back(L.ntiles);
        gy.push_back((c->nitems + per - 1) / per);
    }
    return group_build(gb, G_RES32, jobs, gx, gy);
}

GStage group_finish(GroupBlob& gb, const std::vector<SolveCtx*>& cs) {
    std::vector<FinJob> jobs;
    std::vector<int> gx, gy;
    for (const SolveCtx* c : cs) {
        const mbp_plan* P = c->P;
        jobs.push_back(FinJob{P->d_part, P->levels[0].ntiles, P->d_act, P->d_nact, P->d_rnorm, P->d_pnorm});
        gx.push_back(c->nitems);
        gy.push_back(1);
    }
    return group_build(gb, G_FINISH, jobs, gx, gy);
}

GStage group_update(GroupBlob& gb, const std::vector<SolveCtx*>& cs) {
    std::vector<UpdJob> jobs;
    std::vector<int> gx, gy;
    for (const SolveCtx* c : cs) {
        const mbp_plan* P = c->P;
        jobs.push_back(UpdJob{P->g.nz, P->d_rnorm, P->d_fnorm, P->d_pnorm, P->d_sabs, c->rtol2, c->etol2,
                              c->retire ? 1 : 0, P->opt.max_cycles, P->d_act, P->d_nact, P->d_cyc, P->d_scal,
                              P->d_flag});
        gx.push_back(1);
        gy.push_back(1);
    }
    GStage st = group_build(gb, G_UPDATE, jobs, gx, gy);
    st.threads = 1024;
    return st;
}

GStage group_addcorr(GroupBlob& gb, const std::vector<SolveCtx*>& cs) {
    std::vector<AddJob> jobs;
    std::vector<int> gx, gy;
    for (const SolveCtx* c : cs) {
        const mbp_plan* P = c->P;
        const Level& L = P->levels[0];
        jobs.push_back(AddJob{P->phat, P->p32[0], (long long)L.plane, P->d_act, P->d_nact});
        gx.push_back(add_chunks(L.plane));
        gy.push_back(c->nitems);
    }
    return group_build(gb, G_ADDCORR, jobs, gx, gy);
}

GStage group_lds32(GroupBlob& gb, const std::vector<SolveCtx*>& cs) {
    std::vector<LdsJob<float>> jobs;
    std::vector<int> gx, gy;
    size_t bytes = 0;
    for (const SolveCtx* c : cs) {
        const mbp_plan* P = c->P;
        const int L = P->lds_level32;
        jobs.push_back(LdsJob<float>{lds_args(P, L), P->p32[L], P->f32[L], (long long)P->levels[L].plane,
                                     P->d_shift, P->d_act, P->d_nact});
        gx.push_back(c->nitems);
        gy.push_back(1);
        bytes = std::max(bytes, size_t(P->lds_bytes32));
    }
    GStage st = group_build(gb, G_LDS32, jobs, gx, gy);
    st.lds = bytes;
    // as many workgroups per CU as the largest image allows (at most four;
    // the kernel's register use caps a CU at 16 of its waves), and the
    // waves split between them
    const int64_t per_cu = cs.empty() ? 1 : cs[0]->P->lds_limit;
    const int wgs_per_cu = int(std::min<int64_t>(4, std::max<int64_t>(1, per_cu / int64_t(std::max<size_t>(bytes, 1)))));
    st.threads = wgs_per_cu >= 4 ? 256 : wgs_per_cu >= 2 ? 512 : 1024;
    set_lds(reinterpret_cast<const void*>(k_lds_vcycle_group), bytes);
    return st;
}

void group_launch_mg(const GStage& st, const unsigned char* dev, hipStream_t s) {
    if (st.wgs <= 0) return;
    const GEnt* e = reinterpret_cast<const GEnt*>(dev + st.ent_off);
    const void* j = dev + st.job_off;
    const dim3 tile(kTileX, kRowsPerPass);
    switch (st.kind) {
        case G_RES32:
            hipLaunchKernelGGL(k_residual32_group, dim3(st.wgs), tile, 0, s, e, st.nent,
                               reinterpret_cast<const ResJob*>(j));
            break;
        case G_FINISH:
            hipLaunchKernelGGL(k_finish_group, dim3(st.wgs), dim3(256), 0, s, e, st.nent,
                               reinterpret_cast<const FinJob*>(j));
            break;
        case G_UPDATE:
            hipLaunchKernelGGL(k_update_group, dim3(st.wgs), dim3(1024), 0, s, e, st.nent,
                               reinterpret_cast<const UpdJob*>(j));
            break;
        case G_ADDCORR:
            hipLaunchKernelGGL(k_addcorr_group, dim3(st.wgs), dim3(256), 0, s, e, st.nent,
                               reinterpret_cast<const AddJob*>(j));
            break;
        case G_LDS32:
            hipLaunchKernelGGL(k_lds_vcycle_group, dim3(st.wgs), dim3(st.threads), st.lds, s, e, st.nent,
                               reinterpret_cast<const LdsJob<float>*>(j));
            break;
        default:
            break;
    }
}

}  // namespace mbp
