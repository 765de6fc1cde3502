// Geometric multigrid on the whole 3D system, without the z synthesis: the
// comparison solver of Sec. 3.3.1 (the paper's "3D MG" against which the
// FFT-accelerated solve is timed, Sec. 4.2).  It solves
//     (L_h - alpha) p = f
// on the same multi-block, stretched x-y grid extruded along z, with the same
// cell-centred finite-volume operator (Eq. (8) on uniform grids).
//
// Hierarchy: each level is one x-y level of the FFT path's plan (full x-y
// coarsening, odd counts merging their last three cells) times nz_l cells
// along z.  Each coarsening step coarsens the direction(s) with the smaller
// spacing, as the paper's PFMG picks its semicoarsening direction: z alone
// when dz is at most half the mean x-y cell width, x-y alone when that width
// is at most half of dz, both otherwise (z only while its count is even and
// >= 4).  Coarse operators are rediscretised.  Smoother: weighted Jacobi
// (the paper's PFMG runs weighted Jacobi), out of place.  Transfers:
// volume-weighted restriction of the residual (fused with its evaluation),
// trilinear prolongation with physical-coordinate weights in x-y and the
// 3/4-1/4 weights of uniform cell-centred z.  The coarsest grid is solved
// exactly by separation: the dense z eigenvectors of the coarsest z operator
// and the x-y eigen-decomposition of the coarsest plane.
//
// Fields use the caller's packed layout on every level: block b occupies
// [nz_l * off_b, nz_l * off_{b+1}) in C order (nz_l, ny_b, nx_b), so the
// finest level reads the caller's rhs and writes the caller's p directly.
#include "internal.h"
#include "mg3d.h"

namespace mbp {

namespace {

__device__ __forceinline__ int xcd_remap3(int g, int n) {
    int x = g & 7, l = g >> 3;
    int per = n >> 3, rem = n & 7;
    return x * per + min(x, rem) + l;
}

__device__ __forceinline__ long long cell3(const DBlock& b, int nz, int k, int j, int i) {
    return (long long)nz * b.off + ((long long)k * b.ny + j) * b.nx + i;
}

// Sum over one workgroup; the result is valid in thread 0.
__device__ __forceinline__ double wg_sum(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int t = threadIdx.x + threadIdx.y * blockDim.x;
    const int w = t >> 6, nw = (blockDim.x * blockDim.y + 63) >> 6;
    __syncthreads();
    if ((t & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (t == 0)
        for (int k = 0; k < nw; ++k) s += red[k];
    return s;
}

// (L_h - alpha) p at cell (b, k, j, i) and its diagonal coefficient.  x-y
// neighbours beyond a joined face come from the partner block; beyond a wall
// the coefficient already holds the boundary condition (Neumann: none,
// Dirichlet: folded into the diagonal).  z ends: periodic wrap, or a mirror
// ghost (Neumann +p, Dirichlet -p) one cell away.
struct Op3 {
    const DBlock* B;
    const double* dp;
    int nz;
    double idz2;
    int zlo, zhi;  // MBP_PERIODIC / MBP_NEUMANN / MBP_DIRICHLET
    double alpha;
};

__device__ __forceinline__ double zdiag(const Op3& o, int k) {
    double d = -2.0 * o.idz2;
    if (k == 0 && o.zlo != MBP_PERIODIC) d += o.zlo == MBP_NEUMANN ? o.idz2 : -o.idz2;
    if (k == o.nz - 1 && o.zhi != MBP_PERIODIC) d += o.zhi == MBP_NEUMANN ? o.idz2 : -o.idz2;
    return d;
}

// Off-diagonal part sum_n a_n p_n at (b, k, j, i).
__device__ __forceinline__ double offdiag(const Op3& o, const double* __restrict__ p, const DBlock& b, int bi,
                                          int k, int j, int i, long long c) {
    const double* dp = o.dp;
    double xm = 0.0, xp = 0.0, ym = 0.0, yp = 0.0;
    if (i > 0) xm = p[c - 1];
    else if (b.nbr[XM] >= 0) { const DBlock& n = o.B[b.nbr[XM]]; xm = p[cell3(n, o.nz, k, j, n.nx - 1)]; }
    if (i < b.nx - 1) xp = p[c + 1];
    else if (b.nbr[XP] >= 0) { const DBlock& n = o.B[b.nbr[XP]]; xp = p[cell3(n, o.nz, k, j, 0)]; }
    if (j > 0) ym = p[c - b.nx];
    else if (b.nbr[YM] >= 0) { const DBlock& n = o.B[b.nbr[YM]]; ym = p[cell3(n, o.nz, k, n.ny - 1, i)]; }
    if (j < b.ny - 1) yp = p[c + b.nx];
    else if (b.nbr[YP] >= 0) { const DBlock& n = o.B[b.nbr[YP]]; yp = p[cell3(n, o.nz, k, 0, i)]; }
    const long long kz = (long long)b.nx * b.ny;
    double zs = 0.0;
    if (k > 0) zs += p[c - kz];
    else if (o.zlo == MBP_PERIODIC) zs += p[c + (o.nz - 1) * kz];
    if (k < o.nz - 1) zs += p[c + kz];
    else if (o.zhi == MBP_PERIODIC) zs += p[c - (o.nz - 1) * kz];
    (void)bi;
    return dp[b.cx + i] * xm + dp[b.cx + b.nx + i] * xp + dp[b.cy + j] * ym + dp[b.cy + b.ny + j] * yp +
           o.idz2 * zs;
}

__device__ __forceinline__ double diag(const Op3& o, const DBlock& b, int k, int j, int i) {
    return o.dp[b.cx + 2 * b.nx + i] + o.dp[b.cy + 2 * b.ny + j] + zdiag(o, k) - o.alpha;
}

}  // namespace

// ---------------------------------------------------------------------------
// Weighted Jacobi sweep: pout = pin + omega D^-1 (f - fshift - A pin).
// ZERO: pin is zero (not read).  NORM: per-workgroup partial sums of the
// squared residual of pin into part[0, nw) and of pin^2 into part[nw, 2 nw)
// (nw = workgroups of the launch).  WRITE: store pout.
// ---------------------------------------------------------------------------
template <bool ZERO, bool NORM, bool WRITE>
__global__ void __launch_bounds__(256)
k3_jacobi(Op3 o, const int4* __restrict__ tiles, int ntiles, const double* __restrict__ pin,
          double* __restrict__ pout, const double* __restrict__ f, double fshift, double omega,
          double* __restrict__ part) {
    const int k = blockIdx.y;
    const int4 t = tiles[xcd_remap3(blockIdx.x, ntiles)];
    const DBlock b = o.B[t.x];
    const int i = t.y + threadIdx.x;
    double acc = 0.0, accp = 0.0;
    if (i < b.nx) {
        for (int r = threadIdx.y; r < kTileY; r += kRowsPerPass) {
            const int j = t.z + r;
            if (j >= b.ny) break;
            const long long c = cell3(b, o.nz, k, j, i);
            const double d = diag(o, b, k, j, i);
            double res = f[c] - fshift;
            double v = 0.0;
            if (!ZERO) {
                v = pin[c];
                res -= offdiag(o, pin, b, t.x, k, j, i, c) + d * v;
            }
            if (NORM) {
                acc += res * res;
                accp += v * v;
            }
            if (WRITE) pout[c] = v + omega * res / d;
        }
    }
    if (NORM) {
        __shared__ double red[8];
        const long long w = (long long)blockIdx.y * gridDim.x + blockIdx.x;
        const long long nw = (long long)gridDim.y * gridDim.x;
        const double s = wg_sum(acc, red);
        if (threadIdx.x == 0 && threadIdx.y == 0) part[w] = s;
        const double sp = wg_sum(accp, red);
        if (threadIdx.x == 0 && threadIdx.y == 0) part[nw + w] = sp;
    }
}

// ---------------------------------------------------------------------------
// The same sweep (pin read, so not the zero start) marching along z: a
// workgroup owns one 64 x 16 x-y tile and a chunk of kZChunk planes; each
// thread keeps its four cells' values at planes k-1, k, k+1 in registers and
// the plane-k tile (with a one-cell ring from the tile's neighbours, or from
// the partner block across a joined face) in LDS.  Every value of p is read
// from device memory once per sweep, plus the ring.
// ---------------------------------------------------------------------------
constexpr int kZChunk = 32;

namespace {

// p at (k, jj, ii) of block b where (ii, jj) may lie one cell outside the
// block: the partner's cell across a joined face, 0 beyond a wall (its
// coupling coefficient is zero) or diagonally outside.
__device__ __forceinline__ double ring_value(const Op3& o, const double* __restrict__ p, const DBlock& b, int k,
                                             int ii, int jj) {
    const bool xin = ii >= 0 && ii < b.nx, yin = jj >= 0 && jj < b.ny;
    if (xin && yin) return p[cell3(b, o.nz, k, jj, ii)];
    if (yin) {
        if (ii == -1 && b.nbr[XM] >= 0) { const DBlock& n = o.B[b.nbr[XM]]; return p[cell3(n, o.nz, k, jj, n.nx - 1)]; }
        if (ii == b.nx && b.nbr[XP] >= 0) { const DBlock& n = o.B[b.nbr[XP]]; return p[cell3(n, o.nz, k, jj, 0)]; }
    } else if (xin) {
        if (jj == -1 && b.nbr[YM] >= 0) { const DBlock& n = o.B[b.nbr[YM]]; return p[cell3(n, o.nz, k, n.ny - 1, ii)]; }
        if (jj == b.ny && b.nbr[YP] >= 0) { const DBlock& n = o.B[b.nbr[YP]]; return p[cell3(n, o.nz, k, 0, ii)]; }
    }
    return 0.0;
}

// Plane index of z neighbour k (periodic wrap) or -1 where the ghost rule
// applies (its coupling is folded into the diagonal).
__device__ __forceinline__ int zplane(const Op3& o, int k) {
    if (k >= 0 && k < o.nz) return k;
    if (o.zlo == MBP_PERIODIC) return (k + o.nz) % o.nz;
    return -1;
}

}  // namespace

// The coarse level a restricting march writes to.
struct Rst3 {
    const DBlock* Bc;
    int nzc;
    double* fc;
};

// MODE 0: the sweep; 1: the sweep and the partial sums of NORM above; 2: no
// sweep, the residual restricted to the next level instead (x-y and z both
// coarsened, even x-y block sizes: children 2I, 2I + 1 of coarse cell I lie
// in the same tile; the pair of planes 2K, 2K + 1 is summed in registers,
// the 2 x 2 x-y children through LDS).
template <int MODE>
__global__ void __launch_bounds__(256)
k3_jacobi_zm(Op3 o, const int4* __restrict__ tiles, int ntiles, const double* __restrict__ pin,
             double* __restrict__ pout, const double* __restrict__ f, double fshift, double omega,
             double* __restrict__ part, Rst3 rs) {
    constexpr bool NORM = MODE == 1;
    __shared__ double sp[kTileY + 2][kTileX + 2];
    __shared__ double sr[MODE == 2 ? kTileY : 1][MODE == 2 ? kTileX : 1];
    const int4 t = tiles[xcd_remap3(blockIdx.x, ntiles)];
    const DBlock b = o.B[t.x];
    const int k0 = blockIdx.y * kZChunk;
    const int k1 = min(k0 + kZChunk, o.nz);
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int tid = ty * kTileX + tx;
    const int i = t.y + tx;
    const bool in_i = i < b.nx;
    const double* dp = o.dp;
    const long long kz = (long long)b.nx * b.ny;
    const long long base = (long long)o.nz * b.off;
    constexpr int R = kTileY / kRowsPerPass;  // rows per thread
    int j[R];
    bool act[R];
    double wym[R], wyp[R], dxy[R];
    const double wxm = in_i ? dp[b.cx + i] : 0.0, wxp = in_i ? dp[b.cx + b.nx + i] : 0.0;
    const double dx = in_i ? dp[b.cx + 2 * b.nx + i] : 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        j[r] = t.z + ty + kRowsPerPass * r;
        act[r] = in_i && j[r] < b.ny;
        wym[r] = act[r] ? dp[b.cy + j[r]] : 0.0;
        wyp[r] = act[r] ? dp[b.cy + b.ny + j[r]] : 0.0;
        dxy[r] = act[r] ? dx + dp[b.cy + 2 * b.ny + j[r]] - o.alpha : 1.0;
    }
    auto load = [&](int kp, double* v) {
        const int q = zplane(o, kp);
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = (act[r] && q >= 0) ? pin[base + q * kz + (long long)j[r] * b.nx + i] : 0.0;
    };
    auto loadf = [&](int kp, double* v) {
#pragma unroll
        for (int r = 0; r < R; ++r)
            v[r] = (act[r] && kp < o.nz) ? f[base + kp * kz + (long long)j[r] * b.nx + i] - fshift : 0.0;
    };
    double pm[R], pc[R], pp[R], fc[R], pn[R], fn[R];
    load(k0 - 1, pm);
    load(k0, pc);
    load(k0 + 1, pp);
    loadf(k0, fc);
    double acc = 0.0, accp = 0.0;
    double racc[R], rw[R];
    if (MODE == 2) {
        const double wx = in_i ? dp[b.rwx + i] : 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            racc[r] = 0.0;
            rw[r] = act[r] ? 0.5 * wx * dp[b.rwy + j[r]] : 0.0;  // volume fraction: x, y and the z pair
        }
    }
    for (int k = k0; k < k1; ++k) {
        if (k + 1 < k1) {  // next plane's loads in flight during this plane's work
            load(k + 2, pn);
            loadf(k + 1, fn);
        }
        // plane k into LDS: own cells from registers, the ring and cells of a
        // ragged tile's edge through ring_value
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int ly = ty + kRowsPerPass * r;
            sp[ly + 1][tx + 1] = act[r] ? pc[r] : ring_value(o, pin, b, k, i, t.z + ly);
        }
        if (tid < 2 * kTileX) {
            const int side = tid / kTileX, lx = tid % kTileX;
            const int jj = side == 0 ? t.z - 1 : t.z + kTileY;
            sp[side == 0 ? 0 : kTileY + 1][lx + 1] = ring_value(o, pin, b, k, t.y + lx, jj);
        } else if (tid < 2 * kTileX + 2 * kTileY) {
            const int e = tid - 2 * kTileX, side = e / kTileY, ly = e % kTileY;
            const int ii = side == 0 ? t.y - 1 : t.y + kTileX;
            sp[ly + 1][side == 0 ? 0 : kTileX + 1] = ring_value(o, pin, b, k, ii, t.z + ly);
        }
        __syncthreads();
        const double zd = zdiag(o, k);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!act[r]) continue;
            const int ly = ty + kRowsPerPass * r + 1, lx = tx + 1;
            const double d = dxy[r] + zd;
            const double off = wxm * sp[ly][lx - 1] + wxp * sp[ly][lx + 1] + wym[r] * sp[ly - 1][lx] +
                               wyp[r] * sp[ly + 1][lx] + o.idz2 * (pm[r] + pp[r]);
            const double res = fc[r] - off - d * pc[r];
            if (NORM) {
                acc += res * res;
                accp += pc[r] * pc[r];
            }
            if (MODE == 2) racc[r] += rw[r] * res;
            else pout[base + k * kz + (long long)j[r] * b.nx + i] = pc[r] + omega * res / d;
        }
        __syncthreads();
        if (MODE == 2 && (k & 1)) {  // planes 2K, 2K + 1 done: sum the x-y children
#pragma unroll
            for (int r = 0; r < R; ++r) {
                sr[ty + kRowsPerPass * r][tx] = racc[r];
                racc[r] = 0.0;
            }
            __syncthreads();
            const int ci = tid % (kTileX / 2), cj = tid / (kTileX / 2);  // 32 x 8 coarse cells
            const DBlock bc = rs.Bc[t.x];
            const int I = t.y / 2 + ci, J = t.z / 2 + cj;
            if (I < bc.nx && J < bc.ny)
                rs.fc[cell3(bc, rs.nzc, k >> 1, J, I)] = sr[2 * cj][2 * ci] + sr[2 * cj][2 * ci + 1] +
                                                         sr[2 * cj + 1][2 * ci] + sr[2 * cj + 1][2 * ci + 1];
            __syncthreads();
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            pm[r] = pc[r];
            pc[r] = pp[r];
            pp[r] = pn[r];
            fc[r] = fn[r];
        }
    }
    if (NORM) {
        __shared__ double red[8];
        const long long w = (long long)blockIdx.y * gridDim.x + blockIdx.x;
        const long long nw = (long long)gridDim.y * gridDim.x;
        const double sr = wg_sum(acc, red);
        if (tid == 0) part[w] = sr;
        const double sq = wg_sum(accp, red);
        if (tid == 0) part[nw + w] = sq;
    }
}

// ---------------------------------------------------------------------------
// Residual of level l restricted to level l+1 (volume-weighted average of
// the children), written to fc; one thread per coarse cell.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k3_restrict(Op3 of, const DBlock* __restrict__ Bc, const int4* __restrict__ tiles_c, int ntiles_c,
            int nzc, const int* __restrict__ ip, const double* __restrict__ p, const double* __restrict__ f,
            double fshift, double* __restrict__ fc, int xycoarse, int zcoarse) {
    const int K = blockIdx.y;
    const int4 t = tiles_c[xcd_remap3(blockIdx.x, ntiles_c)];
    const DBlock bc = Bc[t.x];
    const DBlock bf = of.B[t.x];
    const double* dp = of.dp;
    const int I = t.y + threadIdx.x;
    if (I >= bc.nx) return;
    // children: the x-y transfer tables when x-y coarsens, else the same cell
    const int i0 = xycoarse ? ip[bf.rsx + I] : I, i1 = xycoarse ? ip[bf.rsx + I + 1] : I + 1;
    const int k0 = zcoarse ? 2 * K : K, k1 = zcoarse ? 2 * K + 2 : K + 1;
    const double wz = zcoarse ? 0.5 : 1.0;
    for (int r = threadIdx.y; r < kTileY; r += kRowsPerPass) {
        const int J = t.z + r;
        if (J >= bc.ny) break;
        const int j0 = xycoarse ? ip[bf.rsy + J] : J, j1 = xycoarse ? ip[bf.rsy + J + 1] : J + 1;
        double acc = 0.0;
        for (int k = k0; k < k1; ++k)
            for (int j = j0; j < j1; ++j) {
                const double wy = xycoarse ? dp[bf.rwy + j] : 1.0;
                double row = 0.0;
                for (int i = i0; i < i1; ++i) {
                    const long long c = cell3(bf, of.nz, k, j, i);
                    const double res =
                        f[c] - fshift - offdiag(of, p, bf, t.x, k, j, i, c) - diag(of, bf, k, j, i) * p[c];
                    row += (xycoarse ? dp[bf.rwx + i] : 1.0) * res;
                }
                acc += wy * row;
            }
        fc[cell3(bc, nzc, K, J, I)] = wz * acc;
    }
}

namespace {

// Coarse value at (I, J) of plane K (K inside [0, nzc)) of block b, I in
// [-1, nx], J in [-1, ny]: beyond a joined face the partner's cell, beyond a
// wall the mirror image (Neumann +, Dirichlet -); corners through y first.
__device__ __forceinline__ double cvalue(const double* __restrict__ pc, const DBlock* __restrict__ B, int nzc,
                                         int b, int I, int J, int K) {
    double s = 1.0;
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
    return s * pc[cell3(*bb, nzc, K, J, I)];
}

// Bilinear (physical weights) value of coarse plane K at fine cell (i, j).
__device__ __forceinline__ double bilinear(const double* __restrict__ pc, const DBlock* __restrict__ Bc, int nzc,
                                           const DBlock& bf, int b, const double* __restrict__ dp,
                                           const int* __restrict__ ip, int i, int j, int K) {
    const int cx = ip[bf.pcx + i], cy = ip[bf.pcy + j];
    const double wx = dp[bf.pwx + i], wy = dp[bf.pwy + j];
    const double e00 = cvalue(pc, Bc, nzc, b, cx, cy, K), e10 = cvalue(pc, Bc, nzc, b, cx + 1, cy, K);
    const double e01 = cvalue(pc, Bc, nzc, b, cx, cy + 1, K), e11 = cvalue(pc, Bc, nzc, b, cx + 1, cy + 1, K);
    return wy * (wx * e00 + (1.0 - wx) * e10) + (1.0 - wy) * (wx * e01 + (1.0 - wx) * e11);
}

}  // namespace

// ---------------------------------------------------------------------------
// p_l += P e_{l+1}: trilinear interpolation of the coarse correction.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k3_prolong(const DBlock* __restrict__ Bf, const DBlock* __restrict__ Bc, const int4* __restrict__ tiles_f,
           int ntiles_f, int nzf, int nzc, const double* __restrict__ dp, const int* __restrict__ ip,
           const double* __restrict__ pc, double* __restrict__ pf, int xycoarse, int zcoarse, int zlo, int zhi) {
    const int k = blockIdx.y;
    const int4 t = tiles_f[xcd_remap3(blockIdx.x, ntiles_f)];
    const DBlock bf = Bf[t.x];
    const int i = t.y + threadIdx.x;
    if (i >= bf.nx) return;
    // z: the two coarse planes around the fine centre, weight of the lower one
    int K0 = k, K1 = k;
    double w0 = 1.0, s0 = 1.0, s1 = 1.0;
    if (zcoarse) {
        const int K = k >> 1;
        if (k & 1) { K0 = K; K1 = K + 1; w0 = 0.75; }
        else { K0 = K - 1; K1 = K; w0 = 0.25; }
        if (K0 < 0) {  // below the first coarse cell: periodic wrap or mirror ghost
            if (zlo == MBP_PERIODIC) K0 = nzc - 1;
            else { K0 = 0; s0 = zlo == MBP_DIRICHLET ? -1.0 : 1.0; }
        }
        if (K1 >= nzc) {
            if (zhi == MBP_PERIODIC) K1 = 0;
            else { K1 = nzc - 1; s1 = zhi == MBP_DIRICHLET ? -1.0 : 1.0; }
        }
    }
    for (int r = threadIdx.y; r < kTileY; r += kRowsPerPass) {
        const int j = t.z + r;
        if (j >= bf.ny) break;
        double e;
        if (xycoarse) {
            e = w0 * s0 * bilinear(pc, Bc, nzc, bf, t.x, dp, ip, i, j, K0);
            if (zcoarse) e += (1.0 - w0) * s1 * bilinear(pc, Bc, nzc, bf, t.x, dp, ip, i, j, K1);
        } else {  // same x-y grid: the coarse cell under the fine one
            e = w0 * s0 * pc[cell3(bf, nzc, K0, j, i)];
            if (zcoarse) e += (1.0 - w0) * s1 * pc[cell3(bf, nzc, K1, j, i)];
        }
        pf[cell3(bf, nzf, k, j, i)] += e;
    }
}

// ---------------------------------------------------------------------------
// The same correction when both x-y and z coarsen, marching along z: a
// workgroup owns one 64 x 16 fine tile and kPZChunk fine planes (pairs 2K,
// 2K+1).  Each coarse plane the chunk needs is staged once into LDS (the
// tile's coarse cells and their ring, through cvalue), and its bilinear
// interpolant at the thread's four cells kept in registers; fine plane 2K
// takes 1/4 of plane K-1 and 3/4 of plane K, plane 2K+1 3/4 of K and 1/4 of
// K+1 (mirror or wrap beyond the z ends).
// ---------------------------------------------------------------------------
constexpr int kPZChunk = 16;             // fine planes per workgroup (even)
constexpr int kPX = kTileX / 2 + 4;      // staged coarse columns (with ring and merge slack)
constexpr int kPY = kTileY / 2 + 4;      // staged coarse rows

__global__ void __launch_bounds__(256)
k3_prolong_zm(const DBlock* __restrict__ Bf, const DBlock* __restrict__ Bc, const int4* __restrict__ tiles_f,
              int ntiles_f, int nzf, int nzc, const double* __restrict__ dp, const int* __restrict__ ip,
              const double* __restrict__ pc, double* __restrict__ pf, int zlo, int zhi) {
    __shared__ double sc[kPY][kPX];
    const int4 t = tiles_f[xcd_remap3(blockIdx.x, ntiles_f)];
    const DBlock bf = Bf[t.x];
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * kTileX + tx;
    const int i = t.y + tx;
    const bool in_i = i < bf.nx;
    // coarse range of the tile (the lower-neighbour tables are monotone)
    const int ilast = min(t.y + kTileX - 1, bf.nx - 1), jlast = min(t.z + kTileY - 1, bf.ny - 1);
    const int cx0 = ip[bf.pcx + t.y], cy0 = ip[bf.pcy + t.z];
    const int ncx = ip[bf.pcx + ilast] + 2 - cx0, ncy = ip[bf.pcy + jlast] + 2 - cy0;
    constexpr int R = kTileY / kRowsPerPass;
    int lx = 0;
    double wx = 0.0;
    if (in_i) {
        lx = ip[bf.pcx + i] - cx0;
        wx = dp[bf.pwx + i];
    }
    int ly[R];
    double wy[R];
    bool act[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int j = t.z + ty + kRowsPerPass * r;
        act[r] = in_i && j < bf.ny;
        ly[r] = act[r] ? ip[bf.pcy + j] - cy0 : 0;
        wy[r] = act[r] ? dp[bf.pwy + j] : 0.0;
    }
    // bilinear values of coarse plane K (inside [0, nzc)) at the thread's cells
    auto interp = [&](int K, double* e) {
        __syncthreads();
        for (int q = tid; q < ncx * ncy; q += kTileX * kRowsPerPass) {
            const int a = q % ncx, b = q / ncx;
            sc[b][a] = cvalue(pc, Bc, nzc, t.x, cx0 + a, cy0 + b, K);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!act[r]) {
                e[r] = 0.0;
                continue;
            }
            const double e00 = sc[ly[r]][lx], e10 = sc[ly[r]][lx + 1];
            const double e01 = sc[ly[r] + 1][lx], e11 = sc[ly[r] + 1][lx + 1];
            e[r] = wy[r] * (wx * e00 + (1.0 - wx) * e10) + (1.0 - wy[r]) * (wx * e01 + (1.0 - wx) * e11);
        }
    };
    // beyond a non-periodic z end the coarse ghost is the end plane mirrored
    // (Neumann +, Dirichlet -)
    const double slo = zlo == MBP_DIRICHLET ? -1.0 : 1.0, shi = zhi == MBP_DIRICHLET ? -1.0 : 1.0;
    const bool per = zlo == MBP_PERIODIC;
    const int K0 = blockIdx.y * (kPZChunk / 2);
    const long long base = (long long)nzf * bf.off, kz = (long long)bf.nx * bf.ny;
    double em[R], ec[R], ep[R];
    interp(K0, ec);
    if (K0 > 0 || per) interp((K0 - 1 + nzc) % nzc, em);
    else
#pragma unroll
        for (int r = 0; r < R; ++r) em[r] = slo * ec[r];
    for (int K = K0; K < K0 + kPZChunk / 2; ++K) {
        if (K + 1 < nzc || per) interp((K + 1) % nzc, ep);
        else
#pragma unroll
            for (int r = 0; r < R; ++r) ep[r] = shi * ec[r];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!act[r]) continue;
            const long long c = base + ((long long)t.z + ty + kRowsPerPass * r) * bf.nx + i;
            pf[c + (2 * K) * kz] += 0.25 * em[r] + 0.75 * ec[r];
            pf[c + (2 * K + 1) * kz] += 0.75 * ec[r] + 0.25 * ep[r];
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            em[r] = ec[r];
            ec[r] = ep[r];
        }
    }
}

// ---------------------------------------------------------------------------
// Exact coarsest solve by separation.  Stage 1, one workgroup per z mode m:
// fz = sum_k V[k][m] f_k (z eigenvectors), then the x-y solve
// x_m = WL diag(1 / (mu + muz_m - alpha)) WR fz, with the null mode dropped.
// Stage 2: p_k = sum_m V[k][m] x_m.  Plane cells are indexed like the x-y
// eigen tables; cmap gives each one's packed offset at z = 0 and its z stride.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k3_coarse_modes(const double* __restrict__ f, const int2* __restrict__ cmap, int nc, int nzc,
                const double* __restrict__ vz, const double* __restrict__ muz, const double* __restrict__ wl,
                const double* __restrict__ wr, const double* __restrict__ mu, double alpha,
                double* __restrict__ xhat) {
    extern __shared__ double sm[];
    double* fz = sm;       // nc
    double* tmp = sm + nc; // nc
    const int m = blockIdx.x;
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        const int2 cm = cmap[c];
        double a = 0.0;
        for (int k = 0; k < nzc; ++k) a += vz[k * nzc + m] * f[cm.x + (long long)k * cm.y];
        fz[c] = a;
    }
    __syncthreads();
    double mumax = 0.0;
    for (int q = 0; q < nc; ++q) mumax = fmax(mumax, fabs(mu[q]));
    const double sh = muz[m] - alpha;
    for (int q = threadIdx.x; q < nc; q += blockDim.x) {
        double a = 0.0;
        const double* row = wr + (long long)q * nc;
        for (int c = 0; c < nc; ++c) a += row[c] * fz[c];
        const double d = mu[q] + sh;
        tmp[q] = fabs(d) > 1e-11 * (mumax + fabs(sh)) ? a / d : 0.0;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        double a = 0.0;
        const double* row = wl + (long long)c * nc;
        for (int q = 0; q < nc; ++q) a += row[q] * tmp[q];
        xhat[(long long)m * nc + c] = a;
    }
}

__global__ void __launch_bounds__(256)
k3_coarse_back(const double* __restrict__ xhat, const int2* __restrict__ cmap, int nc, int nzc,
               const double* __restrict__ vz, double* __restrict__ p) {
    const long long n = (long long)nc * nzc;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const int k = int(e / nc), c = int(e % nc);
        double a = 0.0;
        for (int m = 0; m < nzc; ++m) a += vz[k * nzc + m] * xhat[(long long)m * nc + c];
        const int2 cm = cmap[c];
        p[cm.x + (long long)k * cm.y] = a;
    }
}

// ---------------------------------------------------------------------------
// Reductions on the packed finest field: partial sums of area * x (the
// volume-weighted sum, dz being uniform) per workgroup, and their total.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k3_area_sum(const DBlock* __restrict__ B, const int4* __restrict__ tiles, int ntiles, int nz,
            const double* __restrict__ area, const double* __restrict__ x, double* __restrict__ part) {
    const int k = blockIdx.y;
    const int4 t = tiles[xcd_remap3(blockIdx.x, ntiles)];
    const DBlock b = B[t.x];
    const int i = t.y + threadIdx.x;
    double acc = 0.0;
    if (i < b.nx)
        for (int r = threadIdx.y; r < kTileY; r += kRowsPerPass) {
            const int j = t.z + r;
            if (j >= b.ny) break;
            acc += area[b.off + j * b.nx + i] * x[cell3(b, nz, k, j, i)];
        }
    __shared__ double red[8];
    const double s = wg_sum(acc, red);
    if (threadIdx.x == 0 && threadIdx.y == 0) part[(long long)blockIdx.y * gridDim.x + blockIdx.x] = s;
}

__global__ void __launch_bounds__(1024) k3_total(const double* __restrict__ part, long long n, double scale,
                                                  double* __restrict__ out) {
    double acc = 0.0;
    for (long long e = threadIdx.x; e < n; e += blockDim.x) acc += part[e];
    __shared__ double red[16];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < int(blockDim.x >> 6); ++w) s += red[w];
        *out = s * scale;
    }
}

// x -= *mean (device scalar) over n elements.
__global__ void __launch_bounds__(256) k3_sub(double* __restrict__ x, long long n, const double* __restrict__ mean) {
    const double m = *mean;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
        x[e] -= m;
}

__global__ void __launch_bounds__(256) k3_copy(const double* __restrict__ a, double* __restrict__ b, long long n) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
        b[e] = a[e];
}

// ============================== launchers ==============================

namespace {
Op3 op_of(const Mg3Plan& M, int l) {
    const Mg3Level& L = M.lev[l];
    return Op3{M.d_blk + L.blk_off, M.d_dbl, L.nz, L.idz2, M.zlo, M.zhi, M.alpha};
}
dim3 grid_of(const Mg3Level& L) { return dim3(unsigned(L.ntiles), unsigned(L.nz)); }
const dim3 kBlk(kTileX, kRowsPerPass);
}  // namespace

long long m3_jacobi(const Mg3Plan& M, int l, const double* pin, double* pout, const double* f, double fshift,
                    bool zero, double* part, hipStream_t s) {
    const Mg3Level& L = M.lev[l];
    const Op3 o = op_of(M, l);
    const int4* tl = M.d_tiles + L.tile_off;
    if (zero) {  // elementwise: no neighbour is read
        if (part) hipLaunchKernelGGL((k3_jacobi<true, true, true>), grid_of(L), kBlk, 0, s, o, tl, L.ntiles, pin, pout, f,
                                     fshift, M.omega, part);
        else hipLaunchKernelGGL((k3_jacobi<true, false, true>), grid_of(L), kBlk, 0, s, o, tl, L.ntiles, pin, pout, f,
                                fshift, M.omega, part);
        return (long long)L.ntiles * L.nz;
    }
    const dim3 g(unsigned(L.ntiles), unsigned((L.nz + kZChunk - 1) / kZChunk));
    const Rst3 none{nullptr, 0, nullptr};
    if (part) hipLaunchKernelGGL(k3_jacobi_zm<1>, g, kBlk, 0, s, o, tl, L.ntiles, pin, pout, f, fshift, M.omega,
                                 part, none);
    else hipLaunchKernelGGL(k3_jacobi_zm<0>, g, kBlk, 0, s, o, tl, L.ntiles, pin, pout, f, fshift, M.omega, part,
                            none);
    return (long long)g.x * g.y;
}

// Squared norms of the finest residual of p and of p itself into out[0], out[1].
void m3_residual_norm(const Mg3Plan& M, const double* p, const double* f, double fshift, bool zero, double* part,
                      double* out, hipStream_t s) {
    const Mg3Level& L = M.lev[0];
    const Op3 o = op_of(M, 0);
    const int4* tl = M.d_tiles + L.tile_off;
    if (zero)
        hipLaunchKernelGGL((k3_jacobi<true, true, false>), grid_of(L), kBlk, 0, s, o, tl, L.ntiles, p, nullptr, f,
                           fshift, M.omega, part);
    else
        hipLaunchKernelGGL((k3_jacobi<false, true, false>), grid_of(L), kBlk, 0, s, o, tl, L.ntiles, p, nullptr, f,
                           fshift, M.omega, part);
    const long long nw = (long long)L.ntiles * L.nz;
    m3_total(part, nw, 1.0, out, s);
    m3_total(part + nw, nw, 1.0, out + 1, s);
}

void m3_total(const double* part, long long n, double scale, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k3_total, dim3(1), dim3(1024), 0, s, part, n, scale, out);
}

void m3_restrict(const Mg3Plan& M, int l, const double* p, const double* f, double fshift, double* fc,
                 hipStream_t s) {
    const Mg3Level& F = M.lev[l];
    const Mg3Level& C = M.lev[l + 1];
    const Op3 o = op_of(M, l);
    if (F.xyc && F.zc && F.xy22 && F.even_xy && F.nz % kZChunk == 0) {  // marching form
        const dim3 g(unsigned(F.ntiles), unsigned(F.nz / kZChunk));
        hipLaunchKernelGGL(k3_jacobi_zm<2>, g, kBlk, 0, s, o, M.d_tiles + F.tile_off, F.ntiles, p, nullptr, f, fshift,
                           M.omega, nullptr, Rst3{M.d_blk + C.blk_off, C.nz, fc});
        return;
    }
    hipLaunchKernelGGL(k3_restrict, grid_of(C), kBlk, 0, s, o, M.d_blk + C.blk_off, M.d_tiles + C.tile_off, C.ntiles,
                       C.nz, M.d_int, p, f, fshift, fc, M.lev[l].xyc, M.lev[l].zc);
}

void m3_prolong(const Mg3Plan& M, int l, const double* pc, double* pf, hipStream_t s) {
    const Mg3Level& F = M.lev[l];
    const Mg3Level& C = M.lev[l + 1];
    if (F.xyc && F.zc && F.xy22 && F.nz % kPZChunk == 0) {  // staged tile: x-y halved
        const dim3 g(unsigned(F.ntiles), unsigned(F.nz / kPZChunk));
        hipLaunchKernelGGL(k3_prolong_zm, g, kBlk, 0, s, M.d_blk + F.blk_off, M.d_blk + C.blk_off,
                           M.d_tiles + F.tile_off, F.ntiles, F.nz, C.nz, M.d_dbl, M.d_int, pc, pf, M.zlo, M.zhi);
        return;
    }
    hipLaunchKernelGGL(k3_prolong, grid_of(F), kBlk, 0, s, M.d_blk + F.blk_off, M.d_blk + C.blk_off,
                       M.d_tiles + F.tile_off, F.ntiles, F.nz, C.nz, M.d_dbl, M.d_int, pc, pf, F.xyc, F.zc,
                       M.zlo, M.zhi);
}

void m3_coarse(const Mg3Plan& M, const double* f, double* p, hipStream_t s) {
    const Mg3Level& L = M.lev[M.nlev - 1];
    const size_t lds = 2 * size_t(M.nc) * sizeof(double);
    hipLaunchKernelGGL(k3_coarse_modes, dim3(unsigned(L.nz)), dim3(256), lds, s, f, M.d_cmap, M.nc, L.nz, M.d_vz,
                       M.d_muz, M.d_cwl, M.d_cwr, M.d_cmu, M.alpha, M.d_xhat);
    const long long n = (long long)M.nc * L.nz;
    const unsigned g = unsigned(std::min<long long>((n + 255) / 256, 4096));
    hipLaunchKernelGGL(k3_coarse_back, dim3(g), dim3(256), 0, s, M.d_xhat, M.d_cmap, M.nc, L.nz, M.d_vz, p);
}

void m3_area_sum(const Mg3Plan& M, const double* x, double* part, double* out, double scale, hipStream_t s) {
    const Mg3Level& L = M.lev[0];
    hipLaunchKernelGGL(k3_area_sum, grid_of(L), kBlk, 0, s, M.d_blk + L.blk_off, M.d_tiles + L.tile_off, L.ntiles,
                       L.nz, M.d_area0, x, part);
    m3_total(part, (long long)L.ntiles * L.nz, scale, out, s);
}

void m3_sub(double* x, long long n, const double* mean, hipStream_t s) {
    hipLaunchKernelGGL(k3_sub, dim3(2048), dim3(256), 0, s, x, n, mean);
}

void m3_copy(const double* a, double* b, long long n, hipStream_t s) {
    hipLaunchKernelGGL(k3_copy, dim3(4096), dim3(256), 0, s, a, b, n);
}

}  // namespace mbp
