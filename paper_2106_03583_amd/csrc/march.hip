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
#include "internal.h"

namespace mbp {

struct MTile {
    int b, x0, w, y0, y1, pad0, pad1, pad2;
};

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
__device__ __forceinline__ T correction(const MArgs<T>& a, const T* __restrict__ ecq, int fb, int ci, int cj) {
    const DBlock& d = a.B[fb];
    const int cx = a.ip[d.pcx + ci], cy = a.ip[d.pcy + cj];
    const T wx = T(a.dp[d.pwx + ci]), wy = T(a.dp[d.pwy + cj]);
    const T e00 = coarse_at(ecq, a.Bc, fb, cx, cy), e10 = coarse_at(ecq, a.Bc, fb, cx + 1, cy);
    const T e01 = coarse_at(ecq, a.Bc, fb, cx, cy + 1), e11 = coarse_at(ecq, a.Bc, fb, cx + 1, cy + 1);
    return wy * (wx * e00 + (T(1) - wx) * e10) + (T(1) - wy) * (wx * e01 + (T(1) - wx) * e11);
}

template <typename T, bool PRO, bool RES, bool NRM>
__global__ void __launch_bounds__(256) k_march(MArgs<T> a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwg = (a.ntiles + 3) >> 2;
    const int tix = xcd_remap_m(blockIdx.x, nwg) * 4 + wave;
    if (tix >= a.ntiles) return;
    const int item = blockIdx.y;
    if (item >= *a.nact) return;
    const int q = a.act[item];
    const MTile t = a.tiles[tix];
    const DBlock& b = a.B[t.b];
    const int bny = b.ny;
    const T sig = T(a.shift[q]);
    const T* __restrict__ po = a.pold + q * a.plane;
    T* __restrict__ pn = a.pnew + q * a.plane;
    const T* __restrict__ fq = a.f + q * a.plane;
    const T* __restrict__ ecq = PRO ? a.ec + q * a.plane_c : nullptr;

    // ---- the lane's cells: block and column index per row region ----
    // Rows inside the strip's block use the block's x neighbours for the halo
    // columns.  Rows below / above it belong to the y neighbour M; there a halo
    // column is M's own x neighbour when that exists, else the y neighbour of
    // the side block (the two agree wherever both exist; the host checks).
    const int c = t.x0 - 3 + lane;
    const bool live = lane < t.w + 6;  // beyond the right halo: unused
    const bool inb = c >= 0 && c < b.nx;
    int cid = -1, ci = 0;
    if (live) {
        if (c < 0) { cid = b.nbr[XM]; ci = cid >= 0 ? a.B[cid].nx + c : 0; }
        else if (c >= b.nx) { cid = b.nbr[XP]; ci = c - b.nx; }
        else { cid = t.b; ci = c; }
    }
    auto halo_col = [&](int fy, int& hc) -> int {
        hc = 0;
        if (!live) return -1;
        const int M = b.nbr[fy];
        if (inb) { hc = c; return M; }
        const int fx = c < 0 ? XM : XP;
        if (M >= 0 && a.B[M].nbr[fx] >= 0) {
            const int X = a.B[M].nbr[fx];
            hc = c < 0 ? a.B[X].nx + c : c - b.nx;
            return X;
        }
        if (cid >= 0 && a.B[cid].nbr[fy] >= 0) { hc = ci; return a.B[cid].nbr[fy]; }
        return -1;
    };
    int cim, cip;
    const int kmb = halo_col(YM, cim), kpb = halo_col(YP, cip);
    const ColBlk K0 = colblk(a.B, cid);  // rows inside [0, ny)
    const ColBlk Km = colblk(a.B, kmb);  // rows below
    const ColBlk Kp = colblk(a.B, kpb);  // rows above
    const bool out_lane = lane >= 3 && lane < 3 + t.w;

    // region of virtual row k for this lane: block geometry, row and column
    auto region = [&](int k, ColBlk& R, int& cj, int& cc) -> bool {
        if (k < 0) { R = Km; cj = Km.ny + k; cc = cim; }
        else if (k >= bny) { R = Kp; cj = k - bny; cc = cip; }
        else { R = K0; cj = k; cc = ci; }
        return R.id >= 0;
    };

    // restriction bookkeeping (block b's tables; output lanes lie in block b)
    int Ipar = 0, Inext1 = -1, Inext2 = -1, ncx = 0, ncy = 0;
    T wrx = T(0);
    bool leader = false;
    if (RES) {
        const DBlock& bc = a.Bc[t.b];
        ncx = bc.nx;
        ncy = bc.ny;
        auto parent = [&](int col) { return min(col >> 1, ncx - 1); };
        if (c >= 0 && c < b.nx) {
            Ipar = parent(c);
            wrx = T(a.dp[b.rwx + c]);
            leader = out_lane && (c == 2 * Ipar);
        }
        Inext1 = (c + 1 < b.nx && c + 1 >= 0) ? parent(c + 1) : -1;
        Inext2 = (c + 2 < b.nx && c + 2 >= 0) ? parent(c + 2) : -1;
    }

    // ---- register window ----
    T p0 = T(0), p1 = T(0), p2 = T(0), p3 = T(0), p4 = T(0);  // rows k-4 .. k
    T f1 = T(0), f2 = T(0), f3 = T(0), f4 = T(0);             // rows k-3 .. k
    T accy = T(0);
    double nrm = 0.0, pnr = 0.0;
    int curJ = -1;

    // relax one cell of the given colour (row values: dn = row below, up = row above)
    auto relax = [&](T& cen, T dn, T up, T fv, int k, int colour) {
        const T xm = shfl_up1(cen), xp = shfl_dn1(cen);
        ColBlk R;
        int cj, cc;
        if (!region(k, R, cj, cc)) return;
        if (((cc + cj + R.par) & 1) != colour) return;
        const double* dp = a.dp;
        const T d = T(dp[R.cx + 2 * R.nx + cc]) + T(dp[R.cy + 2 * R.ny + cj]) + sig;
        const T off = T(dp[R.cx + cc]) * xm + T(dp[R.cx + R.nx + cc]) * xp + T(dp[R.cy + cj]) * dn +
                      T(dp[R.cy + R.ny + cj]) * up;
        cen = (fv - off) / d;
    };

    const int kbeg = t.y0 - 3, kend = t.y1 + 2;
    for (int k = kbeg; k <= kend; ++k) {
        // shift the window and load row k
        p0 = p1; p1 = p2; p2 = p3; p3 = p4;
        f1 = f2; f2 = f3; f3 = f4;
        {
            ColBlk R;
            int cj, cc;
            T pv = T(0), fv = T(0);
            if (region(k, R, cj, cc)) {
                const long long o = R.off + (long long)cj * R.nx + cc;
                pv = po[o];
                fv = fq[o];
                if (PRO) pv += correction(a, ecq, R.id, cc, cj);
            }
            p4 = pv;
            f4 = fv;
        }
        // red cells of row k-1 (old black neighbours), black cells of row k-2
        if (k - 1 >= t.y0 - 2) relax(p3, p2, p4, f3, k - 1, 0);
        if (k - 2 >= t.y0 - 1) relax(p2, p1, p3, f2, k - 2, 1);
        // row k-2 is final: store it
        if (k - 2 >= t.y0 && k - 2 < t.y1 && out_lane) {
            const long long o = K0.off + (long long)(k - 2) * K0.nx + ci;
            pn[o] = p2;
        }
        // residual of row k-3 (rows k-4 .. k-2 are final)
        if (RES || NRM) {
            const int kr = k - 3;
            const T xm = shfl_up1(p1), xp = shfl_dn1(p1);
            T r = T(0);
            if (kr >= t.y0 && kr < t.y1 && out_lane) {
                const double* dp = a.dp;
                const T d = T(dp[K0.cx + 2 * K0.nx + ci]) + T(dp[K0.cy + 2 * K0.ny + kr]) + sig;
                r = f1 - (T(dp[K0.cx + ci]) * xm + T(dp[K0.cx + K0.nx + ci]) * xp +
                          T(dp[K0.cy + kr]) * p0 + T(dp[K0.cy + K0.ny + kr]) * p2 + d * p1);
                if (NRM) {
                    nrm += double(r) * double(r);
                    pnr += double(p1) * double(p1);
                }
            }
            if (RES) {
                const bool inrow = kr >= t.y0 && kr < t.y1;
                T rw = (inrow && out_lane) ? r * wrx : T(0);
                const T v1 = shfl_dn1(rw);
                const T v2 = __shfl_down(rw, 2);
                if (inrow) {
                    const int J = min(kr >> 1, ncy - 1);
                    T sx = rw;
                    if (Inext1 == Ipar) sx += v1;
                    if (Inext2 == Ipar) sx += v2;
                    accy += T(a.dp[b.rwy + kr]) * sx;
                    curJ = J;
                    // flush when the next row belongs to another coarse row (or the strip ends)
                    const int Jn = (kr + 1 < t.y1) ? min((kr + 1) >> 1, ncy - 1) : -1;
                    if (Jn != J) {
                        if (leader) {
                            const DBlock& bc = a.Bc[t.b];
                            const long long o = q * a.plane_c + bc.off + (long long)J * bc.nx + Ipar;
                            a.fc[o] = accy;
                            a.pc[o] = T(0);
                        }
                        accy = T(0);
                    }
                }
            }
        }
    }
    (void)curJ;
    if (NRM) {
        for (int o = 32; o > 0; o >>= 1) {
            nrm += __shfl_xor(nrm, o);
            pnr += __shfl_xor(pnr, o);
        }
        if (lane == 0) {
            a.part[2 * ((long long)q * a.ntiles + tix)] = nrm;
            a.part[2 * ((long long)q * a.ntiles + tix) + 1] = pnr;
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
        auto cuts = [&](int n, int nc, int maxw) {
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
        for (size_t yi = 0; yi + 1 < ey.size(); ++yi)
            for (size_t xi = 0; xi + 1 < ex.size(); ++xi) {
                MTile t{};
                t.b = b;
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
    const int nwg = (a.ntiles + 3) / 4;
    hipLaunchKernelGGL((k_march<T, PRO, RES, NRM>), dim3(nwg, nitems), dim3(256), 0, s, a);
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
