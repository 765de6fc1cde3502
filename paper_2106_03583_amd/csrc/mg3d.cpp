// Host side of the 3D multigrid solver without z synthesis (Sec. 3.3.1, the
// "3D MG" of the comparison in Sec. 4.2): plan creation and the cycle loop
// behind the mbp3_* entry points of mbp.h.
//
// The cycle loop is pipelined: the first smoothing sweep of every V-cycle
// also sums the squared residual of the cycle's input, and that number is
// copied to pinned memory right after the sweep, so the host reads it while
// the rest of the cycle is still running and decides whether to queue the
// next cycle (stop when the input already met the tolerance, or when the
// measured contraction predicts the output meets half of it).  The device
// never waits for the host between cycles.  A final residual evaluation of
// the returned iterate confirms the tolerance (more cycles run if it does
// not hold).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>

#include "internal.h"
#include "mg3d.h"

struct mbp3_plan {
    mbp_plan host;  // x-y hierarchy, coefficient and transfer tables, coarsest x-y eigen-decomposition
    mbp::Mg3Plan M;
    int device = -1;
    mbp::BusyFlag busy;
    void* dmem = nullptr;
    size_t dbytes = 0;
    void* pinned = nullptr;  // readback slots
    hipEvent_t ev_norm[2] = {nullptr, nullptr};
    hipEvent_t ev_t[2] = {nullptr, nullptr};
};

namespace mbp {

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// The 3D hierarchy: pairs (x-y level, nz).  Each step coarsens the
// direction(s) with the smaller spacing (PFMG's rule of semicoarsening along
// the smallest spacing): z alone when dz <= h/2, x-y alone when h <= dz/2,
// both otherwise, h being the mean x-y cell width sqrt(area / cells).  z is
// halved only while its count is even and >= 4; the last level is always
// the coarsest x-y level (its eigen-decomposition is the coarse solve).
std::vector<std::pair<int, int>> hierarchy(const mbp_plan& H) {
    std::vector<std::pair<int, int>> out;
    int xl = 0, nz = H.g.nz;
    out.emplace_back(xl, nz);
    for (;;) {
        const bool can_xy = xl + 1 < H.nlev;
        const bool can_z = nz % 2 == 0 && nz >= 4;
        if (!can_xy && !can_z) break;
        const double h = std::sqrt(H.area_sum / double(H.levels[xl].plane));
        const double dz = H.g.lz / nz;
        bool cx = can_xy, cz = can_z;
        if (can_xy && can_z) {
            if (dz <= 0.5 * h * (1.0 + 1e-9)) cx = false;
            else if (h <= 0.5 * dz * (1.0 + 1e-9)) cz = false;
        }
        if (cx) ++xl;
        if (cz) nz /= 2;
        out.emplace_back(xl, nz);
    }
    return out;
}

// Eigen-decomposition of the 1D z operator (uniform spacing dz, ghost rules
// of the end conditions): symmetric tridiagonal, solved by Jacobi rotations.
void z_eigen(int n, double dz, int lo, int hi, std::vector<double>& V, std::vector<double>& mu) {
    std::vector<double> A(size_t(n) * n, 0.0);
    const double w = 1.0 / (dz * dz);
    for (int k = 0; k < n; ++k) {
        A[size_t(k) * n + k] = -2.0 * w;
        if (k > 0) A[size_t(k) * n + k - 1] += w;
        if (k < n - 1) A[size_t(k) * n + k + 1] += w;
    }
    if (lo == MBP_PERIODIC) {
        A[size_t(0) * n + (n - 1)] += w;
        A[size_t(n - 1) * n + 0] += w;
    } else {
        A[0] += lo == MBP_NEUMANN ? w : -w;
        A[size_t(n - 1) * n + (n - 1)] += hi == MBP_NEUMANN ? w : -w;
    }
    jacobi_eig(A, n, V, mu);
}

}  // namespace

int mg3_create(const mbp_block_desc* blocks, int nblocks, const mbp_synth_desc* z, const mbp_options* opt,
               mbp3_plan* X) {
    mbp_options o;
    if (opt) {
        o = *opt;
    } else {
        options_default(&o);
        o.nu1 = 2;
        o.nu2 = 2;
        o.max_cycles = 100;
    }
    if (o.precision != MBP_FP64) return MBP_ERR_INVALID;  // the comparison solver is FP64 only
    if (o.smoother != MBP_SMOOTHER_DEFAULT && o.smoother != MBP_SMOOTHER_JACOBI) return MBP_ERR_INVALID;
    if (o.nu1 < 1 || o.nu2 < 1) return MBP_ERR_INVALID;
    mbp_options o2 = o;
    o2.smoother = MBP_SMOOTHER_DEFAULT;
    std::string err;
    // the x-y tables of the FFT path's plan (uniform x-y steps unless they
    // leave more than 256 coarsest cells, as there); its LDS budget does not
    // apply here
    int st = build_plan_host_limits(blocks, nblocks, z, &o2, int64_t(1) << 40, &X->host, &err, false);
    if (st != MBP_OK) return st;
    X->host.opt.smoother = o.smoother;
    mbp_plan& H = X->host;
    Mg3Plan& M = X->M;
    M.zlo = H.g.zlo;
    M.zhi = H.g.zhi;
    M.alpha = o.helmholtz;
    M.nc = H.coarse_n;
    const auto hier = hierarchy(H);
    M.nlev = int(hier.size());
    M.lev.assign(M.nlev, Mg3Level{});
    for (int l = 0; l < M.nlev; ++l) {
        Mg3Level& L = M.lev[l];
        L.xl = hier[l].first;
        const Level& X2 = H.levels[L.xl];
        L.blk_off = X2.blk_off;
        L.tile_off = X2.tile_off;
        L.ntiles = X2.ntiles;
        L.nz = hier[l].second;
        const double dz = H.g.lz / L.nz;
        L.idz2 = 1.0 / (dz * dz);
        L.plane = X2.plane;
        L.ncell = L.plane * L.nz;
        if (l + 1 < M.nlev) {
            L.xyc = hier[l + 1].first != L.xl ? 1 : 0;
            L.zc = hier[l + 1].second != L.nz ? 1 : 0;
        }
        L.even_xy = 1;
        for (int b = 0; b < X2.nb; ++b)
            if ((X2.nx[b] & 1) || (X2.ny[b] & 1)) L.even_xy = 0;
        L.xy22 = X2.cx && X2.cy ? 1 : 0;
    }
    return MBP_OK;
}

int mg3_device_init(mbp3_plan* X) {
    mbp_plan& H = X->host;
    Mg3Plan& M = X->M;
    const Mg3Level& C = M.lev[M.nlev - 1];
    const int nc = M.nc, nzc = C.nz;
    // coarsest z eigen-decomposition and the coarsest plane's cell map
    std::vector<double> vz, muz;
    z_eigen(nzc, H.g.lz / nzc, M.zlo, M.zhi, vz, muz);
    // smallest non-null eigenvalue magnitude of the coarsest 3D operator: an
    // estimate of the fine operator's, for the error test
    {
        double mx = 0.0;
        for (double a : H.coarse_mu)
            for (double b : muz) mx = std::max(mx, std::fabs(a + b - M.alpha));
        double mn = mx;
        for (double a : H.coarse_mu)
            for (double b : muz) {
                const double v = std::fabs(a + b - M.alpha);
                if (v > 1e-9 * mx) mn = std::min(mn, v);
            }
        M.mu_min = mn;
    }
    std::vector<int2> cmap(nc);
    {
        const Level& L = H.levels[C.xl];
        for (int b = 0; b < L.nb; ++b)
            for (int j = 0; j < L.ny[b]; ++j)
                for (int i = 0; i < L.nx[b]; ++i)
                    cmap[L.off[b] + j * L.nx[b] + i] =
                        make_int2(nzc * L.off[b] + j * L.nx[b] + i, L.nx[b] * L.ny[b]);
    }
    const Mg3Level& F = M.lev[0];
    const size_t nparts = size_t(F.ntiles) * F.nz;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    const size_t o_blk = take(H.hblk.size() * sizeof(DBlock));
    const size_t o_int = take(H.hint.size() * sizeof(int));
    const size_t o_dbl = take(H.hdbl.size() * sizeof(double));
    const size_t o_til = take(H.htiles.size() * sizeof(int4));
    const size_t o_cwl = take(size_t(nc) * nc * sizeof(double));
    const size_t o_cwr = take(size_t(nc) * nc * sizeof(double));
    const size_t o_cmu = take(size_t(nc) * sizeof(double));
    const size_t o_cmap = take(size_t(nc) * sizeof(int2));
    const size_t o_vz = take(vz.size() * sizeof(double));
    const size_t o_muz = take(muz.size() * sizeof(double));
    const size_t o_xh = take(size_t(nc) * nzc * sizeof(double));
    const size_t o_area = take(H.areas0.size() * sizeof(double));
    const size_t o_part = take(2 * nparts * sizeof(double));
    const size_t o_scal = take(8 * sizeof(double));
    const size_t o_q0 = take(size_t(F.ncell) * sizeof(double));
    std::vector<size_t> o_f(M.nlev, 0), o_p(M.nlev, 0), o_q(M.nlev, 0);
    for (int l = 1; l < M.nlev; ++l) {
        o_f[l] = take(size_t(M.lev[l].ncell) * sizeof(double));
        o_p[l] = take(size_t(M.lev[l].ncell) * sizeof(double));
        o_q[l] = take(size_t(M.lev[l].ncell) * sizeof(double));
    }
    void* mem = nullptr;
    if (hipMalloc(&mem, o) != hipSuccess) {
        (void)hipGetLastError();
        return MBP_ERR_NOMEM;
    }
    X->dmem = mem;
    X->dbytes = o;
    unsigned char* b = static_cast<unsigned char*>(mem);
    M.d_blk = reinterpret_cast<DBlock*>(b + o_blk);
    M.d_int = reinterpret_cast<int*>(b + o_int);
    M.d_dbl = reinterpret_cast<double*>(b + o_dbl);
    M.d_tiles = reinterpret_cast<int4*>(b + o_til);
    M.d_cwl = reinterpret_cast<double*>(b + o_cwl);
    M.d_cwr = reinterpret_cast<double*>(b + o_cwr);
    M.d_cmu = reinterpret_cast<double*>(b + o_cmu);
    M.d_cmap = reinterpret_cast<int2*>(b + o_cmap);
    M.d_vz = reinterpret_cast<double*>(b + o_vz);
    M.d_muz = reinterpret_cast<double*>(b + o_muz);
    M.d_xhat = reinterpret_cast<double*>(b + o_xh);
    M.d_area0 = reinterpret_cast<double*>(b + o_area);
    M.d_part = reinterpret_cast<double*>(b + o_part);
    M.d_scal = reinterpret_cast<double*>(b + o_scal);
    M.q0 = reinterpret_cast<double*>(b + o_q0);
    for (int l = 1; l < M.nlev; ++l) {
        M.lev[l].f = reinterpret_cast<double*>(b + o_f[l]);
        M.lev[l].p = reinterpret_cast<double*>(b + o_p[l]);
        M.lev[l].q = reinterpret_cast<double*>(b + o_q[l]);
    }
    auto up = [&](void* dst, const void* src, size_t bytes) {
        return bytes == 0 || hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    const bool ok = up(M.d_blk, H.hblk.data(), H.hblk.size() * sizeof(DBlock)) &&
                    up(M.d_int, H.hint.data(), H.hint.size() * sizeof(int)) &&
                    up(M.d_dbl, H.hdbl.data(), H.hdbl.size() * sizeof(double)) &&
                    up(M.d_tiles, H.htiles.data(), H.htiles.size() * sizeof(int4)) &&
                    up(M.d_cwl, H.coarse_wl.data(), H.coarse_wl.size() * sizeof(double)) &&
                    up(M.d_cwr, H.coarse_wr.data(), H.coarse_wr.size() * sizeof(double)) &&
                    up(M.d_cmu, H.coarse_mu.data(), H.coarse_mu.size() * sizeof(double)) &&
                    up(M.d_cmap, cmap.data(), cmap.size() * sizeof(int2)) &&
                    up(M.d_vz, vz.data(), vz.size() * sizeof(double)) &&
                    up(M.d_muz, muz.data(), muz.size() * sizeof(double)) &&
                    up(M.d_area0, H.areas0.data(), H.areas0.size() * sizeof(double));
    if (!ok) return MBP_ERR_HIP;
    if (hipHostMalloc(&X->pinned, 4096, hipHostMallocDefault) != hipSuccess) return MBP_ERR_NOMEM;
    for (int k = 0; k < 2; ++k) {
        if (hipEventCreateWithFlags(&X->ev_norm[k], hipEventDisableTiming) != hipSuccess) return MBP_ERR_HIP;
        if (hipEventCreate(&X->ev_t[k]) != hipSuccess) return MBP_ERR_HIP;
    }
    return MBP_OK;
}

void mg3_free(mbp3_plan* X) {
    for (int k = 0; k < 2; ++k) {
        if (X->ev_norm[k]) (void)hipEventDestroy(X->ev_norm[k]);
        if (X->ev_t[k]) (void)hipEventDestroy(X->ev_t[k]);
    }
    if (X->pinned) (void)hipHostFree(X->pinned);
    if (X->dmem) (void)hipFree(X->dmem);
    X->pinned = nullptr;
    X->dmem = nullptr;
}

namespace {

// Pinned readback layout (doubles): per cycle slot k, [8k] residual^2 and
// [8k+1] |p|^2 of the cycle's input; [16] the rhs mean; [17], [18] residual^2
// and |p|^2 of a residual evaluation.
constexpr int kPinMean = 16, kPinRes = 17;

// One V-cycle on the iterate p (finest level = the caller's buffer).  The
// first sweep's residual and iterate sums of squares land in d_scal[0..1] and
// are copied to pinned slot `slot` behind event ev (skipped when ev is null).
void mg3_cycle(mbp3_plan* X, double* p, const double* f, double fshift, bool zero_p, int slot, hipEvent_t ev,
               hipStream_t s) {
    const Mg3Plan& M = X->M;
    const int nu1 = X->host.opt.nu1, nu2 = X->host.opt.nu2;
    const int L = M.nlev - 1;
    std::vector<double*> cur(M.nlev), oth(M.nlev);
    std::vector<const double*> rhs(M.nlev);
    cur[0] = p;
    oth[0] = M.q0;
    rhs[0] = f;
    for (int l = 1; l < M.nlev; ++l) {
        cur[l] = M.lev[l].p;
        oth[l] = M.lev[l].q;
        rhs[l] = M.lev[l].f;
    }
    double* pin = static_cast<double*>(X->pinned);
    for (int l = 0; l < L; ++l) {
        const double sh = l == 0 ? fshift : 0.0;
        for (int k = 0; k < nu1; ++k) {
            const bool zero = k == 0 && (l > 0 || zero_p);
            const bool norm = l == 0 && k == 0 && ev;
            const long long nw = m3_jacobi(M, l, cur[l], oth[l], rhs[l], sh, zero, norm ? M.d_part : nullptr, s);
            std::swap(cur[l], oth[l]);
            if (norm) {
                m3_total(M.d_part, nw, 1.0, M.d_scal, s);
                m3_total(M.d_part + nw, nw, 1.0, M.d_scal + 1, s);
                (void)hipMemcpyAsync(pin + 8 * slot, M.d_scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
                (void)hipEventRecord(ev, s);
            }
        }
        m3_restrict(M, l, cur[l], rhs[l], sh, M.lev[l + 1].f, s);
    }
    m3_coarse(M, M.lev[L].f, cur[L], s);
    for (int l = L - 1; l >= 0; --l) {
        m3_prolong(M, l, cur[l + 1], cur[l], s);
        const double sh = l == 0 ? fshift : 0.0;
        for (int k = 0; k < nu2; ++k) {
            m3_jacobi(M, l, cur[l], oth[l], rhs[l], sh, false, nullptr, s);
            std::swap(cur[l], oth[l]);
        }
    }
    if (cur[0] != p) m3_copy(cur[0], p, M.lev[0].ncell, s);
}

}  // namespace

// Stopping rule (the readings of the FFT path, on the whole 3D field):
// ||f - L_h p|| <= rtol ||f|| and the error estimate 2 ||r|| / mu_min <=
// etol ||p||, mu_min being the smallest non-null eigenvalue magnitude of the
// coarsest operator (etol = 10 rtol by default, negative = off).
int mg3_solve(mbp3_plan* X, const double* f, double* p, double rtol, int flags, hipStream_t s,
              mbp_solve_info* info) {
    const Mg3Plan& M = X->M;
    const mbp_plan& H = X->host;
    const Mg3Level& F = M.lev[0];
    const bool singular = H.g.singular && M.alpha == 0.0;
    const bool warm = (flags & MBP_WARM_START) != 0;
    const int maxc = H.opt.max_cycles;
    const double etol = H.opt.etol == 0.0 ? 10.0 * rtol : H.opt.etol;
    const double etol2 = etol < 0.0 ? -1.0 : etol * etol;
    double* pin = static_cast<double*>(X->pinned);
    (void)hipEventRecord(X->ev_t[0], s);
    int status = MBP_OK;
    // compatibility of a singular problem: volume-weighted mean of f
    double fshift = 0.0, removed = 0.0;
    const double vol = H.area_sum * F.nz;
    if (singular) {
        m3_area_sum(M, f, M.d_part, M.d_scal + 2, 1.0 / vol, s);
        if (hipMemcpyAsync(pin + kPinMean, M.d_scal + 2, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return MBP_ERR_HIP;
        if (flags & MBP_PROJECT_RHS) {
            fshift = pin[kPinMean];
            removed = fshift;
        }
    }
    // ||f - fshift||^2 (the residual of p = 0)
    m3_residual_norm(M, p, f, fshift, true, M.d_part, M.d_scal + 3, s);
    if (hipMemcpyAsync(pin + kPinRes, M.d_scal + 3, 2 * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return MBP_ERR_HIP;
    const double fn2 = pin[kPinRes];
    if (!std::isfinite(fn2)) status = MBP_ERR_NONFINITE;
    if (status == MBP_OK && singular && !(flags & MBP_PROJECT_RHS)) {
        const double rms = std::sqrt(fn2 / double(F.ncell));
        if (std::fabs(pin[kPinMean]) > 1e-12 * (rms + 1e-300)) status = MBP_ERR_INCOMPATIBLE;
    }
    const double mu2 = M.mu_min * M.mu_min;
    auto passes = [&](double r2, double p2, double scale) {
        return r2 <= scale * scale * rtol * rtol * fn2 && (etol2 < 0.0 || 4.0 * r2 <= scale * scale * etol2 * mu2 * p2);
    };
    int cycles = 0;  // V-cycles queued (each one runs to completion)
    double res = 0.0;
    if (status == MBP_OK && fn2 == 0.0) {
        launch_zero(p, size_t(F.ncell), s);  // f = 0 (after projection): p = 0
    } else if (status == MBP_OK) {
        bool zero_p = !warm;
        for (;;) {
            // cycles run back to back; the host reads each cycle's input
            // residual while the rest of that cycle runs, then queues the next
            double prev = -1.0;
            int slot = 0;
            mg3_cycle(X, p, f, fshift, zero_p, slot, X->ev_norm[slot], s);
            ++cycles;
            zero_p = false;
            for (;;) {
                if (hipEventSynchronize(X->ev_norm[slot]) != hipSuccess) return MBP_ERR_HIP;
                const double r2 = pin[8 * slot], p2 = pin[8 * slot + 1];
                if (!std::isfinite(r2)) {
                    status = MBP_ERR_NONFINITE;
                    break;
                }
                // the input already passes, or the measured contraction
                // predicts that this cycle's output passes with margin 2
                const double rho2 = prev > 0.0 ? r2 / prev : 1e300;
                if (passes(r2, p2, 1.0) || (rho2 < 1.0 && passes(r2 * rho2, p2, 0.5)) || cycles >= maxc) break;
                prev = r2;
                slot ^= 1;
                mg3_cycle(X, p, f, fshift, false, slot, X->ev_norm[slot], s);
                ++cycles;
            }
            // the returned iterate
            m3_residual_norm(M, p, f, fshift, false, M.d_part, M.d_scal + 3, s);
            if (hipMemcpyAsync(pin + kPinRes, M.d_scal + 3, 2 * sizeof(double), hipMemcpyDeviceToHost, s) !=
                    hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return MBP_ERR_HIP;
            res = std::sqrt(pin[kPinRes] / fn2);
            if (status != MBP_OK) break;
            if (!std::isfinite(res)) {
                status = MBP_ERR_NONFINITE;
                break;
            }
            if (passes(pin[kPinRes], pin[kPinRes + 1], 1.0)) break;
            if (cycles >= maxc) {
                status = MBP_ERR_NOT_CONVERGED;
                break;
            }
        }
        if (singular && (status == MBP_OK || status == MBP_ERR_NOT_CONVERGED)) {
            // gauge: zero volume-weighted mean of p
            m3_area_sum(M, p, M.d_part, M.d_scal + 5, 1.0 / vol, s);
            m3_sub(p, F.ncell, M.d_scal + 5, s);
        }
    }
    (void)hipEventRecord(X->ev_t[1], s);
    if (hipStreamSynchronize(s) != hipSuccess) return MBP_ERR_HIP;
    if (hipGetLastError() != hipSuccess) return MBP_ERR_HIP;
    if (info) {
        info->status = status;
        info->cycles = cycles;
        info->rel_residual = res;
        info->removed_mean = status == MBP_ERR_NONFINITE ? 0.0 : removed;
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, X->ev_t[0], X->ev_t[1]);
        info->t_ms[0] = 0.0;
        info->t_ms[1] = ms;
        info->t_ms[2] = 0.0;
        info->t_ms[3] = ms;
    }
    return status;
}

}  // namespace mbp

extern "C" {

int mbp3_plan_create(const mbp_block_desc* blocks, int nblocks, const mbp_synth_desc* z, const mbp_options* opt,
                     mbp3_plan** out) {
    if (!out) return MBP_ERR_INVALID;
    *out = nullptr;
    int dev = 0, count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
        (void)hipGetLastError();
        return MBP_ERR_NO_DEVICE;
    }
    if (hipGetDevice(&dev) != hipSuccess) return MBP_ERR_HIP;
    mbp3_plan* X = new (std::nothrow) mbp3_plan();
    if (!X) return MBP_ERR_NOMEM;
    int st = mbp::mg3_create(blocks, nblocks, z, opt, X);
    if (st == MBP_OK) {
        X->device = dev;
        st = mbp::mg3_device_init(X);
    }
    if (st != MBP_OK) {
        mbp::mg3_free(X);
        delete X;
        return st;
    }
    *out = X;
    return MBP_OK;
}

int mbp3_plan_levels(const mbp3_plan* plan, int* nlevels, int* nz_per_level, int64_t* cells_per_level,
                     size_t* workspace_bytes) {
    if (!plan) return MBP_ERR_INVALID;
    if (nlevels) *nlevels = plan->M.nlev;
    for (int l = 0; l < plan->M.nlev; ++l) {
        if (nz_per_level) nz_per_level[l] = plan->M.lev[l].nz;
        if (cells_per_level) cells_per_level[l] = plan->M.lev[l].ncell;
    }
    if (workspace_bytes) *workspace_bytes = plan->dbytes;
    return MBP_OK;
}

int mbp3_jacobi_sweep(mbp3_plan* plan, const double* pin_dev, double* pout_dev, const double* f_dev,
                      void* stream) {
    if (!plan || !pin_dev || !pout_dev || !f_dev || pin_dev == pout_dev) return MBP_ERR_INVALID;
    mbp::m3_jacobi(plan->M, 0, pin_dev, pout_dev, f_dev, 0.0, false, nullptr, static_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? MBP_OK : MBP_ERR_HIP;
}

int mbp3_solve(mbp3_plan* plan, const double* rhs_dev, double* p_dev, double rtol, int flags, void* stream,
               mbp_solve_info* info) {
    if (!plan || !rhs_dev || !p_dev || !(rtol > 0.0) || rhs_dev == p_dev) return MBP_ERR_INVALID;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != plan->device) return MBP_ERR_INVALID;
    if (!plan->busy.claim()) return MBP_ERR_BUSY;
    const int st = mbp::mg3_solve(plan, rhs_dev, p_dev, rtol, flags | plan->host.opt.flags,
                                  static_cast<hipStream_t>(stream), info);
    plan->busy.release();
    return st;
}

void mbp3_plan_destroy(mbp3_plan* plan) {
    if (!plan) return;
    mbp::mg3_free(plan);
    delete plan;
}

}  // extern "C"
