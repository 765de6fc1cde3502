// Device workspace and the solve drivers (Algorithm 1 on one plan).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace mbp {

void launch_lds_full(const mbp_plan* P, double* p, const double* f, const int* act, const int* nact,
                     int nitems, int maxc, double rtol2, double etol2, int* cyc, double* rnorm,
                     double* fnorm, hipStream_t s);
void launch_reset_active(const mbp_plan* P, hipStream_t s);
void launch_area_dot(const mbp_plan* P, const double* plane, double* out_sum, hipStream_t s);
void launch_fill_int(int* p, int n, int v, hipStream_t s);

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct Layout {
    size_t blk, ints, dbls, tiles, shift, cwl, cwr, cmu, area0, ftf, fti, mt, fhat, phat, phatB, part,
        fnorm, rnorm, pnorm, sabs, act, nact, cyc, flag, scal;
    std::vector<size_t> p64, f64, p32, f32, p64B, p32B;
    size_t total;
};

Layout layout(const mbp_plan* P, size_t ftile_bytes, size_t mtile_bytes, int nparts) {
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    const size_t nz = size_t(P->g.nz);
    const size_t nc = size_t(P->coarse_n);
    L.blk = take(P->hblk.size() * sizeof(DBlock));
    L.ints = take(P->hint.size() * sizeof(int));
    L.dbls = take(P->hdbl.size() * sizeof(double));
    L.tiles = take(P->htiles.size() * sizeof(int4));
    L.shift = take(nz * sizeof(double));
    L.cwl = take(nc * nc * sizeof(double));
    L.cwr = take(nc * nc * sizeof(double));
    L.cmu = take(nc * sizeof(double));
    L.area0 = take(size_t(P->plane0) * sizeof(double));
    L.ftf = take(ftile_bytes);
    L.fti = take(ftile_bytes);
    L.mt = take(mtile_bytes);
    L.fhat = take(nz * P->plane0 * sizeof(double));
    L.phat = take(nz * P->plane0 * sizeof(double));
    const bool mixed = P->opt.precision == MBP_MIXED;
    // out-of-place sweeps need a second buffer on every level that runs them
    const int Lg = mixed ? P->lds_level32 : P->lds_level;  // levels below run in LDS
    auto march = [&](int l) { return l < Lg && l < int(P->march_ok.size()) && P->march_ok[l]; };
    L.phatB = (!mixed && march(0)) ? take(nz * P->plane0 * sizeof(double)) : 0;
    L.p64.assign(P->nlev, 0);
    L.f64.assign(P->nlev, 0);
    L.p64B.assign(P->nlev, 0);
    for (int l = 1; l < P->nlev; ++l) {
        L.p64[l] = take(nz * P->levels[l].plane * sizeof(double));
        L.f64[l] = take(nz * P->levels[l].plane * sizeof(double));
        if (!mixed && march(l)) L.p64B[l] = take(nz * P->levels[l].plane * sizeof(double));
    }
    L.p32.assign(P->nlev, 0);
    L.f32.assign(P->nlev, 0);
    L.p32B.assign(P->nlev, 0);
    if (mixed)
        for (int l = 0; l < P->nlev; ++l) {
            L.p32[l] = take(nz * P->levels[l].plane * sizeof(float));
            L.f32[l] = take(nz * P->levels[l].plane * sizeof(float));
            if (march(l)) L.p32B[l] = take(nz * P->levels[l].plane * sizeof(float));
        }
    L.part = take(2 * nz * size_t(std::max(nparts, P->levels[0].ntiles)) * sizeof(double));
    L.fnorm = take(nz * sizeof(double));
    L.rnorm = take(nz * sizeof(double));
    L.pnorm = take(nz * sizeof(double));
    L.sabs = take(nz * sizeof(double));
    L.act = take(nz * sizeof(int));
    L.nact = take(sizeof(int) * 4);
    L.cyc = take(nz * sizeof(int));
    L.flag = take(sizeof(int) * 4);
    L.scal = take(sizeof(double) * 8);
    L.total = o;
    return L;
}

}  // namespace

constexpr int kMarchSeg = 30;  // rows per fused-sweep strip (the LDS tile height)

// Fused-sweep strips of every level (host tables); fills march_ok.
void plan_march_tables(mbp_plan* P, std::vector<unsigned char>& bytes) {
    P->march_ok.assign(P->nlev, 0);
    P->mtile_off.assign(P->nlev, 0);
    P->mtile_cnt.assign(P->nlev, 0);
    bytes.clear();
    int off = 0;
    for (int l = 0; l < P->nlev; ++l) {
        P->march_ok[l] = march_level_ok(P, l) ? 1 : 0;
        if (!P->march_ok[l]) continue;
        std::vector<unsigned char> b;
        int cnt = 0;
        march_build_tiles_bytes(P, l, kMarchSeg, b, &cnt);
        P->mtile_off[l] = off;
        P->mtile_cnt[l] = cnt;
        off += cnt;
        bytes.insert(bytes.end(), b.begin(), b.end());
    }
}

size_t plan_device_bytes(const mbp_plan* P) {
    mbp_plan tmp = *P;
    std::vector<unsigned char> mt;
    plan_march_tables(&tmp, mt);
    const int W = fft_columns_per_wg(P);
    size_t nt = 0;
    for (int b = 0; b < P->g.nb; ++b) nt += (size_t(P->g.nx[b]) * P->g.ny[b] + W - 1) / W;
    return layout(&tmp, nt * 32, mt.size(), tmp.mtile_cnt.empty() ? 0 : tmp.mtile_cnt[0]).total;
}

int plan_device_init(mbp_plan* P) {
    std::vector<unsigned char> ftf, fti, mt;
    fft_build_tiles(P, ftf, fti, &P->fft_ntiles);
    plan_march_tables(P, mt);
    Layout L = layout(P, ftf.size(), mt.size(), P->mtile_cnt[0]);
    void* mem = nullptr;
    if (hipMalloc(&mem, L.total) != hipSuccess) {
        (void)hipGetLastError();
        return MBP_ERR_NOMEM;
    }
    P->dmem = mem;
    P->dbytes = L.total;
    unsigned char* b = static_cast<unsigned char*>(mem);
    P->d_blk = reinterpret_cast<DBlock*>(b + L.blk);
    P->d_int = reinterpret_cast<int*>(b + L.ints);
    P->d_dbl = reinterpret_cast<double*>(b + L.dbls);
    P->d_tiles = reinterpret_cast<int4*>(b + L.tiles);
    P->d_shift = reinterpret_cast<double*>(b + L.shift);
    P->d_cwl = reinterpret_cast<double*>(b + L.cwl);
    P->d_cwr = reinterpret_cast<double*>(b + L.cwr);
    P->d_cmu = reinterpret_cast<double*>(b + L.cmu);
    P->d_area0 = reinterpret_cast<double*>(b + L.area0);
    P->d_ftiles_fwd = b + L.ftf;
    P->d_ftiles_inv = b + L.fti;
    P->d_mtiles = b + L.mt;
    P->mtile_bytes = mt.size();
    P->fhat = reinterpret_cast<double*>(b + L.fhat);
    P->phat = reinterpret_cast<double*>(b + L.phat);
    P->phatB = L.phatB ? reinterpret_cast<double*>(b + L.phatB) : nullptr;
    P->p64.assign(P->nlev, nullptr);
    P->f64.assign(P->nlev, nullptr);
    P->p64B.assign(P->nlev, nullptr);
    P->p32.assign(P->nlev, nullptr);
    P->f32.assign(P->nlev, nullptr);
    P->p32B.assign(P->nlev, nullptr);
    for (int l = 1; l < P->nlev; ++l) {
        P->p64[l] = reinterpret_cast<double*>(b + L.p64[l]);
        P->f64[l] = reinterpret_cast<double*>(b + L.f64[l]);
        if (L.p64B[l]) P->p64B[l] = reinterpret_cast<double*>(b + L.p64B[l]);
    }
    if (P->opt.precision == MBP_MIXED)
        for (int l = 0; l < P->nlev; ++l) {
            P->p32[l] = reinterpret_cast<float*>(b + L.p32[l]);
            P->f32[l] = reinterpret_cast<float*>(b + L.f32[l]);
            if (L.p32B[l]) P->p32B[l] = reinterpret_cast<float*>(b + L.p32B[l]);
        }
    P->d_part = reinterpret_cast<double*>(b + L.part);
    P->nparts = P->levels[0].ntiles;
    P->d_fnorm = reinterpret_cast<double*>(b + L.fnorm);
    P->d_rnorm = reinterpret_cast<double*>(b + L.rnorm);
    P->d_pnorm = reinterpret_cast<double*>(b + L.pnorm);
    P->d_sabs = reinterpret_cast<double*>(b + L.sabs);
    P->d_act = reinterpret_cast<int*>(b + L.act);
    P->d_nact = reinterpret_cast<int*>(b + L.nact);
    P->d_cyc = reinterpret_cast<int*>(b + L.cyc);
    P->d_flag = reinterpret_cast<int*>(b + L.flag);
    P->d_scal = reinterpret_cast<double*>(b + L.scal);
    auto up = [&](void* dst, const void* src, size_t bytes) {
        if (bytes == 0) return true;
        return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    bool ok = up(P->d_blk, P->hblk.data(), P->hblk.size() * sizeof(DBlock)) &&
              up(P->d_int, P->hint.data(), P->hint.size() * sizeof(int)) &&
              up(P->d_dbl, P->hdbl.data(), P->hdbl.size() * sizeof(double)) &&
              up(P->d_tiles, P->htiles.data(), P->htiles.size() * sizeof(int4)) &&
              up(P->d_shift, P->shift.data(), P->shift.size() * sizeof(double)) &&
              up(P->d_sabs, P->sabs.data(), P->sabs.size() * sizeof(double)) &&
              up(P->d_cwl, P->coarse_wl.data(), P->coarse_wl.size() * sizeof(double)) &&
              up(P->d_cwr, P->coarse_wr.data(), P->coarse_wr.size() * sizeof(double)) &&
              up(P->d_cmu, P->coarse_mu.data(), P->coarse_mu.size() * sizeof(double)) &&
              up(P->d_area0, P->areas0.data(), P->areas0.size() * sizeof(double)) &&
              up(P->d_ftiles_fwd, ftf.data(), ftf.size()) && up(P->d_ftiles_inv, fti.data(), fti.size()) &&
              up(P->d_mtiles, mt.data(), mt.size());
    if (!ok) return MBP_ERR_HIP;
    void* hp = nullptr;
    if (hipHostMalloc(&hp, 4096, hipHostMallocDefault) != hipSuccess) return MBP_ERR_NOMEM;
    P->host_pinned = hp;
    return MBP_OK;
}

// Event pairs around a finest-level sweep launch (only while profiling).
// The plan object is logically const for the kernels; the record is mutable.
void prof_begin(const mbp_plan* Pc, int cls, hipStream_t s, double cells) {
    mbp_plan* P = const_cast<mbp_plan*>(Pc);
    if (!P->prof) return;
    auto& v = P->prof_ev[cls];
    const size_t i = P->prof_used[cls];
    if (i == v.size()) {
        std::array<void*, 2> e{nullptr, nullptr};
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return;
        e[0] = a;
        e[1] = b;
        v.push_back(e);
        P->prof_cells[cls].push_back(0.0);
    }
    P->prof_cells[cls][i] = cells;
    (void)hipEventRecord(static_cast<hipEvent_t>(v[i][0]), s);
}

void prof_end(const mbp_plan* Pc, int cls, hipStream_t s) {
    mbp_plan* P = const_cast<mbp_plan*>(Pc);
    if (!P->prof) return;
    const size_t i = P->prof_used[cls];
    if (i >= P->prof_ev[cls].size()) return;
    (void)hipEventRecord(static_cast<hipEvent_t>(P->prof_ev[cls][i][1]), s);
    P->prof_used[cls] = i + 1;
}

void plan_device_free(mbp_plan* P) {
    for (int c = 0; c < 2; ++c)
        for (auto& e : P->prof_ev[c]) {
            (void)hipEventDestroy(static_cast<hipEvent_t>(e[0]));
            (void)hipEventDestroy(static_cast<hipEvent_t>(e[1]));
        }
    if (P->dmem) (void)hipFree(P->dmem);
    if (P->host_pinned) (void)hipHostFree(P->host_pinned);
    P->dmem = nullptr;
    P->host_pinned = nullptr;
}

namespace {

struct Readback {
    double maxratio;
    int nact;
    int flag;
    double s1, s2;
};

}  // namespace

// Algorithm 1: forward transform, per-mode multigrid to the tolerance,
// inverse transform.  Host-driven: convergence data is read back once per
// cycle (the plain form; the batched form replays a captured graph instead).
int solve_one(mbp_plan* P, const double* rhs, double* p, double rtol, int flags, hipStream_t s,
              mbp_solve_info* info) {
    const int nz = P->g.nz;
    const bool mixed = P->opt.precision == MBP_MIXED;
    const bool retire = (flags & MBP_RETIRE) != 0;
    const int maxc = P->opt.max_cycles;
    const double rtol2 = rtol * rtol;
    const double etol = P->opt.etol == 0.0 ? 10.0 * rtol : P->opt.etol;
    const double etol2 = etol < 0.0 ? -1.0 : etol * etol;
    hipEvent_t ev[4];
    for (auto& e : ev) (void)hipEventCreate(&e);
    (void)hipEventRecord(ev[0], s);
    launch_fill_int(P->d_flag, 4, 0, s);
    launch_forward(P, rhs, P->fhat, P->d_flag, s);
    if (P->g.singular) {
        if (flags & MBP_PROJECT_RHS) launch_singular_fix(P, P->fhat, P->d_scal + 1, s);
        else launch_area_dot(P, P->fhat, P->d_scal + 1, s);
    }
    launch_plane_norm(P, P->fhat, P->d_fnorm, s);
    if (flags & MBP_WARM_START) launch_forward(P, p, P->phat, nullptr, s);
    else launch_zero(P->phat, size_t(nz) * P->plane0, s);
    launch_reset_active(P, s);
    (void)hipEventRecord(ev[1], s);

    double* hs = static_cast<double*>(P->host_pinned);
    int* hi = reinterpret_cast<int*>(hs + 16);
    (void)hipMemcpyAsync(hi, P->d_flag, sizeof(int), hipMemcpyDeviceToHost, s);
    (void)hipMemcpyAsync(hs + 1, P->d_scal + 1, sizeof(double), hipMemcpyDeviceToHost, s);
    if (hipStreamSynchronize(s) != hipSuccess) return MBP_ERR_HIP;
    int status = MBP_OK;
    double removed = 0.0;
    if (hi[0]) status = MBP_ERR_NONFINITE;
    if (status == MBP_OK && P->g.singular) {
        const double mean_q0 = hs[1] / P->area_sum;  // area-weighted mean of fhat_0
        removed = mean_q0 / std::sqrt(double(nz));   // volume-weighted mean of f
        if (!(flags & MBP_PROJECT_RHS)) {
            // compatible if the mean is at rounding level of the plane's rms
            std::vector<double> fn(1);
            (void)hipMemcpy(fn.data(), P->d_fnorm, sizeof(double), hipMemcpyDeviceToHost);
            const double rms = std::sqrt(fn[0] / double(P->plane0));
            if (std::fabs(mean_q0) > 1e-12 * (rms + 1e-300)) status = MBP_ERR_INCOMPATIBLE;
            removed = 0.0;
        }
    }
    int cycles = 0;
    double maxratio = 0.0;
    std::vector<int> cyc(nz, 0);
    if (status == MBP_OK) {
        if (!mixed && P->lds_level == 0) {
            launch_lds_full(P, P->phat, P->fhat, P->d_act, P->d_nact, nz, maxc, rtol2, etol2, P->d_cyc,
                            P->d_rnorm, P->d_fnorm, s);
            std::vector<double> rn(nz), fn(nz);
            (void)hipMemcpyAsync(cyc.data(), P->d_cyc, nz * sizeof(int), hipMemcpyDeviceToHost, s);
            (void)hipMemcpyAsync(rn.data(), P->d_rnorm, nz * sizeof(double), hipMemcpyDeviceToHost, s);
            (void)hipMemcpyAsync(fn.data(), P->d_fnorm, nz * sizeof(double), hipMemcpyDeviceToHost, s);
            if (hipStreamSynchronize(s) != hipSuccess) return MBP_ERR_HIP;
            for (int q = 0; q < nz; ++q) {
                const double r = fn[q] > 0 ? rn[q] / fn[q] : (rn[q] > 0 ? 1e300 : 0.0);
                maxratio = std::max(maxratio, r);
                cycles = std::max(cycles, cyc[q]);
            }
            if (maxratio > rtol2) status = MBP_ERR_NOT_CONVERGED;
        } else {
            int nitems = nz;
            int fused_parts = 0;  // > 0: the last V-cycle already produced the residual partials
            for (int c = 0;; ++c) {
                if (mixed)
                    launch_residual_to32(P, P->phat, P->fhat, P->f32[0], P->p32[0], P->d_rnorm,
                                         P->d_act, P->d_nact, nitems, s);
                else if (fused_parts > 0)
                    launch_finish(P, fused_parts, P->d_rnorm, P->d_act, P->d_nact, nitems, s);
                else
                    launch_residual_norm(P, P->phat, P->fhat, P->d_rnorm, P->d_act, P->d_nact, nitems, s);
                launch_update_active(P, rtol2, etol2, retire ? 1 : 0, c, s);
                (void)hipMemcpyAsync(hs, P->d_scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
                (void)hipMemcpyAsync(hi + 1, P->d_nact, sizeof(int), hipMemcpyDeviceToHost, s);
                if (hipStreamSynchronize(s) != hipSuccess) return MBP_ERR_HIP;
                cycles = c;
                if (retire) {
                    nitems = hi[1];
                    if (nitems == 0) break;
                } else if (hs[1] == 0.0) {  // every mode passed
                    maxratio = hs[0];
                    break;
                }
                maxratio = hs[0];
                if (c >= maxc) {
                    status = MBP_ERR_NOT_CONVERGED;
                    break;
                }
                if (mixed) {
                    launch_vcycle<float>(P, P->p32[0], P->p32B[0], P->f32[0], P->d_act, P->d_nact, nitems,
                                         false, s);
                    launch_add_correction(P, P->phat, P->p32[0], P->d_act, P->d_nact, nitems, s);
                } else {
                    fused_parts = launch_vcycle<double>(P, P->phat, P->phatB, P->fhat, P->d_act, P->d_nact,
                                                        nitems, true, s);
                }
            }
            (void)hipMemcpyAsync(cyc.data(), P->d_cyc, nz * sizeof(int), hipMemcpyDeviceToHost, s);
            if (retire) {
                std::vector<double> rn(nz), fn(nz);
                (void)hipMemcpyAsync(rn.data(), P->d_rnorm, nz * sizeof(double), hipMemcpyDeviceToHost, s);
                (void)hipMemcpyAsync(fn.data(), P->d_fnorm, nz * sizeof(double), hipMemcpyDeviceToHost, s);
                if (hipStreamSynchronize(s) != hipSuccess) return MBP_ERR_HIP;
                maxratio = 0.0;
                for (int q = 0; q < nz; ++q)
                    maxratio = std::max(maxratio, fn[q] > 0 ? rn[q] / fn[q] : (rn[q] > 0 ? 1e300 : 0.0));
            }
            if (hipStreamSynchronize(s) != hipSuccess) return MBP_ERR_HIP;
            if (retire)
                for (int q = 0; q < nz; ++q) cycles = std::max(cycles, cyc[q]);
        }
    }
    (void)hipEventRecord(ev[2], s);
    if (status == MBP_OK || status == MBP_ERR_NOT_CONVERGED) {
        if (P->g.singular) launch_singular_fix(P, P->phat, P->d_scal + 2, s);
        launch_inverse(P, P->phat, p, s);
    }
    (void)hipEventRecord(ev[3], s);
    if (hipStreamSynchronize(s) != hipSuccess) return MBP_ERR_HIP;
    if (hipGetLastError() != hipSuccess) return MBP_ERR_HIP;
    if (info) {
        info->status = status;
        info->cycles = cycles;
        info->rel_residual = std::sqrt(maxratio);
        info->removed_mean = removed;
        if (info->cycles_per_mode) std::memcpy(info->cycles_per_mode, cyc.data(), nz * sizeof(int));
        float t01 = 0, t12 = 0, t23 = 0, t03 = 0;
        (void)hipEventElapsedTime(&t01, ev[0], ev[1]);
        (void)hipEventElapsedTime(&t12, ev[1], ev[2]);
        (void)hipEventElapsedTime(&t23, ev[2], ev[3]);
        (void)hipEventElapsedTime(&t03, ev[0], ev[3]);
        info->t_ms[0] = t01;
        info->t_ms[1] = t12;
        info->t_ms[2] = t23;
        info->t_ms[3] = t03;
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    return status;
}

}  // namespace mbp
