// Device workspace and the solve drivers (Algorithm 1 on one plan).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace mbp {

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

constexpr int kMarchSeg = 26;  // rows per fused-sweep strip (the LDS tile height)

// Fused-sweep strips of every level (host tables); fills march_ok.  Two
// sets per level: short strips for the LDS form, tall ones for the
// register march; both live in one descriptor array.
constexpr int kRMarchSeg = 128;  // rows per register-march strip

void plan_march_tables(mbp_plan* P, std::vector<unsigned char>& bytes) {
    P->march_ok.assign(P->nlev, 0);
    P->mtile_off.assign(P->nlev, 0);
    P->mtile_cnt.assign(P->nlev, 0);
    P->rtile_off.assign(P->nlev, 0);
    P->rtile_cnt.assign(P->nlev, 0);
    P->use_rmarch.assign(P->nlev, 0);
    bytes.clear();
    int off = 0;
    for (int l = 0; l < P->nlev; ++l) {
        // the fused transfers take 2 x 2 children (restriction) and two fine
        // rows per coarse row (correction): not above a semicoarsened step
        const bool full_step = l + 1 >= P->nlev || (P->levels[l].cx && P->levels[l].cy);
        P->march_ok[l] = full_step && march_level_ok(P, l) ? 1 : 0;
        if (!P->march_ok[l]) continue;
        for (int set = 0; set < 2; ++set) {
            std::vector<unsigned char> b;
            int cnt = 0;
            march_build_tiles_bytes(P, l, set == 0 ? kMarchSeg : kRMarchSeg, b, &cnt);
            (set == 0 ? P->mtile_off : P->rtile_off)[l] = off;
            (set == 0 ? P->mtile_cnt : P->rtile_cnt)[l] = cnt;
            off += cnt;
            bytes.insert(bytes.end(), b.begin(), b.end());
        }
        P->use_rmarch[l] = char(P->opt.march);  // the autotuner may change it per level
    }
}

static int partial_count(const mbp_plan* P) {
    if (P->mtile_cnt.empty()) return 0;
    return std::max(4 * P->mtile_cnt[0], P->rtile_cnt[0]);
}

size_t plan_device_bytes(const mbp_plan* P) {
    mbp_plan tmp = *P;
    std::vector<unsigned char> mt;
    plan_march_tables(&tmp, mt);
    const int W = fft_columns_per_wg(P);
    size_t nt = 0;
    for (int b = 0; b < P->g.nb; ++b) nt += (size_t(P->g.nx[b]) * P->g.ny[b] + W - 1) / W;
    return layout(&tmp, nt * 32, mt.size(), partial_count(&tmp)).total;
}

int plan_device_init(mbp_plan* P, void* ext_mem, size_t ext_bytes, void* ext_pinned) {
    std::vector<unsigned char> ftf, fti, mt;
    fft_build_tiles(P, ftf, fti, &P->fft_ntiles);
    if (const int st = fft_stream_setup(P)) return st;
    plan_march_tables(P, mt);
    Layout L = layout(P, ftf.size(), mt.size(), partial_count(P));
    void* mem = ext_mem;
    if (ext_mem) {
        if (ext_bytes < L.total) return MBP_ERR_NOMEM;
        P->owns_mem = false;
    } else {
        if (hipMalloc(&mem, L.total) != hipSuccess) {
            (void)hipGetLastError();
            return MBP_ERR_NOMEM;
        }
        P->owns_mem = true;
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
    // every table sits below fhat in the allocation: one host image, one copy
    std::vector<unsigned char> img(L.fhat, 0);
    auto put = [&](size_t off, const void* src, size_t bytes) {
        if (bytes) std::memcpy(img.data() + off, src, bytes);
    };
    put(L.blk, P->hblk.data(), P->hblk.size() * sizeof(DBlock));
    put(L.ints, P->hint.data(), P->hint.size() * sizeof(int));
    put(L.dbls, P->hdbl.data(), P->hdbl.size() * sizeof(double));
    put(L.tiles, P->htiles.data(), P->htiles.size() * sizeof(int4));
    put(L.shift, P->shift.data(), P->shift.size() * sizeof(double));
    put(L.cwl, P->coarse_wl.data(), P->coarse_wl.size() * sizeof(double));
    put(L.cwr, P->coarse_wr.data(), P->coarse_wr.size() * sizeof(double));
    put(L.cmu, P->coarse_mu.data(), P->coarse_mu.size() * sizeof(double));
    put(L.area0, P->areas0.data(), P->areas0.size() * sizeof(double));
    put(L.ftf, ftf.data(), ftf.size());
    put(L.fti, fti.data(), fti.size());
    put(L.mt, mt.data(), mt.size());
    if (hipMemcpy(mem, img.data(), img.size(), hipMemcpyHostToDevice) != hipSuccess) return MBP_ERR_HIP;
    // (the error-test bounds sit after the fields)
    if (hipMemcpy(P->d_sabs, P->sabs.data(), P->sabs.size() * sizeof(double), hipMemcpyHostToDevice) !=
        hipSuccess)
        return MBP_ERR_HIP;
    if (ext_pinned) {
        P->host_pinned = ext_pinned;
        P->owns_pinned = false;
        return MBP_OK;
    }
    void* hp = nullptr;
    if (hipHostMalloc(&hp, 4096, hipHostMallocDefault) != hipSuccess) return MBP_ERR_NOMEM;
    P->host_pinned = hp;
    P->owns_pinned = true;
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
    if (P->dmem && P->owns_mem) (void)hipFree(P->dmem);
    if (P->host_pinned && P->owns_pinned) (void)hipHostFree(P->host_pinned);
    P->dmem = nullptr;
    P->host_pinned = nullptr;
}

// ---------------------------------------------------------------------------
// Solve stages.  Algorithm 1 as a sequence of stream-ordered stages so that
// the single solve and the batched form share them: prologue (forward
// transform, compatibility, norms), cycles (convergence test, then one
// V-cycle of every mode still active; the device keeps the active list and
// the cycle count), epilogue (gauge, inverse transform).
// ---------------------------------------------------------------------------

namespace {
// layout of the plan's pinned readback buffer
constexpr int kPinScal = 0;     // doubles 0..7: d_scal
constexpr int kPinSum = 8;      // double: singular-plane area sum
constexpr int kPinInts = 32;    // ints (byte offset 256): flag[0..3], nact
constexpr int kPinSlots = 64;   // doubles from byte 512: state slots of the pipelined loop
constexpr int kSlotDoubles = 8; //   each scal[0..1], then ints flag[0..3], nact
constexpr int kSlots = 3;
}  // namespace

void ctx_init(SolveCtx& c, mbp_plan* P, const double* rhs, double* p, double rtol, int flags) {
    c = SolveCtx{};
    c.P = P;
    c.rhs = rhs;
    c.p = p;
    c.rtol2 = rtol * rtol;
    const double etol = P->opt.etol == 0.0 ? 10.0 * rtol : P->opt.etol;
    c.etol2 = etol < 0.0 ? -1.0 : etol * etol;
    c.flags = flags;
    c.mixed = P->opt.precision == MBP_MIXED;
    c.retire = (flags & MBP_RETIRE) != 0;
    c.warm = (flags & MBP_WARM_START) != 0;
    c.full_lds = !c.mixed && P->lds_level == 0;
    c.nitems = P->g.nz;
}

static double* pin_d(const mbp_plan* P) { return static_cast<double*>(P->host_pinned); }
static int* pin_i(const mbp_plan* P) { return reinterpret_cast<int*>(pin_d(P) + kPinInts); }

void ctx_prologue(SolveCtx& c, hipStream_t s) {
    mbp_plan* P = c.P;
    const int nz = P->g.nz;
    launch_fill_int(P->d_flag, 4, 0, s);
    launch_forward(P, c.rhs, P->fhat, P->d_flag, s);
    if (P->g.singular) {
        if (c.flags & MBP_PROJECT_RHS) launch_singular_fix(P, P->fhat, P->d_scal + 4, s);
        else launch_area_dot(P, P->fhat, P->d_scal + 4, s);
    }
    launch_plane_norm(P, P->fhat, P->d_fnorm, s);
    if (c.warm) launch_forward(P, c.p, P->phat, nullptr, s);
    else if (!c.lazy_zero) launch_zero(P->phat, size_t(nz) * P->plane0, s);
    launch_reset_active(P, s);
    (void)hipMemcpyAsync(pin_i(P), P->d_flag, 4 * sizeof(int), hipMemcpyDeviceToHost, s);
    (void)hipMemcpyAsync(pin_d(P) + kPinSum, P->d_scal + 4, sizeof(double), hipMemcpyDeviceToHost, s);
}

void ctx_check(SolveCtx& c) {
    mbp_plan* P = c.P;
    const int nz = P->g.nz;
    if (pin_i(P)[0]) c.status = MBP_ERR_NONFINITE;
    if (c.status == MBP_OK && P->g.singular) {
        const double mean_q0 = pin_d(P)[kPinSum] / P->area_sum;  // area-weighted mean of fhat_0
        c.removed = mean_q0 / std::sqrt(double(nz));               // volume-weighted mean of f
        if (!(c.flags & MBP_PROJECT_RHS)) {
            // compatible if the mean is at rounding level of the plane's rms
            double fn0 = 0.0;
            (void)hipMemcpy(&fn0, P->d_fnorm, sizeof(double), hipMemcpyDeviceToHost);
            const double rms = std::sqrt(fn0 / double(P->plane0));
            if (std::fabs(mean_q0) > 1e-12 * (rms + 1e-300)) c.status = MBP_ERR_INCOMPATIBLE;
            c.removed = 0.0;
        }
    }
    if (c.status != MBP_OK) c.done = true;
}

// Convergence test of the current iterate (Sec. 3's per-mode systems each
// stop on their own when retiring).
void ctx_test(SolveCtx& c, hipStream_t s, double* state_out) {
    mbp_plan* P = c.P;
    const bool zero = c.cycles == 0 && !c.warm;  // p = 0: the residual is f itself
    if (c.mixed)
        launch_residual_to32(P, P->phat, P->fhat, P->f32[0], fp32_guess_to_zero(P), P->d_rnorm, P->d_act, P->d_nact,
                             c.nitems, s, zero);
    else if (zero)
        launch_norm_from_rhs(P, c.nitems, s);
    else if (c.fused_parts > 0)
        launch_finish(P, c.fused_parts, P->d_rnorm, P->d_act, P->d_nact, c.nitems, s);
    else
        launch_residual_norm(P, P->phat, P->fhat, P->d_rnorm, P->d_act, P->d_nact, c.nitems, s);
    launch_update_active(P, c.rtol2, c.etol2, c.retire ? 1 : 0, P->opt.max_cycles, s, state_out);
}

void ctx_vcycle(SolveCtx& c, hipStream_t s) {
    mbp_plan* P = c.P;
    const bool zero = c.cycles == 0 && !c.warm;
    if (c.mixed) {
        // refinement step: the FP32 correction equation is solved by `inner`
        // V-cycles from zero, then the correction is added in FP64
        for (int k = 0; k < P->opt.inner; ++k)
            launch_vcycle<float>(P, P->p32[0], P->p32B[0], P->f32[0], P->d_act, P->d_nact, c.nitems, false,
                                 k == 0, s);
        launch_add_correction(P, P->phat, P->p32[0], P->d_act, P->d_nact, c.nitems, s, zero);
    } else {
        c.fused_parts = launch_vcycle<double>(P, P->phat, P->phatB, P->fhat, P->d_act, P->d_nact, c.nitems,
                                              true, zero, s);
    }
    ++c.cycles;
}

void ctx_state_readback(SolveCtx& c, hipStream_t s) {
    mbp_plan* P = c.P;
    (void)hipMemcpyAsync(pin_d(P) + kPinScal, P->d_scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
    (void)hipMemcpyAsync(pin_i(P), P->d_flag, 4 * sizeof(int), hipMemcpyDeviceToHost, s);
    (void)hipMemcpyAsync(pin_i(P) + 4, P->d_nact, sizeof(int), hipMemcpyDeviceToHost, s);
}

// After the readback synchronised: stop when every mode retired (retiring
// form) or every mode passed (lockstep), or when the cycle budget ran out.
// hi: flag[0..3], nact; scal1: the lockstep count of unconverged modes.
static void state_apply(SolveCtx& c, const int* hi, double scal1) {
    const bool hitmax = hi[2] != 0;
    bool converged;
    if (c.retire) {
        c.nitems = hi[4];
        converged = c.nitems == 0 && !hitmax;
    } else {
        converged = scal1 == 0.0;
    }
    if (converged) {
        c.done = true;
    } else if (hitmax) {
        c.status = MBP_ERR_NOT_CONVERGED;
        c.done = true;
    }
}

void ctx_state_apply(SolveCtx& c) { state_apply(c, pin_i(c.P), pin_d(c.P)[kPinScal + 1]); }

void ctx_epilogue(SolveCtx& c, hipStream_t s) {
    mbp_plan* P = c.P;
    if (c.status == MBP_OK || c.status == MBP_ERR_NOT_CONVERGED) {
        if (c.lazy_zero) launch_zero_unrelaxed(P, P->phat, s);
        if (P->g.singular) launch_singular_fix(P, P->phat, P->d_scal + 5, s);
        launch_inverse(P, P->phat, c.p, s);
    }
}

// Host-side result record; synchronises the stream.
int ctx_info(SolveCtx& c, hipStream_t s, mbp_solve_info* info) {
    mbp_plan* P = c.P;
    const int nz = P->g.nz;
    std::vector<int> cyc(nz, 0);
    std::vector<double> rn(nz, 0.0), fn(nz, 0.0);
    (void)hipMemcpyAsync(cyc.data(), P->d_cyc, nz * sizeof(int), hipMemcpyDeviceToHost, s);
    (void)hipMemcpyAsync(rn.data(), P->d_rnorm, nz * sizeof(double), hipMemcpyDeviceToHost, s);
    (void)hipMemcpyAsync(fn.data(), P->d_fnorm, nz * sizeof(double), hipMemcpyDeviceToHost, s);
    if (hipStreamSynchronize(s) != hipSuccess) return MBP_ERR_HIP;
    if (hipGetLastError() != hipSuccess) return MBP_ERR_HIP;
    double maxratio = 0.0;
    int cycles = 0;
    for (int q = 0; q < nz; ++q) {
        maxratio = std::max(maxratio, fn[q] > 0 ? rn[q] / fn[q] : (rn[q] > 0 ? 1e300 : 0.0));
        cycles = std::max(cycles, cyc[q]);
    }
    if (c.status == MBP_OK && c.full_lds && maxratio > c.rtol2) c.status = MBP_ERR_NOT_CONVERGED;
    if (info) {
        info->status = c.status;
        info->cycles = cycles;
        info->rel_residual = std::sqrt(maxratio);
        info->removed_mean = c.status == MBP_ERR_NONFINITE ? 0.0 : c.removed;
        if (info->cycles_per_mode) std::memcpy(info->cycles_per_mode, cyc.data(), nz * sizeof(int));
    }
    return MBP_OK;
}

// Algorithm 1 for one problem: forward transform, per-mode multigrid to the
// tolerance, inverse transform.  Host-driven: the convergence state is read
// back once per cycle (the batched form replays captured cycles instead).
int solve_one(mbp_plan* P, const double* rhs, double* p, double rtol, int flags, hipStream_t s,
              mbp_solve_info* info) {
    SolveCtx c;
    ctx_init(c, P, rhs, p, rtol, flags);
    // the retiring solve whose first step reads no iterate skips the up-front
    // zero fill of the modal solution (one write of the whole field)
    // (mixed: the first refinement step takes r = f and writes p = e)
    c.lazy_zero = c.retire && !c.warm && !c.full_lds && (c.mixed || vcycle_zero_start_reads_none(P));
    hipEvent_t ev[4];
    for (auto& e : ev) (void)hipEventCreate(&e);
    (void)hipEventRecord(ev[0], s);
    ctx_prologue(c, s);
    (void)hipEventRecord(ev[1], s);
    int st = MBP_OK;
    if (hipStreamSynchronize(s) != hipSuccess) st = MBP_ERR_HIP;
    if (st == MBP_OK) {
        ctx_check(c);
        if (!c.done && c.full_lds) {
            launch_lds_full(P, P->phat, P->fhat, P->d_act, P->d_nact, P->g.nz, P->opt.max_cycles, c.rtol2,
                            c.etol2, P->d_cyc, P->d_rnorm, P->d_fnorm, s);
        } else if (c.retire) {
            // Pipelined: the next V-cycle and test are queued before the host
            // reads the state of the previous test, so the device never waits
            // for the host.  Once every mode has retired the queued work runs
            // on an empty active list (no-op launches).
            double* slots = pin_d(P) + kPinSlots;
            double* dslots = nullptr;
            if (hipHostGetDevicePointer(reinterpret_cast<void**>(&dslots), slots, 0) != hipSuccess) {
                st = MBP_ERR_HIP;
            } else {
                hipEvent_t sev[kSlots];
                for (auto& e : sev) (void)hipEventCreateWithFlags(&e, hipEventDisableTiming);
                auto test = [&](int k) {
                    ctx_test(c, s, dslots + (k % kSlots) * kSlotDoubles);
                    (void)hipEventRecord(sev[k % kSlots], s);
                };
                test(0);
                for (int k = 0;; ++k) {
                    ctx_vcycle(c, s);
                    test(k + 1);
                    if (hipEventSynchronize(sev[k % kSlots]) != hipSuccess) {
                        st = MBP_ERR_HIP;
                        break;
                    }
                    const double* sl = slots + (k % kSlots) * kSlotDoubles;
                    state_apply(c, reinterpret_cast<const int*>(sl + 2), sl[1]);
                    if (c.done) break;
                }
                for (auto& e : sev) (void)hipEventDestroy(e);
            }
        } else {
            while (!c.done) {
                ctx_test(c, s);
                ctx_state_readback(c, s);
                if (hipStreamSynchronize(s) != hipSuccess) {
                    st = MBP_ERR_HIP;
                    break;
                }
                ctx_state_apply(c);
                if (c.done) break;
                ctx_vcycle(c, s);
            }
        }
    }
    (void)hipEventRecord(ev[2], s);
    if (st == MBP_OK) ctx_epilogue(c, s);
    (void)hipEventRecord(ev[3], s);
    if (st == MBP_OK) st = ctx_info(c, s, info);
    if (st == MBP_OK && info) {
        float t[3] = {0, 0, 0}, tt = 0;
        (void)hipEventElapsedTime(&t[0], ev[0], ev[1]);
        (void)hipEventElapsedTime(&t[1], ev[1], ev[2]);
        (void)hipEventElapsedTime(&t[2], ev[2], ev[3]);
        (void)hipEventElapsedTime(&tt, ev[0], ev[3]);
        info->t_ms[0] = t[0];
        info->t_ms[1] = t[1];
        info->t_ms[2] = t[2];
        info->t_ms[3] = tt;
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    return st != MBP_OK ? st : c.status;
}

}  // namespace mbp
