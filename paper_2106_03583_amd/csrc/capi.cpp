// The extern "C" surface declared in include/mbp.h.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "internal.h"

using namespace mbp;

namespace mbp {
void launch_fill_int(int* p, int n, int v, hipStream_t s);
int solve_batch(mbp_plan* const* plans, const double* const* rhs, double* const* p, int count,
                double rtol, int flags, hipStream_t s, mbp_solve_info* infos);
int batch_tuning(mbp_plan* const* plans, int count, int* streams, int* chunk);
}

extern "C" {

const char* mbp_status_string(int status) {
    switch (status) {
        case MBP_OK: return "ok";
        case MBP_PENDING: return "pending";
        case MBP_ERR_INVALID: return "invalid argument or problem description";
        case MBP_ERR_NOMEM: return "out of memory";
        case MBP_ERR_HIP: return "HIP runtime error";
        case MBP_ERR_NOT_CONVERGED: return "not converged within max_cycles";
        case MBP_ERR_NONFINITE: return "rhs holds NaN or Inf";
        case MBP_ERR_INCOMPATIBLE: return "singular problem with an incompatible rhs";
        case MBP_ERR_BUSY: return "plan busy";
        case MBP_ERR_TOO_LARGE: return "request larger than the server budget";
        case MBP_ERR_NO_DEVICE: return "no HIP device";
        default: return "unknown status";
    }
}

int mbp_version(void) { return 200; }

int mbp_grid_tanh(int n, double lmin, double lmax, int type, double factor, double* faces_out) {
    return grid_tanh(n, lmin, lmax, type, factor, faces_out);
}

int mbp_plan_check(const mbp_block_desc* blocks, int nblocks, const mbp_synth_desc* z,
                   const mbp_options* opt, mbp_plan_summary* out) {
    mbp_plan* P = new (std::nothrow) mbp_plan();
    if (!P) return MBP_ERR_NOMEM;
    std::string err;
    int st = build_plan_host(blocks, nblocks, z, opt, P, &err);
    if (st == MBP_OK && out) {
        std::memset(out, 0, sizeof(*out));
        out->ncells = P->ncells;
        out->nlevels = P->nlev;
        out->coarse_cells = P->coarse_n;
        out->singular = P->g.singular ? 1 : 0;
        out->nblocks = P->g.nb;
        out->workspace_bytes = int64_t(plan_device_bytes(P));
        for (int b = 0; b < P->g.nb && b < 64; ++b)
            for (int f = 0; f < 4; ++f) out->nbr[b][f] = P->g.nbr[b][f];
    }
    delete P;
    return st;
}

int mbp_plan_create(const mbp_block_desc* blocks, int nblocks, const mbp_synth_desc* z,
                    const mbp_options* opt, mbp_plan** out) {
    if (!out) return MBP_ERR_INVALID;
    *out = nullptr;
    int dev = 0, count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
        (void)hipGetLastError();
        return MBP_ERR_NO_DEVICE;
    }
    if (hipGetDevice(&dev) != hipSuccess) return MBP_ERR_HIP;
    int lds = 65536;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        lds = 65536;
    mbp_plan* P = new (std::nothrow) mbp_plan();
    if (!P) return MBP_ERR_NOMEM;
    std::string err;
    int st = build_plan_host_limits(blocks, nblocks, z, opt, int64_t(lds), P, &err);
    if (st != MBP_OK) {
        delete P;
        return st;
    }
    P->device = dev;
    st = plan_device_init(P);
    if (st != MBP_OK) {
        plan_device_free(P);
        delete P;
        return st;
    }
    *out = P;
    return MBP_OK;
}

int mbp_plan_set_helmholtz(mbp_plan* plan, double alpha) {
    if (!plan || !(alpha >= 0.0) || !std::isfinite(alpha)) return MBP_ERR_INVALID;
    if (!plan->busy.claim()) return MBP_ERR_BUSY;
    plan->opt.helmholtz = alpha;
    plan_set_shifts(plan);
    const size_t nz = plan->shift.size();
    int st = MBP_OK;
    if (hipMemcpy(plan->d_shift, plan->shift.data(), nz * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(plan->d_sabs, plan->sabs.data(), nz * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        st = MBP_ERR_HIP;
    plan->busy.release();
    return st;
}

int mbp_plan_layout(const mbp_plan* plan, int64_t* block_offsets, size_t* workspace_bytes,
                    int* singular) {
    if (!plan) return MBP_ERR_INVALID;
    if (block_offsets)
        for (int b = 0; b <= plan->g.nb; ++b) block_offsets[b] = plan->block_off[b];
    if (workspace_bytes) *workspace_bytes = plan->dbytes;
    if (singular) *singular = plan->g.singular ? 1 : 0;
    return MBP_OK;
}

int mbp_solve(mbp_plan* plan, const double* rhs_dev, double* p_dev, double rtol, int flags,
              void* stream, mbp_solve_info* info) {
    if (!plan || !rhs_dev || !p_dev || !(rtol > 0.0) || rhs_dev == p_dev) return MBP_ERR_INVALID;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != plan->device) return MBP_ERR_INVALID;
    if (!plan->busy.claim()) return MBP_ERR_BUSY;
    int st = solve_one(plan, rhs_dev, p_dev, rtol, flags | plan->opt.flags,
                       static_cast<hipStream_t>(stream), info);
    plan->busy.release();
    return st;
}

int mbp_solve_batch(mbp_plan* const* plans, const double* const* rhs_dev, double* const* p_dev,
                    int count, double rtol, int flags, void* stream, mbp_solve_info* infos) {
    if (!plans || !rhs_dev || !p_dev || count < 1 || !(rtol > 0.0)) return MBP_ERR_INVALID;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return MBP_ERR_HIP;
    for (int i = 0; i < count; ++i) {
        if (!plans[i] || !rhs_dev[i] || !p_dev[i] || rhs_dev[i] == p_dev[i]) return MBP_ERR_INVALID;
        if (plans[i]->device != dev) return MBP_ERR_INVALID;
        for (int k = 0; k < i; ++k)
            if (plans[k] == plans[i]) return MBP_ERR_INVALID;
    }
    for (int i = 0; i < count; ++i)
        if (!plans[i]->busy.claim()) {
            for (int k = 0; k < i; ++k) plans[k]->busy.release();
            return MBP_ERR_BUSY;
        }
    int st = solve_batch(plans, rhs_dev, p_dev, count, rtol, flags, static_cast<hipStream_t>(stream),
                         infos);
    for (int i = 0; i < count; ++i) plans[i]->busy.release();
    return st;
}

int mbp_batch_schedule(mbp_plan* const* plans, int count, int* streams, int* cycles_per_replay) {
    if (!plans || count < 1 || !streams || !cycles_per_replay) return MBP_ERR_INVALID;
    for (int i = 0; i < count; ++i)
        if (!plans[i]) return MBP_ERR_INVALID;
    return batch_tuning(plans, count, streams, cycles_per_replay);
}

int mbp_forward_transform(mbp_plan* plan, const double* f_dev, double* fhat_dev, void* stream) {
    if (!plan || !f_dev || !fhat_dev) return MBP_ERR_INVALID;
    launch_forward(plan, f_dev, fhat_dev, nullptr, static_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? MBP_OK : MBP_ERR_HIP;
}

int mbp_inverse_transform(mbp_plan* plan, const double* phat_dev, double* p_dev, void* stream) {
    if (!plan || !phat_dev || !p_dev) return MBP_ERR_INVALID;
    launch_inverse(plan, phat_dev, p_dev, static_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? MBP_OK : MBP_ERR_HIP;
}

int mbp_apply_operator(mbp_plan* plan, const double* p_dev, double* out_dev, void* stream) {
    if (!plan || !p_dev || !out_dev || p_dev == out_dev) return MBP_ERR_INVALID;
    launch_apply3d(plan, p_dev, out_dev, static_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? MBP_OK : MBP_ERR_HIP;
}

int mbp_residual_norm(mbp_plan* plan, const double* rhs_dev, const double* p_dev, double rhs_shift,
                      double* out_dev, void* stream) {
    if (!plan || !rhs_dev || !p_dev || !out_dev) return MBP_ERR_INVALID;
    // the plan's partial-sum buffer holds 2 nz max(nparts, finest tiles) doubles
    if (resnorm_scratch_doubles(plan) >
        2 * size_t(plan->g.nz) * size_t(std::max(plan->nparts, plan->levels[0].ntiles)))
        return MBP_ERR_INVALID;
    if (!plan->busy.claim()) return MBP_ERR_BUSY;
    launch_resnorm3d(plan, rhs_dev, p_dev, rhs_shift, plan->d_part, out_dev, static_cast<hipStream_t>(stream));
    plan->busy.release();
    return hipGetLastError() == hipSuccess ? MBP_OK : MBP_ERR_HIP;
}

int mbp_velocity_layout(const mbp_plan* plan, int64_t* u_off, int64_t* v_off, int64_t* w_off) {
    if (!plan) return MBP_ERR_INVALID;
    velocity_offsets(plan, u_off, v_off, w_off);
    return MBP_OK;
}

int mbp_divergence(mbp_plan* plan, const double* u_dev, const double* v_dev, const double* w_dev, double scale,
                   double* out_dev, void* stream) {
    if (!plan || !u_dev || !v_dev || !w_dev || !out_dev) return MBP_ERR_INVALID;
    launch_divergence(plan, u_dev, v_dev, w_dev, scale, out_dev, static_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? MBP_OK : MBP_ERR_HIP;
}

int mbp_project(mbp_plan* plan, double* u_dev, double* v_dev, double* w_dev, double gamma_dt, double* phi_dev,
                double* rhs_work_dev, double rtol, int flags, void* stream, mbp_solve_info* info) {
    if (!plan || !u_dev || !v_dev || !w_dev || !phi_dev || !rhs_work_dev || !(gamma_dt > 0.0) ||
        !std::isfinite(gamma_dt) || !(rtol > 0.0) || phi_dev == rhs_work_dev)
        return MBP_ERR_INVALID;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != plan->device) return MBP_ERR_INVALID;
    if (!plan->busy.claim()) return MBP_ERR_BUSY;
    hipStream_t s = static_cast<hipStream_t>(stream);
    launch_divergence(plan, u_dev, v_dev, w_dev, 1.0 / gamma_dt, rhs_work_dev, s);
    int st = solve_one(plan, rhs_work_dev, phi_dev, rtol, flags | plan->opt.flags | MBP_PROJECT_RHS, s, info);
    if (st == MBP_OK || st == MBP_ERR_NOT_CONVERGED) launch_gradient_update(plan, phi_dev, gamma_dt, u_dev, v_dev, w_dev, s);
    plan->busy.release();
    if (hipGetLastError() != hipSuccess) return MBP_ERR_HIP;
    return st;
}

int mbp_modal_shift(const mbp_plan* plan, double* shift_host) {
    if (!plan || !shift_host) return MBP_ERR_INVALID;
    std::memcpy(shift_host, plan->shift.data(), plan->shift.size() * sizeof(double));
    return MBP_OK;
}

int mbp_plan_autotune(mbp_plan* plan, const double* rhs_dev, void* stream, mbp_tuning* out) {
    if (!plan || !rhs_dev) return MBP_ERR_INVALID;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != plan->device) return MBP_ERR_INVALID;
    if (!plan->busy.claim()) return MBP_ERR_BUSY;
    const int st = plan_autotune(plan, rhs_dev, static_cast<hipStream_t>(stream), out);
    plan->busy.release();
    return st;
}

int mbp_profile_enable(mbp_plan* plan, int enable) {
    if (!plan) return MBP_ERR_INVALID;
    plan->prof = enable != 0;
    plan->prof_used[0] = plan->prof_used[1] = 0;
    return MBP_OK;
}

int mbp_profile_read(mbp_plan* plan, mbp_profile_info* out) {
    if (!plan || !out) return MBP_ERR_INVALID;
    std::memset(out, 0, sizeof(*out));
    for (int c = 0; c < 2; ++c)
        for (size_t i = 0; i < plan->prof_used[c]; ++i) {
            hipEvent_t a = static_cast<hipEvent_t>(plan->prof_ev[c][i][0]);
            hipEvent_t b = static_cast<hipEvent_t>(plan->prof_ev[c][i][1]);
            if (hipEventSynchronize(b) != hipSuccess) return MBP_ERR_HIP;
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return MBP_ERR_HIP;
            out->launches[c] += 1;
            out->total_ms[c] += ms;
            out->cells[c] += plan->prof_cells[c][i];
        }
    return MBP_OK;
}

void mbp_plan_destroy(mbp_plan* plan) {
    if (!plan) return;
    plan_device_free(plan);
    delete plan;
}

}  // extern "C"
