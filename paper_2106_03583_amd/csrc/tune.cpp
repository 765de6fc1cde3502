// Per-plan autotuner.  Times a few V-cycles of every mode for candidate
// schedules on the plan's own workspace and keeps the fastest:
//   * the number of workgroups a strip-form launch aims at (which sets how
//     many modes each workgroup runs in turn), and
//   * per fused level, the pre-smoothing form: LDS strip tiles or the
//     register march.
// The schedule only changes how the same arithmetic is distributed; every
// candidate runs the same red-black sweeps.
#include <algorithm>
#include <cstring>
#include <vector>

#include "internal.h"

namespace mbp {

void launch_reset_active(const mbp_plan* P, hipStream_t s);

namespace {

// Mean time of `reps` V-cycles over all modes (after one untimed cycle).
float time_cycles(SolveCtx& c, hipStream_t s, hipEvent_t a, hipEvent_t b, int reps) {
    mbp_plan* P = c.P;
    launch_reset_active(P, s);
    c.nitems = P->g.nz;
    ctx_vcycle(c, s);
    (void)hipEventRecord(a, s);
    for (int i = 0; i < reps; ++i) ctx_vcycle(c, s);
    (void)hipEventRecord(b, s);
    if (hipEventSynchronize(b) != hipSuccess) return 1e30f;
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, a, b);
    return ms / float(reps);
}

}  // namespace

int plan_autotune(mbp_plan* P, const double* rhs, hipStream_t s, mbp_tuning* out) {
    SolveCtx c;
    ctx_init(c, P, rhs, nullptr, 1e-10, MBP_PROJECT_RHS);
    ctx_prologue(c, s);
    if (hipStreamSynchronize(s) != hipSuccess) return MBP_ERR_HIP;
    ctx_check(c);
    if (c.status == MBP_ERR_NONFINITE) return MBP_ERR_NONFINITE;
    const int nlev = std::min(P->nlev, 16);
    if (out) {
        std::memset(out, 0, sizeof(*out));
        out->levels = nlev;
    }
    if (c.full_lds) {  // the whole solve runs in one LDS kernel: nothing to choose
        if (out) out->wg_target = P->wg_target;
        return MBP_OK;
    }
    // Fill every buffer a V-cycle reads before timing it: the test computes
    // the finest residual (and, for a mixed plan, its FP32 copy, the rhs of
    // the FP32 V-cycles), so no candidate runs on uninitialised memory.
    ctx_test(c, s);
    c.cycles = 1;  // from here on the iterate is not zero
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    const int reps = 3;
    std::fill(P->use_rmarch.begin(), P->use_rmarch.end(), 0);
    P->wg_target = 256 * 3;
    const float t_default = time_cycles(c, s, a, b, reps);
    float best = t_default;
    // workgroups per launch (sets the modes each workgroup runs in turn)
    for (int target : {256 * 1, 256 * 12}) {
        const int keep = P->wg_target;
        P->wg_target = target;
        const float t = time_cycles(c, s, a, b, reps);
        if (t < 0.98f * best) best = t;
        else P->wg_target = keep;
    }
    // pre-smoothing form per fused level (finest first)
    for (int l = 0; l < P->nlev; ++l) {
        if (!P->march_ok[l] || P->rtile_cnt[l] == 0) continue;
        P->use_rmarch[l] = 1;
        const float t = time_cycles(c, s, a, b, reps);
        if (t < 0.98f * best) best = t;
        else P->use_rmarch[l] = 0;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (out) {
        out->wg_target = P->wg_target;
        for (int l = 0; l < nlev; ++l) out->form[l] = P->use_rmarch[l];
        out->ms_default = t_default;
        out->ms_tuned = best;
    }
    return hipGetLastError() == hipSuccess ? MBP_OK : MBP_ERR_HIP;
}

}  // namespace mbp
