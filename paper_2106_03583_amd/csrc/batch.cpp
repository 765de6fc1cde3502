// Batched solves (placeholder: sequential until the graph-replayed form lands).
#include "internal.h"

namespace mbp {

int solve_batch(mbp_plan* const* plans, const double* const* rhs, double* const* p, int count,
                double rtol, int flags, hipStream_t s, mbp_solve_info* infos) {
    int first = MBP_OK;
    for (int i = 0; i < count; ++i) {
        int st = solve_one(plans[i], rhs[i], p[i], rtol, flags | plans[i]->opt.flags | MBP_RETIRE, s,
                           infos ? &infos[i] : nullptr);
        if (st != MBP_OK && first == MBP_OK) first = st;
    }
    return first;
}

}  // namespace mbp

extern "C" {
int mbp_server_create(size_t, int, const mbp_options*, mbp_server**) { return MBP_ERR_INVALID; }
int mbp_server_submit(mbp_server*, const mbp_block_desc*, int, const mbp_synth_desc*, const double*,
                      double*, double, int, uint64_t*) { return MBP_ERR_INVALID; }
int mbp_server_poll(mbp_server*, uint64_t, mbp_solve_info*, double*) { return MBP_ERR_INVALID; }
int mbp_server_wait(mbp_server*, uint64_t, mbp_solve_info*, double*) { return MBP_ERR_INVALID; }
void mbp_server_destroy(mbp_server*) {}
}
