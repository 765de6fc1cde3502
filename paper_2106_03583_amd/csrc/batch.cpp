// Batched solves: many independent problems (each with all of its modes)
// driven together.  After the prologue (and, unless the grouped form runs,
// one eager cycle), the cycles of every unfinished problem are captured into
// one HIP graph and replayed chunk by chunk: inside a replay the device runs
// the convergence test and retires converged modes (and so finished
// problems, whose kernels then exit at once); the host reads the active
// counts after each replay and re-captures when the set has shrunk enough to
// pay off.  Two graph shapes: the grouped form (mixed precision, strip
// levels only) launches each stage of the refinement step once for all
// problems; otherwise each problem's kernels form one branch per stream.
// The number of streams and the cycles per replay come from a small online
// autotuner, cached per batch signature; streams and events are pooled.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "internal.h"

namespace mbp {

namespace {

struct BatchTune {
    int streams = 4;
    int chunk = 4;
    bool grouped = false;  // every replay of the set's last batch ran in the grouped form
};

std::mutex g_tune_mu;
std::map<uint64_t, BatchTune> g_tune;

uint64_t mix(uint64_t h, uint64_t v) {
    h ^= v + 0x9e3779b97f4a7c15ULL + (h << 6) + (h >> 2);
    return h;
}

uint64_t batch_signature(mbp_plan* const* plans, int count) {
    uint64_t h = 1469598103934665603ULL;
    for (int i = 0; i < count; ++i) {
        h = mix(h, uint64_t(plans[i]->ncells));
        h = mix(h, uint64_t(plans[i]->g.nz));
        h = mix(h, uint64_t(plans[i]->opt.precision));
    }
    return h;
}

constexpr int kMaxStreams = 8;

struct Graph {
    hipGraph_t g = nullptr;
    hipGraphExec_t e = nullptr;
    std::vector<int> members;
    long long modes = 0;  // active modes captured (grid sizes)
    void reset() {
        if (e) (void)hipGraphExecDestroy(e);
        if (g) (void)hipGraphDestroy(g);
        e = nullptr;
        g = nullptr;
        members.clear();
        modes = 0;
    }
};

// Streams and events of one batch call, kept for later calls on the same
// device (creating them costs about as much as a small problem's cycle).
struct StreamSet {
    int dev = -1;
    hipStream_t st[kMaxStreams] = {};
    hipEvent_t ev_join[kMaxStreams] = {};
    hipEvent_t ev_fork = nullptr, t0 = nullptr, t1 = nullptr;
};
std::mutex g_pool_mu;
std::vector<StreamSet*> g_pool;

StreamSet* acquire_streams() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        for (size_t i = 0; i < g_pool.size(); ++i)
            if (g_pool[i]->dev == dev) {
                StreamSet* p = g_pool[i];
                g_pool.erase(g_pool.begin() + long(i));
                return p;
            }
    }
    StreamSet* p = new StreamSet;
    p->dev = dev;
    bool ok = true;
    for (int k = 0; k < kMaxStreams; ++k) {
        ok = ok && hipStreamCreateWithFlags(&p->st[k], hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&p->ev_join[k], hipEventDisableTiming) == hipSuccess;
    }
    ok = ok && hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreate(&p->t0) == hipSuccess && hipEventCreate(&p->t1) == hipSuccess;
    if (!ok) {
        for (int k = 0; k < kMaxStreams; ++k) {
            if (p->st[k]) (void)hipStreamDestroy(p->st[k]);
            if (p->ev_join[k]) (void)hipEventDestroy(p->ev_join[k]);
        }
        if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
        if (p->t0) (void)hipEventDestroy(p->t0);
        if (p->t1) (void)hipEventDestroy(p->t1);
        delete p;
        return nullptr;
    }
    return p;
}

void release_streams(StreamSet* p) {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    g_pool.push_back(p);
}

}  // namespace

int solve_batch(mbp_plan* const* plans, const double* const* rhs, double* const* p, int count,
                double rtol, int flags, hipStream_t s, mbp_solve_info* infos) {
    std::vector<SolveCtx> cx(count);
    for (int i = 0; i < count; ++i)
        ctx_init(cx[i], plans[i], rhs[i], p[i], rtol, flags | plans[i]->opt.flags | MBP_RETIRE);

    const uint64_t sig = batch_signature(plans, count);
    BatchTune tune;
    bool have = false;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(sig);
        if (it != g_tune.end()) {
            tune = it->second;
            have = true;
        }
    }
    std::vector<BatchTune> trials;
    if ((flags & MBP_AUTOTUNE) && !have)
        trials = {{4, 4}, {1, 4}, {8, 4}, {2, 4}, {4, 2}, {4, 8}};

    // streams: [0] is the capture origin; all of them are forked from s
    StreamSet* ss = acquire_streams();
    if (!ss) return MBP_ERR_HIP;
    hipStream_t* st = ss->st;
    hipEvent_t* ev_join = ss->ev_join;
    hipEvent_t ev_fork = ss->ev_fork, t0 = ss->t0, t1 = ss->t1;
    auto fork = [&](hipStream_t from, int S) {
        (void)hipEventRecord(ev_fork, from);
        for (int k = 0; k < S; ++k)
            if (st[k] != from) (void)hipStreamWaitEvent(st[k], ev_fork, 0);
    };
    auto join = [&](hipStream_t to, int S) {
        for (int k = 0; k < S; ++k) {
            if (st[k] == to) continue;
            (void)hipEventRecord(ev_join[k], st[k]);
            (void)hipStreamWaitEvent(to, ev_join[k], 0);
        }
    };
    int status = MBP_OK;
    auto fail = [&](int e) {
        if (status == MBP_OK) status = e;
    };

    // prologue of every problem, then the checks that need the host
    int S = std::min(std::max(1, tune.streams), std::min(count, kMaxStreams));
    fork(s, S);
    for (int i = 0; i < count; ++i) ctx_prologue(cx[i], st[i % S]);
    join(s, S);
    if (hipStreamSynchronize(s) != hipSuccess) fail(MBP_ERR_HIP);
    for (int i = 0; i < count && status == MBP_OK; ++i) ctx_check(cx[i]);

    // problems whose whole hierarchy fits in LDS: one launch each; the
    // others run their first cycle (from zero) eagerly, unless they all take
    // the grouped form, whose captured cycles do not depend on the iterate
    bool all_grouped = true;
    int inner0 = -1;
    for (int i = 0; i < count; ++i) {
        const SolveCtx& c = cx[i];
        if (c.done || c.full_lds) continue;
        if (inner0 < 0) inner0 = c.P->opt.inner;
        all_grouped = all_grouped && group_ok(c) && c.P->opt.inner == inner0;
    }
    if (status == MBP_OK) {
        fork(s, S);
        for (int i = 0; i < count; ++i) {
            SolveCtx& c = cx[i];
            if (c.done) continue;
            if (c.full_lds) {
                mbp_plan* P = c.P;
                launch_lds_full(P, P->phat, P->fhat, P->d_act, P->d_nact, P->g.nz, P->opt.max_cycles, c.rtol2,
                                c.etol2, P->d_cyc, P->d_rnorm, P->d_fnorm, st[i % S]);
                c.done = true;
                continue;
            }
            if (all_grouped) continue;
            ctx_test(c, st[i % S]);
            ctx_vcycle(c, st[i % S]);
        }
        join(s, S);
    }

    // captured cycles, replayed until every problem is done
    Graph G;
    int captures = 0, grouped_captures = 0;
    void* table = nullptr;  // stage tables of the grouped form
    size_t table_bytes = 0;
    size_t trial = 0;
    BatchTune cur = trials.empty() ? tune : trials[0];
    double best_cost = 1e300;
    BatchTune best = cur;
    while (status == MBP_OK) {
        std::vector<int> act;
        long long modes = 0;
        for (int i = 0; i < count; ++i)
            if (!cx[i].done) {
                act.push_back(i);
                modes += cx[i].nitems;
            }
        if (act.empty()) break;
        const bool retune = trial < trials.size();
        if (retune) cur = trials[trial];
        const int Sc = std::min(std::max(1, cur.streams), std::min(int(act.size()), kMaxStreams));
        bool recapture = G.e == nullptr || retune || act.size() < G.members.size() ||
                         modes * 4 < G.modes * 3;
        if (recapture) {
            G.reset();
            // grouped form: every unfinished problem is a mixed strip V-cycle
            // with the same inner cycle count
            bool grouped = true;
            for (int i : act)
                grouped = grouped && group_ok(cx[i]) && cx[i].P->opt.inner == cx[act[0]].P->opt.inner;
            std::vector<GStage> stages;
            if (grouped) {
                std::vector<SolveCtx*> cs;
                int maxL = 0;
                for (int i : act) {
                    cs.push_back(&cx[i]);
                    maxL = std::max(maxL, cx[i].P->lds_level32);
                }
                GroupBlob gb;
                stages.push_back(group_res32(gb, cs));
                stages.push_back(group_finish(gb, cs));
                stages.push_back(group_update(gb, cs));
                for (int k = 0; k < cx[act[0]].P->opt.inner; ++k) {
                    for (int l = 0; l < maxL; ++l) stages.push_back(group_march32(gb, cs, l, false, k == 0));
                    stages.push_back(group_lds32(gb, cs));
                    for (int l = maxL - 1; l >= 0; --l) stages.push_back(group_march32(gb, cs, l, true, false));
                }
                stages.push_back(group_addcorr(gb, cs));
                if (gb.host.size() > table_bytes) {
                    if (table) (void)hipFree(table);
                    table = nullptr;
                    table_bytes = 0;
                    if (hipMalloc(&table, gb.host.size()) != hipSuccess) {
                        fail(MBP_ERR_NOMEM);
                        break;
                    }
                    table_bytes = gb.host.size();
                }
                if (hipMemcpy(table, gb.host.data(), gb.host.size(), hipMemcpyHostToDevice) != hipSuccess) {
                    fail(MBP_ERR_HIP);
                    break;
                }
            }
            if (hipStreamBeginCapture(st[0], hipStreamCaptureModeThreadLocal) != hipSuccess) {
                fail(MBP_ERR_HIP);
                break;
            }
            ++captures;
            if (grouped) {
                ++grouped_captures;
                const unsigned char* dev = static_cast<const unsigned char*>(table);
                for (int it = 0; it < cur.chunk; ++it)
                    for (const GStage& g : stages) {
                        if (g.kind == G_PRE32 || g.kind == G_POST32) group_launch_march(g, dev, st[0]);
                        else group_launch_mg(g, dev, st[0]);
                    }
                for (int i : act) cx[i].cycles += cur.chunk;
            } else {
                fork(st[0], Sc);
                for (int it = 0; it < cur.chunk; ++it)
                    for (size_t a = 0; a < act.size(); ++a) {
                        SolveCtx& c = cx[act[a]];
                        ctx_test(c, st[a % Sc]);
                        ctx_vcycle(c, st[a % Sc]);
                    }
                join(st[0], Sc);
            }
            if (hipStreamEndCapture(st[0], &G.g) != hipSuccess ||
                hipGraphInstantiate(&G.e, G.g, nullptr, nullptr, 0) != hipSuccess) {
                (void)hipGetLastError();
                G.reset();
                fail(MBP_ERR_HIP);
                break;
            }
            G.members = act;
            G.modes = modes;
        }
        (void)hipEventRecord(t0, s);
        if (hipGraphLaunch(G.e, s) != hipSuccess) {
            fail(MBP_ERR_HIP);
            break;
        }
        (void)hipEventRecord(t1, s);
        for (int i : act) ctx_state_readback(cx[i], s);
        if (hipStreamSynchronize(s) != hipSuccess) {
            fail(MBP_ERR_HIP);
            break;
        }
        if (retune) {
            // cost per active mode-cell and cycle of this replay
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, t0, t1);
            double work = 0.0;
            for (int i : act) work += double(cx[i].nitems) * double(cx[i].P->plane0);
            const double cost = ms / std::max(1.0, work * cur.chunk);
            if (cost < best_cost) {
                best_cost = cost;
                best = cur;
            }
            if (++trial == trials.size()) {
                std::lock_guard<std::mutex> lk(g_tune_mu);
                g_tune[sig] = best;
                tune = best;
                cur = best;
                G.reset();
            }
        }
        for (int i : act) ctx_state_apply(cx[i]);
    }
    G.reset();
    if (table) (void)hipFree(table);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        // the batch finished before every candidate ran: keep the best seen
        if (trial > 0 && trial < trials.size()) g_tune[sig] = best;
        auto it = g_tune.find(sig);
        if (it != g_tune.end()) it->second.grouped = captures > 0 && grouped_captures == captures;
    }

    // epilogue and results
    fork(s, S);
    for (int i = 0; i < count; ++i) ctx_epilogue(cx[i], st[i % S]);
    join(s, S);
    for (int i = 0; i < count; ++i) {
        const int r = ctx_info(cx[i], s, infos ? &infos[i] : nullptr);
        if (r != MBP_OK) fail(r);
        else if (cx[i].status != MBP_OK) fail(cx[i].status);
    }
    release_streams(ss);
    return status;
}

// Schedule chosen for a batch signature (for reports and tests).
int batch_tuning(mbp_plan* const* plans, int count, int* streams, int* chunk) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(batch_signature(plans, count));
    if (it == g_tune.end()) return MBP_PENDING;
    *streams = it->second.grouped ? 0 : it->second.streams;
    *chunk = it->second.chunk;
    return MBP_OK;
}

}  // namespace mbp
