// Serving loop: continuous batching of solve requests of any size and
// conditions.  A worker thread owns every HIP call: it admits waiting
// requests in arrival order as soon as a slot (stream) is free and the plan
// memory fits the budget (evicting idle cached plans, least recently used
// first), then advances every running request through the solve stages
// without blocking on any of them: each request issues a few cycles, records
// an event, and is looked at again when that event has completed.  Requests
// therefore overlap on the device, and one that arrives while others run
// starts at once when a slot and memory are free.
//
// The budget is one device allocation made at creation (the arena): plans
// are placed in it and their ranges returned on eviction, so admission never
// calls hipMalloc or hipFree (hipFree waits for the whole device, which
// would stall every running request).  The host part of a plan (validation,
// hierarchy, tables) is built in the submitting thread, so the worker only
// places the plan and uploads its tables in one copy; readbacks use pinned
// buffers owned by the slots.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

using namespace mbp;

namespace {

using Clock = std::chrono::steady_clock;

constexpr int kCyclesPerStep = 2;  // cycles issued between looks at a request

struct CachedPlan {
    std::string key;
    mbp_plan* plan = nullptr;
    size_t bytes = 0;
    size_t off = 0;  // range in the arena
    bool busy = false;
    uint64_t last_use = 0;
};

// First-fit allocator over the arena with coalescing free ranges.
class Arena {
  public:
    void init(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
    }
    // offset of a range of `bytes` (256-byte aligned), or SIZE_MAX
    size_t alloc(size_t bytes) {
        bytes = (bytes + 255) & ~size_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= bytes) {
                const size_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > bytes) free_[off + bytes] = len - bytes;
                return off;
            }
        return SIZE_MAX;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + 255) & ~size_t(255);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

  private:
    std::map<size_t, size_t> free_;
};

enum Stage { kQueued, kPrologue, kCycles, kEpilogue, kDone };

struct Request {
    uint64_t ticket = 0;
    std::string key;
    size_t bytes = 0;
    std::vector<mbp_block_desc> blocks;
    std::vector<std::vector<double>> faces;  // copies: the caller may free its arrays
    mbp_synth_desc z{};
    const double* rhs = nullptr;
    double* p = nullptr;
    double rtol = 1e-10;
    int flags = 0;
    Clock::time_point t_submit;
    // in flight
    CachedPlan* cp = nullptr;
    int slot = -1;
    Stage stage = kQueued;
    SolveCtx ctx;
    hipEvent_t ev = nullptr;
    std::unique_ptr<mbp_plan> host;  // host plan built at submission (none when cached)
    // result
    int status = MBP_OK;
    mbp_solve_info info{};
    std::vector<int32_t> cycles;  // per mode, handed out by poll / wait
    double latency_ms = 0.0;
};

// Descriptor bytes (blocks, faces, z, options): the cache key.
std::string describe(const mbp_block_desc* blocks, int nblocks, const mbp_synth_desc* z,
                     const mbp_options& opt) {
    std::string k;
    auto put = [&](const void* p, size_t n) { k.append(static_cast<const char*>(p), n); };
    put(&nblocks, sizeof(nblocks));
    for (int b = 0; b < nblocks; ++b) {
        const mbp_block_desc& d = blocks[b];
        put(d.lo, sizeof(d.lo));
        put(d.hi, sizeof(d.hi));
        put(d.bc, sizeof(d.bc));
        const int nx = d.hi[0] - d.lo[0] + 1, ny = d.hi[1] - d.lo[1] + 1;
        if (d.xf && nx > 0) put(d.xf, sizeof(double) * (nx + 1));
        if (d.yf && ny > 0) put(d.yf, sizeof(double) * (ny + 1));
    }
    put(&z->nz, sizeof(z->nz));
    put(&z->lz, sizeof(z->lz));
    put(&z->bc_lo, sizeof(z->bc_lo));
    put(&z->bc_hi, sizeof(z->bc_hi));
    put(&opt.precision, sizeof(opt.precision));
    put(&opt.nu1, sizeof(opt.nu1));
    put(&opt.nu2, sizeof(opt.nu2));
    put(&opt.max_cycles, sizeof(opt.max_cycles));
    put(&opt.etol, sizeof(opt.etol));
    put(&opt.inner, sizeof(opt.inner));
    put(&opt.march, sizeof(opt.march));
    put(&opt.smoother, sizeof(opt.smoother));
    put(&opt.helmholtz, sizeof(opt.helmholtz));
    return k;
}

}  // namespace

struct mbp_server {
    int device = 0;
    int lds_limit = 65536;
    size_t budget = 0;
    int slots = 1;
    mbp_options opt{};
    std::vector<hipStream_t> streams;
    std::vector<char> slot_busy;
    void* arena_mem = nullptr;      // the budget, allocated once
    Arena arena;
    void* pinned = nullptr;         // 4 KB readback buffer per slot

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> waiting;
    std::vector<Request*> running;
    std::map<uint64_t, Request*> finished;
    std::map<uint64_t, Request*> all;  // every live ticket
    std::vector<std::unique_ptr<CachedPlan>> cache;
    size_t resident = 0;
    uint64_t use_clock = 0;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;

    // ---- worker side (no lock held during HIP work) ----
    void evict(CachedPlan* victim) {
        plan_device_free(victim->plan);  // arena memory and slot buffers are not owned: nothing to free
        delete victim->plan;
        arena.release(victim->off, victim->bytes);
        resident -= victim->bytes;
        cache.erase(std::find_if(cache.begin(), cache.end(),
                                 [&](const std::unique_ptr<CachedPlan>& c) { return c.get() == victim; }));
    }

    CachedPlan* acquire_plan(Request* r, int slot) {
        void* pin = static_cast<unsigned char*>(pinned) + size_t(slot) * 4096;
        for (auto& c : cache)
            if (!c->busy && c->key == r->key) {
                c->busy = true;
                c->last_use = ++use_clock;
                c->plan->host_pinned = pin;
                return c.get();
            }
        // make room: drop idle plans, least recently used first, until a
        // contiguous range of the arena fits the plan
        size_t off;
        while ((off = arena.alloc(r->bytes)) == SIZE_MAX) {
            CachedPlan* victim = nullptr;
            for (auto& c : cache)
                if (!c->busy && (!victim || c->last_use < victim->last_use)) victim = c.get();
            if (!victim) return nullptr;  // waits for memory held by running requests
            evict(victim);
        }
        mbp_plan* P = r->host.release();
        P->device = device;
        int st = plan_device_init(P, static_cast<unsigned char*>(arena_mem) + off, r->bytes, pin);
        if (st != MBP_OK) {
            plan_device_free(P);
            delete P;
            arena.release(off, r->bytes);
            r->status = st;
            return nullptr;
        }
        auto c = std::make_unique<CachedPlan>();
        c->key = r->key;
        c->plan = P;
        c->bytes = r->bytes;
        c->off = off;
        c->busy = true;
        c->last_use = ++use_clock;
        resident += c->bytes;
        cache.push_back(std::move(c));
        return cache.back().get();
    }

    // Start (or move on) one request; returns true if it made progress.
    bool step(Request* r) {
        hipStream_t s = streams[r->slot];
        SolveCtx& c = r->ctx;
        switch (r->stage) {
            case kQueued:
                ctx_init(c, r->cp->plan, r->rhs, r->p, r->rtol, r->flags | opt.flags | MBP_RETIRE);
                ctx_prologue(c, s);
                (void)hipEventRecord(r->ev, s);
                r->stage = kPrologue;
                return true;
            case kPrologue:
            case kCycles: {
                const hipError_t q = hipEventQuery(r->ev);
                if (q == hipErrorNotReady) return false;
                if (q != hipSuccess) {
                    c.status = MBP_ERR_HIP;
                    c.done = true;
                } else if (r->stage == kPrologue) {
                    ctx_check(c);
                    if (!c.done && c.full_lds) {
                        mbp_plan* P = c.P;
                        launch_lds_full(P, P->phat, P->fhat, P->d_act, P->d_nact, P->g.nz, P->opt.max_cycles,
                                        c.rtol2, c.etol2, P->d_cyc, P->d_rnorm, P->d_fnorm, s);
                        c.done = true;
                    }
                } else {
                    ctx_state_apply(c);
                }
                if (c.done) {
                    ctx_epilogue(c, s);
                    (void)hipEventRecord(r->ev, s);
                    r->stage = kEpilogue;
                    return true;
                }
                for (int k = 0; k < kCyclesPerStep; ++k) {
                    ctx_test(c, s);
                    ctx_vcycle(c, s);
                }
                ctx_state_readback(c, s);
                (void)hipEventRecord(r->ev, s);
                r->stage = kCycles;
                return true;
            }
            case kEpilogue: {
                const hipError_t q = hipEventQuery(r->ev);
                if (q == hipErrorNotReady) return false;
                r->cycles.assign(size_t(c.P->g.nz), 0);
                r->info.cycles_per_mode = r->cycles.data();
                int st = q == hipSuccess ? ctx_info(c, s, &r->info) : MBP_ERR_HIP;
                r->info.cycles_per_mode = nullptr;
                r->status = st != MBP_OK ? st : c.status;
                r->info.status = r->status;
                r->latency_ms =
                    std::chrono::duration<double, std::milli>(Clock::now() - r->t_submit).count();
                r->stage = kDone;
                return true;
            }
            case kDone:
                return false;
        }
        return false;
    }

    void run() {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            if (stop && waiting.empty() && running.empty()) break;
            // admission, in arrival order
            while (!waiting.empty()) {
                int slot = -1;
                for (int k = 0; k < slots; ++k)
                    if (!slot_busy[k]) {
                        slot = k;
                        break;
                    }
                if (slot < 0) break;
                Request* r = waiting.front();
                lk.unlock();
                r->status = MBP_OK;
                CachedPlan* cp = acquire_plan(r, slot);
                lk.lock();
                if (!cp) {
                    if (r->status != MBP_OK) {  // the plan could not be built
                        waiting.pop_front();
                        r->info.status = r->status;
                        r->latency_ms =
                            std::chrono::duration<double, std::milli>(Clock::now() - r->t_submit).count();
                        r->stage = kDone;
                        finished[r->ticket] = r;
                        cv_done.notify_all();
                        continue;
                    }
                    break;  // waits for memory held by running requests
                }
                waiting.pop_front();
                r->cp = cp;
                r->slot = slot;
                slot_busy[slot] = 1;
                running.push_back(r);
            }
            // progress
            std::vector<Request*> run_now = running;
            lk.unlock();
            bool progressed = false;
            for (Request* r : run_now) progressed |= step(r);
            lk.lock();
            for (size_t i = 0; i < running.size();) {
                Request* r = running[i];
                if (r->stage == kDone) {
                    slot_busy[r->slot] = 0;
                    r->cp->busy = false;
                    r->cp->last_use = ++use_clock;
                    finished[r->ticket] = r;
                    running.erase(running.begin() + long(i));
                    progressed = true;
                    cv_done.notify_all();
                } else {
                    ++i;
                }
            }
            if (!progressed) {
                if (running.empty() && waiting.empty())
                    cv_work.wait(lk, [&] { return stop || !waiting.empty(); });
                else
                    cv_work.wait_for(lk, std::chrono::microseconds(20));
            }
        }
    }
};

extern "C" {

int mbp_server_create(size_t hbm_budget, int slots, const mbp_options* opt, mbp_server** out) {
    if (!out || slots < 1 || slots > 64 || hbm_budget == 0) return MBP_ERR_INVALID;
    *out = nullptr;
    int count = 0, dev = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
        (void)hipGetLastError();
        return MBP_ERR_NO_DEVICE;
    }
    if (hipGetDevice(&dev) != hipSuccess) return MBP_ERR_HIP;
    mbp_server* S = new (std::nothrow) mbp_server();
    if (!S) return MBP_ERR_NOMEM;
    S->device = dev;
    S->budget = hbm_budget;
    S->slots = slots;
    if (opt) S->opt = *opt;
    else options_default(&S->opt);
    // served requests are solved one per slot, most of them small: there two
    // FP32 V-cycles per refinement step measured faster than the four that
    // single and batched solves default to (finer retirement per step)
    if (S->opt.inner == 0 || !opt) S->opt.inner = 2;
    int lds = 65536;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) lds = 65536;
    S->lds_limit = lds;
    S->streams.resize(slots);
    S->slot_busy.assign(slots, 0);
    if (hipMalloc(&S->arena_mem, hbm_budget) != hipSuccess) {
        (void)hipGetLastError();
        delete S;
        return MBP_ERR_NOMEM;
    }
    S->arena.init(hbm_budget);
    if (hipHostMalloc(&S->pinned, size_t(slots) * 4096, hipHostMallocDefault) != hipSuccess) {
        (void)hipFree(S->arena_mem);
        delete S;
        return MBP_ERR_NOMEM;
    }
    for (int k = 0; k < slots; ++k)
        if (hipStreamCreateWithFlags(&S->streams[k], hipStreamNonBlocking) != hipSuccess) {
            for (int j = 0; j < k; ++j) (void)hipStreamDestroy(S->streams[j]);
            (void)hipHostFree(S->pinned);
            (void)hipFree(S->arena_mem);
            delete S;
            return MBP_ERR_HIP;
        }
    S->worker = std::thread([S] { S->run(); });
    *out = S;
    return MBP_OK;
}

int mbp_server_submit(mbp_server* S, const mbp_block_desc* blocks, int nblocks, const mbp_synth_desc* z,
                      const double* rhs_dev, double* p_dev, double rtol, int flags, uint64_t* ticket) {
    if (!S || !blocks || nblocks < 1 || !z || !rhs_dev || !p_dev || rhs_dev == p_dev || !(rtol > 0.0) ||
        !ticket)
        return MBP_ERR_INVALID;
    auto r = std::make_unique<Request>();
    r->key = describe(blocks, nblocks, z, S->opt);
    // validate and build the host part of the plan in this thread (no device
    // memory yet); the worker places it in the arena when it admits the
    // request, or drops it when a cached plan with the same key is idle
    auto P = std::unique_ptr<mbp_plan>(new (std::nothrow) mbp_plan());
    if (!P) return MBP_ERR_NOMEM;
    std::string err;
    const int st = build_plan_host_limits(blocks, nblocks, z, &S->opt, int64_t(S->lds_limit), P.get(), &err);
    if (st != MBP_OK) return st;
    const size_t bytes = plan_device_bytes(P.get());
    r->host = std::move(P);
    if (bytes > S->budget) return MBP_ERR_TOO_LARGE;
    r->bytes = bytes;
    r->blocks.assign(blocks, blocks + nblocks);
    r->faces.resize(2 * size_t(nblocks));
    for (int b = 0; b < nblocks; ++b) {
        const int nx = blocks[b].hi[0] - blocks[b].lo[0] + 1, ny = blocks[b].hi[1] - blocks[b].lo[1] + 1;
        r->faces[2 * b].assign(blocks[b].xf, blocks[b].xf + nx + 1);
        r->faces[2 * b + 1].assign(blocks[b].yf, blocks[b].yf + ny + 1);
        r->blocks[b].xf = r->faces[2 * b].data();
        r->blocks[b].yf = r->faces[2 * b + 1].data();
    }
    r->z = *z;
    r->rhs = rhs_dev;
    r->p = p_dev;
    r->rtol = rtol;
    r->flags = flags;
    if (hipEventCreateWithFlags(&r->ev, hipEventDisableTiming) != hipSuccess) return MBP_ERR_HIP;
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) {
        (void)hipEventDestroy(r->ev);
        return MBP_ERR_INVALID;
    }
    r->ticket = S->next_ticket++;
    *ticket = r->ticket;
    Request* raw = r.release();
    S->all[raw->ticket] = raw;
    S->waiting.push_back(raw);
    S->cv_work.notify_all();
    return MBP_OK;
}

static int take_result(mbp_server* S, uint64_t ticket, mbp_solve_info* info, double* latency_ms) {
    auto it = S->finished.find(ticket);
    Request* r = it->second;
    const int st = r->status;
    if (info) {
        int32_t* keep = info->cycles_per_mode;
        *info = r->info;
        info->cycles_per_mode = keep;
        if (keep && !r->cycles.empty()) std::memcpy(keep, r->cycles.data(), r->cycles.size() * sizeof(int32_t));
    }
    if (latency_ms) *latency_ms = r->latency_ms;
    S->finished.erase(it);
    S->all.erase(ticket);
    (void)hipEventDestroy(r->ev);
    delete r;
    S->cv_done.notify_all();  // other waiters on this ticket re-check and leave
    return st;
}

int mbp_server_poll(mbp_server* S, uint64_t ticket, mbp_solve_info* info, double* latency_ms) {
    if (!S) return MBP_ERR_INVALID;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->all.find(ticket) == S->all.end()) return MBP_ERR_INVALID;
    if (S->finished.find(ticket) == S->finished.end()) return MBP_PENDING;
    return take_result(S, ticket, info, latency_ms);
}

int mbp_server_wait(mbp_server* S, uint64_t ticket, mbp_solve_info* info, double* latency_ms) {
    if (!S) return MBP_ERR_INVALID;
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->all.find(ticket) == S->all.end()) return MBP_ERR_INVALID;
    // Another thread may collect the same ticket first (wait or poll): then
    // the ticket is gone from `all` and this waiter reports it as invalid
    // instead of waiting for a result that will never come.
    S->cv_done.wait(lk, [&] {
        return S->finished.find(ticket) != S->finished.end() || S->all.find(ticket) == S->all.end();
    });
    if (S->finished.find(ticket) == S->finished.end()) return MBP_ERR_INVALID;
    return take_result(S, ticket, info, latency_ms);
}

void mbp_server_destroy(mbp_server* S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv_work.notify_all();
    }
    if (S->worker.joinable()) S->worker.join();
    for (auto& kv : S->all) {
        (void)hipEventDestroy(kv.second->ev);
        delete kv.second;
    }
    for (auto& c : S->cache) {
        plan_device_free(c->plan);
        delete c->plan;
    }
    for (hipStream_t s : S->streams) (void)hipStreamDestroy(s);
    if (S->pinned) (void)hipHostFree(S->pinned);
    if (S->arena_mem) (void)hipFree(S->arena_mem);
    delete S;
}

}  // extern "C"
