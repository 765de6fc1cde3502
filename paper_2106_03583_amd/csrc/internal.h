// Internal structures of the multi-block Poisson library (host + device).
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <atomic>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "mbp.h"

namespace mbp {

// Kinds of the z expansion (Table 1 rows; DN is the sine counterpart of ND).
enum ZKind { Z_PP = 0, Z_NN = 1, Z_DD = 2, Z_ND = 3, Z_DN = 4 };

enum Face { XM = 0, XP = 1, YM = 2, YP = 3 };

// Tile of the global-memory multigrid kernels: 64 cells along x (one wave),
// kTileY rows, 256 threads.
constexpr int kTileX = 64;
constexpr int kTileY = 16;
constexpr int kRowsPerPass = 4;  // threadIdx.y extent (256 threads = 64 x 4)

// One block of one multigrid level, as the kernels read it.
struct DBlock {
    int nx, ny;   // cells
    int off;      // first cell of this block inside a packed plane
    int nbr[4];   // neighbour block per face (-1 = wall)
    int bc[4];    // face condition (MBP_DIRICHLET / MBP_NEUMANN / joined)
    int par;      // colour parity offset (red-black ordering across blocks)
    int oddwrap;  // bit 0: odd periodic x wrap, bit 1: odd periodic y wrap (extra colours)
    int cx, cy;   // coefficient pool offsets: x -> [wm(nx) | wp(nx) | d(nx)], y alike
    // transfer from this level to the next coarser one
    int rsx, rsy;  // int pool: coarse -> first fine index (nc + 1 entries)
    int rwx, rwy;  // double pool: per fine index dc_fine / dc_coarse(parent)
    int pcx, pcy;  // int pool: per fine index coarse lower neighbour (-1 .. nc-1)
    int pwx, pwy;  // double pool: per fine index weight of that lower neighbour
};

// Host view of one multigrid level.
struct Level {
    int nb = 0;
    int64_t plane = 0;            // cells per plane
    std::vector<int> nx, ny, off;
    std::vector<std::vector<double>> xf, yf;  // face coordinates per block
    int blk_off = 0;              // first DBlock of this level in the block table
    int ntiles = 0;               // global-kernel tiles covering the plane
    int tile_off = 0;             // first tile in the tile table
    int64_t lds_off = 0;          // element offset of this level in the LDS image
    bool oddwrap = false;         // some block needs the two extra smoothing colours
    int cx = 1, cy = 1;           // the next coarser level halves x / y in every block (the transfer
                                  // tables carry each block's own step)
    int dp_begin = 0, ip_begin = 0;  // first entries of this level's tables in the pools
};

struct Geometry {
    int nb = 0;
    std::vector<int> lo0, lo1, hi0, hi1, nx, ny;
    std::vector<std::vector<double>> xf, yf;
    std::vector<std::array<int, 4>> bc, nbr;
    int nz = 0;
    double lz = 0.0, dz = 0.0;
    int zlo = 0, zhi = 0;
    ZKind zkind = Z_PP;
    bool dirichlet_xy = false;
    bool singular = false;
};

// The per-mode work description of one solve (batched launches list many).
struct Item {
    int plan;   // index into the batch's plan table
    int mode;   // z mode q
};

struct DevPlan;  // device pointers of one plan (see below)

// "One solve in flight per plan": claimed atomically so that two host
// threads calling into the same plan cannot both pass the check.  Copyable
// (the value is copied) so that plan descriptions can still be copied.
struct BusyFlag {
    std::atomic<bool> v{false};
    BusyFlag() = default;
    BusyFlag(const BusyFlag& o) : v(o.v.load()) {}
    BusyFlag& operator=(const BusyFlag& o) {
        v.store(o.v.load());
        return *this;
    }
    bool claim() {
        bool expect = false;
        return v.compare_exchange_strong(expect, true);
    }
    void release() { v.store(false); }
    bool held() const { return v.load(); }
};

struct FFTPlan {
    int n = 0, m = 0;              // real length, complex length n/2
    std::vector<int> radices;      // Stockham stages, product = m
};

}  // namespace mbp

struct mbp_plan {
    mbp::Geometry g;
    mbp_options opt{};
    std::vector<mbp::Level> levels;
    int nlev = 0;
    int lds_level = 0;            // first level handled by the LDS-resident kernel (FP64)
    int lds_level32 = 0;          // same for FP32 V-cycles
    int dp_levels_end = 0, ip_levels_end = 0;  // pool entries of all level tables
    int64_t lds_bytes64 = 0, lds_bytes32 = 0;
    int lds_fglob64 = 0;          // FP64: level lds_level's rhs read from device memory
    int coarse_n = 0;             // cells of the coarsest plane
    std::vector<double> lambda;   // Table-1 eigenvalues
    std::vector<double> shift;    // lambda_q / dz^2
    double mu0 = 0.0;             // smallest non-zero |eigenvalue| of the coarsest plane operator
    std::vector<double> sabs;     // mu0 + |shift_q|: lower bound of |eigenvalues| of mode q
    mbp::FFTPlan fft;
    int fft_tw = 0, fft_twn = 0, fft_post = 0, fft_pre4 = 0, fft_post4 = 0;  // double-pool offsets
    int fft_ntiles = 0;
    int fft_stream_nt = 0, fft_grid = 0;  // streaming transform: threads per workgroup, grid (0 = per-tile kernel)
    void* d_ftiles_fwd = nullptr;
    void* d_ftiles_inv = nullptr;
    int64_t lds_limit = 64 * 1024;  // LDS bytes one workgroup may use
    int lvinfo = 0;               // int-pool offset: per level {plane, blk_off, tile_off, ntiles}
    int proj_tab = 0;             // int-pool offset: per block {dcx, dcy, gx, gy, rows before, columns before}
    std::vector<int> mtile_off, mtile_cnt;  // fused-sweep strips per level (LDS strip form)
    std::vector<int> rtile_off, rtile_cnt;  // taller strips of the register-march form
    std::vector<char> use_rmarch;           // level runs its pre-smoothing as a register march
    int wg_target = 256 * 3;               // strip-form launches: workgroups aimed at
    std::vector<char> march_ok;   // level runs the fused one-pass sweeps
    void* d_mtiles = nullptr;
    size_t mtile_bytes = 0;
    // host tables (uploaded into one device allocation)
    std::vector<mbp::DBlock> hblk;
    std::vector<int> hint;
    std::vector<double> hdbl;
    std::vector<int4> htiles;
    std::vector<double> coarse_wl, coarse_wr, coarse_mu;  // nc x nc, nc x nc, nc
    std::vector<double> areas0;   // cell areas of the finest plane
    double area_sum = 0.0;
    int64_t ncells = 0;
    int64_t plane0 = 0;
    std::vector<int64_t> block_off;  // packed-field element offsets, nb + 1
    // ---- device state ----
    int device = -1;
    mbp::BusyFlag busy;
    void* dmem = nullptr;         // one allocation holding everything below
    bool owns_mem = true;         // false: dmem lies in a caller's arena (server)
    bool owns_pinned = true;      // false: host_pinned belongs to the caller (server slot)
    size_t dbytes = 0;
    mbp::DBlock* d_blk = nullptr;
    int* d_int = nullptr;
    double* d_dbl = nullptr;
    int4* d_tiles = nullptr;
    double* d_shift = nullptr;    // nz
    float* d_shift32 = nullptr;   // nz
    double* d_cwl = nullptr;      // coarse eigen tables
    double* d_cwr = nullptr;
    double* d_cmu = nullptr;
    double* d_area0 = nullptr;    // finest plane areas
    double* fhat = nullptr;       // nz * plane0 modal rhs
    double* phat = nullptr;       // nz * plane0 modal solution
    std::vector<double*> p64, f64;  // levels >= 1, FP64
    std::vector<float*> p32, f32;   // levels >= 0, FP32 (mixed precision)
    double* phatB = nullptr;        // second buffer of the finest level (out-of-place sweeps)
    std::vector<double*> p64B;      // levels >= 1
    std::vector<float*> p32B;       // levels >= 0
    double* d_part = nullptr;     // per-mode partial sums (nz * nparts * 2)
    int nparts = 0;
    double* d_fnorm = nullptr;    // nz: ||fhat_q||^2
    double* d_rnorm = nullptr;    // nz: ||rhat_q||^2
    double* d_pnorm = nullptr;    // nz: ||phat_q||^2
    double* d_sabs = nullptr;     // nz: mu0 + |shift_q|
    int* d_act = nullptr;         // active mode list (nz)
    int* d_nact = nullptr;        // 1 int
    int* d_cyc = nullptr;         // nz: cycles per mode
    int* d_flag = nullptr;        // 4 ints: [0] non-finite rhs
    double* d_scal = nullptr;     // 8 doubles of scratch scalars
    void* graph_exec = nullptr;   // cached batched replay (hipGraphExec_t)
    void* host_pinned = nullptr;  // small pinned buffer for convergence readback
    // kernel timing (mbp_profile_*): event pairs around finest-level sweeps
    bool prof = false;
    std::vector<std::array<void*, 2>> prof_ev[2];  // hipEvent_t pairs per kernel class
    std::vector<double> prof_cells[2];
    size_t prof_used[2] = {0, 0};
};

namespace mbp {

// plan.cpp
// uniform_levels: every block takes each coarsening step (the hierarchy ends
// when one block cannot), instead of each class of blocks sharing cells
// across joined faces stepping on its own
int build_plan_host_limits(const mbp_block_desc* blocks, int nblocks, const mbp_synth_desc* z,
                           const mbp_options* opt, int64_t lds_limit, mbp_plan* P, std::string* err,
                           bool uniform_levels = false);
int build_plan_host(const mbp_block_desc* blocks, int nblocks, const mbp_synth_desc* z,
                    const mbp_options* opt, mbp_plan* P, std::string* err);
void options_default(mbp_options* o);
void plan_set_shifts(mbp_plan* P);  // shift, sabs, singular from lambda and opt.helmholtz
// Symmetric eigen-decomposition (cyclic Jacobi); A (n x n, row-major) is
// overwritten, V gets the eigenvectors as columns, w the eigenvalues.
void jacobi_eig(std::vector<double>& A, int n, std::vector<double>& V, std::vector<double>& w);
int grid_tanh(int n, double lmin, double lmax, int type, double factor, double* out);

// fft.hip (host helpers)
int fft_columns_per_wg(const mbp_plan* P);
int fft_col_stride(const mbp_plan* P);
int fft_stream_setup(mbp_plan* P);
void fft_build_tiles(const mbp_plan* P, std::vector<unsigned char>& fwd, std::vector<unsigned char>& inv,
                     int* ntiles);

// device launchers (fft.hip, mg.hip)
void launch_forward(const mbp_plan* P, const double* f, double* fhat, int* nonfinite_flag,
                    hipStream_t s);
void launch_inverse(const mbp_plan* P, const double* phat, double* p, hipStream_t s);
void launch_apply3d(const mbp_plan* P, const double* p, double* out, hipStream_t s);
// project.hip: staggered velocities (packed face fields) and the projection
void velocity_offsets(const mbp_plan* P, int64_t* uo, int64_t* vo, int64_t* wo);
void launch_divergence(const mbp_plan* P, const double* u, const double* v, const double* w, double scale,
                       double* out, hipStream_t s);
void launch_gradient_update(const mbp_plan* P, const double* phi, double gdt, double* u, double* v, double* w,
                            hipStream_t s);
// Final check: out[0] = ||f - shift - (L_h - alpha) p||_2, out[1] = ||f - shift||_2
// (device doubles), per-workgroup partials in part (resnorm_scratch_doubles).
size_t resnorm_scratch_doubles(const mbp_plan* P);
void launch_resnorm3d(const mbp_plan* P, const double* f, const double* p, double shift, double* part,
                      double* out, hipStream_t s);

// One V-cycle on every active mode.  p0 / f0: finest-level iterate and rhs;
// p0B: second finest buffer for the out-of-place sweeps (the result is
// always left in p0).  With norm0 the finest post-smoothing sweep also
// produces per-strip squared residuals; returns the partial count then (0 if
// the caller must evaluate the residual itself).  zero0: p0 holds zeros
// (the first cycle), so the fused finest sweeps need not read it.
template <typename T>
int launch_vcycle(const mbp_plan* P, T* p0, T* p0B, T* f0, const int* act, const int* nact,
                  int nitems, bool norm0, bool zero0, hipStream_t s);
void launch_finish(const mbp_plan* P, int nparts, double* out, const int* act, const int* nact,
                   int nitems, hipStream_t s);
// Whole solve of every mode for plans whose hierarchy fits in LDS.
void launch_lds_full(const mbp_plan* P, double* p, const double* f, const int* act, const int* nact,
                     int nitems, int maxc, double rtol2, double etol2, int* cyc, double* rnorm,
                     double* fnorm, hipStream_t s);
// First cycle from a zero guess: residual norms are the rhs norms.
void launch_norm_from_rhs(const mbp_plan* P, int nitems, hipStream_t s);

// kernel timing helpers (solve.cpp)
void prof_begin(const mbp_plan* P, int cls, hipStream_t s, double cells);
void prof_end(const mbp_plan* P, int cls, hipStream_t s);

// march.hip
struct MTile;
bool march_level_ok(const mbp_plan* P, int l);
void march_build_tiles_bytes(const mbp_plan* P, int l, int seg, std::vector<unsigned char>& out, int* count);
template <typename T>
void march_pre(const mbp_plan* P, int l, const T* pold, T* pnew, const T* f, T* fc, T* pc,
               const int* act, const int* nact, int nitems, bool zero_in, hipStream_t s);
template <typename T>
void march_sweep(const mbp_plan* P, int l, const T* pold, T* pnew, const T* f, const int* act,
                 const int* nact, int nitems, bool zero_in, hipStream_t s);
template <typename T>
void march_post(const mbp_plan* P, int l, const T* pold, T* pnew, const T* f, const T* ec, bool norm,
                const int* act, const int* nact, int nitems, hipStream_t s);
void launch_residual_norm(const mbp_plan* P, const double* p, const double* f, double* rnorm,
                          const int* act, const int* nact, int nitems, hipStream_t s);
// pzero: p is zero (the first refinement step), r = f without reading p
void launch_residual_to32(const mbp_plan* P, const double* p, const double* f, float* r32,
                          float* e32, double* rnorm, const int* act, const int* nact, int nitems,
                          hipStream_t s, bool pzero = false);
// FP32 finest guess the refinement residual must zero (nullptr: none).
float* fp32_guess_to_zero(const mbp_plan* P);
// first: p is zero before the add (it is written, not read)
void launch_add_correction(const mbp_plan* P, double* p, const float* e32, const int* act,
                           const int* nact, int nitems, hipStream_t s, bool first = false);
void launch_plane_norm(const mbp_plan* P, const double* f, double* out, hipStream_t s);
void launch_update_active(const mbp_plan* P, double rtol2, double etol2, int retire, int maxc,
                          hipStream_t s, double* out = nullptr);
void launch_zero(double* p, size_t n, hipStream_t s);
void launch_zero_unrelaxed(const mbp_plan* P, double* p, hipStream_t s);  // modes with cyc == 0
bool vcycle_zero_start_reads_none(const mbp_plan* P);
void launch_zero32(float* p, size_t n, hipStream_t s);
void launch_singular_fix(const mbp_plan* P, double* plane, double* out_mean, hipStream_t s);

// solve.cpp
size_t plan_device_bytes(const mbp_plan* P);
// Device part of a plan.  ext_mem (optional): place the plan in that region
// of ext_bytes instead of allocating; ext_pinned (optional): a 4 KB pinned
// host buffer to use for readbacks.
int plan_device_init(mbp_plan* P, void* ext_mem = nullptr, size_t ext_bytes = 0, void* ext_pinned = nullptr);
void plan_device_free(mbp_plan* P);
int solve_one(mbp_plan* P, const double* rhs, double* p, double rtol, int flags, hipStream_t s,
              mbp_solve_info* info);

// One solve in flight: the stages of Algorithm 1 shared by the single and
// the batched forms.
struct SolveCtx {
    mbp_plan* P = nullptr;
    const double* rhs = nullptr;
    double* p = nullptr;
    double rtol2 = 0.0, etol2 = 0.0;
    int flags = 0;
    bool mixed = false, retire = false, warm = false, full_lds = false;
    int status = 0;
    double removed = 0.0;
    int nitems = 0;       // host upper bound on the active modes (grid sizes)
    int fused_parts = 0;  // partials left by the last V-cycle (0: explicit residual)
    int cycles = 0;       // V-cycles launched so far
    bool done = false;
    bool lazy_zero = false;  // p is not zeroed up front: the planes of modes no V-cycle
                             // relaxed are zeroed before the inverse transform
};
void ctx_init(SolveCtx& c, mbp_plan* P, const double* rhs, double* p, double rtol, int flags);
void ctx_prologue(SolveCtx& c, hipStream_t s);  // ends with an async readback of the checks
void ctx_check(SolveCtx& c);                    // after that readback synchronised
void ctx_test(SolveCtx& c, hipStream_t s, double* state_out = nullptr);  // residual norms + convergence
                                                                        // update (state copied to state_out)
void ctx_vcycle(SolveCtx& c, hipStream_t s);    // one V-cycle of the active modes
void ctx_state_readback(SolveCtx& c, hipStream_t s);
void ctx_state_apply(SolveCtx& c);              // after that readback synchronised
void ctx_epilogue(SolveCtx& c, hipStream_t s);
int ctx_info(SolveCtx& c, hipStream_t s, mbp_solve_info* info);  // synchronises s
int plan_autotune(mbp_plan* P, const double* rhs, hipStream_t s, mbp_tuning* out);

// ---- grouped launches: one launch runs one stage of the refinement step for
//      many problems.  Workgroups [wg0, next entry's wg0) belong to job `job`;
//      a workgroup's local index splits into (bx, by) with gx columns. ----
struct GEnt {
    int wg0, gx, job, pad;
};
enum GKind { G_RES32 = 0, G_FINISH, G_UPDATE, G_PRE32, G_LDS32, G_POST32, G_ADDCORR };
struct GStage {
    int kind = 0;
    int wgs = 0;            // workgroups of the launch
    int nent = 0;
    size_t ent_off = 0;     // byte offsets in the table image
    size_t job_off = 0;
    size_t lds = 0;         // dynamic LDS bytes (LDS-resident stage)
    int threads = 256;
};
// Host image of the tables of every stage; uploaded once per capture.
struct GroupBlob {
    std::vector<unsigned char> host;
    size_t add(const void* src, size_t bytes) {
        const size_t off = (host.size() + 255) & ~size_t(255);
        host.resize(off + bytes);
        if (bytes) std::memcpy(host.data() + off, src, bytes);
        return off;
    }
};
// Stage record for jobs with (gx, gy) workgroups each; empty jobs are skipped.
template <typename Job>
GStage group_build(GroupBlob& gb, int kind, const std::vector<Job>& jobs, const std::vector<int>& gx,
                   const std::vector<int>& gy) {
    std::vector<GEnt> ents;
    long long wg = 0;
    for (size_t i = 0; i < jobs.size(); ++i) {
        const long long n = (long long)gx[i] * gy[i];
        if (n <= 0) continue;
        ents.push_back(GEnt{int(wg), gx[i], int(i), 0});
        wg += n;
    }
    GStage st;
    st.kind = kind;
    st.wgs = int(wg);
    st.nent = int(ents.size());
    st.ent_off = gb.add(ents.data(), ents.size() * sizeof(GEnt));
    st.job_off = gb.add(jobs.data(), jobs.size() * sizeof(Job));
    return st;
}
// Job of this workgroup in a grouped launch, and its (bx, by) inside the job.
// A record every lane of the wave read from the same address: say so, so
// that what is computed from it stays in scalar registers.
template <typename R>
__device__ __forceinline__ R wave_uniform(const R& v) {
    static_assert(sizeof(R) % 4 == 0, "whole 32-bit words");
    R out;
    const int* src = reinterpret_cast<const int*>(&v);
    int* dst = reinterpret_cast<int*>(&out);
#pragma unroll
    for (int k = 0; k < int(sizeof(R) / 4); ++k) dst[k] = __builtin_amdgcn_readfirstlane(src[k]);
    return out;
}

__device__ __forceinline__ int group_locate(const GEnt* __restrict__ e, int n, int& bx, int& by) {
    const int g = blockIdx.x;
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (e[mid].wg0 <= g) lo = mid;
        else hi = mid - 1;
    }
    const int local = g - e[lo].wg0;
    bx = local % e[lo].gx;
    by = local / e[lo].gx;
    return e[lo].job;
}
// A problem joins the grouped form when every level above its LDS-resident
// ones runs the strip kernels (mixed precision, one pre- and one post-sweep).
bool group_ok(const SolveCtx& c);
// Stage tables for the problems `cs` (phase 1, host only) ...
GStage group_res32(GroupBlob& gb, const std::vector<SolveCtx*>& cs);
GStage group_finish(GroupBlob& gb, const std::vector<SolveCtx*>& cs);
GStage group_update(GroupBlob& gb, const std::vector<SolveCtx*>& cs);
GStage group_lds32(GroupBlob& gb, const std::vector<SolveCtx*>& cs);
GStage group_addcorr(GroupBlob& gb, const std::vector<SolveCtx*>& cs);
GStage group_march32(GroupBlob& gb, const std::vector<SolveCtx*>& cs, int level, bool post, bool zero0);
// ... and their launches from the uploaded image (phase 2, capturable).
void group_launch_mg(const GStage& st, const unsigned char* dev, hipStream_t s);
void group_launch_march(const GStage& st, const unsigned char* dev, hipStream_t s);

}  // namespace mbp
