/*
 * mbp.h -- C ABI of the multi-block FFT-accelerated Poisson solver (gfx950).
 *
 * Problem (paper Sec. 2, Eqs. (8)-(9); Sec. 3.1, Table 2): the cell-centred
 * second-order finite-volume Laplacian L_h p = f on a multi-block x-y
 * cross-section (logically rectangular blocks, spacing free to vary in x and
 * y) extruded along a uniform z direction with nz cells.  Along z the field is
 * expanded in the eigenfunctions of Table 1 (periodic, Neumann-Neumann,
 * Dirichlet-Dirichlet, Neumann-Dirichlet, plus Dirichlet-Neumann), which
 * splits the 3D system into nz independent 2D Helmholtz systems
 *     (A_2D + lambda_q / dz^2) phat_q = fhat_q          (Eq. (9))
 * solved here by geometric-multigrid V-cycles, then transformed back
 * (Algorithm 1).
 *
 * Conventions shared by every entry point:
 *   - Every call returns an int status: MBP_OK (0) or a negative MBP_ERR_*.
 *     Nothing throws across this interface.  mbp_status_string() names codes.
 *   - Fields (rhs, p) are ONE packed float64 buffer: block after block in the
 *     order given to mbp_plan_create, each block in C order (nz, ny, nx), x
 *     fastest.  mbp_plan_layout() returns the offsets.
 *   - Pointers named *_dev are device pointers on the plan's HIP device; all
 *     other pointers are host pointers.  Descriptors are copied at plan
 *     creation; the caller may free them afterwards.
 *   - "stream" is a hipStream_t passed as void* (NULL = the null stream).
 *   - Homogeneous boundary conditions only (inhomogeneous data belongs in the
 *     rhs).  Unknowns are cell centred; a Dirichlet / Neumann face holds p = 0 /
 *     dp/dn = 0 on the face (staggered conditions of Table 1).
 */
#ifndef MBP_H
#define MBP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define MBP_OK                 0
#define MBP_PENDING            1   /* server ticket not finished yet */
#define MBP_ERR_INVALID       -1   /* bad descriptor / argument */
#define MBP_ERR_NOMEM         -2   /* device or host allocation failed */
#define MBP_ERR_HIP           -3   /* a HIP runtime call failed */
#define MBP_ERR_NOT_CONVERGED -4   /* max_cycles reached; p holds the last iterate */
#define MBP_ERR_NONFINITE     -5   /* rhs holds NaN or Inf */
#define MBP_ERR_INCOMPATIBLE  -6   /* singular problem, rhs not compatible, no projection asked */
#define MBP_ERR_BUSY          -7   /* plan already has a solve in flight */
#define MBP_ERR_TOO_LARGE     -8   /* request footprint exceeds the server budget */
#define MBP_ERR_NO_DEVICE     -9   /* no HIP device available */

/* ---- face / end conditions (Sec. 3.1: Dirichlet, Neumann, block-block
 *      connectivity; periodic = cyclic connectivity) ---------------------- */
#define MBP_DIRICHLET 1
#define MBP_NEUMANN   2
#define MBP_CONNECT   3   /* joined to the block touching this face in index space */
#define MBP_PERIODIC  4   /* joined cyclically to the opposite PERIODIC face */

/* ---- options ------------------------------------------------------------ */
#define MBP_FP64  0       /* every V-cycle in float64 */
#define MBP_MIXED 1       /* float32 V-cycles inside float64 iterative refinement */

#define MBP_PROJECT_RHS 1 /* singular problems: remove the volume-weighted mean of rhs */
#define MBP_WARM_START  2 /* p_dev holds the initial guess (Sec. 3.3.1: latest solution) */
#define MBP_RETIRE      4 /* retire each z mode as soon as it converges (else lockstep) */
#define MBP_AUTOTUNE    8 /* mbp_solve_batch: time candidate schedules on this call and keep
                             the fastest for later calls with the same plan set */

/* One block of the x-y cross-section (Table 2: lo / hi in index space,
 * inclusive, cells = hi - lo + 1; physical face coordinates).
 *   lo, hi : index-space corners (x, y).
 *   xf, yf : host arrays of nx+1 / ny+1 increasing face coordinates.
 *   bc     : condition of the faces -x, +x, -y, +y (MBP_DIRICHLET ...).
 * A CONNECT face must touch exactly one block over exactly the same
 * tangential index range, and both sides must carry the same face
 * coordinates (the congruence rule of Sec. 3.1).  A PERIODIC face on the
 * lower side joins the PERIODIC upper face of the block with the same
 * tangential range (itself for a single block). */
typedef struct {
    int32_t lo[2];
    int32_t hi[2];
    const double* xf;
    const double* yf;
    int32_t bc[4];
} mbp_block_desc;

/* The homogeneous (synthesis) direction: nz uniform cells on [0, lz) (the
 * grid must be uniform along it, Sec. 2).  nz must be even (Table 1).
 * (bc_lo, bc_hi) is one of (P,P), (N,N), (D,D), (N,D), (D,N). */
typedef struct {
    int32_t nz;
    double lz;
    int32_t bc_lo;
    int32_t bc_hi;
} mbp_synth_desc;

/* Smoothers (Sec. 3.3.1: the paper's PFMG offers weighted Jacobi and
 * red-black Gauss-Seidel point smoothers). */
#define MBP_SMOOTHER_DEFAULT 0 /* the solver's own: RB-GS (FFT path), weighted Jacobi (mbp3_*) */
#define MBP_SMOOTHER_RBGS    1 /* red-black Gauss-Seidel; FFT-accelerated path only */
#define MBP_SMOOTHER_JACOBI  2 /* weighted Jacobi, omega = 6/7; 3D multigrid (mbp3_*) only */

/* Solver options (Sec. 3.3.1: the multigrid solver's settings; Sec. 2: the
 * Helmholtz systems of implicit diffusion).  Pass NULL for the defaults in
 * brackets.
 *   precision  MBP_FP64 | MBP_MIXED                              [MBP_FP64]
 *   nu1, nu2   smoothing sweeps before / after the coarse-grid
 *              correction                                        [1, 1]
 *   max_cycles cap on V-cycles (or refinement steps)             [100]
 *   flags      default solve flags OR-ed into each solve          [0]
 *   etol       target of the estimated relative solution error of
 *              each mode, ||rhat_q|| / (mu_0 + |sigma_q|) <= etol ||phat_q||
 *              / 2, with mu_0 the smallest non-zero eigenvalue magnitude
 *              of the coarsest plane operator (a lower bound of the fine
 *              one, so the estimate is conservative); 0 = 10 * rtol,
 *              negative = off                                    [0]
 *   inner      MBP_MIXED: FP32 V-cycles per FP64 refinement step
 *              (residual in FP64, correction solved in FP32, added in
 *              FP64); 0 = default                [4; 2 in a server]
 *   march      pre-smoothing form of the fused levels: 0 LDS strip
 *              tiles, 1 register march (mbp_plan_autotune may change
 *              it per level)                                     [0]
 *   smoother   MBP_SMOOTHER_DEFAULT | _RBGS (FFT path) | _JACOBI (mbp3_*)
 *                                                                [DEFAULT]
 *   helmholtz  alpha >= 0: solve (L_h - alpha) p = f, the Helmholtz
 *              systems of implicit diffusion, which the paper solves
 *              by the same method as the Poisson equation (Sec. 2);
 *              every modal shift becomes lambda_q/dz^2 - alpha.
 *              With alpha > 0 no problem is singular.  Change it between
 *              solves with mbp_plan_set_helmholtz                  [0]
 * In the mixed form max_cycles and the reported cycles count refinement
 * steps (each one convergence test). */
typedef struct {
    int32_t precision;
    int32_t nu1, nu2;
    int32_t max_cycles;
    int32_t flags;
    double etol;
    int32_t inner;
    int32_t march;
    int32_t smoother;
    double helmholtz;
} mbp_options;

/* Per-solve report (caller-owned).
 *   status          MBP_OK or the asynchronous error of this solve
 *   cycles          V-cycles (refinement steps) taken by the slowest mode
 *   rel_residual    max over modes of ||rhat_q|| / ||fhat_q|| at exit; since
 *                   the transforms are orthonormal this bounds the 3D
 *                   relative residual ||f - L_h p|| / ||f||
 *   removed_mean    volume-weighted mean removed from rhs (singular, projected)
 *   cycles_per_mode optional caller array of nz ints, or NULL
 *   t_ms            [0] forward transform, [1] multigrid, [2] inverse, [3] total
 *                   (filled only when the solve is timed, else 0) */
typedef struct {
    int32_t status;
    int32_t cycles;
    double rel_residual;
    double removed_mean;
    int32_t* cycles_per_mode;
    double t_ms[4];
} mbp_solve_info;

/* Host-side summary of a validated problem (mbp_plan_check). */
typedef struct {
    int64_t ncells;          /* total cells nz * sum(nx*ny) */
    int32_t nlevels;         /* multigrid levels of the x-y plane */
    int32_t coarse_cells;    /* cells of the coarsest plane (dense solve) */
    int32_t singular;        /* 1 if no Dirichlet condition anywhere */
    int32_t nblocks;
    int64_t workspace_bytes; /* device bytes the plan allocates (FP64 + FP32 work) */
    int32_t nbr[64][4];      /* neighbour block per face (first 64 blocks; -1 = wall) */
} mbp_plan_summary;

typedef struct mbp_plan mbp_plan;
typedef struct mbp_server mbp_server;

/* Static text for a status code (library plumbing; no passage of the paper). */
const char* mbp_status_string(int status);

/* ABI version (major*100 + minor; library plumbing). */
int mbp_version(void);

/* Face coordinates of a hyperbolic-tangent clustered 1D grid (Sec. 3.1,
 * Table 2 caption: type 0 clusters at both ends, -1 / +1 at the lower /
 * upper end, factor 0 is uniform).  Writes n+1 faces into faces_out (host,
 * caller-owned) from lmin to lmax.  MBP_ERR_INVALID for n < 1, lmax <= lmin,
 * an unknown type or a negative factor. */
int mbp_grid_tanh(int n, double lmin, double lmax, int type, double factor, double* faces_out);

/* Validate a problem and describe the plan it would build, on the host only
 * (no HIP call, no allocation on the device): the checks of the problem
 * statement of Sec. 3.1 and Table 2 (blocks, faces, conditions) and the
 * Sec. 3.3.1 multigrid hierarchy.  Same errors as mbp_plan_create's
 * validation; out may be NULL. */
int mbp_plan_check(const mbp_block_desc* blocks, int nblocks, const mbp_synth_desc* z,
                   const mbp_options* opt, mbp_plan_summary* out);

/* Build a plan on the current HIP device (the set-up of Algorithm 1 for the
 * problem of Sec. 3.1 / Table 2): validation, connectivity, grid metrics per
 * multigrid level, modal shifts lambda_q / dz^2 (Table 1, Eq. (9)),
 * transform tables, the coarsest-level eigen-decomposition, device workspace.
 * Blocking.  The plan owns its device memory.  Errors: MBP_ERR_INVALID
 * (odd or < 2 nz, invalid pair, non-congruent or partial interface, a face
 * with two neighbours, overlapping blocks, bad faces), MBP_ERR_NOMEM,
 * MBP_ERR_HIP, MBP_ERR_NO_DEVICE. */
int mbp_plan_create(const mbp_block_desc* blocks, int nblocks, const mbp_synth_desc* z,
                    const mbp_options* opt, mbp_plan** out);

/* Change the Helmholtz term alpha (>= 0) of an idle plan, as the implicit
 * diffusion of each Runge-Kutta substep needs (footnote of Sec. 3.3.1: the
 * matrix diagonal is modified every substep).  Updates the modal shifts
 * lambda_q/dz^2 - alpha on the host and the device (a blocking copy) and the
 * plan's singular flag; no other table changes.  Errors: MBP_ERR_INVALID
 * (NULL plan, alpha < 0 or not finite), MBP_ERR_BUSY, MBP_ERR_HIP. */
int mbp_plan_set_helmholtz(mbp_plan* plan, double alpha);

/* Layout query (the packed field layout is this library's own; no passage).
 * block_offsets (nblocks+1 int64, may be NULL): element offsets of each
 * block in the packed field; workspace_bytes and singular may be NULL. */
int mbp_plan_layout(const mbp_plan* plan, int64_t* block_offsets, size_t* workspace_bytes,
                    int* singular);

/* Solve L_h p = rhs (Algorithm 1) to a relative residual rtol.
 *   rhs_dev  packed float64 device field, read only.
 *   p_dev    packed float64 device field, written (read first if
 *            MBP_WARM_START).  May not alias rhs_dev.
 *   rtol     per-mode stopping rule ||rhat_q|| <= rtol * ||fhat_q||, which
 *            implies ||f - L_h p|| <= rtol * ||f||.  Must be > 0.
 *   flags    MBP_PROJECT_RHS | MBP_WARM_START | MBP_RETIRE, OR-ed with the
 *            plan's default flags.
 * The work is ordered on `stream`; the call returns when the solve has
 * finished (it reads convergence data back to decide when to stop) and
 * info (optional) is then valid.  One solve at a time per plan
 * (MBP_ERR_BUSY otherwise).  Returns the same status as info->status. */
int mbp_solve(mbp_plan* plan, const double* rhs_dev, double* p_dev, double rtol, int flags,
              void* stream, mbp_solve_info* info);

/* Many independent solves in one call (Algorithm 1 for each).  After the
 * forward transforms and one eager cycle, the cycles of every unfinished
 * problem are captured into one HIP graph (one branch per internal stream)
 * and replayed, a few cycles per replay; inside a replay the device tests
 * every mode and retires converged ones, so finished problems cost only
 * empty launches until the host, reading the active counts after each
 * replay, captures a smaller graph.  Plans may differ in size, conditions
 * and precision and must be distinct; each must be idle.  Every item runs
 * with per-mode retirement.  The stream count and cycles per replay come
 * from a cache keyed by the plan set, filled when a call passes
 * MBP_AUTOTUNE (default 4 streams, 4 cycles).  Stream-ordered on `stream`
 * at entry and exit; the call returns after the results are read back.
 * Returns MBP_OK if every item converged, else the first failing item's
 * status; infos (optional, count entries) hold the per-item reports.
 * Grouped form: when every unfinished item is a mixed-precision plan whose
 * levels above the LDS-resident ones all run the strip kernels (one pre- and
 * one post-smoothing sweep) with the same inner cycle count, each stage of
 * the refinement step is one launch across all items (the stream count is
 * then unused). */
int mbp_solve_batch(mbp_plan* const* plans, const double* const* rhs_dev, double* const* p_dev,
                    int count, double rtol, int flags, void* stream, mbp_solve_info* infos);

/* Schedule the batch autotuner chose for this plan set (the batched form is
 * this library's; the paper solves one problem at a time): MBP_OK with the
 * stream count and cycles per replay, or MBP_PENDING if none is cached.
 * streams is 0 when every replay of the last batch of this plan set ran in
 * the grouped form. */
int mbp_batch_schedule(mbp_plan* const* plans, int count, int* streams, int* cycles_per_replay);

/* Building blocks of the solve, exposed for checking and for callers that
 * compose their own pipelines.  All are stream-ordered and asynchronous.
 *   mbp_forward_transform: fhat = T^T f along z for every x-y cell; modal
 *     layout is plane-major: mode q occupies [q*P, (q+1)*P) with P the cells
 *     of one x-y plane, blocks packed inside a plane in block order, each
 *     (ny, nx).  Orthonormal transforms (Table 1 kinds, scaled to theta = 1).
 *   mbp_inverse_transform: the inverse map, modal -> packed field.
 *   mbp_apply_operator: out = L_h p on the packed field (float64).
 *   mbp_modal_shift: writes the nz shifts lambda_q / dz^2 (host array). */
int mbp_forward_transform(mbp_plan* plan, const double* f_dev, double* fhat_dev, void* stream);

/* Final check of a solve (Eq. (8) on the whole field; the paper validates
 * its solver by checking the result up to the tolerance, Sec. 4.1):
 *   out_dev[0] = ||f - s - (L_h - alpha) p||_2,  out_dev[1] = ||f - s||_2
 * over every cell, with f = rhs_dev, p = p_dev (packed float64 device
 * fields), s = rhs_shift (pass info.removed_mean of a projected singular
 * solve, else 0), alpha the plan's Helmholtz term.  out_dev: two device
 * doubles, written by the stream's work.  Stream-ordered and asynchronous;
 * per-workgroup partial sums go to the plan's workspace, so it must not
 * overlap a solve on the same plan.  Errors: MBP_ERR_INVALID (NULL
 * argument), MBP_ERR_BUSY (a solve is running in another thread),
 * MBP_ERR_HIP. */
int mbp_residual_norm(mbp_plan* plan, const double* rhs_dev, const double* p_dev, double rhs_shift,
                      double* out_dev, void* stream);

/* The same check for callers that cannot allocate (code under HIP graph
 * capture, serving loops, harnesses that forbid allocation): allocates
 * nothing and does not touch the plan's workspace (only its read-only
 * tables), so it may also run while a solve on the plan is in flight.  Its
 * partial sums live in a fixed per-device scratch array of
 * mbp_noalloc_scratch_bytes() bytes (8 MiB; the check needs
 * 16 * nz * (finest-level tiles of 64 x 16 cells) bytes); larger problems
 * get MBP_ERR_TOO_LARGE.  Every call on a GPU shares that GPU's array:
 * calls that overlap on one GPU (several streams or threads) race and must
 * be ordered by the caller.  Same arguments and results as
 * mbp_residual_norm; the plan must live on the current device
 * (MBP_ERR_INVALID otherwise). */
int mbp_residual_norm_noalloc(const mbp_plan* plan, const double* rhs_dev, const double* p_dev,
                              double rhs_shift, double* out_dev, void* stream);
size_t mbp_noalloc_scratch_bytes(void);
int mbp_inverse_transform(mbp_plan* plan, const double* phat_dev, double* p_dev, void* stream);
int mbp_apply_operator(mbp_plan* plan, const double* p_dev, double* out_dev, void* stream);
int mbp_modal_shift(const mbp_plan* plan, double* shift_host);

/* ---- pressure projection (Eqs. (3)-(6)) --------------------------------- */
/* The steps on either side of the Poisson solve in the paper's fractional
 * step, on the staggered grid (Sec. 2: velocities on cell faces):
 *     rhs = D u* / (gamma dt),  L_h Phi = rhs,  u = u* - gamma dt G Phi,
 * after which D u = 0 to the solver's tolerance (the check of Sec. 4.1).  D
 * is the finite-volume divergence, G the face gradient, D G = L_h: a Neumann
 * face (prescribed normal velocity) keeps its velocity, a Dirichlet face
 * (prescribed pressure) sees the mirrored ghost -Phi, joined and periodic
 * faces couple the partner's cell.
 * Face fields are packed float64 device buffers, block after block in plan
 * order: u (nz, ny, nx + 1), v (nz, ny + 1, nx), w (nz, ny, nx) when z is
 * periodic (face k - 1/2, cyclic) and (nz + 1, ny, nx) otherwise.  A face
 * shared by two joined blocks is stored in both (the caller keeps the two
 * copies equal; the update keeps them equal).
 *   mbp_velocity_layout: element offsets of each block in u, v, w (nblocks +
 *     1 int64 each; any may be NULL).
 *   mbp_divergence: out_dev (a packed cell field) = scale * D(u, v, w).
 *     Stream-ordered and asynchronous.
 *   mbp_project: one projection: rhs_work_dev (a cell field, caller-owned
 *     scratch) = D u / gamma_dt, Phi solved into phi_dev as mbp_solve does
 *     (flags as there, MBP_PROJECT_RHS implied: a singular problem whose net
 *     boundary flux is not zero is projected; MBP_WARM_START starts from the
 *     previous Phi, as the paper's time loop does), then u, v, w -= gamma_dt G
 *     Phi in place.  Returns the solve's status (info as mbp_solve's); the
 *     velocity is corrected also when the solve stops at max_cycles.
 *     Errors: MBP_ERR_INVALID (NULL pointer, gamma_dt <= 0, rtol <= 0,
 *     phi_dev == rhs_work_dev, wrong device), MBP_ERR_BUSY, MBP_ERR_HIP and
 *     the solve's codes. */
int mbp_velocity_layout(const mbp_plan* plan, int64_t* u_off, int64_t* v_off, int64_t* w_off);
int mbp_divergence(mbp_plan* plan, const double* u_dev, const double* v_dev, const double* w_dev,
                   double scale, double* out_dev, void* stream);
int mbp_project(mbp_plan* plan, double* u_dev, double* v_dev, double* w_dev, double gamma_dt,
                double* phi_dev, double* rhs_work_dev, double rtol, int flags, void* stream,
                mbp_solve_info* info);

/* Kernel timing for roofline reports.  While enabled, the finest-level
 * fused smoothing launches of every solve on the plan are bracketed by HIP
 * events on the solve's stream.  mbp_profile_read waits for those events and
 * returns, per kernel class (0: pre-smoothing sweep + restriction, 1:
 * correction + post-smoothing sweep + residual norm), the launch count, the
 * summed duration in ms and the cells processed (plane cells x active modes,
 * summed over launches); enabling again clears the record.  Errors:
 * MBP_ERR_INVALID for a NULL plan. */
typedef struct {
    int64_t launches[2];
    double total_ms[2];
    double cells[2];
} mbp_profile_info;
int mbp_profile_enable(mbp_plan* plan, int enable);
int mbp_profile_read(mbp_plan* plan, mbp_profile_info* out);

/* Schedule autotuner for one plan.  Runs the forward transform of rhs_dev
 * and, for each candidate schedule, a few V-cycles of every mode on the
 * plan's own workspace, timed with events on `stream`; the fastest
 * candidate stays in the plan for every later solve.  Candidates: the
 * number of workgroups a strip-form launch aims at (which sets how many
 * modes one workgroup runs in turn) and, per fused multigrid level, the
 * pre-smoothing form (LDS strip tiles of 26 x 58 cells, or a register
 * march down strips of 128 x 58 cells).  All candidates run the same
 * red-black sweeps.  Blocking; the plan must be idle.  out (optional):
 *   wg_target  chosen workgroups per launch
 *   levels     multigrid levels reported in form[] (at most 16)
 *   form[l]    0 strip tiles, 1 register march
 *   ms_default / ms_tuned  time of one V-cycle over all modes before / after
 * Errors: MBP_ERR_INVALID, MBP_ERR_NONFINITE (rhs), MBP_ERR_HIP. */
typedef struct {
    int32_t wg_target;
    int32_t levels;
    int32_t form[16];
    double ms_default;
    double ms_tuned;
} mbp_tuning;
int mbp_plan_autotune(mbp_plan* plan, const double* rhs_dev, void* stream, mbp_tuning* out);

/* Release the plan's device memory (library plumbing).  The caller ensures
 * no work is in flight on it.  NULL is ignored. */
void mbp_plan_destroy(mbp_plan* plan);

/* ---- 3D multigrid without the z synthesis ----------------------------- */
/* The comparison solver of Sec. 3.3.1 (the paper's "3D MG", timed against
 * the FFT-accelerated solve in Sec. 4.2): geometric multigrid V-cycles on the
 * whole 3D system (L_h - alpha) p = f of Eq. (8), on the same multi-block,
 * stretched x-y grid and uniform z.  Level l = x-y level l of the FFT path's
 * hierarchy times nz_l z cells (z halved with x-y while its count is even and
 * >= 4); rediscretised coarse operators; weighted Jacobi smoothing (omega =
 * 6/7, the smoother the paper runs in PFMG); volume-weighted restriction of
 * the residual; trilinear prolongation (physical weights in x-y); exact
 * coarsest solve by separation (dense z and x-y eigen-decompositions).
 * FP64 only.  Fields use the packed layout of mbp_plan_layout, on the
 * caller's buffers directly.
 *   mbp3_plan_create: same descriptors as mbp_plan_create.  opt (NULL =
 *     defaults nu1 = nu2 = 2, max_cycles 100): precision must be MBP_FP64,
 *     smoother MBP_SMOOTHER_DEFAULT or _JACOBI, nu1, nu2 >= 1, helmholtz =
 *     alpha >= 0.  Blocking; owns its device memory (about 1.5 x 8 B per
 *     cell beyond the caller's fields).  Errors as mbp_plan_create.
 *   mbp3_plan_levels: levels, nz and cells per level (caller arrays of
 *     nlevels entries, each may be NULL), device bytes (may be NULL).
 *   mbp3_jacobi_sweep: one weighted-Jacobi sweep of the finest level,
 *     pout = pin + omega D^-1 (f - (L_h - alpha) pin), packed fields, out of
 *     place (pin != pout); stream-ordered and asynchronous.  Exposed for
 *     checking and timing the smoother alone.
 *   mbp3_solve: stopping rule ||f - L_h p||_2 <= rtol ||f||_2 on the whole
 *     3D field (checked on the returned iterate).  Flags MBP_PROJECT_RHS
 *     (singular problems: remove the volume-weighted mean of f, without
 *     writing rhs_dev) and MBP_WARM_START.  Ordered on `stream`; returns when
 *     the solve is done (it reads each cycle's residual to decide whether to
 *     queue the next).  info: status, cycles, rel_residual (of the returned
 *     p), removed_mean, t_ms[1] = t_ms[3] = solve time; cycles_per_mode is
 *     not used.  Same error codes as mbp_solve.
 *   mbp3_plan_destroy: frees the plan (no work may be in flight). */
typedef struct mbp3_plan mbp3_plan;
int mbp3_plan_create(const mbp_block_desc* blocks, int nblocks, const mbp_synth_desc* z,
                     const mbp_options* opt, mbp3_plan** out);
int mbp3_plan_levels(const mbp3_plan* plan, int* nlevels, int* nz_per_level, int64_t* cells_per_level,
                     size_t* workspace_bytes);
int mbp3_jacobi_sweep(mbp3_plan* plan, const double* pin_dev, double* pout_dev, const double* f_dev,
                      void* stream);
int mbp3_solve(mbp3_plan* plan, const double* rhs_dev, double* p_dev, double rtol, int flags,
               void* stream, mbp_solve_info* info);
void mbp3_plan_destroy(mbp3_plan* plan);

/* ---- serving loop ------------------------------------------------------- */
/* The serving form is this library's own (the paper runs one problem per
 * job); each request is the solve of Algorithm 1.
 * A server admits solve requests of any size and conditions, keeps plans
 * (hierarchies, tables, workspaces) resident in an LRU cache keyed by the
 * descriptor, and runs up to `slots` requests concurrently on their own HIP
 * streams: a request that arrives while others run starts as soon as a slot
 * and `hbm_budget` bytes of plan memory are free (continuous batching).
 *   mbp_server_create: opt may be NULL.  slots in [1, 64].
 *   mbp_server_submit: rhs_dev / p_dev stay owned by the caller and must stay
 *     valid until the ticket completes; rhs_dev must already hold its data
 *     (its producing stream synchronised).  The descriptor is copied.
 *     Returns MBP_ERR_TOO_LARGE when the request alone exceeds the budget,
 *     MBP_ERR_INVALID for a bad problem.  Requests run with per-mode
 *     retirement and the server's options.
 *   mbp_server_poll: MBP_PENDING, or the request's final status with info
 *     filled (info->cycles_per_mode, when not NULL, receives the request's
 *     nz per-mode cycle counts); latency_ms (optional) = completion -
 *     submission, wall clock.  A ticket is collected once: a later poll or
 *     wait on it (also a wait already blocked on it in another thread)
 *     returns MBP_ERR_INVALID.
 *   mbp_server_wait: blocks until the ticket completes, then as poll.
 *   mbp_server_destroy: waits for all work, frees every cached plan. */
int mbp_server_create(size_t hbm_budget, int slots, const mbp_options* opt, mbp_server** out);
int mbp_server_submit(mbp_server* s, const mbp_block_desc* blocks, int nblocks,
                      const mbp_synth_desc* z, const double* rhs_dev, double* p_dev,
                      double rtol, int flags, uint64_t* ticket);
int mbp_server_poll(mbp_server* s, uint64_t ticket, mbp_solve_info* info, double* latency_ms);
int mbp_server_wait(mbp_server* s, uint64_t ticket, mbp_solve_info* info, double* latency_ms);
void mbp_server_destroy(mbp_server* s);

#ifdef __cplusplus
}
#endif
#endif /* MBP_H */
