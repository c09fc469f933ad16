/*
 * lap.h — C ABI of liblap, a gfx950 (MI355X) solver library for the 5-point
 * discretisation of the 2D Laplace / Poisson equation
 *
 *     d2psi/dx2 + d2psi/dy2 = f   on a rectangle,   psi = g on its boundary,
 *
 * with the methods compared in M. M. Ahmed, "A Comparison of SOR, ADI and
 * Multigrid Methods for Solving Partial Differential Equations" (arXiv:2208.02427):
 * red-black SOR (the parallel ordering of SOR, Eq. (7)), line ADI with
 * Thomas solves (SLOR/ADI sections, Eqs. (8)-(10)) and the multigrid
 * V-cycle (Multigrid section, Eqs. (11)-(15)), plus mixed-precision defect
 * correction (FP32 V-cycle, FP64 residual and accumulation).
 *
 * Conventions used by every entry point
 * -------------------------------------
 * - Grid: m nodes along x (index i), n along y (index j), spacings dx, dy.
 *   The discrete operator is (L_h psi)_ij = cx (psi_{i-1,j} + psi_{i+1,j})
 *   + cy (psi_{i,j-1} + psi_{i,j+1}) - 2 (cx + cy) psi_ij with cx = 1/dx^2,
 *   cy = 1/dy^2 (Eq. (2)/(11) with dy^2 under the y term).  The residual is
 *   r = f - L_h psi on interior nodes and 0 on the perimeter.
 * - Dense host-visible layout ("m x n row-major"): element (i, j) at offset
 *   j*m + i, FP64.  Every pointer passed to the library is a DEVICE pointer
 *   unless the parameter name ends in _host.
 * - Pitched device layout (the op-level calls, lap_op_*): element (i, j) at
 *   offset j*ld + i with ld >= m, ld a multiple of 64 elements, and the base
 *   256-byte aligned.  Columns m..ld-1 are padding: read, never used for a
 *   result, never written.
 * - All work is ordered on the HIP stream given to lap_ctx_create (or to the
 *   lap_op_* call).  Calls that return host-visible results synchronise that
 *   stream; the others only enqueue.
 * - Errors: every call returns a lap_status; on failure lap_last_error()
 *   returns a thread-local message.  No C++ exception crosses the ABI.
 *   HIP runtime failures map to LAP_EHIP with hipGetErrorString's text.
 */
#ifndef LAP_H
#define LAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lap_ctx lap_ctx;
typedef struct lap_grid lap_grid;

typedef enum lap_status {
    LAP_OK = 0,
    LAP_EINVAL = -1,      /* bad argument (sizes, spacings, omega, method, layout) */
    LAP_ENOMEM = -2,      /* the context's device arena cannot hold the request   */
    LAP_ENOTCONV = -3,    /* max_iter reached before the stopping rule held        */
    LAP_EDIVERGED = -4,   /* residual became NaN/Inf or grew by 1e6 over its start */
    LAP_EHIP = -5         /* a HIP runtime call failed                             */
} lap_status;

/* Methods (lap_solve). */
enum {
    LAP_SOR_RB = 1,  /* red-black SOR sweeps: colour (i+j) even, then odd (Eq. (7) reordered) */
    LAP_ADI = 2,     /* line ADI: all row systems, then all column systems, zebra order       */
    LAP_MG = 3,      /* multigrid V(nu1,nu2) cycles, red-black smoother, exact coarsest solve */
    /* The paper's sequential orderings, exactly (same update order and
     * expressions as the methods' definitions), for grids that fit one
     * workgroup's LDS (2 m n + 3 max(m, n) doubles: up to about 100 x 100 on
     * gfx950); the whole solve runs in one launch of one workgroup. */
    LAP_JACOBI = 4,  /* Jacobi, Eq. (5)                                                       */
    LAP_SOR_LEX = 5, /* lexicographic SOR, Eq. (7) (Gauss-Seidel, Eq. (6), at omega = 1)      */
    LAP_SLOR_LEX = 6,/* line SOR by rows, ascending: adi_form AFTER = SLORA (Eqs. (8)-(9)),
                      * INSIDE = SLORB (Eq. (10))                                             */
    LAP_ADI_LEX = 7  /* ADI: every row line ascending, then every column line ascending,
                      * relaxation placement by adi_form (ADI section)                        */
};

/* Precision (lap_solve, lap_grid_footprint). */
enum {
    LAP_FP64 = 0,    /* every kernel in FP64                                                  */
    LAP_MIXED = 1    /* MG only: FP32 V-cycle on the error equation, FP64 residual and update */
};

/* Stopping rules (lap_opts.stop). */
enum {
    LAP_STOP_REL_L2 = 0,   /* ||r_k||_2 / ||r_0||_2 < tol, r_0 at the start of the call */
    LAP_STOP_RES_INF = 1,  /* max |r_k| < tol (physical units of L_h)                   */
    LAP_STOP_DELTA = 2     /* max |psi^{k+1} - psi^k| < tol, Eq. (16) (LAP_JACOBI ..
                            * LAP_ADI_LEX only)                                         */
};

/* ADI relaxation placement (lap_opts.adi_form). */
enum {
    LAP_ADI_RELAX_AFTER = 0,  /* solve the line, then psi += w (psi~ - psi)     (SLORA, Eqs. (8)-(9)) */
    LAP_ADI_RELAX_INSIDE = 1  /* w folded into the line system (SLORB, Eq. (10)); needs w < 1 + beta^2 */
};

/* Multigrid smoother (lap_opts.smoother; "Multigrid Method (V-Cycle)" with
 * the line relaxation of the SLOR / ADI sections, Eqs. (8)-(9)). */
enum {
    LAP_SMOOTH_RB = 0,     /* red-black SOR sweeps; nu1 / nu2 count sweeps                     */
    LAP_SMOOTH_ZEBRA = 1   /* alternating zebra line relaxation: one smoothing step = odd rows,
                            * even rows, odd columns, even columns, each line solved exactly
                            * (relaxation after the solve with omega); nu1 / nu2 count steps
                            * (1, 1 is the usual choice).  Robust when dx != dy makes the
                            * operator anisotropic.  Every level's lines must fit the segmented
                            * line solver: sides of at most 4097 (LAP_EINVAL otherwise). */
};

/* Allocation flags (lap_grid_create_ex). */
enum {
    LAP_ALLOC_FP64 = 1,       /* FP64 multigrid hierarchy (LAP_MG with LAP_FP64) */
    LAP_ALLOC_MIXED = 2,      /* FP32 hierarchy for LAP_MIXED                    */
    LAP_ALLOC_ADI = 4,        /* line-solve scratch for LAP_ADI                  */
    LAP_ALLOC_ALL = 7
};

typedef struct lap_info {
    int32_t iterations;   /* sweeps (SOR), iterations (ADI), cycles (MG) or outer steps (MIXED) */
    int32_t status;       /* lap_status of the solve                                          */
    double rel_res_l2;    /* ||r||_2 / ||r_0||_2 of the returned psi                          */
    double res_l2;        /* ||r||_2 of the returned psi                                      */
    double res_linf;      /* max |r| of the returned psi                                      */
    double res0_l2;       /* ||r_0||_2 at the start of the call                               */
    double seconds;       /* wall time of the call, host clock                                */
    double monitor;       /* LAP_JACOBI .. LAP_ADI_LEX: the stopping rule's quantity after the
                           * last iteration (max update, max |r| or relative l2); else 0      */
} lap_info;

typedef struct lap_opts {
    int32_t method;       /* LAP_SOR_RB, LAP_ADI or LAP_MG                                 */
    int32_t precision;    /* LAP_FP64 or LAP_MIXED (MIXED requires LAP_MG)               */
    double omega;         /* SOR / ADI relaxation factor; MG smoother factor, in (0, 2)   */
    double tol;           /* stopping tolerance (rule in .stop); 0 runs exactly max_iter  */
    int32_t max_iter;     /* upper bound on iterations / cycles / outer steps             */
    int32_t stop;         /* LAP_STOP_REL_L2 or LAP_STOP_RES_INF                           */
    int32_t nu1, nu2;     /* MG pre- and post-smoothing sweeps (default 2, 2)             */
    int32_t check_every;  /* SOR/ADI: test the stopping rule every k iterations (>= 1)    */
    int32_t adi_form;     /* LAP_ADI_RELAX_AFTER or LAP_ADI_RELAX_INSIDE                  */
    int32_t use_graph;    /* MG: replay a captured hipGraph per cycle (1) or launch (0);
                           * a grid's graph is captured on its second solve with the same
                           * method options (its first solve launches directly)           */
    int32_t smoother;     /* MG: LAP_SMOOTH_RB or LAP_SMOOTH_ZEBRA                        */
    int32_t fmg;          /* MG, FP64, red-black smoother, one grid (lap_solve): 1 = start
                           * with one full-multigrid pass (the problem posed on every level
                           * with its boundary nodes and the full-weighted source, exact
                           * coarsest solve, bilinear interpolation of each coarse solution,
                           * one V-cycle per level); it counts as the first iteration, the
                           * stopping test's r_0 is the residual of the incoming field      */
    int32_t inner;        /* MIXED, red-black smoother (lap_solve, lap_solve_batch): FP32
                           * V-cycles per FP64 defect correction, 1..8 (default 1); the first
                           * starts from zero, each next from the previous correction.
                           * LAP_EINVAL outside 1..8 and for inner > 1 with FP64 or zebra
                           * smoothing (lap_batch_step always runs one cycle per step)      */
} lap_opts;

/* Fill *o with the defaults: MG, FP64, omega 1, tol 1e-10, max_iter 100,
 * REL_L2, nu1 = nu2 = 2, check_every 1, ADI relax-after, use_graph 1,
 * smoother LAP_SMOOTH_RB, fmg 0, inner 1. */
void lap_opts_default(lap_opts* o);

/* ---------------------------------------------------------------- context */

/* Create a context over a caller-owned device buffer `dev_arena` of
 * `arena_bytes` (>= 1 MiB, 256-byte aligned) that must outlive the context;
 * every grid allocation is carved from it (the library never calls hipMalloc
 * for grid data).  `hip_stream` (a hipStream_t, may be NULL = default
 * stream) orders all work.  The context is not thread-safe: use one per host
 * thread.  Errors: LAP_EINVAL on a NULL/unaligned/too-small arena. */
lap_status lap_ctx_create(void* dev_arena, size_t arena_bytes, void* hip_stream, lap_ctx** out);
lap_status lap_ctx_destroy(lap_ctx* ctx);   /* destroys remaining grids; the arena stays the caller's */

/* Bytes of arena in use and largest free block. */
lap_status lap_ctx_usage(lap_ctx* ctx, size_t* used, size_t* largest_free);

/* Timing of kernel launches (off by default).  on = 1: the library records a
 * pair of HIP events on its stream around every launch; on = 2: around the
 * finest-level launches only (the others are counted without events).  It
 * accumulates, per kernel class and for the finest level separately, the
 * launch count, the summed device time and the algorithmic bytes the launches
 * move (interior nodes x bytes per node of that kernel).  Solves run as with
 * timing off (steps enqueued ahead of the stopping test, no graph replay);
 * launches after the stopping test that ended a solve exit at once on the
 * device and are left out of the statistics.  Classes: 0 RB sweep, 1 RB sweep
 * with fused prolongation, 2 residual + full weighting, 3 defect correction
 * (FP64), 4 coarse solve, 5 norm finalise, 6 ADI row lines, 7 ADI column
 * lines, 8 residual, 9 small-level subtree (one launch per sub-V-cycle; its
 * bytes are the top level's right-hand side read and result written),
 * 10 fused pre-smoothing pass (one or two sweeps + residual + full
 * weighting), 11 fused two-sweep pass with the prolongation (post-smoothing),
 * 12 fused two-sweep pass without a transfer (red-black SOR, further
 * smoothing passes), 13 one whole solve of a paper-order method
 * (LAP_JACOBI .. LAP_ADI_LEX; no algorithmic bytes), 14 fused four-sweep pass
 * (a mixed step's FP32 cycle: the level-0 post-smoothing after the bilinear
 * correction, then the next cycle's pre-smoothing, residual and full
 * weighting).  Class 3 also holds the mixed loop's fused FP32
 * post-smoothing + FP64 defect pass.  `fine_only` selects the finest-level
 * bucket.
 * lap_ctx_kernel_stats synchronises the stream. */
lap_status lap_ctx_set_timing(lap_ctx* ctx, int32_t on);
lap_status lap_ctx_kernel_stats(lap_ctx* ctx, int32_t kernel_class, int32_t fine_only,
                                int64_t* launches, double* device_ms, double* alg_bytes);
lap_status lap_ctx_reset_stats(lap_ctx* ctx);

/* Tilings of the stencil kernels.  Each kernel class (as numbered above) has,
 * per dtype (0 FP64, 1 FP32) and per size class of the level (k = 0..7: the
 * level has fewer than 2^(12+2k) interior nodes, 7: 2^24 or more, so every
 * level of a (2^j + 1)-sided hierarchy has a class of its own;
 * lap_size_class), a tiling: V columns per lane (1, 2 or 4) and chunks of ty
 * rows (even, >= 2), or ty = 0 for chunks (of at least 16 rows) sized so a
 * launch has about target_waves wavefronts.  The tilings that produce norm
 * partials are fixed and not in this table.  Every tiling produces bitwise
 * identical fields; only speed differs. */
int32_t lap_size_class(int32_t m, int32_t n);
lap_status lap_ctx_set_tiling(lap_ctx* ctx, int32_t kernel_class, int32_t dtype, int32_t size_class,
                              int32_t V, int32_t ty, int32_t target_waves);
lap_status lap_ctx_get_tiling(lap_ctx* ctx, int32_t kernel_class, int32_t dtype, int32_t size_class,
                              int32_t* V, int32_t* ty, int32_t* target_waves);

/* Small-level subtree (the V-cycle of "Multigrid Method (V-Cycle)",
 * Eqs. (11)-(15), below a size): from the first zero-start level whose
 * remaining hierarchy (u and b of every level below it, plus the coarsest
 * right-hand side) fits one workgroup's LDS, the
 * rest of the V-cycle (pre-smoothing, full weighting, coarsest solve,
 * bilinear correction, post-smoothing on every level below) runs as ONE
 * launch of one workgroup (per grid, in a batch) instead of five launches per
 * level.  The result is bitwise the one of the multi-launch schedule.
 * max_nodes caps the subtree's top level at m*n nodes: -1 (default) = any
 * level that fits LDS, 0 = never use the subtree.  lap_ctx_get_subtree also
 * reports the LDS bytes one workgroup may use on this device.  Changing the
 * setting drops captured graphs and batch plans. */
lap_status lap_ctx_set_subtree(lap_ctx* ctx, int64_t max_nodes);
lap_status lap_ctx_get_subtree(lap_ctx* ctx, int64_t* max_nodes, int32_t* lds_bytes);

/* Fused smoothing passes (the V-cycle of "Multigrid Method (V-Cycle)",
 * Eqs. (11)-(15)): with fusion on (the default) a level's pre-smoothing
 * runs as passes of up to two red-black sweeps, the last of which also
 * forms the residual of its result and full-weights it onto the coarse
 * right-hand side, and the post-smoothing as
 * passes of up to two sweeps, the first of which adds the bilinear
 * correction; each pass reads and writes the level once.  The fields are
 * bitwise those of one launch per sweep (fusion off).  A level holding the
 * iterate keeps an even number of passes (one two-sweep pass is split when
 * needed).  Changing the setting drops captured graphs and batch plans. */
lap_status lap_ctx_set_fusion(lap_ctx* ctx, int32_t on);
lap_status lap_ctx_get_fusion(lap_ctx* ctx, int32_t* on);

/* Autotuner: time every candidate tiling (V in {1,2,4}; ty in {16,32,64,128};
 * auto with 1 or 2 device wave rounds) of the sweep, sweep+prolongation,
 * residual+restriction, residual, defect, fused pre-smoothing and fused
 * two-sweep kernels on scratch buffers of an
 * m x n level (odd m, n >= 5; carved from the arena and released), keep the
 * fastest per kernel class and dtype for that size class, and write a JSON
 * report of the choices into `report` (host buffer of report_bytes, may be
 * NULL).  `reps` timed launches per candidate.  Levels with arrays of 16 MB
 * or more are timed from a cold cache (a 512 MB copy through the arena before
 * each timed launch, when the arena can hold it; "cold_cache" in the report).
 * Synchronises the stream. */
lap_status lap_autotune(lap_ctx* ctx, int32_t m, int32_t n, int32_t reps, char* report, size_t report_bytes);

/* ------------------------------------------------------------------ grids */

/* Arena bytes a grid of m x n takes with the hierarchies of `alloc_flags`
 * (LAP_ALLOC_*), so a scheduler can admit requests by footprint. */
size_t lap_grid_footprint(int32_t m, int32_t n, int32_t alloc_flags);

/* Create a grid: m, n >= 3; dx, dy > 0 and finite.  `psi0` (device, FP64,
 * m x n row-major) holds the Dirichlet data on its perimeter and the initial
 * guess inside; `source` (device, FP64, m x n row-major) is f, or NULL for
 * f = 0 (Laplace).  Both are copied into the grid's device-resident storage
 * (stream-ordered; the caller may reuse them after the next synchronising
 * call).  The multigrid hierarchy coarsens while both sides are odd and stay
 * >= 5 (m_{l+1} = (m_l - 1)/2 + 1); the coarsest level must have at most
 * 1024 interior nodes (choose sizes c*2^k+1), else an explicit
 * LAP_ALLOC_FP64 / LAP_ALLOC_MIXED request fails with LAP_EINVAL while
 * LAP_ALLOC_ALL ("everything this grid supports") quietly leaves the
 * multigrid hierarchies out.  lap_grid_create allocates LAP_ALLOC_ALL. */
lap_status lap_grid_create(lap_ctx* ctx, int32_t m, int32_t n, double dx, double dy,
                           const double* psi0, const double* source, lap_grid** out);
lap_status lap_grid_create_ex(lap_ctx* ctx, int32_t m, int32_t n, double dx, double dy,
                              const double* psi0, const double* source, int32_t alloc_flags,
                              lap_grid** out);
lap_status lap_grid_destroy(lap_grid* g);

/* Copy the current solution (FP64, m x n row-major, perimeter included) to
 * the caller's device buffer `dst` (stream-ordered, no synchronisation). */
lap_status lap_grid_read(lap_grid* g, double* dst);

/* Replace the solution with `psi` (device, FP64, m x n row-major): new
 * boundary data and a new initial guess.  Stream-ordered. */
lap_status lap_grid_write(lap_grid* g, const double* psi);

/* Number of multigrid levels and the size of level l. */
lap_status lap_grid_levels(lap_grid* g, int32_t* nlevels);
lap_status lap_grid_level_shape(lap_grid* g, int32_t l, int32_t* m, int32_t* n);

/* ------------------------------------------------------------------ solve */

/* Solve with `method` (LAP_SOR_RB, LAP_ADI, LAP_MG) and `precision` until
 * ||r||_2/||r_0||_2 < tol or max_iter iterations; the solution stays resident
 * and a second call continues from it.  omega: the SOR/ADI factor, or the MG
 * smoother factor, in (0, 2).  Returns LAP_OK, LAP_ENOTCONV (info filled),
 * LAP_EDIVERGED, or LAP_EINVAL (omega outside (0,2), MIXED with a method
 * other than MG, or a hierarchy the grid was created without).
 * Synchronises the stream.  `info` may be NULL. */
lap_status lap_solve(lap_grid* g, int32_t method, double omega, double tol, int32_t max_iter,
                     int32_t precision, lap_info* info);
lap_status lap_solve_ex(lap_grid* g, const lap_opts* opts, lap_info* info);

/* FP64 residual of the current solution: ||r||_2 relative to the r_0 of the
 * last solve call (or to itself if none) and max |r|.  Synchronises. */
lap_status lap_residual(lap_grid* g, double* l2_rel, double* linf);
lap_status lap_residual_ex(lap_grid* g, double* l2, double* linf);

/* ------------------------------------------------------------------ batch */

/* Solve `count` grids of one context together.  Grids are advanced in
 * lockstep: each step runs one cycle (MG; a mixed step its opts->inner FP32
 * cycles, or one where the step's test predicts one is enough, chosen per
 * grid on the device) or one iteration (ADI/SOR) of every grid that has not
 * yet met its stopping rule, with the launches of all grids
 * of one level merged into one persistent launch over a tile table.  Each
 * grid's arithmetic is the same as in a lap_solve_ex of that grid alone.
 * infos[k] (may be NULL) receives grid k's result.  Returns LAP_OK if all
 * converged, else the first failing status. */
lap_status lap_solve_batch(lap_ctx* ctx, lap_grid* const* grids, int32_t count,
                           const lap_opts* opts, lap_info* infos);

/* One scheduling tick for continuous batching: advance every listed grid by
 * `steps` (>= 1) outer steps (MG cycle / mixed outer step) with merged
 * per-level launches, enqueued back to back, then read every grid's control
 * block once.  A grid whose stopping rule holds during the tick stops there
 * (its later launches exit on the device), so each grid's iterate sequence
 * is the same for any `steps`; more steps per tick mean fewer host round
 * trips.  A grid already done is left unchanged and reports done.  tol per
 * grid is taken from lap_grid_set_tol (default 1e-10), the smoother's
 * relaxation from lap_grid_set_omega (default 1).  done_host[k] (host array)
 * is set to 1 when grid k has converged or failed. */
lap_status lap_batch_step(lap_ctx* ctx, lap_grid* const* grids, int32_t count,
                          int32_t precision, int32_t steps, int32_t* done_host, lap_info* infos);
lap_status lap_grid_set_tol(lap_grid* g, double tol);
/* Relaxation of the red-black multigrid smoother in the grid's batched steps
 * (the omega of LAP_MG, as in "Successive over relaxation", Eq. (7)): default 1
 * (Gauss-Seidel); LAP_EINVAL unless 0 < omega < 2.  Takes effect when the
 * grid's batched solve starts (after lap_grid_reset or a finished solve). */
lap_status lap_grid_set_omega(lap_grid* g, double omega);
/* Restart the stopping test of a grid (r_0 is re-taken at its next step). */
lap_status lap_grid_reset(lap_grid* g);

/* ------------------------------------------------------------- op level */
/*
 * Single-kernel entry points on caller-owned pitched device arrays (layout
 * in the header comment), for users who drive their own schedule and for
 * kernel-level parity checks.  dtype: 0 = FP64, 1 = FP32.  `stream` is a
 * hipStream_t (NULL = default).  All are stream-ordered and do not
 * synchronise.  Errors: LAP_EINVAL for m or n < 3, non-positive spacings,
 * ld not a multiple of 64 or < m, or a misaligned pointer.
 */

/* One red-black SOR sweep (colour (i+j) even, then odd), out of place: reads
 * u_in (and f, NULL = 0), writes the interior of u_out; u_out's perimeter is
 * not touched (keep it equal to u_in's).  If ec != NULL the sweep starts
 * from u_in + P(ec), the bilinear interpolation of the coarse correction ec
 * ((m-1)/2+1 x (n-1)/2+1, pitch ldc, zero perimeter) — the multigrid
 * correction step fused into the first post-smoothing sweep.  u_in may be
 * NULL: the sweep then starts from zero (also on the perimeter). */
lap_status lap_op_rb_sweep(int32_t dtype, int32_t m, int32_t n, int32_t ld, double dx, double dy,
                           double omega, const void* u_in, const void* f, const void* ec, int32_t ldc,
                           void* u_out, void* stream);

/* Residual r = f - L_h u (f NULL = 0): writes r (interior; r's perimeter is
 * not touched) if r != NULL, and if norms != NULL writes norms[0] = sum r^2,
 * norms[1] = max |r| over the interior (FP64, device).  `work` must hold
 * lap_op_work_bytes(m, n) bytes of device memory. */
lap_status lap_op_residual(int32_t dtype, int32_t m, int32_t n, int32_t ld, double dx, double dy,
                           const void* u, const void* f, void* r, double* norms, void* work, void* stream);
size_t lap_op_work_bytes(int32_t m, int32_t n);

/* lap_op_residual without a work buffer, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the per-tile norm partials go to a fixed
 * 1 MiB device array of the library (one per GPU, held until the process
 * ends; its address is looked up once per device on the first call, the only
 * call that is not purely stream-ordered).  The call allocates nothing.
 * Arguments, layout and results are those of lap_op_residual; the kernels
 * are the same, so r and norms are bitwise equal to it.  Limit: at most
 * 65536 norm tiles (windows of 124 FP64 / 252 FP32 columns x chunks of 32
 * rows; square grids up to 16121^2 in FP64, 22931^2 in FP32; 8193^2 FP64
 * uses 17152); larger grids are rejected with LAP_EINVAL when norms != NULL,
 * before anything is enqueued.
 * All calls on one GPU share the array: calls that overlap on that GPU (on
 * different streams, or from different host threads) race and may return
 * each other's norms; serialise them. */
lap_status lap_op_residual_static(int32_t dtype, int32_t m, int32_t n, int32_t ld, double dx, double dy,
                                  const void* u, const void* f, void* r, double* norms, void* stream);

/* Residual followed by full weighting onto the coarse grid: writes the
 * interior of bc ((m-1)/2+1 x (n-1)/2+1, pitch ldc); m and n must be odd. */
lap_status lap_op_restrict(int32_t dtype, int32_t m, int32_t n, int32_t ld, double dx, double dy,
                           const void* u, const void* f, void* bc, int32_t ldc, void* stream);

/* One ADI half-iteration in zebra order: rows (dir 0: odd rows j, then even)
 * or columns (dir 1: odd columns i, then even), each line's tridiagonal
 * system (SLOR / ADI sections, Eqs. (8)-(10)) solved by Gaussian elimination
 * without pivoting, relaxation placement `form`.  Lines of up to 4095
 * unknowns are solved in parallel blocks of 15 unknowns coupled through a
 * reduced system over the block separators (equal to the sequential Thomas
 * recurrence up to rounding); longer lines by the sequential recurrence.
 * In place on u (FP64 only: dtype must be 0).  `work` must hold
 * lap_op_work_bytes(m, n) bytes.  The line tables are copied from the host
 * into `work` first; the call waits for that copy (a stream synchronisation),
 * then enqueues the two launches. */
lap_status lap_op_adi_half(int32_t dtype, int32_t m, int32_t n, int32_t ld, double dx, double dy,
                           double omega, int32_t dir, int32_t form, void* u, const void* f,
                           void* work, void* stream);

/* Plain streaming copy of `bytes` (a multiple of 16; 16-byte aligned
 * pointers) from src to dst with `blocks` workgroups of 256 threads: the
 * achievable-bandwidth reference for roofline figures and the calibration
 * kernel for hardware byte counters.  Stream-ordered. */
lap_status lap_op_stream_copy(const void* src, void* dst, size_t bytes, int32_t blocks, void* stream);

/* ---------------------------------------------------------------- errors */
const char* lap_last_error(void);
/* Library version string. */
const char* lap_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LAP_H */
