// Internal interface between the liblap runtime and its gfx950 kernels.
//
// Data layout of a field on one level: element (i, j) at ptr[j * P + i] with
// the pitch P a multiple of 64 elements and the base 256-byte aligned; the
// perimeter (i = 0, m-1 or j = 0, n-1) holds Dirichlet data (zero on coarse
// levels and for corrections).  Columns m..P-1 are padding.
//
// Stencil kernels are "streaming-window" kernels: one 64-lane wavefront owns
// a window of 64*V consecutive columns (V per lane, one vector load per lane
// and row) and a chunk of `ty` rows, marches down the chunk keeping a few
// rows in registers, and exchanges the left/right neighbours of its lanes
// with cross-lane shuffles.  Windows overlap by 4 columns (2 halo columns on
// each side), so a wave needs no LDS and no barrier; the overlap re-reads
// hit L2.  All kernels are out of place, so a wave's halo rows are never
// being written by a neighbour.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace lap {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kXcds = 8;          // MI355X: workgroups are dealt round-robin over 8 XCDs

// Window geometry for V columns per lane and a halo of H columns on each
// side (columns a window reads but does not own: 2 per red-black sweep fused
// into one pass, 2 more for a fused residual + full weighting): step between
// windows and the left offset of window 0 (keeps every vector load V-aligned).
__host__ __device__ constexpr int win_step(int V, int H = 2) { return 64 * V - 2 * H; }
__host__ __device__ constexpr int win_left(int V, int H = 2) { return (H + V - 1) / V * V; }

struct Tiling {
    int V = 2;       // columns per lane
    int ty = 64;     // rows per chunk (even)
    int nwin = 0;    // windows across
    int nchunk = 0;  // chunks down
    int ntiles = 0;  // nwin * nchunk (one wavefront each)
    int H = 2;       // halo columns per side
};

// Halo of the canonical norm tiling: wide enough for a fused pass of two
// sweeps and a residual + full weighting.
constexpr int kNormH = 6;
// Waves the canonical tiling of the stencil passes aims at.  On 8193^2 the
// finest pre-smoothing pass took 259 us with 16384 waves (36-row chunks),
// 252 us with 32768 (18 rows), 267 us with 49152 or 65536: halo rows shared
// by neighbouring chunks come from L2, so shorter chunks pay little and
// buy parallelism, up to a point.  Below ~6000 rows the 16-row minimum
// decides instead.
constexpr int kNormWaves = 32768;

// Tiling of an m x n level with V columns per lane.  ty > 0: chunks of ty
// rows.  ty == 0: size the chunks so the launch has about `target` waves
// (one full occupancy round of the device when target = its wave capacity),
// which avoids a nearly empty last round.  Chunks are never shorter than 16
// rows, which bounds the number of tiles (and norm partials) of a level.
inline Tiling make_tiling(int m, int n, int V, int ty, int target = 0, int H = 2, int min_rows = 16) {
    Tiling t;
    t.V = V;
    t.H = H;
    const int S = win_step(V, H), L = win_left(V, H);
    // outputs of window w: columns [w*S - L + H, w*S - L + 64V - H); need to reach m-2
    int nw = 1;
    while ((nw - 1) * S - L + 64 * V - H - 1 < m - 2) ++nw;
    t.nwin = nw;
    const int rows = n - 2 > 0 ? n - 2 : 1;
    if (ty <= 0) {
        int chunks = target > 0 ? target / nw : 1;
        if (chunks < 1) chunks = 1;
        ty = (rows + chunks - 1) / chunks;
        ty += ty & 1;
        if (ty < min_rows) ty = min_rows;
    }
    t.ty = ty;
    t.nchunk = (rows + ty - 1) / ty;
    if (t.nchunk < 1) t.nchunk = 1;
    t.ntiles = t.nwin * t.nchunk;
    return t;
}

// Fixed tiling of every kernel that produces norm partials (the first
// pre-sweep with norms, residual norms, the FP64 defect correction): the
// partial sums, and so the stopping decisions, then do not depend on the
// tuning table or on whether the grid runs alone or inside a batch.
// Canonical tilings by producer: the stencil passes (sweeps with norms,
// fused pre-smoothing, residual norms), the FP64 defect correction of the
// mixed loop, and the fused FP32 post-smoothing + FP64 defect pass (halo of
// two sweeps and the residual); a norm finalisation reduces the partials of
// the kind that produced them.
enum NormKind { NORM_PASS = 0, NORM_DEFECT = 1, NORM_POSTDEF = 2 };
// The defect pass keeps chunks of >= 64 rows on levels of more than 257
// rows, >= 16 below.  Grids whose whole FP32 cycle fits one workgroup's LDS
// (up to ~15k nodes) take this pass at every outer step; in a batch they
// share a launch that the row walk of their chunks makes latency-bound
// (64-row chunks: ~67 us per launch; 16-row chunks: 512-grid batch
// 15.9 -> 15.4 ms).
constexpr int kDefectMinRows = 64;
constexpr int kDefectShortRowsN = 257;
// The post-smoothing + defect pass reads 2 * 2 + 1 halo rows above and below
// each chunk: chunks of >= 64 rows up to 4097 rows (faster by 4% at 4097^2,
// and by far in batches of small grids), of >= 16 rows beyond (the 16384
// waves' chunks of 8193^2 are 36 rows; 64-row chunks were 1.5% slower).
constexpr int kPostDefShortRowsN = 4097;
// Levels of at most this many rows take the post-smoothing + defect pass's
// norms per (window, block of 16 rows): one grid alone then walks 16-row
// chunks (4x the waves of 64-row chunks: mixed solves of 129^2 / 257^2 /
// 513^2 / 1025^2 grids 0.91 / 1.06 / 1.21 / 1.38 -> 0.62 / 0.73 / 0.85 /
// 1.03 ms) while merged batch launches keep 64-row chunks (a 512-grid batch
// with 16-row chunks: 15.4 -> 16.0 ms; with the block partials 15.6 ms),
// and both reduce the same partials in the same order.
constexpr int kRowPartN = 1025;
constexpr int kRowBlock = 16;
inline bool postdef_rowpart(int n) { return n <= kRowPartN; }
__host__ __device__ inline int row_blocks(int n) { return (n - 2 + kRowBlock - 1) / kRowBlock; }
// Columns per lane of the stencil passes' and the defect correction's
// canonical tilings (the merged batch kernels of the residual norms and the
// defect correction are compiled for these only).
constexpr int kNormPassV = 2;
constexpr int kNormDefectV = 1;
inline Tiling norm_tiling(int m, int n, int kind = NORM_PASS) {
    if (kind == NORM_DEFECT)
        return make_tiling(m, n, kNormDefectV, 0, 16384, 2, n <= kDefectShortRowsN ? 16 : kDefectMinRows);
    if (kind == NORM_POSTDEF) return make_tiling(m, n, 2, 0, 16384, kNormH, n > kPostDefShortRowsN ? 16 : 64);
    return make_tiling(m, n, kNormPassV, 0, kNormWaves, kNormH);
}
// Tiling of the post-smoothing + defect pass alone or in a merged launch.
inline Tiling postdef_tiling(int m, int n, bool merged) {
    if (postdef_rowpart(n)) return make_tiling(m, n, 2, merged ? 4 * kRowBlock : kRowBlock, 0, kNormH);
    return norm_tiling(m, n, NORM_POSTDEF);
}
// Norm partials a finalisation of this kind reduces.
inline int norm_partials(int m, int n, int kind) {
    const Tiling t = norm_tiling(m, n, kind);
    if (kind == NORM_POSTDEF && postdef_rowpart(n)) return t.nwin * row_blocks(n);
    return t.ntiles;
}

// Blocks of 4 waves; the grid is padded to a multiple of the XCD count so
// the XCD-aware remap below is a bijection.
inline int xcd_pad(int nb) { return ((nb + kXcds - 1) / kXcds) * kXcds; }
inline int blocks_for(const Tiling& t) { return xcd_pad((t.ntiles + kWavesPerBlock - 1) / kWavesPerBlock); }

// Kernel-side control block of one solve (device memory).
struct Ctrl {
    double r0;          // ||r_0||_2 of this solve
    double rel;         // last ||r||_2 / r0
    double res_l2;      // last ||r||_2
    double res_inf;     // last max|r|
    double tol;         // stopping tolerance
    int32_t stop;       // 0: rel l2, 1: max-abs
    int32_t max_iter;
    int32_t iters;      // iterations completed on the iterate that was last tested
    int32_t checks;     // number of norm finalisations so far in this solve
    int32_t done;       // nonzero: stop; every kernel of the solve becomes a no-op
    int32_t status;     // lap_status when done
    int32_t step;       // iterations between two tests (SOR / ADI check interval)
    int32_t cycles;     // mixed steps with several FP32 cycles: cycles the last step runs
};

// Flags of the red-black sweep.
enum : int {
    SW_F = 1,        // source / right-hand side present
    SW_ZERO = 2,     // input is identically zero (u_in ignored)
    SW_PROLONG = 4,  // input is u_in + P(ec)
    SW_NORM = 8,     // accumulate residual norms of the input into partials
    SW_RESTRICT = 16,// fused pass: residual + full weighting of the result into bc
    SW_TWO = 32,     // fused pass: two sweeps
    SW_DEF = 64,     // fused FP32 post-smoothing pass (with SW_PROLONG | SW_TWO | SW_F) whose result, the
                     // correction, goes straight into the next FP64 defect correction (psi_in -> psi_out,
                     // the residual's norms, its FP32 copy into rhs_out); the correction is not stored
    SW_PONLY = 128,  // with SW_PROLONG: only u_in + P(ec), no colour updates (u_out may equal u_in:
                     // every stored value depends on its own node only); the multigrid correction
                     // step when the smoother is zebra line relaxation
    SW_PROBE = 256,  // with SW_NORM: the input's residual norms only, exactly as the pass with the
                     // other flags computes them (same tiles, walk and order); nothing is stored
    SW_RDIFF = 512,  // with SW_RESTRICT: the residual in difference form, cx ((W - C) + (E - C)) +
                     // cy ((S - C) + (N - C)), accurate for a smooth iterate of large values (an FP32
                     // cycle that continues from a correction)
    SW_FOUR = 1024,  // fused pass: four sweeps (a cycle's two post-smoothing sweeps after its bilinear
                     // correction, then the next cycle's two pre-smoothing sweeps, residual and full
                     // weighting: SW_PROLONG | SW_RESTRICT)
};

template <typename T>
struct SweepArgs {
    const T* uin;
    T* uout;
    const T* f;
    const T* ec;        // coarse correction (SW_PROLONG)
    T* bc;              // coarse right-hand side (SW_RESTRICT)
    double* partials;   // 2 doubles per tile (SW_NORM)
    const Ctrl* ctrl;   // nullable: kernel returns at once if ctrl->done
    int m, n, P;
    int mc, nc, Pc;
    // row strides of (uin, uout, f) and of (ec, bc) as the tile sees them:
    // 0 = P / Pc; the fused kernels walk some chunks through a vertically
    // flipped view (base at the last row, stride -P)
    int Ps, Pcs;
    T cx, cy, d, inv_d, omega;
    Tiling tl;
    // SW_DEF: the FP64 iterate, its update, the FP64 source and the next FP32 right-hand side
    const double* psi_in;
    double* psi_out;
    const double* f64;
    T* rhs_out;
    double dcx, dcy, dd;
    int nt;             // nonzero: the pass's row stores are nontemporal (streamed past the caches)
    // SW_DEF with rowpart: chunks of a multiple of kRowBlock rows walk downwards and the norm
    // partials are per (window, block of kRowBlock rows), at win * row_blocks(n) + (row - 1) /
    // kRowBlock, instead of per tile: the same sums whatever the chunk length (rp_off: set by the kernel)
    int rowpart, rp_off;
};

template <typename T>
struct RestrictArgs {
    const T* u;
    const T* f;
    T* bc;
    T* uc0;             // nullable: coarse iterate set to zero at every coarse interior node (zero start)
    const Ctrl* ctrl;
    int m, n, P;
    int mc, nc, Pc;
    T cx, cy, d;
    Tiling tl;
    int rdiff;          // nonzero: the residual in difference form (as SW_RDIFF)
};

template <typename T>
struct ResidualArgs {
    const T* u;
    const T* f;
    T* r;               // nullable
    double* partials;   // nullable
    const Ctrl* ctrl;
    int m, n, P;
    T cx, cy, d;
    Tiling tl;
};

// FP64 defect correction: psi_out = psi_in + e (e nullable), r = f - L psi_out,
// rhs = fl32(r) on the interior, norms of r.
struct DefectArgs {
    const double* psi_in;
    double* psi_out;
    const float* e;
    const double* f;
    float* rhs;
    float* ezero;       // nullable: FP32 level-0 buffer set to zero at every interior node (next cycle's start)
    double* partials;
    const Ctrl* ctrl;
    int m, n, P;
    double cx, cy, d;
    Tiling tl;
};

template <typename T>
struct CoarseArgs {
    const T* u;         // boundary source (level 0) or nullptr (zero boundary)
    const T* b;         // right-hand side (nullable = 0)
    T* out;             // solution (interior written)
    const double* minv; // dense: (N x N) inverse of L_h on the interior unknowns, FP64, symmetric
                        // lines: the short-side sine transform (p x p), then per mode the
                        // Thomas factors c' and 1/pivot (q each) along the long side
    double* work;       // lines: N doubles of FP64 scratch (the mode coefficients)
    const Ctrl* ctrl;
    int m, n, P;
    double cx, cy;
    int bw;             // 0: dense inverse; > 0: separable solve, p = the short interior side
    int ifast;          // separable solve: 1 = the short side runs along x (i), 0 = along y
};

// The small-level tail of a V-cycle run by one workgroup with every level
// resident in LDS: from a zero-start level (the subtree's top) down to the
// coarsest and back (nu1 sweeps, full weighting, recursion, exact coarsest
// solve, bilinear correction, nu2 sweeps).  Only the top level's right-hand
// side is read from HBM and only its result is written back; the levels
// below it are internal to one launch.
constexpr int kMaxSub = 16;
constexpr int kSubBlock = 1024;

template <typename T>
struct SubLevel {
    int m, n;          // level size (LDS pitch m)
    int ou, ob;        // LDS offsets (elements of T) of the level's u and b
    T cx, cy, d, inv_d;
};

template <typename T>
struct SubtreeArgs {
    T* out;              // top-level result, HBM, pitch P (boundary written as 0)
    const T* b;          // top-level right-hand side, HBM, pitch P (nullable = 0)
    int P;
    int nlev, nu1, nu2;
    T omega;
    int lds_elems;       // elements of T for all levels' u and b
    int lds_bytes;       // dynamic LDS of the launch (levels + coarse rhs)
    const double* minv;  // coarsest factor (dense inverse or separable), see CoarseArgs
    double* work;
    int bw, ifast;
    double ccx, ccy;     // coarsest-level coefficients in FP64
    const Ctrl* ctrl;
    SubLevel<T> lv[kMaxSub];
};

// ---- launchers (stencil_kernels.hip) ----
template <typename T> hipError_t launch_sweep(const SweepArgs<T>& a, int flags, hipStream_t s);
template <typename T> hipError_t launch_restrict(const RestrictArgs<T>& a, hipStream_t s);
template <typename T> hipError_t launch_residual(const ResidualArgs<T>& a, hipStream_t s);
template <typename T> hipError_t launch_coarse(const CoarseArgs<T>& a, hipStream_t s);
hipError_t launch_defect(const DefectArgs& a, hipStream_t s);
template <typename T> hipError_t launch_subtree(const SubtreeArgs<T>& a, hipStream_t s);
// fused streaming pass (fused_kernels.hip): one or two sweeps (SW_TWO), input
// zero / + prolongation / with norms, result optionally restricted (SW_RESTRICT)
template <typename T> hipError_t launch_fused(const SweepArgs<T>& a, int flags, hipStream_t s);
// merged subtree launch: one workgroup per item, items[k].sub -> SubtreeArgs<T> in device memory
hipError_t launch_batch_subtree(int dt, const struct BatchItem* items, int count, int lds_bytes, hipStream_t s);
// allow dynamic LDS up to `bytes` for the subtree kernels (once per device)
hipError_t subtree_set_lds_limit(int bytes);
// Sum the per-tile partials in a fixed order and run the stopping test.
// mode 0: stopping test of a solve; mode 1: write norms only (out2 = {sum, max});
// mode 2: a probe of the test the next step opens with: recorded (and the
// solve stopped) only if it ends the solve, else the control block is left
// as it was.
// gate: when not null, the launch does nothing while gate->done is set (a
// finalisation of one of two alternative step openings).
// cyc (mode 0, mixed steps of up to `cycles & 255` FP32 V-cycles): after the
// test, choose how many cycles the step runs, one or all, and write the
// choice into the gate pair cyc[2 p], cyc[2 p + 1] (p = cycles >> 8):
// cyc[2 p].done is set when the step runs one cycle (it gates the cycles
// after the first and the next step's opening that finishes the last of
// them), cyc[2 p + 1].done when it runs all (it gates the next step's
// opening after a one-cycle step).  A test that ends the solve sets the done
// flags of all four.  One cycle is chosen when, with the per-cycle factor
// rho = (q / q_prev)^(1 / c) of the previous step's c cycles, 1.5 q rho < tol
// (q: the test's quantity; never on the first test).
hipError_t launch_finalize(const double* partials, int ntiles, Ctrl* ctrl, double* out2, int mode,
                           hipStream_t s, const Ctrl* gate = nullptr, Ctrl* cyc = nullptr, int cycles = 0);
// Reset a control block for a new solve (stream-ordered, graph-safe).
hipError_t launch_ctrl_init(Ctrl* ctrl, double tol, int stop, int max_iter, int step, hipStream_t s);
// The same for `count` control blocks (device array of pointers).
hipError_t launch_ctrl_init_many(Ctrl* const* ctrls, int count, double tol, int stop, int max_iter, int step,
                                 hipStream_t s);
// Gather the control blocks of a batch of grids into one array.
hipError_t launch_gather_ctrl(Ctrl* const* src, Ctrl* dst, int count, hipStream_t s);
// Streaming copy of `bytes` (a multiple of 16) with `blocks` workgroups.
hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, int blocks, hipStream_t s);
// Dense m x n FP64 field (row pitch m) into pitched fields d0 and (if not NULL) d1.
hipError_t launch_write_field(const double* src, double* d0, double* d1, int m, int n, int P, hipStream_t s);
// Copies of whole buffers (16-byte vectors), one launch for all of them.
struct CopyItem {
    const double2* src;
    double2* dst;
    size_t nvec;
};
hipError_t launch_copy_many(const CopyItem* items, int count, hipStream_t s);
// Copy interior of src into dst (FP64 fields of the same layout).
hipError_t launch_copy(const double* src, double* dst, int m, int n, int P, const Ctrl* ctrl,
                       hipStream_t s);

// Perimeter of a level's buffers d0 (and d1, nullable): the finest level's
// Dirichlet data src (pitch Ps) at every stride-th node, or zero if src is NULL.
hipError_t launch_level_boundary(double* d0, double* d1, const double* src, int m, int n, int P, int Ps, int stride,
                                 const Ctrl* ctrl, hipStream_t s);

// ---- the paper's sequential orderings in one workgroup (paper_kernels.hip) ----
struct PaperArgs {
    double* u;               // the grid (pitched, perimeter = Dirichlet data), in and out
    const double* f;         // nullable
    Ctrl* ctrl;              // iterations, done, status, last monitored quantity (rel), r0
    int m, n, P;
    double cx, cy, d, inv_d, omega;
    int method;              // LAP_JACOBI, LAP_SOR_LEX, LAP_SLOR_LEX, LAP_ADI_LEX
    int form;                // line methods: 0 relaxation after the solve, 1 inside
    int stop;                // LAP_STOP_DELTA, LAP_STOP_RES_INF or LAP_STOP_REL_L2
    double tol;
    int max_iter;
};
size_t paper_lds_bytes(int m, int n);
hipError_t paper_set_lds_limit(int bytes);
hipError_t launch_paper(const PaperArgs& a, hipStream_t s);

// ---- ADI (adi_kernels.hip) ----
// T: element type of the field (the sequential solver is FP64 only; the
// segmented one is also built for FP32, for line smoothing in the FP32 cycle)
template <typename T>
struct LineArgsT {
    T* u;                    // in place
    const T* f;              // nullable
    double* scratch;         // forward-sweep values, same layout as u (sequential solver)
    const double* cprime;    // c'_k of the constant-coefficient factorisation, k = 0..K-1
    const double* piv;       // pivot_k (piv_0 = d)
    const Ctrl* ctrl;
    int m, n, P;
    double cx, cy, d, omega;
    double a_off;            // off-diagonal of the line matrix (-cx or -w cx, rows; -cy.. cols)
    int form;                // 0 relax after, 1 relax inside
    int parity;              // 1: odd lines, 0: even lines
    const T* seg;            // segment table of this direction (adi_seg_table), or NULL
};
using LineArgs = LineArgsT<double>;
constexpr int kRowTile = 64;   // row lines per ADI row block (sequential solver)
hipError_t launch_adi_rows(const LineArgs& a, hipStream_t s);
hipError_t launch_adi_cols(const LineArgs& a, hipStream_t s);
// One zebra line-smoothing half inside a V-cycle: all lines of a.parity along
// rows (dir 0) or columns (dir 1), segmented solver only (every line must
// fit it: hipErrorInvalidValue otherwise), in place on a.u.
template <typename T>
hipError_t launch_zebra_lines(const LineArgsT<T>& a, int dir, hipStream_t s);

// Segmented line solver.  A line of K unknowns is cut into S blocks of
// kSegL unknowns, each followed by one separator unknown (the last block
// holds the remaining 0..kSegL).  Every block is solved on its own with zero
// end values (one thread per block, values kept in registers); the block
// solutions enter a reduced tridiagonal system over the S-1 separators,
// solved per line; each block then adds the responses to its two separator
// values.  The line matrix is constant along the line, so the block factors,
// the response vectors and the reduced system's factors depend only on
// (K, d, E) and are tabulated once per solve on the host.
constexpr int kSegL = 15;
constexpr int kSegMaxS = 256;
constexpr int kSegColMaxS = 256;       // columns: S <= 256 as rows (4 or more lines per workgroup)
// table layout (doubles)
constexpr int SEG_IPIV = 0;                       // 1/pivot_k of a block, k < kSegL
constexpr int SEG_CQ = kSegL;                     // E/pivot_k
constexpr int SEG_G = 2 * kSegL;                  // response of a full block to a unit left value
constexpr int SEG_GL = 3 * kSegL;                 // the same for the last block
constexpr int SEG_IPIVR = 4 * kSegL;              // reduced system: 1/pivot_p
constexpr int SEG_CQR = 4 * kSegL + kSegMaxS;     // reduced system: E_R/pivot_p
constexpr int SEG_E = 4 * kSegL + 2 * kSegMaxS;   // E, E_R
constexpr int kSegTab = SEG_E + 2;
__host__ __device__ constexpr int seg_count(int K) { return K <= 0 ? 0 : (K + kSegL + 1) / (kSegL + 1); }
// Workgroup sizes: rows stage their lines in LDS (8.5 bytes per unknown), so
// small workgroups keep several resident per CU; columns keep 8 or more
// lines per workgroup so a wavefront's row accesses stay contiguous.
// Size code c of a line length: rows use 128 << c threads (c = 0, 1),
// columns 256 << c (c = 0 for lines of at most 4 blocks, else 2: 1024
// threads, 4 or more lines per workgroup).
__host__ __device__ constexpr int seg_code(int dir, int K) {
    return dir == 0 ? (seg_count(K) <= 128 ? 0 : 1) : (seg_count(K) <= 4 ? 0 : 2);
}
__host__ __device__ constexpr int seg_threads(int dir, int code) { return (dir == 0 ? 128 : 256) << code; }
// lines per workgroup of the segmented kernels (one thread per block of a line)
__host__ __device__ constexpr int seg_lines(int dir, int K) {
    return seg_threads(dir, seg_code(dir, K)) / seg_count(K);
}
// q / d for 0 <= q < 2^20, 1 <= d <= 2^12, through single precision: the
// quotient's fractional part is at least 0.5 / d away from an integer, far
// above the rounding error
__device__ __forceinline__ int seg_div(int q, float inv_d) { return (int)(((float)q + 0.5f) * inv_d); }
__host__ __device__ constexpr bool seg_fits(int dir, int K) {
    return K >= 1 && seg_count(K) <= (dir == 0 ? kSegMaxS : kSegColMaxS);
}
// Tabulate the segmented solve of the line matrix tridiag(-E, D, -E) of
// order K (host, extended precision).
void adi_seg_table(double D, double E, int K, double* tab);
void adi_seg_table(double D, double E, int K, float* tab);   // the same, rounded once to FP32

// Coarsest levels with at most this many unknowns use a dense inverse (all
// lanes in parallel); larger ones (long thin grids) a separable solve: sine
// transform along the short side, a tridiagonal solve per mode along the long.
constexpr int kDenseCoarseMax = 256;

// ---- merged ragged-batch launches (batch_kernels.hip) ----
// One grid's share of a merged launch: the arguments of the single-grid
// kernel plus its tiling and the offset of its first tile in the launch.
struct BatchItem {
    const void* in;          // sweep input / residual u / defect psi_in / coarse boundary source
    void* out;               // sweep / coarse output, defect psi_out
    const void* f;           // right-hand side
    const void* ec;          // sweep: coarse correction; defect: FP32 correction
    void* bc;                // restrict: coarse right-hand side; defect: FP32 rhs
    const double* minv;      // coarse solve (dense inverse or separable factor)
    double* cwork;           // separable coarse solve scratch
    int cbw, cifast;
    double* partials;        // norm partials
    Ctrl* ctrl;
    double* scratch;         // ADI
    const double* cprime;
    const double* piv;
    const void* seg;         // ADI segment table of the item's element type (NULL: sequential solver)
    int m, n, P, mc, nc, Pc;
    double cx, cy, d, inv_d, omega, a_off;
    int V, ty, nwin, nchunk, H;
    int ntiles, tile0;       // tiles (or line blocks) of this item; prefix offset in the launch
    int flags;               // SW_F for sweeps; SW_RDIFF for restrictions; ADI relaxation form
    int parity;              // ADI line parity
    const void* sub;         // BK_SUBTREE: device SubtreeArgs<T> of this grid
    // fused post-smoothing + defect pass (SW_DEF; in / out: the FP64 iterate,
    // f / bc: this and the next FP32 right-hand side, ec: coarse correction)
    const void* e;           // post + defect: the FP32 level-0 buffer the post-smoothing starts from;
                             // defect: the FP32 buffer it sets to zero (nullable)
    const double* f64;       // FP64 source (nullable)
    int rowpart;             // norm partials per (window, row block) (see SweepArgs)
    // finalisation of a mixed step of several FP32 cycles (see launch_finalize):
    // the item is skipped while gate->done is set (nullable); after the test
    // the cycle choice goes to the gate pair of cyc (nullable) by `cycles`.
    // The other kinds take a gated operation's gate as ctrl.
    const Ctrl* gate;
    Ctrl* cyc;
    int cycles;
};

enum BatchKind { BK_SWEEP = 0, BK_RESTRICT, BK_COARSE, BK_FINALIZE, BK_RESNORM, BK_DEFECT, BK_ADI_ROWS, BK_ADI_COLS,
                 BK_SUBTREE, BK_FUSED };
// Launch one merged operation over `count` items (device array) covering
// `total` tiles with a persistent grid of `blocks` workgroups; tmap[t] is the
// item of tile t (kinds with tiles; one workgroup per item otherwise).
hipError_t launch_batch(int kind, int dt, int step_flags, const BatchItem* items, const int* tmap, int count,
                        int total, int blocks, hipStream_t s);
// ADI lines of all items; flags ADI_SEG: the segmented solver (every item
// has a segment table and fits it), else the sequential one.
constexpr int ADI_SEG = 2;
constexpr int ADI_CODE_SHIFT = 2;   // segmented: size code (seg_code) in bits 2..3
constexpr int ADI_MG = 16;          // zebra line smoothing of a multigrid level (operation flag)
hipError_t launch_batch_adi(int kind, int flags, int dt, const BatchItem* items, const int* tmap, int total,
                            int blocks, hipStream_t s);
// merged fused passes (batch_fused.hip); step_flags without SW_F; every item has V columns per lane
hipError_t launch_batch_fused(int dt, int step_flags, int V, const BatchItem* items, const int* tmap, int total,
                              int blocks, hipStream_t s);

}  // namespace lap
