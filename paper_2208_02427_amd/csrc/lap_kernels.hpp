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

// Tiling of an m x n level with V columns per lane.  ty > 0: chunks of ty
// rows.  ty == 0: size the chunks so the launch has about `target` waves
// (one full occupancy round of the device when target = its wave capacity),
// which avoids a nearly empty last round.  Chunks are never shorter than 16
// rows, which bounds the number of tiles (and norm partials) of a level.
inline Tiling make_tiling(int m, int n, int V, int ty, int target = 0, int H = 2) {
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
        if (ty < 16) ty = 16;
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
// Two canonical tilings, by producer: the stencil passes (sweeps with
// norms, fused pre-smoothing, residual norms) and the FP64 defect correction
// of the mixed loop; a norm finalisation reduces the partials of the kind
// that produced them.
enum NormKind { NORM_PASS = 0, NORM_DEFECT = 1 };
inline Tiling norm_tiling(int m, int n, int kind = NORM_PASS) {
    return kind == NORM_DEFECT ? make_tiling(m, n, 1, 0, 16384, 2) : make_tiling(m, n, 2, 0, 16384, kNormH);
}

// Blocks of 4 waves; the grid is padded to a multiple of the XCD count so
// the XCD-aware remap below is a bijection.
inline int blocks_for(const Tiling& t) {
    int nb = (t.ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
    return ((nb + kXcds - 1) / kXcds) * kXcds;
}

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
    int32_t pad;
};

// Flags of the red-black sweep.
enum : int {
    SW_F = 1,        // source / right-hand side present
    SW_ZERO = 2,     // input is identically zero (u_in ignored)
    SW_PROLONG = 4,  // input is u_in + P(ec)
    SW_NORM = 8,     // accumulate residual norms of the input into partials
    SW_RESTRICT = 16,// fused pass: residual + full weighting of the result into bc
    SW_TWO = 32,     // fused pass: two sweeps
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
};

template <typename T>
struct RestrictArgs {
    const T* u;
    const T* f;
    T* bc;
    const Ctrl* ctrl;
    int m, n, P;
    int mc, nc, Pc;
    T cx, cy, d;
    Tiling tl;
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
// mode 0: stopping test of a solve; mode 1: write norms only (out2 = {sum, max}).
hipError_t launch_finalize(const double* partials, int ntiles, Ctrl* ctrl, double* out2, int mode,
                           hipStream_t s);
// Reset a control block for a new solve (stream-ordered, graph-safe).
hipError_t launch_ctrl_init(Ctrl* ctrl, double tol, int stop, int max_iter, int step, hipStream_t s);
// Gather the control blocks of a batch of grids into one array.
hipError_t launch_gather_ctrl(Ctrl* const* src, Ctrl* dst, int count, hipStream_t s);
// Streaming copy of `bytes` (a multiple of 16) with `blocks` workgroups.
hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, int blocks, hipStream_t s);
// Dense m x n FP64 field (row pitch m) into pitched fields d0 and (if not NULL) d1.
hipError_t launch_write_field(const double* src, double* d0, double* d1, int m, int n, int P, hipStream_t s);
// Copy interior of src into dst (FP64 fields of the same layout).
hipError_t launch_copy(const double* src, double* dst, int m, int n, int P, const Ctrl* ctrl,
                       hipStream_t s);

// ---- ADI (adi_kernels.hip) ----
struct LineArgs {
    double* u;               // in place
    const double* f;         // nullable
    double* scratch;         // forward-sweep values, same layout as u
    const double* cprime;    // c'_k of the constant-coefficient factorisation, k = 0..K-1
    const double* piv;       // pivot_k (piv_0 = d)
    const Ctrl* ctrl;
    int m, n, P;
    double cx, cy, d, omega;
    double a_off;            // off-diagonal of the line matrix (-cx or -w cx, rows; -cy.. cols)
    int form;                // 0 relax after, 1 relax inside
    int parity;              // 1: odd lines, 0: even lines
};
constexpr int kRowTile = 64;   // row lines per ADI row block
hipError_t launch_adi_rows(const LineArgs& a, hipStream_t s);
hipError_t launch_adi_cols(const LineArgs& a, hipStream_t s);

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
    int m, n, P, mc, nc, Pc;
    double cx, cy, d, inv_d, omega, a_off;
    int V, ty, nwin, nchunk, H;
    int ntiles, tile0;       // tiles (or line blocks) of this item; prefix offset in the launch
    int flags;               // SW_F for sweeps; ADI relaxation form
    int parity;              // ADI line parity
    const void* sub;         // BK_SUBTREE: device SubtreeArgs<T> of this grid
};

enum BatchKind { BK_SWEEP = 0, BK_RESTRICT, BK_COARSE, BK_FINALIZE, BK_RESNORM, BK_DEFECT, BK_ADI_ROWS, BK_ADI_COLS,
                 BK_SUBTREE, BK_FUSED };
// Launch one merged operation over `count` items (device array) covering
// `total` tiles with a persistent grid of `blocks` workgroups.
hipError_t launch_batch(int kind, int dt, int step_flags, const BatchItem* items, int count, int total, int blocks,
                        hipStream_t s);
hipError_t launch_batch_adi(int kind, const BatchItem* items, int count, int total, int blocks, hipStream_t s);
// merged fused passes (fused_kernels.hip); step_flags without SW_F
hipError_t launch_batch_fused(int dt, int step_flags, const BatchItem* items, int count, int total, int blocks,
                              hipStream_t s);

}  // namespace lap
