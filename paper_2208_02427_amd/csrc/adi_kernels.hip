// gfx950 kernels of line ADI: batched Thomas solves of all rows (or all
// columns) of one parity (zebra order), SLOR/ADI sections of the paper,
// Eqs. (8)-(10).
//
// Line system of row j (unknowns i = 1..m-2), relaxation after (SLORA):
//     -cx t_{i-1} + d t_i - cx t_{i+1} = cy (u_{i,j-1} + u_{i,j+1}) - f_ij
//     (+ cx u_{0,j} on the first, + cx u_{m-1,j} on the last unknown),
//     then u <- u + w (t - u);
// relaxation inside (SLORB):
//     -w cx t_{i-1} + d t_i - w cx t_{i+1} = (1-w) d u_ij + w (cy (...) - f_ij)
//     (+ w cx times the end values), then u <- t.
// Columns mirror it with x and y exchanged.  The coefficients are constant
// along a line, so the factorisation c'_k, pivot_k is computed once on the
// host; the kernels do the forward elimination and back substitution.
// Expression order and divisions follow the plain definition exactly (no
// fused multiply-add: the file is built with -ffp-contract=off).
//
// Columns: one thread per column line, marching j; consecutive threads own
// consecutive lines, so every row access of a wavefront is one contiguous
// span.  Rows: one 64-lane wavefront owns 64 row lines and moves through
// 64-column chunks; each chunk is loaded / stored row by row (coalesced)
// through an LDS tile in which each lane walks its own line.
#include "lap_kernels.hpp"

namespace lap {

// ------------------------------------------------------------------ columns
// Column line number t of the parity in A (no-op past the last line).
static __device__ void adi_col_line(const LineArgs& A, int t) {
    const int i = (A.parity ? 1 : 2) + 2 * t;
    if (i > A.m - 2) return;
    const int K = A.n - 2;
    const size_t P = (size_t)A.P;
    // in the column frame the coupling along the line is cy and across it cx
    const double cl = A.cy, cc = A.cx, d = A.d, w = A.omega, a = A.a_off;
    double rp = 0.0;
    for (int k = 0; k < K; ++k) {
        const int j = k + 1;
        const double* row = A.u + (size_t)j * P;
        const double base = cc * (row[i - 1] + row[i + 1]) - (A.f != nullptr ? A.f[(size_t)j * P + i] : 0.0);
        double r;
        if (A.form == 0) {
            r = base;
            if (k == 0) r = r + cl * A.u[i];
            if (k == K - 1) r = r + cl * A.u[(size_t)(A.n - 1) * P + i];
        } else {
            r = (1.0 - w) * d * row[i] + w * base;
            if (k == 0) r = r + w * cl * A.u[i];
            if (k == K - 1) r = r + w * cl * A.u[(size_t)(A.n - 1) * P + i];
        }
        rp = (k == 0) ? r / A.piv[0] : (r - a * rp) / A.piv[k];
        A.scratch[(size_t)j * P + t] = rp;
    }
    double x = 0.0;
    for (int k = K - 1; k >= 0; --k) {
        const int j = k + 1;
        const double q = A.scratch[(size_t)j * P + t];
        x = (k == K - 1) ? q : q - A.cprime[k] * x;
        double* p = A.u + (size_t)j * P + i;
        const double old = *p;
        *p = (A.form == 0) ? old + w * (x - old) : x;
    }
}

__global__ __launch_bounds__(kBlock) void k_adi_cols(LineArgs A) {
    if (A.ctrl != nullptr && A.ctrl->done) return;
    adi_col_line(A, blockIdx.x * blockDim.x + threadIdx.x);
}

hipError_t launch_adi_cols(const LineArgs& a, hipStream_t s) {
    const int first = a.parity ? 1 : 2;
    const int lines = a.m - 2 >= first ? (a.m - 2 - first) / 2 + 1 : 0;
    if (lines <= 0) return hipSuccess;
    const int nb = (lines + kBlock - 1) / kBlock;
    k_adi_cols<<<nb, kBlock, 0, s>>>(a);
    return hipGetLastError();
}

// --------------------------------------------------------------------- rows

// Row lines 64*blk .. 64*blk+63 of the parity in A, one lane per line
// (block of 64 threads; tile / told are LDS scratch of 64 x 65 doubles).
static __device__ void adi_rows_block(const LineArgs& A, int blk, double (*tile)[kRowTile + 1],
                               double (*told)[kRowTile + 1]) {
    const int lane = threadIdx.x;
    const int first = A.parity ? 1 : 2;
    const int nlines = A.n - 2 >= first ? (A.n - 2 - first) / 2 + 1 : 0;
    const int line0 = blk * kRowTile;
    const int mylines = min(kRowTile, nlines - line0);
    const int K = A.m - 2;
    const size_t P = (size_t)A.P;
    const double cl = A.cx, cc = A.cy, d = A.d, w = A.omega, a = A.a_off;
    const int myj = first + 2 * (line0 + lane);          // this lane's row (valid if lane < mylines)
    const int nchunks = (K + kRowTile - 1) / kRowTile;
    // scratch row of line l: the line's own row j (distinct lines never share it)
    double rp = 0.0;
    for (int ch = 0; ch < nchunks; ++ch) {
        const int ic = 1 + ch * kRowTile;                 // first unknown of the chunk
        const int i = ic + lane;                          // column loaded by this lane
        for (int rr = 0; rr < mylines; ++rr) {
            const int j = first + 2 * (line0 + rr);
            if (i <= A.m - 2) {
                const double* row = A.u + (size_t)j * P;
                const double base = cc * (A.u[(size_t)(j - 1) * P + i] + A.u[(size_t)(j + 1) * P + i]) -
                                    (A.f != nullptr ? A.f[(size_t)j * P + i] : 0.0);
                tile[rr][lane] = (A.form == 0) ? base : (1.0 - w) * d * row[i] + w * base;
            }
        }
        __syncthreads();
        if (lane < mylines) {
            const int kend = min(kRowTile, K - ch * kRowTile);
            for (int kk = 0; kk < kend; ++kk) {
                const int k = ch * kRowTile + kk;
                double r = tile[lane][kk];
                if (k == 0) r = r + (A.form == 0 ? cl : w * cl) * A.u[(size_t)myj * P];
                if (k == K - 1) r = r + (A.form == 0 ? cl : w * cl) * A.u[(size_t)myj * P + A.m - 1];
                rp = (k == 0) ? r / A.piv[0] : (r - a * rp) / A.piv[k];
                tile[lane][kk] = rp;
            }
        }
        __syncthreads();
        for (int rr = 0; rr < mylines; ++rr) {
            const int j = first + 2 * (line0 + rr);
            if (i <= A.m - 2) A.scratch[(size_t)j * P + i] = tile[rr][lane];
        }
        __syncthreads();
    }
    double x = 0.0;
    for (int ch = nchunks - 1; ch >= 0; --ch) {
        const int ic = 1 + ch * kRowTile;
        const int i = ic + lane;
        for (int rr = 0; rr < mylines; ++rr) {
            const int j = first + 2 * (line0 + rr);
            if (i <= A.m - 2) {
                tile[rr][lane] = A.scratch[(size_t)j * P + i];
                told[rr][lane] = A.u[(size_t)j * P + i];
            }
        }
        __syncthreads();
        if (lane < mylines) {
            const int kend = min(kRowTile, K - ch * kRowTile);
            for (int kk = kend - 1; kk >= 0; --kk) {
                const int k = ch * kRowTile + kk;
                const double q = tile[lane][kk];
                x = (k == K - 1) ? q : q - A.cprime[k] * x;
                const double old = told[lane][kk];
                tile[lane][kk] = (A.form == 0) ? old + w * (x - old) : x;
            }
        }
        __syncthreads();
        for (int rr = 0; rr < mylines; ++rr) {
            const int j = first + 2 * (line0 + rr);
            if (i <= A.m - 2) A.u[(size_t)j * P + i] = tile[rr][lane];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(64) void k_adi_rows(LineArgs A) {
    if (A.ctrl != nullptr && A.ctrl->done) return;
    __shared__ double tile[kRowTile][kRowTile + 1];
    __shared__ double told[kRowTile][kRowTile + 1];
    adi_rows_block(A, blockIdx.x, tile, told);
}

hipError_t launch_adi_rows(const LineArgs& a, hipStream_t s) {
    const int first = a.parity ? 1 : 2;
    const int lines = a.n - 2 >= first ? (a.n - 2 - first) / 2 + 1 : 0;
    if (lines <= 0) return hipSuccess;
    const int nb = (lines + kRowTile - 1) / kRowTile;
    k_adi_rows<<<nb, kRowTile, 0, s>>>(a);
    return hipGetLastError();
}

// ------------------------------------------------------- merged batch launches
__device__ __forceinline__ int find_item(const BatchItem* it, int count, int t) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (it[mid].tile0 <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ LineArgs line_args(const BatchItem& it) {
    LineArgs a{};
    a.u = (double*)it.out;
    a.f = (const double*)it.f;
    a.scratch = it.scratch;
    a.cprime = it.cprime;
    a.piv = it.piv;
    a.ctrl = nullptr;
    a.m = it.m;
    a.n = it.n;
    a.P = it.P;
    a.cx = it.cx;
    a.cy = it.cy;
    a.d = it.d;
    a.omega = it.omega;
    a.a_off = it.a_off;
    a.form = it.flags;
    a.parity = it.parity;
    return a;
}

// Row lines of all grids: one 64-lane block per 64-line block of a grid,
// the grid loops over all (grid, line block) tiles.
__global__ __launch_bounds__(64) void k_batch_adi_rows(const BatchItem* items, int count, int total) {
    __shared__ double tile[kRowTile][kRowTile + 1];
    __shared__ double told[kRowTile][kRowTile + 1];
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        const BatchItem& it = items[find_item(items, count, t)];
        if (it.ctrl->done) continue;
        adi_rows_block(line_args(it), t - it.tile0, tile, told);
    }
}

// Column lines of all grids: one thread per line, 256 lines per tile.
__global__ __launch_bounds__(kBlock) void k_batch_adi_cols(const BatchItem* items, int count, int total) {
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        const BatchItem& it = items[find_item(items, count, t)];
        if (it.ctrl->done) continue;
        adi_col_line(line_args(it), (t - it.tile0) * kBlock + threadIdx.x);
    }
}

hipError_t launch_batch_adi(int kind, const BatchItem* items, int count, int total, int blocks, hipStream_t s) {
    if (total <= 0 || count <= 0) return hipSuccess;
    if (kind == BK_ADI_ROWS)
        k_batch_adi_rows<<<blocks, kRowTile, 0, s>>>(items, count, total);
    else
        k_batch_adi_cols<<<blocks, kBlock, 0, s>>>(items, count, total);
    return hipGetLastError();
}

}  // namespace lap
