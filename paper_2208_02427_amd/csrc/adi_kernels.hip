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
// Two solvers.  The segmented one (lines of up to 4095 unknowns along rows,
// 1023 along columns) splits every line into short blocks solved in
// parallel and couples them through a small reduced system (see
// lap_kernels.hpp); it reads and writes every value once.  The sequential
// one serves longer lines: columns, one thread per column line, marching j
// (consecutive threads own consecutive lines, so every row access of a
// wavefront is one contiguous span); rows, one 64-lane wavefront owns 64 row
// lines and moves through 64-column chunks, each chunk loaded / stored row by
// row through an LDS tile in which each lane walks its own line.  The
// sequential solver follows the plain recurrence (divisions, no fused
// multiply-add); the segmented one multiplies by tabulated reciprocals and
// fuses, so the two agree to rounding.
#include <cmath>
#include <cstring>

#include "lap_kernels.hpp"
#include "stencil_tiles.hpp"

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

hipError_t launch_adi_cols_seg(const LineArgs& a, int lines, hipStream_t s);

hipError_t launch_adi_cols(const LineArgs& a, hipStream_t s) {
    const int first = a.parity ? 1 : 2;
    const int lines = a.m - 2 >= first ? (a.m - 2 - first) / 2 + 1 : 0;
    if (lines <= 0) return hipSuccess;
    if (a.seg != nullptr && seg_fits(1, a.n - 2)) return launch_adi_cols_seg(a, lines, s);
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

hipError_t launch_adi_rows_seg(const LineArgs& a, int lines, hipStream_t s);

hipError_t launch_adi_rows(const LineArgs& a, hipStream_t s) {
    const int first = a.parity ? 1 : 2;
    const int lines = a.n - 2 >= first ? (a.n - 2 - first) / 2 + 1 : 0;
    if (lines <= 0) return hipSuccess;
    if (a.seg != nullptr && seg_fits(0, a.m - 2)) return launch_adi_rows_seg(a, lines, s);
    const int nb = (lines + kRowTile - 1) / kRowTile;
    k_adi_rows<<<nb, kRowTile, 0, s>>>(a);
    return hipGetLastError();
}

// --------------------------------------------------------- segmented solver
// Templated on the element type T of the field: FP64 for the ADI method,
// FP32 as well for zebra line smoothing inside the mixed-precision V-cycle.
// Every operation of a T solve is done in T with T coefficients and a T
// table (the FP32 table is the extended-precision one rounded once).
static_assert(kSegL + 1 == 16, "block index arithmetic assumes 16 unknowns per block and separator");
constexpr int kSegBS = kSegL + 2;   // LDS slots of a row block: kSegL unknowns, separator, separator value

template <typename T>
void adi_seg_table_t(double Dd, double Ed, int K, T* tab) {
    std::memset(tab, 0, sizeof(T) * kSegTab);
    if (K <= 0) return;
    typedef long double R;
    const int L = kSegL;
    const int S = seg_count(K);
    const int Ll = K - (S - 1) * (L + 1);
    const R D = Dd, E = Ed;
    R piv[kSegL], cq[kSegL];
    piv[0] = D;
    for (int k = 1; k < L; ++k) piv[k] = D - E * E / piv[k - 1];
    for (int k = 0; k < L; ++k) cq[k] = E / piv[k];
    // response of a block of length len to a unit value left of it:
    // solve tridiag(-E, D, -E) g = E e_1
    auto resp = [&](int len, R* g) {
        R z = 0;
        for (int k = 0; k < len; ++k) {
            z = ((k == 0 ? E : (R)0) + E * z) / piv[k];
            g[k] = z;
        }
        for (int k = len - 2; k >= 0; --k) g[k] = g[k] + cq[k] * g[k + 1];
    };
    R g[kSegL] = {}, gl[kSegL] = {};
    resp(L, g);
    resp(Ll, gl);
    for (int k = 0; k < L; ++k) {
        tab[SEG_IPIV + k] = (T)(1 / piv[k]);
        tab[SEG_CQ + k] = (T)cq[k];
        tab[SEG_G + k] = (T)g[k];
        tab[SEG_GL + k] = (T)gl[k];
    }
    tab[SEG_E] = (T)Ed;
    // one block only, or more separators than the table holds (such lines
    // take the sequential solver)
    if (S < 2 || S > kSegMaxS) return;
    // reduced system over the separators: tridiag(-E_R, D_R, -E_R), the last
    // separator couples to the last block (or, if that is empty, to nothing)
    const R ER = E * g[L - 1];
    const R DR = D - 2 * E * g[0];
    const R DRend = D - E * g[0] - (Ll > 0 ? E * gl[0] : (R)0);
    const int NR = S - 1;
    R pv = 0;
    for (int p = 0; p < NR; ++p) {
        const R dg = (p == NR - 1) ? DRend : DR;
        pv = (p == 0) ? dg : dg - ER * ER / pv;
        tab[SEG_IPIVR + p] = (T)(1 / pv);
        tab[SEG_CQR + p] = (T)(ER / pv);
    }
    tab[SEG_E + 1] = (T)ER;
}

void adi_seg_table(double D, double E, int K, double* tab) { adi_seg_table_t<double>(D, E, K, tab); }
void adi_seg_table(double D, double E, int K, float* tab) { adi_seg_table_t<float>(D, E, K, tab); }

// Right-hand side of one unknown from its own old value, the sum of its two
// neighbours across the line and f (end values are added by the caller).
template <typename T>
__device__ __forceinline__ T seg_rhs(const LineArgsT<T>& A, T cc, T own, T nb, T fv) {
    const T base = cc * nb - fv;
    return A.form == 0 ? base : (T(1) - (T)A.omega) * (T)A.d * own + (T)A.omega * base;
}

// Forward elimination of one block given its right-hand sides r[0..len)
// (len <= kSegL); leaves the block's zero-end solution in r, returns its
// last value in *last.
template <typename T>
__device__ __forceinline__ void seg_block(const T* Tb, T E, int len, T (&r)[kSegL], T* last) {
    T z = 0;
#pragma unroll
    for (int k = 0; k < kSegL; ++k)
        if (k < len) {
            z = fma(E, z, r[k]) * Tb[SEG_IPIV + k];
            r[k] = z;
        }
    T x = 0, e = 0;
#pragma unroll
    for (int k = kSegL - 1; k >= 0; --k)
        if (k < len) {
            x = fma(Tb[SEG_CQ + k], x, r[k]);
            r[k] = x;
            if (k == len - 1) e = x;
        }
    *last = e;
}

// Reduced system of one line, its unknown p held by one thread (act; NR
// and the loop trip counts are uniform over the workgroup, every thread
// reaches every barrier).  The forward elimination z_p = (rho_p + E_R
// z_{p-1}) / pivot_p and the back substitution x_p = z_p + (E_R / pivot_p)
// x_{p+1} are first-order linear recurrences: each is evaluated as a
// Hillis-Steele scan of affine maps in ceil(log2 NR) steps through two LDS
// buffer pairs (a0, b0), (a1, b1) addressed by slot(p).  Returns x_p.
template <typename T, typename Slot>
__device__ __forceinline__ T seg_scan(const T* Tb, int NR, int p, bool act, T rho, Slot slot, T* a0, T* b0,
                                      T* a1, T* b1) {
    T a = 0, b = 0;
    if (act) {
        const T ip = Tb[SEG_IPIVR + p];
        a = p > 0 ? Tb[SEG_E + 1] * ip : T(0);
        b = rho * ip;
        a0[slot(p)] = a;
        b0[slot(p)] = b;
    }
    __syncthreads();
    T *ra = a0, *rb = b0, *wa = a1, *wb = b1;
    for (int h = 1; h < NR; h <<= 1) {
        if (act) {
            if (p >= h) {
                const int q = slot(p - h);
                b = fma(a, rb[q], b);
                a = a * ra[q];
            }
            wa[slot(p)] = a;
            wb[slot(p)] = b;
        }
        __syncthreads();
        T* t = ra; ra = wa; wa = t;
        t = rb; rb = wb; wb = t;
    }
    // b = z_p; now x_p = c_p x_{p+1} + z_p, scanned from the end
    T c = (act && p < NR - 1) ? Tb[SEG_CQR + p] : T(0);
    if (act) {
        ra[slot(p)] = c;
        rb[slot(p)] = b;
    }
    __syncthreads();
    for (int h = 1; h < NR; h <<= 1) {
        if (act) {
            if (p + h < NR) {
                const int q = slot(p + h);
                b = fma(c, rb[q], b);
                c = c * ra[q];
            }
            wa[slot(p)] = c;
            wb[slot(p)] = b;
        }
        __syncthreads();
        T* t = ra; ra = wa; wa = t;
        t = rb; rb = wb; wb = t;
    }
    return b;
}

// Row lines of the parity in A, tile `tile` (W = NT / S lines), one
// workgroup of NT threads.  The lines' right-hand sides are staged in
// LDS row by row (coalesced); thread (line c, block s), s fastest, solves its
// block from LDS; the solution goes back through LDS and is written row by
// row with the relaxation.  lds: W * S * kSegBS values.
template <typename T, int NT>
static __device__ void adi_rows_seg(const LineArgsT<T>& A, int tile, T* lds) {
    const int K = A.m - 2;
    const int S = seg_count(K);
    const int W = NT / S;
    const int first = A.parity ? 1 : 2;
    const int nlines = A.n - 2 >= first ? (A.n - 2 - first) / 2 + 1 : 0;
    const int line0 = tile * W;
    const int nl = min(W, nlines - line0);
    if (nl <= 0) return;
    const size_t P = (size_t)A.P;
    const T* Tb = A.seg;
    const T E = Tb[SEG_E];
    const T cc = (T)A.cy;
    const int LW = S * kSegBS;
    const int tid = threadIdx.x;
    const int total = nl * K;
    // element q of the tile is (line q / K, unknown q % K)
    const float invK = 1.0f / (float)K;
    constexpr int kU = 8;   // elements in flight per thread
    for (int q0 = tid; q0 < total; q0 += kU * NT) {
        T r[kU];
        int slot[kU];
#pragma unroll
        for (int v = 0; v < kU; ++v) {
            const int q = q0 + v * NT;
            slot[v] = -1;
            r[v] = 0;
            if (q < total) {
                const int c = seg_div(q, invK);
                const int k = q - c * K;
                const size_t row = (size_t)(first + 2 * (line0 + c)) * P;
                const size_t o = row + k + 1;
                // the line's own old value enters only with relaxation inside
                const T own = A.form == 0 ? T(0) : A.u[o];
                r[v] = seg_rhs<T>(A, cc, own, A.u[o - P] + A.u[o + P], A.f != nullptr ? A.f[o] : T(0));
                if (k == 0) r[v] = r[v] + E * A.u[row];
                if (k == K - 1) r[v] = r[v] + E * A.u[row + A.m - 1];
                slot[v] = c * LW + (k >> 4) * kSegBS + (k & 15);
            }
        }
#pragma unroll
        for (int v = 0; v < kU; ++v)
            if (slot[v] >= 0) lds[slot[v]] = r[v];
    }
    __syncthreads();
    const int c = seg_div(tid, 1.0f / (float)S);
    const int s = tid - c * S;
    const bool act = c < nl;
    const int len = s < S - 1 ? kSegL : K - (S - 1) * (kSegL + 1);
    T* blk = lds + c * LW + s * kSegBS;
    T y[kSegL];
    if (act) {
#pragma unroll
        for (int k = 0; k < kSegL; ++k) y[k] = k < len ? blk[k] : T(0);
        T e;
        seg_block<T>(Tb, E, len, y, &e);
        blk[0] = len > 0 ? y[0] : T(0);
        blk[1] = e;
    }
    __syncthreads();
    if (S > 1) {
        // slots 2..5 of each block are free now (its unknowns live in y)
        const bool sep = act && s < S - 1;
        const T rho = sep ? fma(E, blk[1] + blk[kSegBS], blk[kSegL]) : T(0);
        T* lb = lds + c * LW;
        const auto slot = [](int p) { return p * kSegBS; };
        const T x = seg_scan<T>(Tb, S - 1, s, sep, rho, slot, lb + 2, lb + 3, lb + 4, lb + 5);
        if (sep) blk[kSegL + 1] = x;
        __syncthreads();
    }
    if (act) {
        const T xl = s > 0 ? blk[kSegL + 1 - kSegBS] : T(0);
        if (s < S - 1) {
            const T xr = blk[kSegL + 1];
#pragma unroll
            for (int k = 0; k < kSegL; ++k)
                blk[k] = fma(xr, Tb[SEG_G + kSegL - 1 - k], fma(xl, Tb[SEG_G + k], y[k]));
            blk[kSegL] = xr;
        } else {
#pragma unroll
            for (int k = 0; k < kSegL; ++k)
                if (k < len) blk[k] = fma(xl, Tb[SEG_GL + k], y[k]);
        }
    }
    __syncthreads();
    const T w = (T)A.omega;
    for (int q0 = tid; q0 < total; q0 += kU * NT) {
        T old[kU], t[kU];
        size_t at[kU];
#pragma unroll
        for (int v = 0; v < kU; ++v) {
            const int q = q0 + v * NT;
            at[v] = 0;
            old[v] = t[v] = 0;
            if (q < total) {
                const int c2 = seg_div(q, invK);
                const int k = q - c2 * K;
                at[v] = (size_t)(first + 2 * (line0 + c2)) * P + k + 1;
                t[v] = lds[c2 * LW + (k >> 4) * kSegBS + (k & 15)];
                if (A.form == 0) old[v] = A.u[at[v]];
            }
        }
#pragma unroll
        for (int v = 0; v < kU; ++v)
            if (q0 + v * NT < total) A.u[at[v]] = (A.form == 0) ? old[v] + w * (t[v] - old[v]) : t[v];
    }
}

// Column lines of the parity in A, tile `tile` (W = NT / S lines), one
// workgroup of NT threads; thread (line c, block s), c fastest,
// so a wavefront's accesses to one row are contiguous.  Each thread keeps
// its block's old values and solution in registers.  sh: 5 * NT values
// (first and last block values, separator values, scan buffers).
template <typename T, int NT>
static __device__ void adi_cols_seg(const LineArgsT<T>& A, int tile, T* sh) {
    const int K = A.n - 2;
    const int S = seg_count(K);
    const int W = NT / S;
    const int first = A.parity ? 1 : 2;
    const int nlines = A.m - 2 >= first ? (A.m - 2 - first) / 2 + 1 : 0;
    const int line0 = tile * W;
    const int nl = min(W, nlines - line0);
    if (nl <= 0) return;
    const size_t P = (size_t)A.P;
    const T* Tb = A.seg;
    const T E = Tb[SEG_E];
    const T cc = (T)A.cx;
    const int tid = threadIdx.x;
    const int s = seg_div(tid, 1.0f / (float)W);
    const int c = tid - s * W;
    const bool act = c < nl && s < S;
    const int len = s < S - 1 ? kSegL : K - (S - 1) * (kSegL + 1);
    const int i = first + 2 * (line0 + c);
    const int k0 = s * (kSegL + 1);
    T* yF = sh;
    T* yE = sh + NT;
    T* xs = sh + 2 * NT;
    const int me = s * W + c;
    T y[kSegL], old[kSegL];
    T osep = 0, rsep = 0, e = 0;
    if (act) {
        const T* up = A.u + (size_t)(k0 + 1) * P + i;
        const T* fp = A.f != nullptr ? A.f + (size_t)(k0 + 1) * P + i : nullptr;
#pragma unroll
        for (int k = 0; k < kSegL; ++k) {
            old[k] = 0;
            y[k] = 0;
            if (k < len) {
                const T* q = up + (size_t)k * P;
                old[k] = q[0];
                y[k] = seg_rhs<T>(A, cc, q[0], q[-1] + q[1], fp != nullptr ? fp[(size_t)k * P] : T(0));
            }
        }
        if (s == 0) y[0] = y[0] + E * A.u[i];
        if (len > 0 && k0 + len == K) {
#pragma unroll
            for (int k = 0; k < kSegL; ++k)
                if (k == len - 1) y[k] = y[k] + E * A.u[(size_t)(A.n - 1) * P + i];
        }
        if (s < S - 1) {
            const T* q = up + (size_t)kSegL * P;
            osep = q[0];
            rsep = seg_rhs<T>(A, cc, q[0], q[-1] + q[1], fp != nullptr ? fp[(size_t)kSegL * P] : T(0));
            if (k0 + kSegL == K - 1) rsep = rsep + E * A.u[(size_t)(A.n - 1) * P + i];
        }
        seg_block<T>(Tb, E, len, y, &e);
        yF[me] = len > 0 ? y[0] : T(0);
        yE[me] = e;
    }
    __syncthreads();
    if (S > 1) {
        const bool sep = act && s < S - 1;
        const T rho = sep ? fma(E, e + yF[me + W], rsep) : T(0);
        const auto slot = [W, c](int p) { return p * W + c; };
        const T x = seg_scan<T>(Tb, S - 1, s, sep, rho, slot, yE, xs, sh + 3 * NT, sh + 4 * NT);
        // yF is read above until every thread has passed the scan's first barrier
        if (sep) xs[me] = x;
        __syncthreads();
    }
    if (act) {
        const T w = (T)A.omega;
        const T xl = s > 0 ? xs[me - W] : T(0);
        T* up = A.u + (size_t)(k0 + 1) * P + i;
        if (s < S - 1) {
            const T xr = xs[me];
#pragma unroll
            for (int k = 0; k < kSegL; ++k) {
                const T t = fma(xr, Tb[SEG_G + kSegL - 1 - k], fma(xl, Tb[SEG_G + k], y[k]));
                up[(size_t)k * P] = (A.form == 0) ? old[k] + w * (t - old[k]) : t;
            }
            up[(size_t)kSegL * P] = (A.form == 0) ? osep + w * (xr - osep) : xr;
        } else {
#pragma unroll
            for (int k = 0; k < kSegL; ++k)
                if (k < len) {
                    const T t = fma(xl, Tb[SEG_GL + k], y[k]);
                    up[(size_t)k * P] = (A.form == 0) ? old[k] + w * (t - old[k]) : t;
                }
        }
    }
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_adi_rows_seg(LineArgsT<T> A, int ntiles) {
    if (A.ctrl != nullptr && A.ctrl->done) return;
    __shared__ T lds[NT * kSegBS];
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    if (t < ntiles) adi_rows_seg<T, NT>(A, t, lds);
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_adi_cols_seg(LineArgsT<T> A, int ntiles) {
    if (A.ctrl != nullptr && A.ctrl->done) return;
    __shared__ T sh[5 * NT];
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    if (t < ntiles) adi_cols_seg<T, NT>(A, t, sh);
}

// ------------------------------------------------------- merged batch launches

template <typename T>
__device__ __forceinline__ LineArgsT<T> line_args(const BatchItem& it) {
    LineArgsT<T> a{};
    a.u = (T*)it.out;
    a.f = (const T*)it.f;
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
    a.seg = (const T*)it.seg;
    return a;
}

// Row lines of all grids: one 64-lane block per 64-line block of a grid,
// the grid loops over all (grid, line block) tiles.
__global__ __launch_bounds__(64) void k_batch_adi_rows(const BatchItem* items, const int* tmap, int total) {
    __shared__ double tile[kRowTile][kRowTile + 1];
    __shared__ double told[kRowTile][kRowTile + 1];
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        const BatchItem& it = items[tmap[t]];
        if (it.ctrl->done) continue;
        adi_rows_block(line_args<double>(it), t - it.tile0, tile, told);
    }
}

// Column lines of all grids: one thread per line, 256 lines per tile.
__global__ __launch_bounds__(kBlock) void k_batch_adi_cols(const BatchItem* items, const int* tmap, int total) {
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        const BatchItem& it = items[tmap[t]];
        if (it.ctrl->done) continue;
        adi_col_line(line_args<double>(it), (t - it.tile0) * kBlock + threadIdx.x);
    }
}

// Segmented solver over all grids: tiles of seg_lines lines of one grid,
// dealt XCD-contiguously (neighbouring tiles share boundary lines).
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_batch_adi_rows_seg(const BatchItem* items, const int* tmap, int total) {
    __shared__ T lds[NT * kSegBS];
    for (int t = xcd_remap(blockIdx.x, gridDim.x); t < total; t += gridDim.x) {
        const BatchItem& it = items[tmap[t]];
        if (it.ctrl->done) continue;
        adi_rows_seg<T, NT>(line_args<T>(it), t - it.tile0, lds);
        __syncthreads();
    }
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_batch_adi_cols_seg(const BatchItem* items, const int* tmap, int total) {
    __shared__ T sh[5 * NT];
    for (int t = xcd_remap(blockIdx.x, gridDim.x); t < total; t += gridDim.x) {
        const BatchItem& it = items[tmap[t]];
        if (it.ctrl->done) continue;
        adi_cols_seg<T, NT>(line_args<T>(it), t - it.tile0, sh);
        __syncthreads();
    }
}

template <typename T>
hipError_t launch_adi_rows_seg(const LineArgsT<T>& a, int lines, hipStream_t s) {
    const int W = seg_lines(0, a.m - 2);
    const int nt = (lines + W - 1) / W;
    if (seg_code(0, a.m - 2) == 1)
        k_adi_rows_seg<T, 256><<<xcd_pad(nt), 256, 0, s>>>(a, nt);
    else
        k_adi_rows_seg<T, 128><<<xcd_pad(nt), 128, 0, s>>>(a, nt);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adi_cols_seg(const LineArgsT<T>& a, int lines, hipStream_t s) {
    const int W = seg_lines(1, a.n - 2);
    const int nt = (lines + W - 1) / W;
    if (seg_code(1, a.n - 2) == 0)
        k_adi_cols_seg<T, 256><<<xcd_pad(nt), 256, 0, s>>>(a, nt);
    else
        k_adi_cols_seg<T, 1024><<<xcd_pad(nt), 1024, 0, s>>>(a, nt);
    return hipGetLastError();
}

hipError_t launch_adi_rows_seg(const LineArgs& a, int lines, hipStream_t s) {
    return launch_adi_rows_seg<double>(a, lines, s);
}
hipError_t launch_adi_cols_seg(const LineArgs& a, int lines, hipStream_t s) {
    return launch_adi_cols_seg<double>(a, lines, s);
}

// Zebra line smoothing half (segmented solver only): lines of one parity of
// one direction, in place on a.u, FP64 or FP32.
template <typename T>
hipError_t launch_zebra_lines(const LineArgsT<T>& a, int dir, hipStream_t s) {
    const int first = a.parity ? 1 : 2;
    const int across = dir == 0 ? a.n - 2 : a.m - 2;
    const int K = dir == 0 ? a.m - 2 : a.n - 2;
    const int lines = across >= first ? (across - first) / 2 + 1 : 0;
    if (lines <= 0) return hipSuccess;
    if (a.seg == nullptr || !seg_fits(dir, K)) return hipErrorInvalidValue;
    return dir == 0 ? launch_adi_rows_seg<T>(a, lines, s) : launch_adi_cols_seg<T>(a, lines, s);
}
template hipError_t launch_zebra_lines<double>(const LineArgsT<double>&, int, hipStream_t);
template hipError_t launch_zebra_lines<float>(const LineArgsT<float>&, int, hipStream_t);

hipError_t launch_batch_adi(int kind, int flags, int dt, const BatchItem* items, const int* tmap, int total,
                            int blocks, hipStream_t s) {
    if (total <= 0) return hipSuccess;
    if (flags & ADI_SEG) {
        blocks = xcd_pad(blocks);
        const int code = (flags >> ADI_CODE_SHIFT) & 3;
        if (kind == BK_ADI_ROWS) {
            if (dt == 0) {
                if (code == 1)
                    k_batch_adi_rows_seg<double, 256><<<blocks, 256, 0, s>>>(items, tmap, total);
                else
                    k_batch_adi_rows_seg<double, 128><<<blocks, 128, 0, s>>>(items, tmap, total);
            } else {
                if (code == 1)
                    k_batch_adi_rows_seg<float, 256><<<blocks, 256, 0, s>>>(items, tmap, total);
                else
                    k_batch_adi_rows_seg<float, 128><<<blocks, 128, 0, s>>>(items, tmap, total);
            }
        } else {
            if (dt == 0) {
                if (code == 0)
                    k_batch_adi_cols_seg<double, 256><<<blocks, 256, 0, s>>>(items, tmap, total);
                else
                    k_batch_adi_cols_seg<double, 1024><<<blocks, 1024, 0, s>>>(items, tmap, total);
            } else {
                if (code == 0)
                    k_batch_adi_cols_seg<float, 256><<<blocks, 256, 0, s>>>(items, tmap, total);
                else
                    k_batch_adi_cols_seg<float, 1024><<<blocks, 1024, 0, s>>>(items, tmap, total);
            }
        }
        return hipGetLastError();
    }
    if (dt != 0) return hipErrorInvalidValue;   // the sequential solver is FP64 only
    if (kind == BK_ADI_ROWS)
        k_batch_adi_rows<<<blocks, kRowTile, 0, s>>>(items, tmap, total);
    else
        k_batch_adi_cols<<<blocks, kBlock, 0, s>>>(items, tmap, total);
    return hipGetLastError();
}

}  // namespace lap
