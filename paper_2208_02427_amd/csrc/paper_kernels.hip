// The paper's own sequential methods on the GPU, with the paper's update
// order: Jacobi (Eq. (5)), lexicographic Gauss-Seidel / SOR (Eqs. (6)-(7)),
// SLOR by rows with the relaxation after the line solve (SLORA, Eqs. (8)-(9))
// or inside it (SLORB, Eq. (10)), and ADI as all rows in ascending order
// followed by all columns in ascending order (ADI section).
//
// One workgroup holds the whole grid in LDS and runs the whole solve: every
// iteration, its stopping test and the next iteration stay on the chip, so a
// small problem such as the 25 x 17 chamber costs a few microseconds per
// iteration instead of several launches.
//
// Order.  Lexicographic SOR updates node (i, j) after (i-1, j) and (i, j-1)
// and before (i+1, j) and (i, j+1).  All nodes of one anti-diagonal i + j = d
// depend only on diagonals d - 1 (already new) and d + 1 (still old), so the
// workgroup updates a diagonal at once and moves to the next after a barrier:
// every node sees exactly the operands of the row-by-row loop.  The line
// methods solve one line after another (each line's Thomas recurrence is
// sequential; its right-hand side and its relaxation are computed by all
// threads).
//
// Arithmetic.  Every expression is the plain one of the methods, unfused
// (the file is built with -ffp-contract=off):
//   t = ((cx (W + E) + cy (S + N)) - f) * inv_d,   psi <- psi + w (t - psi),
// and the line systems by the Thomas recurrences with divisions.
#include <cmath>

#include "lap_kernels.hpp"
#include "../../include/lap.h"

namespace lap {

__device__ __forceinline__ double block_max(double v, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double r = red[0];
    for (int k = 1; k < nw; ++k) r = fmax(r, red[k]);
    __syncthreads();
    return r;
}

// Sum over the workgroup: per-thread partials in index order, then the
// wavefront sums in wave order (fixed for a given grid and block size).
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double r = red[0];
    for (int k = 1; k < nw; ++k) r = r + red[k];
    __syncthreads();
    return r;
}

// One line system of K unknowns (row line: along i; column line: along j),
// solved in place on u (LDS) by the Thomas recurrences.  lc / cc: coupling
// coefficients along / across the line; form 0: relaxation after the solve
// (SLORA), 1: inside (SLORB).  rhs, cp, rp: LDS scratch of K values.
__device__ void paper_line(const PaperArgs& A, double* u, int line, int dir, double* rhs, double* cp,
                           double* rp) {
    const int m = A.m, n = A.n;
    const int K = dir == 0 ? m - 2 : n - 2;
    // element k of the line and its neighbours across the line (LDS index)
    auto at = [&](int k) { return dir == 0 ? line * m + (k + 1) : (k + 1) * m + line; };
    const int across = dir == 0 ? m : 1;
    const double lc = dir == 0 ? A.cx : A.cy, cc = dir == 0 ? A.cy : A.cx;
    const double w = A.omega, d = A.d;
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const int p = at(k);
        const int j = dir == 0 ? line : k + 1, i = dir == 0 ? k + 1 : line;
        const double fv = A.f != nullptr ? A.f[(size_t)j * A.P + i] : 0.0;
        const double base = cc * (u[p - across] + u[p + across]) - fv;
        double r = A.form == 0 ? base : (1.0 - w) * d * u[p] + w * base;
        const double e = A.form == 0 ? lc : w * lc;   // end values enter with the line coupling
        if (k == 0) r = r + e * (dir == 0 ? u[line * m] : u[line]);
        if (k == K - 1) r = r + e * (dir == 0 ? u[line * m + m - 1] : u[(n - 1) * m + line]);
        rhs[k] = r;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // a x_{k-1} + b x_k + c x_{k+1} = r_k with a = c = -lc (-w lc inside), b = d
        const double a = A.form == 0 ? -lc : -w * lc, b = d, c = a;
        cp[0] = c / b;
        rp[0] = rhs[0] / b;
        for (int k = 1; k < K; ++k) {
            const double piv = b - a * cp[k - 1];
            cp[k] = c / piv;
            rp[k] = (rhs[k] - a * rp[k - 1]) / piv;
        }
        rhs[K - 1] = rp[K - 1];
        for (int k = K - 2; k >= 0; --k) rhs[k] = rp[k] - cp[k] * rhs[k + 1];
    }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const int p = at(k);
        const double old = u[p];
        u[p] = A.form == 0 ? old + w * (rhs[k] - old) : rhs[k];
    }
    __syncthreads();
}

// The monitored quantity of the stopping rule after an iteration: the
// largest update max|psi - psi_start| (Eq. (16)), max|r| or ||r||_2 / ||r_0||_2.
__device__ double paper_monitor(const PaperArgs& A, const double* u, const double* u0, double r0, double* red) {
    const int m = A.m, n = A.n, N = (m - 2) * (n - 2);
    double mx = 0.0, s2 = 0.0;
    for (int q = threadIdx.x; q < N; q += blockDim.x) {
        const int i = 1 + q % (m - 2), j = 1 + q / (m - 2);
        const int p = j * m + i;
        if (A.stop == LAP_STOP_DELTA) {
            mx = fmax(mx, fabs(u[p] - u0[p]));
        } else {
            const double Lu = (A.cx * (u[p - 1] + u[p + 1]) + A.cy * (u[p - m] + u[p + m])) - A.d * u[p];
            const double r = (A.f != nullptr ? A.f[(size_t)j * A.P + i] : 0.0) - Lu;
            mx = fmax(mx, fabs(r));
            s2 = s2 + r * r;
        }
    }
    if (A.stop == LAP_STOP_REL_L2) {
        const double s = block_sum(s2, red);
        return r0 > 0.0 ? sqrt(s) / r0 : 0.0;
    }
    return block_max(mx, red);
}

// LDS: u (n x m, row stride m), its copy at the start of the iteration, line
// scratch (3 x max(m, n)), reduction slots (16).
__global__ __launch_bounds__(1024) void k_paper(PaperArgs A) {
    extern __shared__ double lds[];
    const int m = A.m, n = A.n, N = (m - 2) * (n - 2);
    const int L = m > n ? m : n;
    double* u = lds;
    double* u0 = u + (size_t)m * n;
    double* rhs = u0 + (size_t)m * n;
    double* cp = rhs + L;
    double* rp = cp + L;
    double* red = rp + L;
    for (int q = threadIdx.x; q < m * n; q += blockDim.x) {
        const int i = q % m, j = q / m;
        u[q] = A.u[(size_t)j * A.P + i];
    }
    __syncthreads();
    double r0 = 0.0;
    if (A.stop == LAP_STOP_REL_L2) {
        double s2 = 0.0;
        for (int q = threadIdx.x; q < N; q += blockDim.x) {
            const int i = 1 + q % (m - 2), j = 1 + q / (m - 2);
            const int p = j * m + i;
            const double Lu = (A.cx * (u[p - 1] + u[p + 1]) + A.cy * (u[p - m] + u[p + m])) - A.d * u[p];
            const double r = (A.f != nullptr ? A.f[(size_t)j * A.P + i] : 0.0) - Lu;
            s2 = s2 + r * r;
        }
        r0 = sqrt(block_sum(s2, red));
    }
    const double cx = A.cx, cy = A.cy, inv_d = A.inv_d, w = A.omega;
    int it = 0, status = 0, done = 0;
    double q = 0.0;
    while (it < A.max_iter) {
        for (int p = threadIdx.x; p < m * n; p += blockDim.x) u0[p] = u[p];
        __syncthreads();
        if (A.method == LAP_JACOBI) {
            // every node from the values at the start of the iteration
            for (int k = threadIdx.x; k < N; k += blockDim.x) {
                const int i = 1 + k % (m - 2), j = 1 + k / (m - 2);
                const int p = j * m + i;
                const double fv = A.f != nullptr ? A.f[(size_t)j * A.P + i] : 0.0;
                u[p] = ((cx * (u0[p - 1] + u0[p + 1]) + cy * (u0[p - m] + u0[p + m])) - fv) * inv_d;
            }
            __syncthreads();
        } else if (A.method == LAP_SOR_LEX) {
            // anti-diagonals d = i + j in increasing order
            for (int dg = 2; dg <= (m - 2) + (n - 2); ++dg) {
                const int ilo = dg - (n - 2) > 1 ? dg - (n - 2) : 1;
                const int ihi = dg - 1 < m - 2 ? dg - 1 : m - 2;
                for (int i = ilo + (int)threadIdx.x; i <= ihi; i += blockDim.x) {
                    const int j = dg - i;
                    const int p = j * m + i;
                    const double fv = A.f != nullptr ? A.f[(size_t)j * A.P + i] : 0.0;
                    const double t = ((cx * (u[p - 1] + u[p + 1]) + cy * (u[p - m] + u[p + m])) - fv) * inv_d;
                    u[p] = u[p] + w * (t - u[p]);
                }
                __syncthreads();
            }
        } else {
            // SLOR: rows j = 1..n-2; ADI: the rows, then columns i = 1..m-2
            for (int j = 1; j <= n - 2; ++j) paper_line(A, u, j, 0, rhs, cp, rp);
            if (A.method == LAP_ADI_LEX)
                for (int i = 1; i <= m - 2; ++i) paper_line(A, u, i, 1, rhs, cp, rp);
        }
        ++it;
        q = paper_monitor(A, u, u0, r0, red);
        if (!isfinite(q) || q > 1e30) {
            status = LAP_EDIVERGED;
            done = 1;
            break;
        }
        if (q < A.tol) {
            done = 1;
            break;
        }
    }
    for (int p = threadIdx.x; p < m * n; p += blockDim.x) {
        const int i = p % m, j = p / m;
        A.u[(size_t)j * A.P + i] = u[p];
    }
    if (threadIdx.x == 0) {
        A.ctrl->iters = it;
        A.ctrl->done = done;
        A.ctrl->status = status;
        A.ctrl->rel = q;          // the last monitored quantity
        A.ctrl->r0 = r0;
        A.ctrl->checks = it;
    }
}

size_t paper_lds_bytes(int m, int n) {
    const int L = m > n ? m : n;
    return (2 * (size_t)m * n + 3 * (size_t)L + 16) * sizeof(double);
}

hipError_t paper_set_lds_limit(int bytes) {
    return hipFuncSetAttribute((const void*)k_paper, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

hipError_t launch_paper(const PaperArgs& a, hipStream_t s) {
    const int threads = 1024;
    k_paper<<<1, threads, paper_lds_bytes(a.m, a.n), s>>>(a);
    return hipGetLastError();
}

}  // namespace lap
