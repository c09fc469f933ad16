// gfx950 stencil kernels of the multigrid / red-black SOR path.
//
//  k_sweep     one red-black SOR sweep (both colours) in a single HBM pass,
//              optionally from a zero start, with the bilinear prolongation
//              of a coarse correction folded into its input, and/or with the
//              residual norms of its input accumulated on the way
//              (SOR: Eq. (7); colour ordering: (i+j) even first).
//  k_restrict  residual r = f - L_h u (Eqs. (11)-(12)) fused with 9-point
//              full weighting onto the coarse right-hand side.
//  k_residual  residual with optional store and norms.
//  k_defect    FP64 defect correction: psi += e32, r = f - L_h psi, rhs32 = fl32(r).
//  k_coarse    exact solve on the coarsest level with a precomputed inverse.
//  k_finalize  fixed-order reduction of per-tile norm partials + stopping test.
//
// All arithmetic is written with explicit fma() and the file is compiled
// with -ffp-contract=off, so every tiling (V, ty) produces bitwise identical
// fields.  Per-node expression trees:
//   t   = (fma(cy, S+N, cx*(W+E)) - f) * inv_d
//   u'  = fma(omega, t - u, u)
//   L u = fma(-d, C, fma(cy, S+N, cx*(W+E)));   r = f - L u
#include <algorithm>

#include "stencil_tiles.hpp"

namespace lap {

template <typename T, int V, int FL>
__global__ __launch_bounds__(kBlock) void k_sweep(SweepArgs<T> A) {
    if (A.ctrl != nullptr && A.ctrl->done) return;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int tile = b * kWavesPerBlock + wave_in_block();
    if (tile >= A.tl.ntiles) return;
    sweep_tile<T, V, FL>(A, tile, threadIdx.x & 63);
}

template <typename T, int V>
static hipError_t launch_sweep_v(const SweepArgs<T>& a, int flags, hipStream_t s) {
    const dim3 grid(blocks_for(a.tl)), block(kBlock);
    switch (flags) {
        case 0: k_sweep<T, V, 0><<<grid, block, 0, s>>>(a); break;
        case SW_F: k_sweep<T, V, SW_F><<<grid, block, 0, s>>>(a); break;
        case SW_ZERO | SW_F: k_sweep<T, V, SW_ZERO | SW_F><<<grid, block, 0, s>>>(a); break;
        case SW_ZERO: k_sweep<T, V, SW_ZERO><<<grid, block, 0, s>>>(a); break;
        case SW_PROLONG: k_sweep<T, V, SW_PROLONG><<<grid, block, 0, s>>>(a); break;
        case SW_PROLONG | SW_F: k_sweep<T, V, SW_PROLONG | SW_F><<<grid, block, 0, s>>>(a); break;
        case SW_PROLONG | SW_PONLY: k_sweep<T, V, SW_PROLONG | SW_PONLY><<<grid, block, 0, s>>>(a); break;
        case SW_ZERO | SW_PROLONG | SW_PONLY:
            k_sweep<T, V, SW_ZERO | SW_PROLONG | SW_PONLY><<<grid, block, 0, s>>>(a);
            break;
        case SW_NORM: k_sweep<T, V, SW_NORM><<<grid, block, 0, s>>>(a); break;
        case SW_NORM | SW_F: k_sweep<T, V, SW_NORM | SW_F><<<grid, block, 0, s>>>(a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sweep(const SweepArgs<T>& a, int flags, hipStream_t s) {
    switch (a.tl.V) {
        case 1: return launch_sweep_v<T, 1>(a, flags, s);
        case 2: return launch_sweep_v<T, 2>(a, flags, s);
        case 4: return launch_sweep_v<T, 4>(a, flags, s);
        default: return hipErrorInvalidValue;
    }
}
template hipError_t launch_sweep<double>(const SweepArgs<double>&, int, hipStream_t);
template hipError_t launch_sweep<float>(const SweepArgs<float>&, int, hipStream_t);

template <typename T, int V, bool DIFF>
__global__ __launch_bounds__(kBlock) void k_restrict(RestrictArgs<T> A) {
    if (A.ctrl != nullptr && A.ctrl->done) return;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int tile = b * kWavesPerBlock + wave_in_block();
    if (tile >= A.tl.ntiles) return;
    restrict_tile<T, V, DIFF>(A, tile, threadIdx.x & 63);
}

template <typename T, bool DIFF>
hipError_t launch_restrict_as(const RestrictArgs<T>& a, hipStream_t s) {
    const dim3 grid(blocks_for(a.tl)), block(kBlock);
    switch (a.tl.V) {
        case 1: k_restrict<T, 1, DIFF><<<grid, block, 0, s>>>(a); break;
        case 2: k_restrict<T, 2, DIFF><<<grid, block, 0, s>>>(a); break;
        case 4: k_restrict<T, 4, DIFF><<<grid, block, 0, s>>>(a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict(const RestrictArgs<T>& a, hipStream_t s) {
    return a.rdiff ? launch_restrict_as<T, true>(a, s) : launch_restrict_as<T, false>(a, s);
}
template hipError_t launch_restrict<double>(const RestrictArgs<double>&, hipStream_t);
template hipError_t launch_restrict<float>(const RestrictArgs<float>&, hipStream_t);

template <typename T, int V>
__global__ __launch_bounds__(kBlock) void k_residual(ResidualArgs<T> A) {
    if (A.ctrl != nullptr && A.ctrl->done) return;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int tile = b * kWavesPerBlock + wave_in_block();
    if (tile >= A.tl.ntiles) return;
    residual_tile<T, V>(A, tile, threadIdx.x & 63);
}

template <typename T>
hipError_t launch_residual(const ResidualArgs<T>& a, hipStream_t s) {
    const dim3 grid(blocks_for(a.tl)), block(kBlock);
    switch (a.tl.V) {
        case 1: k_residual<T, 1><<<grid, block, 0, s>>>(a); break;
        case 2: k_residual<T, 2><<<grid, block, 0, s>>>(a); break;
        case 4: k_residual<T, 4><<<grid, block, 0, s>>>(a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
template hipError_t launch_residual<double>(const ResidualArgs<double>&, hipStream_t);
template hipError_t launch_residual<float>(const ResidualArgs<float>&, hipStream_t);

template <int V>
__global__ __launch_bounds__(kBlock) void k_defect(DefectArgs A) {
    if (A.ctrl != nullptr && A.ctrl->done) return;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int tile = b * kWavesPerBlock + wave_in_block();
    if (tile >= A.tl.ntiles) return;
    defect_tile<V>(A, tile, threadIdx.x & 63);
}

hipError_t launch_defect(const DefectArgs& a, hipStream_t s) {
    const dim3 grid(blocks_for(a.tl)), block(kBlock);
    switch (a.tl.V) {
        case 1: k_defect<1><<<grid, block, 0, s>>>(a); break;
        case 2: k_defect<2><<<grid, block, 0, s>>>(a); break;
        case 4: k_defect<4><<<grid, block, 0, s>>>(a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarse(CoarseArgs<T> A) {
    if (A.ctrl != nullptr && A.ctrl->done) return;
    __shared__ double rhs[1024];
    coarse_block<T>(A, rhs);
}

template <typename T>
hipError_t launch_coarse(const CoarseArgs<T>& a, hipStream_t s) {
    if (a.bw == 0 && (a.m - 2) * (a.n - 2) > kDenseCoarseMax) return hipErrorInvalidValue;
    k_coarse<T><<<1, kBlock, 0, s>>>(a);
    return hipGetLastError();
}
template hipError_t launch_coarse<double>(const CoarseArgs<double>&, hipStream_t);
template hipError_t launch_coarse<float>(const CoarseArgs<float>&, hipStream_t);

__global__ __launch_bounds__(kFinBlock) void k_finalize(const double* partials, int ntiles, Ctrl* ctrl,
                                                     double* out2, int mode, const Ctrl* gate, Ctrl* cyc,
                                                     int cycles) {
    if (mode != 1 && ctrl->done) return;
    if (gate != nullptr && gate->done) return;
    __shared__ double ss[kFinBlock / 64], sm[kFinBlock / 64];
    finalize_step(partials, ntiles, ctrl, out2, mode, cyc, cycles, ss, sm);
}

__global__ void k_ctrl_init(Ctrl* c, double tol, int stop, int max_iter, int step) {
    c->r0 = 0.0;
    c->rel = 0.0;
    c->res_l2 = 0.0;
    c->res_inf = 0.0;
    c->tol = tol;
    c->stop = stop;
    c->max_iter = max_iter;
    c->iters = 0;
    c->checks = 0;
    c->done = 0;
    c->status = 0;
    c->step = step;
    c->cycles = 0;
}

hipError_t launch_ctrl_init(Ctrl* ctrl, double tol, int stop, int max_iter, int step, hipStream_t s) {
    k_ctrl_init<<<1, 1, 0, s>>>(ctrl, tol, stop, max_iter, step);
    return hipGetLastError();
}

__global__ void k_ctrl_init_many(Ctrl* const* ctrls, int count, double tol, int stop, int max_iter, int step) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    Ctrl c{};
    c.tol = tol;
    c.stop = stop;
    c.max_iter = max_iter;
    c.step = step;
    *ctrls[k] = c;
}

hipError_t launch_ctrl_init_many(Ctrl* const* ctrls, int count, double tol, int stop, int max_iter, int step,
                                 hipStream_t s) {
    if (count <= 0) return hipSuccess;
    k_ctrl_init_many<<<(count + 255) / 256, 256, 0, s>>>(ctrls, count, tol, stop, max_iter, step);
    return hipGetLastError();
}

hipError_t launch_finalize(const double* partials, int ntiles, Ctrl* ctrl, double* out2, int mode,
                           hipStream_t s, const Ctrl* gate, Ctrl* cyc, int cycles) {
    k_finalize<<<1, kFinBlock, 0, s>>>(partials, ntiles, ctrl, out2, mode, gate, cyc, cycles);
    return hipGetLastError();
}

// ------------------------------------------------------------ ctrl gather
__global__ void k_gather_ctrl(Ctrl* const* src, Ctrl* dst, int count) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count) dst[k] = *src[k];
}

hipError_t launch_gather_ctrl(Ctrl* const* src, Ctrl* dst, int count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    k_gather_ctrl<<<(count + 255) / 256, 256, 0, s>>>(src, dst, count);
    return hipGetLastError();
}

// ------------------------------------------------------------- stream copy
// Plain streaming copy (16-byte vectors, grid-stride): the achievable HBM
// bandwidth reference for the roofline and the byte counter calibration.
__global__ __launch_bounds__(kBlock) void k_stream_copy(const double2* __restrict__ src, double2* __restrict__ dst,
                                                        size_t nvec) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < nvec; k += stride) dst[k] = src[k];
}

hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, int blocks, hipStream_t s) {
    const size_t nvec = bytes / 16;
    if (nvec == 0) return hipSuccess;
    k_stream_copy<<<blocks, kBlock, 0, s>>>((const double2*)src, (double2*)dst, nvec);
    return hipGetLastError();
}

// ------------------------------------------------------- field upload/copy
// Dense (m-pitched) FP64 field -> one or two pitched fields (perimeter included).
// Workgroups walk rows, threads the row's columns (no index division).
__global__ __launch_bounds__(kBlock) void k_write_field(const double* __restrict__ src, double* __restrict__ d0,
                                                        double* __restrict__ d1, int m, int n, int P) {
    for (int j = blockIdx.x; j < n; j += gridDim.x) {
        const double* s = src + (size_t)j * m;
        double* a = d0 + (size_t)j * P;
        double* b = d1 != nullptr ? d1 + (size_t)j * P : nullptr;
        for (int i = threadIdx.x; i < m; i += blockDim.x) {
            const double v = s[i];
            a[i] = v;
            if (b != nullptr) b[i] = v;
        }
    }
}

hipError_t launch_write_field(const double* src, double* d0, double* d1, int m, int n, int P, hipStream_t s) {
    if (m <= 0 || n <= 0) return hipSuccess;
    const int nb = std::min(n, 16384);
    k_write_field<<<nb, kBlock, 0, s>>>(src, d0, d1, m, n, P);
    return hipGetLastError();
}

// ---------------------------------------------------- level boundary data
// Perimeter of a level's two buffers: the finest level's Dirichlet data at
// every stride-th node (src), or zero (src == NULL).
__global__ __launch_bounds__(kBlock) void k_level_boundary(double* d0, double* d1, const double* src, int m, int n,
                                                          int P, int Ps, int stride, const Ctrl* ctrl) {
    if (ctrl != nullptr && ctrl->done) return;
    const int per = 2 * m + 2 * (n - 2);
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < per; k += gridDim.x * blockDim.x) {
        int i, j;
        if (k < m) {
            i = k;
            j = 0;
        } else if (k < 2 * m) {
            i = k - m;
            j = n - 1;
        } else if (k < 2 * m + (n - 2)) {
            i = 0;
            j = 1 + (k - 2 * m);
        } else {
            i = m - 1;
            j = 1 + (k - 2 * m - (n - 2));
        }
        const double v = src != nullptr ? src[(size_t)j * stride * Ps + (size_t)i * stride] : 0.0;
        d0[(size_t)j * P + i] = v;
        if (d1 != nullptr) d1[(size_t)j * P + i] = v;
    }
}

hipError_t launch_level_boundary(double* d0, double* d1, const double* src, int m, int n, int P, int Ps, int stride,
                                 const Ctrl* ctrl, hipStream_t s) {
    const int per = 2 * m + 2 * (n - 2);
    k_level_boundary<<<(per + kBlock - 1) / kBlock, kBlock, 0, s>>>(d0, d1, src, m, n, P, Ps, stride, ctrl);
    return hipGetLastError();
}

// -------------------------------------------------------------------- copy
__global__ __launch_bounds__(kBlock) void k_copy(const double* src, double* dst, int m, int n, int P,
                                                 const Ctrl* ctrl) {
    if (ctrl != nullptr && ctrl->done) return;
    const size_t total = (size_t)n * P;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (size_t)gridDim.x * blockDim.x)
        dst[k] = src[k];
}

hipError_t launch_copy(const double* src, double* dst, int m, int n, int P, const Ctrl* ctrl, hipStream_t s) {
    const size_t total = (size_t)n * P;
    int nb = (int)((total + kBlock - 1) / kBlock);
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    k_copy<<<nb, kBlock, 0, s>>>(src, dst, m, n, P, ctrl);
    return hipGetLastError();
}

// Item blockIdx.y, its vectors strided over blockIdx.x.
__global__ __launch_bounds__(kBlock) void k_copy_many(const CopyItem* items) {
    const CopyItem it = items[blockIdx.y];
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < it.nvec; k += (size_t)gridDim.x * blockDim.x)
        it.dst[k] = it.src[k];
}

hipError_t launch_copy_many(const CopyItem* items, int count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    k_copy_many<<<dim3(64, count), kBlock, 0, s>>>(items);
    return hipGetLastError();
}

// ------------------------------------------------------- small-level subtree
// Dynamic LDS: the levels' u and b (T), then the coarsest right-hand side
// (double) at the next 8-byte boundary.
template <typename T>
__device__ __forceinline__ double* subtree_rhs(T* s, int lds_elems) {
    return reinterpret_cast<double*>(s + ((lds_elems * (int)sizeof(T) + 7) / 8) * 8 / (int)sizeof(T));
}

template <typename T>
__global__ __launch_bounds__(kSubBlock) void k_subtree(SubtreeArgs<T> S) {
    if (S.ctrl != nullptr && S.ctrl->done) return;
    extern __shared__ double lds_raw[];
    T* s = reinterpret_cast<T*>(lds_raw);
    subtree_block<T>(S, s, subtree_rhs(s, S.lds_elems));
}

template <typename T>
__global__ __launch_bounds__(kSubBlock) void k_batch_subtree(const BatchItem* items, int count) {
    const BatchItem& it = items[blockIdx.x];
    if (it.ctrl != nullptr && it.ctrl->done) return;
    const SubtreeArgs<T>& S = *reinterpret_cast<const SubtreeArgs<T>*>(it.sub);
    extern __shared__ double lds_raw[];
    T* s = reinterpret_cast<T*>(lds_raw);
    subtree_block<T>(S, s, subtree_rhs(s, S.lds_elems));
}

template <typename T>
hipError_t launch_subtree(const SubtreeArgs<T>& a, hipStream_t s) {
    if (a.nlev < 2 || a.nlev > kMaxSub) return hipErrorInvalidValue;
    k_subtree<T><<<1, kSubBlock, a.lds_bytes, s>>>(a);
    return hipGetLastError();
}
template hipError_t launch_subtree<double>(const SubtreeArgs<double>&, hipStream_t);
template hipError_t launch_subtree<float>(const SubtreeArgs<float>&, hipStream_t);

hipError_t launch_batch_subtree(int dt, const BatchItem* items, int count, int lds_bytes, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    if (dt == 0)
        k_batch_subtree<double><<<count, kSubBlock, lds_bytes, s>>>(items, count);
    else
        k_batch_subtree<float><<<count, kSubBlock, lds_bytes, s>>>(items, count);
    return hipGetLastError();
}

hipError_t subtree_set_lds_limit(int bytes) {
    const void* fns[4] = {(const void*)k_subtree<double>, (const void*)k_subtree<float>,
                          (const void*)k_batch_subtree<double>, (const void*)k_batch_subtree<float>};
    for (const void* f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace lap
