// Merged ("persistent") launches of the ragged batch path: one launch runs
// one operation of a V-cycle (or of an ADI iteration) for every grid of the
// batch at once.  The launch covers the concatenated tile lists of all
// grids; a fixed grid of workgroups walks it (tile t, t + #waves, ...), each
// wavefront finds the grid of its tile by binary search over the tile
// offsets, skips grids whose control block says done, and calls the same
// per-tile function as the single-grid kernel, with that grid's arguments
// and tiling.  Every wavefront's loop is bounded, so the grid drains.
#include "stencil_tiles.hpp"

namespace lap {


__device__ __forceinline__ Tiling item_tiling(const BatchItem& it) {
    Tiling t;
    t.V = it.V;
    t.ty = it.ty;
    t.nwin = it.nwin;
    t.nchunk = it.nchunk;
    t.ntiles = it.ntiles;
    t.H = it.H;
    return t;
}

template <typename T, int FLS>
__device__ __forceinline__ void batch_sweep_tile(const BatchItem& it, int lt, int lane) {
    SweepArgs<T> A{};
    A.uin = (const T*)it.in;
    A.uout = (T*)it.out;
    A.f = (const T*)it.f;
    A.ec = (const T*)it.ec;
    A.partials = it.partials;
    A.ctrl = nullptr;
    A.m = it.m;
    A.n = it.n;
    A.P = it.P;
    A.mc = it.mc;
    A.nc = it.nc;
    A.Pc = it.Pc;
    A.cx = (T)it.cx;
    A.cy = (T)it.cy;
    A.d = (T)it.d;
    A.inv_d = (T)it.inv_d;
    A.omega = (T)it.omega;
    A.tl = item_tiling(it);
    const bool hf = (it.flags & SW_F) != 0;
    switch (it.V) {
        case 1: hf ? sweep_tile<T, 1, FLS | SW_F>(A, lt, lane) : sweep_tile<T, 1, FLS>(A, lt, lane); break;
        case 2: hf ? sweep_tile<T, 2, FLS | SW_F>(A, lt, lane) : sweep_tile<T, 2, FLS>(A, lt, lane); break;
        default: hf ? sweep_tile<T, 4, FLS | SW_F>(A, lt, lane) : sweep_tile<T, 4, FLS>(A, lt, lane); break;
    }
}

template <typename T, int FLS>
__global__ __launch_bounds__(kBlock) void k_batch_sweep(const BatchItem* items, const int* tmap, int total) {
    const int nw = gridDim.x * kWavesPerBlock;
    const int lane = threadIdx.x & 63;
    for (int t = xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + wave_in_block(); t < total; t += nw) {
        const BatchItem& it = items[tmap[t]];
        if (it.ctrl->done) continue;
        batch_sweep_tile<T, FLS>(it, t - it.tile0, lane);
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_batch_restrict(const BatchItem* items, const int* tmap, int total) {
    const int nw = gridDim.x * kWavesPerBlock;
    const int lane = threadIdx.x & 63;
    for (int t = xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + wave_in_block(); t < total; t += nw) {
        const BatchItem& it = items[tmap[t]];
        if (it.ctrl->done) continue;
        RestrictArgs<T> A{};
        A.u = (const T*)it.in;
        A.f = (const T*)it.f;
        A.bc = (T*)it.bc;
        A.uc0 = (T*)it.out;
        A.ctrl = nullptr;
        A.m = it.m;
        A.n = it.n;
        A.P = it.P;
        A.mc = it.mc;
        A.nc = it.nc;
        A.Pc = it.Pc;
        A.cx = (T)it.cx;
        A.cy = (T)it.cy;
        A.d = (T)it.d;
        A.tl = item_tiling(it);
        const int lt = t - it.tile0;
        if (it.flags & SW_RDIFF) {
            switch (it.V) {
                case 1: restrict_tile<T, 1, true>(A, lt, lane); break;
                case 2: restrict_tile<T, 2, true>(A, lt, lane); break;
                default: restrict_tile<T, 4, true>(A, lt, lane); break;
            }
        } else {
            switch (it.V) {
                case 1: restrict_tile<T, 1>(A, lt, lane); break;
                case 2: restrict_tile<T, 2>(A, lt, lane); break;
                default: restrict_tile<T, 4>(A, lt, lane); break;
            }
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_batch_resnorm(const BatchItem* items, const int* tmap, int total) {
    const int nw = gridDim.x * kWavesPerBlock;
    const int lane = threadIdx.x & 63;
    for (int t = xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + wave_in_block(); t < total; t += nw) {
        const BatchItem& it = items[tmap[t]];
        if (it.ctrl->done) continue;
        ResidualArgs<double> A{};
        A.u = (const double*)it.in;
        A.f = (const double*)it.f;
        A.r = nullptr;
        A.partials = it.partials;
        A.ctrl = nullptr;
        A.m = it.m;
        A.n = it.n;
        A.P = it.P;
        A.cx = it.cx;
        A.cy = it.cy;
        A.d = it.d;
        A.tl = item_tiling(it);
        residual_tile<double, kNormPassV>(A, t - it.tile0, lane);   // the canonical norm tiling
    }
}

__global__ __launch_bounds__(kBlock) void k_batch_defect(const BatchItem* items, const int* tmap, int total) {
    const int nw = gridDim.x * kWavesPerBlock;
    const int lane = threadIdx.x & 63;
    for (int t = xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + wave_in_block(); t < total; t += nw) {
        const BatchItem& it = items[tmap[t]];
        if (it.ctrl->done) continue;
        DefectArgs A{};
        A.psi_in = (const double*)it.in;
        A.psi_out = (double*)it.out;
        A.e = (const float*)it.ec;
        A.f = (const double*)it.f;
        A.rhs = (float*)it.bc;
        A.ezero = (float*)it.e;
        A.partials = it.partials;
        A.ctrl = nullptr;
        A.m = it.m;
        A.n = it.n;
        A.P = it.P;
        A.cx = it.cx;
        A.cy = it.cy;
        A.d = it.d;
        A.tl = item_tiling(it);
        defect_tile<kNormDefectV>(A, t - it.tile0, lane);   // the canonical defect tiling
    }
}

// One workgroup per grid.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_batch_coarse(const BatchItem* items, int count) {
    __shared__ double rhs[1024];
    for (int k = blockIdx.x; k < count; k += gridDim.x) {
        const BatchItem& it = items[k];
        if (it.ctrl->done) continue;
        CoarseArgs<T> A{};
        A.u = (const T*)it.in;
        A.b = (const T*)it.f;
        A.out = (T*)it.out;
        A.minv = it.minv;
        A.work = it.cwork;
        A.bw = it.cbw;
        A.ifast = it.cifast;
        A.ctrl = nullptr;
        A.m = it.m;
        A.n = it.n;
        A.P = it.P;
        A.cx = it.cx;
        A.cy = it.cy;
        coarse_block<T>(A, rhs);
        __syncthreads();
    }
}

__global__ __launch_bounds__(kFinBlock) void k_batch_finalize(const BatchItem* items, int count) {
    __shared__ double ss[kFinBlock / 64], sm[kFinBlock / 64];
    for (int k = blockIdx.x; k < count; k += gridDim.x) {
        const BatchItem& it = items[k];
        if (it.ctrl->done || (it.gate != nullptr && it.gate->done)) continue;
        finalize_step(it.partials, it.ntiles, it.ctrl, nullptr, 0, it.cyc, it.cycles, ss, sm);
        __syncthreads();
    }
}

template <typename T>
static hipError_t launch_batch_t(int kind, int fl, const BatchItem* items, const int* tmap, int count, int total,
                                 int blocks,
                                 hipStream_t s) {
    const dim3 g(blocks), b(kBlock);
    switch (kind) {
        case BK_SWEEP:
            switch (fl) {
                case 0: k_batch_sweep<T, 0><<<g, b, 0, s>>>(items, tmap, total); break;
                case SW_ZERO: k_batch_sweep<T, SW_ZERO><<<g, b, 0, s>>>(items, tmap, total); break;
                case SW_PROLONG: k_batch_sweep<T, SW_PROLONG><<<g, b, 0, s>>>(items, tmap, total); break;
                case SW_PROLONG | SW_PONLY:
                    k_batch_sweep<T, SW_PROLONG | SW_PONLY><<<g, b, 0, s>>>(items, tmap, total);
                    break;
                case SW_NORM: k_batch_sweep<T, SW_NORM><<<g, b, 0, s>>>(items, tmap, total); break;
                default: return hipErrorInvalidValue;
            }
            break;
        case BK_RESTRICT: k_batch_restrict<T><<<g, b, 0, s>>>(items, tmap, total); break;
        case BK_COARSE: k_batch_coarse<T><<<g, b, 0, s>>>(items, count); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch(int kind, int dt, int step_flags, const BatchItem* items, const int* tmap, int count, int total,
                        int blocks,
                        hipStream_t s) {
    if (count <= 0) return hipSuccess;
    if (blocks < 1) blocks = 1;
    switch (kind) {
        case BK_SWEEP:
        case BK_RESTRICT:
        case BK_COARSE:
            return dt == 0 ? launch_batch_t<double>(kind, step_flags, items, tmap, count, total, blocks, s)
                           : launch_batch_t<float>(kind, step_flags, items, tmap, count, total, blocks, s);
        case BK_FINALIZE: k_batch_finalize<<<blocks, kFinBlock, 0, s>>>(items, count); break;
        case BK_RESNORM: k_batch_resnorm<<<blocks, kBlock, 0, s>>>(items, tmap, total); break;
        case BK_DEFECT: k_batch_defect<<<blocks, kBlock, 0, s>>>(items, tmap, total); break;
        case BK_ADI_ROWS:
        case BK_ADI_COLS: return launch_batch_adi(kind, step_flags, dt, items, tmap, total, blocks, s);
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lap
