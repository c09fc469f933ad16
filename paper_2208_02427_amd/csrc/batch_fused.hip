// Merged fused passes of the ragged batch path: the tile lists of all grids
// concatenated, a persistent grid of workgroups walking them (see
// batch_kernels.hip), each tile running the same fused_tile as the
// single-grid kernel with its grid's arguments, tiling and halo.
#include "fused_tiles.hpp"

namespace lap {


template <typename T, int FLS, int V>
__device__ __forceinline__ void batch_fused_tile(const BatchItem& it, int lt, int lane) {
    SweepArgs<T> A{};
    A.uin = (const T*)it.in;
    A.uout = (T*)it.out;
    A.f = (const T*)it.f;
    A.ec = (const T*)it.ec;
    A.bc = (T*)it.bc;
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
    A.tl.V = it.V;
    A.tl.ty = it.ty;
    A.tl.nwin = it.nwin;
    A.tl.nchunk = it.nchunk;
    A.tl.ntiles = it.ntiles;
    A.tl.H = it.H;
    if constexpr ((FLS & SW_DEF) != 0) {
        A.uin = (const T*)it.e;
        A.uout = nullptr;
        A.psi_in = (const double*)it.in;
        A.psi_out = (double*)it.out;
        A.f64 = it.f64;
        A.rhs_out = (T*)it.bc;
        A.bc = nullptr;
        A.dcx = it.cx;
        A.dcy = it.cy;
        A.dd = it.d;
        A.rowpart = it.rowpart;
    }
    if (it.flags & SW_F)
        fused_tile<T, V, FLS | SW_F>(A, lt, lane);
    else
        fused_tile<T, V, FLS>(A, lt, lane);
}

// One kernel per columns-per-lane V (the host groups items by V), so a
// launch is compiled, and occupies registers, for its own V only.
template <typename T, int FLS, int V>
__global__ __launch_bounds__(kBlock) void k_batch_fused(const BatchItem* items, const int* tmap, int total) {
    const int nw = gridDim.x * kWavesPerBlock;
    const int lane = threadIdx.x & 63;
    for (int t = xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + (int)(threadIdx.x >> 6); t < total; t += nw) {
        const BatchItem& it = items[tmap[t]];
        if (it.ctrl->done) continue;
        batch_fused_tile<T, FLS, V>(it, t - it.tile0, lane);
    }
}

// step flags without SW_F (the right-hand side is a per-grid runtime choice)
#define LAP_BATCH_FUSED_FLAGS(X)                                                           \
    X(SW_TWO) X(SW_TWO | SW_ZERO) X(SW_TWO | SW_NORM) X(SW_TWO | SW_PROLONG) X(SW_RESTRICT) \
    X(SW_RESTRICT | SW_ZERO) X(SW_RESTRICT | SW_NORM) X(SW_RESTRICT | SW_TWO)              \
    X(SW_RESTRICT | SW_TWO | SW_ZERO) X(SW_RESTRICT | SW_TWO | SW_NORM) X(SW_DEF | SW_PROLONG | SW_TWO)
// FP32 only: the level-0 passes of the cycles after the first of a mixed step
// of several cycles (residual in difference form; four-sweep passes)
#define LAP_BATCH_FUSED_FLAGS32(X) \
    X(SW_RDIFF | SW_RESTRICT | SW_TWO) X(SW_RDIFF | SW_RESTRICT) X(SW_FOUR | SW_PROLONG | SW_RESTRICT | SW_RDIFF)

template <typename T, int V>
static hipError_t launch_batch_fused_v(int fl, const BatchItem* items, const int* tmap, int total, int blocks,
                                       hipStream_t s) {
    const dim3 g(blocks), b(kBlock);
    switch (fl) {
#define LAP_CASE(F)                                                       \
    case (F):                                                             \
        k_batch_fused<T, (F), V><<<g, b, 0, s>>>(items, tmap, total);     \
        break;
        LAP_BATCH_FUSED_FLAGS(LAP_CASE)
        default:
            if constexpr (sizeof(T) == 4) {
                switch (fl) {
                    LAP_BATCH_FUSED_FLAGS32(LAP_CASE)
                    default: return hipErrorInvalidValue;
                }
            } else {
                return hipErrorInvalidValue;
            }
#undef LAP_CASE
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_batch_fused_t(int fl, int V, const BatchItem* items, const int* tmap, int total, int blocks,
                                       hipStream_t s) {
    switch (V) {
        case 1: return launch_batch_fused_v<T, 1>(fl, items, tmap, total, blocks, s);
        case 2: return launch_batch_fused_v<T, 2>(fl, items, tmap, total, blocks, s);
        case 4: return launch_batch_fused_v<T, 4>(fl, items, tmap, total, blocks, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_fused(int dt, int step_flags, int V, const BatchItem* items, const int* tmap, int total,
                              int blocks, hipStream_t s) {
    if (total <= 0) return hipSuccess;
    if (blocks < 1) blocks = 1;
    return dt == 0 ? launch_batch_fused_t<double>(step_flags, V, items, tmap, total, blocks, s)
                   : launch_batch_fused_t<float>(step_flags, V, items, tmap, total, blocks, s);
}

}  // namespace lap
