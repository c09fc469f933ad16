// Fused streaming passes of one grid (see fused_tiles.hpp): pre-smoothing
// (one or two sweeps, from zero / with the input's residual norms) with the
// residual + full weighting of its result, post-smoothing (bilinear
// correction + two sweeps), and the mixed loop's FP32 post-smoothing of the
// finest level merged with the next FP64 defect correction.  One wavefront per (window, chunk) tile, blocks
// of four wavefronts dealt XCD-contiguously as in the one-sweep kernel.
#include "fused_tiles.hpp"

namespace lap {

// FP64 restricting passes of two columns per lane without a source sit just
// above 128 registers with whole ring turns; held to 128, they keep four
// waves per SIMD.
template <typename T, int V, int FL>
constexpr int fused_min_waves() {
    return (sizeof(T) == 8 && V == 2 && (FL & (SW_RESTRICT | SW_F | SW_PROLONG)) == SW_RESTRICT) ? 4 : 1;
}

template <typename T, int V, int FL>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(fused_min_waves<T, V, FL>())))
void k_fused(SweepArgs<T> A) {
    if (A.ctrl != nullptr && A.ctrl->done) return;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    // the wave index stays a vector value here: with a uniform one
    // (wave_in_block) the post-smoothing pass measured 3-7% slower on MI355X
    const int tile = b * kWavesPerBlock + (int)(threadIdx.x >> 6);
    if (tile >= A.tl.ntiles) return;
    fused_tile<T, V, FL>(A, tile, threadIdx.x & 63);
}

// The flag sets a V-cycle plan uses (SW_F added where a right-hand side exists).
#define LAP_FUSED_FLAGS(X)                                                                         \
    X(SW_TWO) X(SW_TWO | SW_F) X(SW_TWO | SW_ZERO | SW_F) X(SW_TWO | SW_NORM)                    \
    X(SW_TWO | SW_NORM | SW_F) X(SW_TWO | SW_PROLONG) X(SW_TWO | SW_PROLONG | SW_F)              \
    X(SW_RESTRICT) X(SW_RESTRICT | SW_F) X(SW_RESTRICT | SW_ZERO | SW_F) X(SW_RESTRICT | SW_NORM) \
    X(SW_RESTRICT | SW_NORM | SW_F) X(SW_RESTRICT | SW_TWO) X(SW_RESTRICT | SW_TWO | SW_F)       \
    X(SW_RESTRICT | SW_TWO | SW_ZERO | SW_F) X(SW_RESTRICT | SW_TWO | SW_NORM)                    \
    X(SW_RESTRICT | SW_TWO | SW_NORM | SW_F) X(SW_DEF | SW_PROLONG | SW_TWO | SW_F)                  \
    X(SW_PROBE | SW_RESTRICT | SW_TWO | SW_NORM) X(SW_PROBE | SW_RESTRICT | SW_TWO | SW_NORM | SW_F)  \
    X(SW_PROBE | SW_RESTRICT | SW_NORM) X(SW_PROBE | SW_RESTRICT | SW_NORM | SW_F)                \
    X(SW_PROBE | SW_TWO | SW_NORM) X(SW_PROBE | SW_TWO | SW_NORM | SW_F)                          \
    X(SW_RDIFF | SW_RESTRICT | SW_TWO | SW_F) X(SW_RDIFF | SW_RESTRICT | SW_F)                   \
    X(SW_FOUR | SW_PROLONG | SW_RESTRICT | SW_RDIFF | SW_F)

template <typename T, int V>
static hipError_t launch_fused_v(const SweepArgs<T>& a, int flags, hipStream_t s) {
    const dim3 grid(blocks_for(a.tl)), block(kBlock);
    switch (flags) {
#define LAP_CASE(F)                                      \
    case (F):                                            \
        k_fused<T, V, (F)><<<grid, block, 0, s>>>(a);    \
        break;
        LAP_FUSED_FLAGS(LAP_CASE)
#undef LAP_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fused(const SweepArgs<T>& a, int flags, hipStream_t s) {
    // the halo must cover every fused stage
    const int need = ((flags & SW_FOUR) ? 8 : (flags & SW_TWO) ? 4 : 2) + ((flags & (SW_RESTRICT | SW_DEF)) ? 2 : 0);
    if (a.tl.H < need) return hipErrorInvalidValue;
    switch (a.tl.V) {
        case 1: return launch_fused_v<T, 1>(a, flags, s);
        case 2: return launch_fused_v<T, 2>(a, flags, s);
        case 4: return launch_fused_v<T, 4>(a, flags, s);
        default: return hipErrorInvalidValue;
    }
}
template hipError_t launch_fused<double>(const SweepArgs<double>&, int, hipStream_t);
template hipError_t launch_fused<float>(const SweepArgs<float>&, int, hipStream_t);

}  // namespace lap
