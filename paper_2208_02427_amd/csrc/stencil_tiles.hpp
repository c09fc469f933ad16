// Per-tile device functions of the stencil kernels (red-black sweep,
// residual + full weighting, residual norms, FP64 defect correction, coarse
// solve, norm finalisation).  The single-grid kernels (stencil_kernels.hip)
// and the merged ragged-batch kernels (batch_kernels.hip) both call these,
// so a grid's arithmetic is the same code whichever way it is launched.
#pragma once

#include "lap_kernels.hpp"

namespace lap {

// ------------------------------------------------------------------ helpers
template <typename T, int V> struct VecT;
template <> struct VecT<double, 1> { using type = double; };
template <> struct VecT<double, 2> { using type = double __attribute__((ext_vector_type(2))); };
template <> struct VecT<double, 4> { using type = double __attribute__((ext_vector_type(4))); };
template <> struct VecT<float, 1> { using type = float; };
template <> struct VecT<float, 2> { using type = float __attribute__((ext_vector_type(2))); };
template <> struct VecT<float, 4> { using type = float __attribute__((ext_vector_type(4))); };

template <typename T, int V>
__device__ __forceinline__ void ldv(T (&x)[V], const T* p) {
    using VT = typename VecT<T, V>::type;
    VT v = *reinterpret_cast<const VT*>(p);
    if constexpr (V == 1) {
        x[0] = v;
    } else {
#pragma unroll
        for (int e = 0; e < V; ++e) x[e] = v[e];
    }
}

template <typename T, int V, bool NT = false>
__device__ __forceinline__ void stv(T* p, const T (&x)[V]) {
    using VT = typename VecT<T, V>::type;
    VT v;
    if constexpr (V == 1) {
        v = x[0];
    } else {
#pragma unroll
        for (int e = 0; e < V; ++e) v[e] = x[e];
    }
    if constexpr (NT)
        __builtin_nontemporal_store(v, reinterpret_cast<VT*>(p));
    else
        *reinterpret_cast<VT*>(p) = v;
}

template <typename T, int V>
__device__ __forceinline__ void zero(T (&x)[V]) {
#pragma unroll
    for (int e = 0; e < V; ++e) x[e] = T(0);
}

template <typename T, int V>
__device__ __forceinline__ void copy(T (&dst)[V], const T (&src)[V]) {
#pragma unroll
    for (int e = 0; e < V; ++e) dst[e] = src[e];
}

// Index of the calling wavefront in its workgroup, as a wave-uniform value
// (threadIdx.x >> 6 is the same on every lane, but the compiler cannot know
// it; read from lane 0, every row and chunk test derived from it becomes a
// scalar branch instead of an exec-masked vector one).
__device__ __forceinline__ int wave_in_block() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Workgroups are dealt to the XCDs round-robin; give XCD x the contiguous
// tile range [x*per, (x+1)*per) so neighbouring tiles share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int per = nb / kXcds;
    return (b % kXcds) * per + (b / kXcds);
}

// The value held by the previous / next lane of the wavefront, moved by a
// DPP wavefront shift: one VALU move per 32 bits instead of a permute
// through LDS.  The first / last lane, which has no such neighbour, gets 0:
// in every tile those lanes' outer columns are halo columns, whose values
// never reach an output.  Every lane must be active (the stencil tiles call
// these in wave-uniform control flow).
constexpr int kDppWaveShr1 = 0x138;   // lane i reads lane i - 1
constexpr int kDppWaveShl1 = 0x130;   // lane i reads lane i + 1
template <int CTRL, typename T>
__device__ __forceinline__ T lane_shift(T x) {
    if constexpr (sizeof(T) == 8) {
        const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
        const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xf, 0xf, true);
        const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xf, 0xf, true);
        return __builtin_bit_cast(T, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
    } else {
        return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, 0xf, 0xf, true));
    }
}
template <typename T>
__device__ __forceinline__ T lane_prev(T x) { return lane_shift<kDppWaveShr1>(x); }
template <typename T>
__device__ __forceinline__ T lane_next(T x) { return lane_shift<kDppWaveShl1>(x); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// Per-lane column bookkeeping of one window (halo H columns per side).
template <int V>
struct Cols {
    int ws, i0;
    bool vin;                 // whole vector inside [0, P)
    bool cint[V];             // interior column
    bool cout[V];             // interior and inside this window's output range
    bool all_out;
    __device__ __forceinline__ Cols(int win, int lane, int m, int P, int H) {
        ws = win * win_step(V, H) - win_left(V, H);
        i0 = ws + lane * V;
        vin = (i0 >= 0) && (i0 + V <= P);
        all_out = true;
#pragma unroll
        for (int e = 0; e < V; ++e) {
            const int i = i0 + e;
            cint[e] = (i >= 1) && (i <= m - 2);
            cout[e] = cint[e] && (i >= ws + H) && (i < ws + 64 * V - H);
            all_out = all_out && cout[e];
        }
    }
};

// The relaxation factor of each of a lane's columns for each row parity JP:
// omega where the node is interior and has the colour the sweep updates on
// that row, else 0.  An update psi <- fma(w, t - psi, psi) with w = 0 leaves
// psi unchanged (up to the sign of a zero), so the sweeps need no per-lane
// branch; for even V the colour of element e is fixed by e and JP and the
// elements of the other colour are skipped at compile time.
template <typename T, int V>
struct OmegaMask {
    T w[2][V];
    __device__ __forceinline__ OmegaMask(const Cols<V>& c, int ipar, T om) {
#pragma unroll
        for (int jp = 0; jp < 2; ++jp)
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const bool upd = ((((V % 2 == 0) ? 0 : ipar) + e + jp) & 1) == 0;
                w[jp][e] = (upd && c.cint[e]) ? om : T(0);
            }
    }
};
template <int V, int JP>
__host__ __device__ constexpr bool colour_skip(int e) { return V % 2 == 0 && ((e + JP) & 1) != 0; }

// P is the row stride (negative for a flipped view); vin says the lane's
// columns lie inside the row.
template <typename T, int V>
__device__ __forceinline__ void load_row(T (&x)[V], const T* base, int j, int n, int P, int i0, bool vin) {
    if (base != nullptr && vin && j >= 0 && j < n)
        ldv<T, V>(x, base + (ptrdiff_t)j * P + i0);
    else
        zero<T, V>(x);
}

template <typename T, int V, bool NT = false>
__device__ __forceinline__ void store_row(T* base, const T (&x)[V], int j, int P, const Cols<V>& c) {
    T* p = base + (ptrdiff_t)j * P + c.i0;
    if (c.vin && c.all_out) {
        stv<T, V, NT>(p, x);
    } else {
#pragma unroll
        for (int e = 0; e < V; ++e) {
            if (!c.cout[e]) continue;
            if constexpr (NT)
                __builtin_nontemporal_store(x[e], p + e);
            else
                p[e] = x[e];
        }
    }
}

// store_row with a wave-uniform runtime choice of nontemporal stores
template <typename T, int V>
__device__ __forceinline__ void store_row_nt(bool nt, T* base, const T (&x)[V], int j, int P, const Cols<V>& c) {
    if (nt)
        store_row<T, V, true>(base, x, j, P, c);
    else
        store_row<T, V, false>(base, x, j, P, c);
}

// Bilinear interpolation of a coarse correction, streamed with the fine rows.
// A lane owning fine columns i0..i0+V-1 needs coarse columns I0 = i0>>1 ..
// I0 + V2 (V2 = max(1, V/2)); it loads I0..I0+V2-1 with one vector load per
// coarse row and takes column I0+V2 from the next lane.  The two coarse rows
// J, J+1 around the current fine row stay in registers, and rows J+2 and J+3
// are already in flight (a raw load is completed with the neighbour's column
// only when it moves up), so the stream of fine rows does not wait on a
// coarse load: fine rows arrive in increasing order and each coarse row is
// loaded once per wave, four to six fine rows before it is used.
template <typename T, int V>
struct Prolong {
    static constexpr int V2 = V >= 2 ? V / 2 : 1;
    T lo[V2 + 1], hi[V2 + 1];   // coarse rows Jcur, Jcur+1 (entry V2 from the next lane)
    T nraw[V2], nlast;          // coarse row Jcur+2 as loaded (nlast: lane 63's column I0+V2)
    T mraw[V2], mlast;          // coarse row Jcur+3 as loaded (two coarse rows in flight)
    int Jcur;
    // Pc: the coarse row length bound (pitch), Ps: the coarse row stride
    __device__ __forceinline__ void issue(T (&raw)[V2], T& last, const T* ec, int J, int nc, int Pc, int Ps,
                                          int I0) {
        if (J >= 0 && J < nc && I0 >= 0 && I0 + V2 <= Pc)
            ldv<T, V2>(raw, ec + (ptrdiff_t)J * Ps + I0);
        else
            zero<T, V2>(raw);
        // the last lane has no right neighbour, but its halo columns still need
        // coarse column I0 + V2 (the sweep reads the window's last column)
        last = T(0);
        if ((threadIdx.x & 63) == 63) {
            const int I = I0 + V2;
            if (J >= 0 && J < nc && I >= 0 && I < Pc) last = ec[(ptrdiff_t)J * Ps + I];
        }
    }
    __device__ __forceinline__ void complete(T (&x)[V2 + 1]) {
#pragma unroll
        for (int q = 0; q < V2; ++q) x[q] = nraw[q];
        const T r = lane_next(nraw[0]);
        x[V2] = (threadIdx.x & 63) == 63 ? nlast : r;
    }
    __device__ __forceinline__ void init(const T* ec, int j, int nc, int Pc, int Ps, int i0) {
        Jcur = j >> 1;
        issue(nraw, nlast, ec, Jcur, nc, Pc, Ps, i0 >> 1);
        complete(lo);
        issue(nraw, nlast, ec, Jcur + 1, nc, Pc, Ps, i0 >> 1);
        complete(hi);
        issue(nraw, nlast, ec, Jcur + 2, nc, Pc, Ps, i0 >> 1);
        issue(mraw, mlast, ec, Jcur + 3, nc, Pc, Ps, i0 >> 1);
    }
    // add P(ec) to fine row j (j non-decreasing between calls)
    __device__ __forceinline__ void add(T (&x)[V], const T* ec, int j, int n, int nc, int Pc, int Ps, int i0,
                                        int m) {
        const int J = j >> 1;
        while (Jcur < J) {   // at most one step per fine row
#pragma unroll
            for (int q = 0; q <= V2; ++q) lo[q] = hi[q];
            complete(hi);
            ++Jcur;
            copy<T, V2>(nraw, mraw);
            nlast = mlast;
            issue(mraw, mlast, ec, Jcur + 3, nc, Pc, Ps, i0 >> 1);
        }
        if (j < 0 || j >= n) return;
        const bool t = (j & 1) != 0;                  // wave-uniform
        // branch-free: every lane evaluates the same instructions; for even V
        // the coarse index and the column parity of element e are compile-time
#pragma unroll
        for (int e = 0; e < V; ++e) {
            const int i = i0 + e;
            T e00, e10, e01, e11;
            bool s;
            if constexpr (V % 2 == 0) {
                s = (e & 1) != 0;
                e00 = lo[e >> 1];
                e10 = lo[(e >> 1) + 1];
                e01 = hi[e >> 1];
                e11 = hi[(e >> 1) + 1];
            } else {
                s = (i & 1) != 0;                      // V == 1: q = 0 for every lane
                e00 = lo[0];
                e10 = lo[1];
                e01 = hi[0];
                e11 = hi[1];
            }
            const T p_even = t ? (e00 + e01) * T(0.5) : e00;
            const T p_odd = t ? ((e00 + e10) + (e01 + e11)) * T(0.25) : (e00 + e10) * T(0.5);
            const T p = s ? p_odd : p_even;
            x[e] = (i >= 0 && i < m) ? x[e] + p : x[e];
        }
    }
};

// ------------------------------------------------------------ red-black sweep
// Input row j as stored (zero for a zero start), before any correction.
template <typename T, int V, int FL>
__device__ __forceinline__ void sweep_load_raw(T (&x)[V], const SweepArgs<T>& A, int j, const Cols<V>& c) {
    if constexpr (FL & SW_ZERO)
        zero<T, V>(x);
    else
        load_row<T, V>(x, A.uin, j, A.n, A.Ps, c.i0, c.vin);
}

// Whether input rows take the bilinear correction P(ec): passes with the
// prolongation, except a zero start without SW_PONLY.  (A zero start with
// SW_PONLY is the interpolated coarse solution alone.)
template <int FL>
__host__ __device__ constexpr bool adds_correction() {
    return (FL & SW_PROLONG) != 0 && ((FL & SW_ZERO) == 0 || (FL & SW_PONLY) != 0);
}

// Input row j of a sweep: as stored, plus the correction where the pass adds it.
template <typename T, int V, int FL>
__device__ __forceinline__ void sweep_load(T (&x)[V], const SweepArgs<T>& A, int j, const Cols<V>& c,
                                           Prolong<T, V>& pr) {
    sweep_load_raw<T, V, FL>(x, A, j, c);
    if constexpr (adds_correction<FL>()) pr.add(x, A.ec, j, A.n, A.nc, A.Pc, A.Pcs, c.i0, A.m);
}

template <typename T, int V, int FL>
__device__ __forceinline__ void sweep_loadf(T (&x)[V], const SweepArgs<T>& A, int j, const Cols<V>& c) {
    if constexpr (FL & SW_F)
        load_row<T, V>(x, A.f, j, A.n, A.Ps, c.i0, c.vin);
    else
        zero<T, V>(x);
}

// State carried down the rows of one window (registers).
template <typename T, int V>
struct SweepRegs {
    T a[V], b[V], c[V], d[V];   // rows j-2 (final), j-1 (red done), j (old -> red), j+1 (old)
    T fb[V], fc[V], fd[V];      // f at rows j-1, j, j+1
    T dn[V], fdn[V];            // prefetched row j+2
    T dnn[V], fdnn[V];          // prefetched row j+3
    T bo[V];                    // old row j-1 (norm of the input)
    double s2, mx;
    Prolong<T, V> pr;           // coarse rows of a fused prolongation
};

template <typename T, int V, int FL, int JP>
__device__ __forceinline__ void sweep_step(const SweepArgs<T>& A, SweepRegs<T, V>& R, const Cols<V>& c,
                                           int j, int j0, int j1, const OmegaMask<T, V>& wm) {
    // rotate in the prefetched row j+1 (the correction is added as it enters),
    // prefetch row j+3 (two rows in flight)
    copy<T, V>(R.d, R.dn);
    if constexpr (adds_correction<FL>()) R.pr.add(R.d, A.ec, j + 1, A.n, A.nc, A.Pc, A.Pcs, c.i0, A.m);
    copy<T, V>(R.fd, R.fdn);
    copy<T, V>(R.dn, R.dnn);
    copy<T, V>(R.fdn, R.fdnn);
    if (j + 3 <= j1 + 2) {
        sweep_load_raw<T, V, FL>(R.dnn, A, j + 3, c);
        sweep_loadf<T, V, FL>(R.fdnn, A, j + 3, c);
    }
    const T cx = A.cx, cy = A.cy, inv_d = A.inv_d;

    // old row j: neighbours across lanes
    const T cW = lane_prev(R.c[V - 1]);
    const T cE = lane_next(R.c[0]);

    if constexpr (FL & SW_NORM) {
        if (j >= j0 && j <= j1) {
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const T W = e > 0 ? R.c[e - 1] : cW;
                const T E = e < V - 1 ? R.c[e + 1] : cE;
                const T L = fma(-A.d, R.c[e], fma(cy, R.bo[e] + R.d[e], cx * (W + E)));
                const double r = c.cout[e] ? (double)(R.fc[e] - L) : 0.0;
                R.s2 = fma(r, r, R.s2);
                R.mx = fmax(R.mx, fabs(r));
            }
        }
        copy<T, V>(R.bo, R.c);
    }

    const bool rj = !(FL & SW_PONLY) && (j >= 1) && (j <= A.n - 2);
    const bool rjm = !(FL & SW_PONLY) && (j - 1 >= 1) && (j - 1 <= A.n - 2);

    // colour 0 ((i+j) even) on row j from old colour-1 neighbours
    if (rj) {
#pragma unroll
        for (int e = 0; e < V; ++e) {
            if (colour_skip<V, JP>(e)) continue;
            const T W = e > 0 ? R.c[e - 1] : cW;
            const T E = e < V - 1 ? R.c[e + 1] : cE;
            const T t = (fma(cy, R.b[e] + R.d[e], cx * (W + E)) - R.fc[e]) * inv_d;
            R.c[e] = fma(wm.w[JP][e], t - R.c[e], R.c[e]);
        }
    }
    // colour 1 on row j-1 ((i+j-1) odd) from the new colour-0 values
    const T bW = lane_prev(R.b[V - 1]);
    const T bE = lane_next(R.b[0]);
    if (rjm) {
#pragma unroll
        for (int e = 0; e < V; ++e) {
            if (colour_skip<V, JP>(e)) continue;
            const T W = e > 0 ? R.b[e - 1] : bW;
            const T E = e < V - 1 ? R.b[e + 1] : bE;
            const T t = (fma(cy, R.a[e] + R.c[e], cx * (W + E)) - R.fb[e]) * inv_d;
            R.b[e] = fma(wm.w[JP][e], t - R.b[e], R.b[e]);
        }
    }
    if (j - 1 >= j0 && j - 1 <= j1) store_row<T, V>(A.uout, R.b, j - 1, A.Ps, c);

    copy<T, V>(R.a, R.b);
    copy<T, V>(R.b, R.c);
    copy<T, V>(R.c, R.d);
    copy<T, V>(R.fb, R.fc);
    copy<T, V>(R.fc, R.fd);
}

template <typename T, int V, int FL>
__device__ __forceinline__ void sweep_tile(const SweepArgs<T>& A0, int tile, int lane) {
    SweepArgs<T> A = A0;
    A.Ps = A.P;
    A.Pcs = A.Pc;
    const int win = tile % A.tl.nwin, chunk = tile / A.tl.nwin;
    const Cols<V> c(win, lane, A.m, A.P, A.tl.H);
    const int j0 = 1 + chunk * A.tl.ty;          // odd
    const int j1 = min(j0 + A.tl.ty - 1, A.n - 2);
    const int ipar = c.i0 & 1;
    const OmegaMask<T, V> wm(c, ipar, A.omega);

    SweepRegs<T, V> R;
    R.s2 = 0.0;
    R.mx = 0.0;
    zero<T, V>(R.a);
    zero<T, V>(R.fb);
    if constexpr (FL & SW_PROLONG) R.pr.init(A.ec, j0 - 2, A.nc, A.Pc, A.Pcs, c.i0);
    sweep_load<T, V, FL>(R.b, A, j0 - 2, c, R.pr);
    sweep_load<T, V, FL>(R.c, A, j0 - 1, c, R.pr);
    sweep_loadf<T, V, FL>(R.fc, A, j0 - 1, c);
    sweep_load_raw<T, V, FL>(R.dn, A, j0, c);
    sweep_loadf<T, V, FL>(R.fdn, A, j0, c);
    sweep_load_raw<T, V, FL>(R.dnn, A, j0 + 1, c);
    sweep_loadf<T, V, FL>(R.fdnn, A, j0 + 1, c);
    if constexpr (FL & SW_NORM) copy<T, V>(R.bo, R.b);

    for (int j = j0 - 1; j <= j1 + 1; j += 2) {   // j0 - 1 is even
        sweep_step<T, V, FL, 0>(A, R, c, j, j0, j1, wm);
        if (j + 1 <= j1 + 1) sweep_step<T, V, FL, 1>(A, R, c, j + 1, j0, j1, wm);
    }
    if constexpr (FL & SW_NORM) {
        const double s = wave_sum(R.s2);
        const double mx = wave_max(R.mx);
        if (lane == 0) {
            A.partials[2 * tile] = s;
            A.partials[2 * tile + 1] = mx;
        }
    }
}

// ------------------------------------------------- residual + full weighting
template <typename T, int V>
__device__ __forceinline__ void residual_row(T (&r)[V], const T (&um)[V], const T (&uc)[V], const T (&up)[V],
                                             const T (&f)[V], bool rowint, const Cols<V>& c, T cx, T cy, T d) {
    const T W0 = lane_prev(uc[V - 1]);
    const T E0 = lane_next(uc[0]);
#pragma unroll
    for (int e = 0; e < V; ++e) {
        const T W = e > 0 ? uc[e - 1] : W0;
        const T E = e < V - 1 ? uc[e + 1] : E0;
        const T L = fma(-d, uc[e], fma(cy, um[e] + up[e], cx * (W + E)));
        r[e] = (rowint && c.cint[e]) ? (f[e] - L) : T(0);
    }
}

// The same residual in difference form: cx ((W - C) + (E - C)) + cy ((S - C)
// + (N - C)) forms each neighbour difference first.  For a smooth u the
// standard form adds terms of size 8|u|/h^2 whose rounding, in FP32 on a fine
// grid, swamps the small smooth residual; the differences are exact or
// nearly so, and the result keeps the accuracy of the second differences.
template <typename T, int V>
__device__ __forceinline__ void residual_row_diff(T (&r)[V], const T (&um)[V], const T (&uc)[V], const T (&up)[V],
                                                  const T (&f)[V], bool rowint, const Cols<V>& c, T cx, T cy) {
    const T W0 = lane_prev(uc[V - 1]);
    const T E0 = lane_next(uc[0]);
#pragma unroll
    for (int e = 0; e < V; ++e) {
        const T W = e > 0 ? uc[e - 1] : W0;
        const T E = e < V - 1 ? uc[e + 1] : E0;
        const T C = uc[e];
        const T L = cx * ((W - C) + (E - C)) + cy * ((um[e] - C) + (up[e] - C));
        r[e] = (rowint && c.cint[e]) ? (f[e] - L) : T(0);
    }
}

// DIFF: the residual in difference form (RestrictArgs::rdiff)
template <typename T, int V, bool DIFF = false>
__device__ __forceinline__ void restrict_tile(const RestrictArgs<T>& A, int tile, int lane) {
    const int win = tile % A.tl.nwin, chunk = tile / A.tl.nwin;
    const Cols<V> c(win, lane, A.m, A.P, A.tl.H);
    const int j0 = 1 + chunk * A.tl.ty;
    const int j1 = min(j0 + A.tl.ty - 1, A.n - 2);

    T um[V], uc[V], up[V], q1[V], q2[V], fr[V], fq1[V], fq2[V];
    T r2[V], r1[V], r0[V];
    zero<T, V>(r2);
    zero<T, V>(r1);
    load_row<T, V>(um, A.u, j0 - 1, A.n, A.P, c.i0, c.vin);
    load_row<T, V>(uc, A.u, j0, A.n, A.P, c.i0, c.vin);
    load_row<T, V>(q1, A.u, j0 + 1, A.n, A.P, c.i0, c.vin);
    load_row<T, V>(q2, A.u, j0 + 2, A.n, A.P, c.i0, c.vin);
    load_row<T, V>(fq1, A.f, j0, A.n, A.P, c.i0, c.vin);
    load_row<T, V>(fq2, A.f, j0 + 1, A.n, A.P, c.i0, c.vin);

    for (int j = j0; j <= j1 + 1; ++j) {   // rows j+1, j+2 (u) and j, j+1 (f) are in flight
        copy<T, V>(up, q1);
        copy<T, V>(fr, fq1);
        copy<T, V>(q1, q2);
        copy<T, V>(fq1, fq2);
        if (j + 3 <= j1 + 2) load_row<T, V>(q2, A.u, j + 3, A.n, A.P, c.i0, c.vin);
        if (j + 2 <= j1 + 1) load_row<T, V>(fq2, A.f, j + 2, A.n, A.P, c.i0, c.vin);
        if constexpr (DIFF)
            residual_row_diff<T, V>(r0, um, uc, up, fr, (j >= 1) && (j <= A.n - 2), c, A.cx, A.cy);
        else
            residual_row<T, V>(r0, um, uc, up, fr, (j >= 1) && (j <= A.n - 2), c, A.cx, A.cy, A.d);
        if ((j & 1) && j >= j0 + 2) {
            const int J = (j - 1) >> 1;               // coarse row at fine row j-1
            const T w2 = lane_prev(r2[V - 1]), w1 = lane_prev(r1[V - 1]), w0 = lane_prev(r0[V - 1]);
            const T e2 = lane_next(r2[0]), e1 = lane_next(r1[0]), e0 = lane_next(r0[0]);
            if (J >= 1 && J <= A.nc - 2) {
                T* brow = A.bc + (size_t)J * A.Pc;
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const int i = c.i0 + e;
                    if ((i & 1) || !c.cout[e]) continue;
                    const int I = i >> 1;
                    if (I < 1 || I > A.mc - 2) continue;
                    const T C = r1[e];
                    const T W = e > 0 ? r1[e - 1] : w1;
                    const T E = e < V - 1 ? r1[e + 1] : e1;
                    const T S = r2[e], N = r0[e];
                    const T SW = e > 0 ? r2[e - 1] : w2;
                    const T SE = e < V - 1 ? r2[e + 1] : e2;
                    const T NW = e > 0 ? r0[e - 1] : w0;
                    const T NE = e < V - 1 ? r0[e + 1] : e0;
                    const T v = (fma(T(4), C, T(2) * ((W + E) + (S + N))) + ((SW + SE) + (NW + NE))) * T(0.0625);
                    brow[I] = v;
                    if (A.uc0 != nullptr) A.uc0[(size_t)J * A.Pc + I] = T(0);
                }
            }
        }
        copy<T, V>(r2, r1);
        copy<T, V>(r1, r0);
        copy<T, V>(um, uc);
        copy<T, V>(uc, up);
    }
}

// ------------------------------------------------------------------ residual
// Rows in the residual kernel's ring (see residual_tile).  8193^2 FP64, the
// canonical 18-row chunks, HIP events: f = 0 106 us with two rows ahead, 95 us
// with a ring of 6 (66 registers, 7 waves per SIMD), 99-104 with 8 or 9; with
// a source 185 -> 178 us.
constexpr int kResRing = 6;

template <typename T, int V>
__device__ __forceinline__ void residual_tile(const ResidualArgs<T>& A, int tile, int lane) {
    const int win = tile % A.tl.nwin, chunk = tile / A.tl.nwin;
    const Cols<V> c(win, lane, A.m, A.P, A.tl.H);
    const int j0 = 1 + chunk * A.tl.ty;
    const int j1 = min(j0 + A.tl.ty - 1, A.n - 2);

    // A ring of R rows: row q of u sits in slot (q - j0 + 1) % R and is
    // loaded R - 2 rows before its first use, row q of f in slot (q - j0) % R,
    // R rows ahead.  The row loop is unrolled by R, so every slot index is a
    // compile-time constant (no register copies that would wait for a load),
    // and the loads are unconditional (rows past the chunk are clamped to its
    // last neighbour row and never used), so the compiler counts them exactly.
    constexpr int R = kResRing;
    T u[R][V], fq[R][V], r[V];
    double s2 = 0.0, mx = 0.0;
#pragma unroll
    for (int k = 0; k < R; ++k) load_row<T, V>(u[k], A.u, min(j0 - 1 + k, j1 + 1), A.n, A.P, c.i0, c.vin);
#pragma unroll
    for (int k = 0; k < R; ++k) load_row<T, V>(fq[k], A.f, min(j0 + k, j1), A.n, A.P, c.i0, c.vin);
    auto row = [&](int k, int j) {
        residual_row<T, V>(r, u[k], u[(k + 1) % R], u[(k + 2) % R], fq[k], true, c, A.cx, A.cy, A.d);
        if (A.r != nullptr) store_row<T, V>(A.r, r, j, A.P, c);
        if (A.partials != nullptr) {
#pragma unroll
            for (int e = 0; e < V; ++e) {
                if (!c.cout[e]) continue;
                const double v = (double)r[e];
                s2 = fma(v, v, s2);
                mx = fmax(mx, fabs(v));
            }
        }
    };
    for (int jb = j0; jb <= j1; jb += R) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int j = jb + k;
            if (j <= j1) row(k, j);
            // slot k of u (row j - 1) and of f (row j) are free now
            load_row<T, V>(u[k], A.u, min(j - 1 + R, j1 + 1), A.n, A.P, c.i0, c.vin);
            load_row<T, V>(fq[k], A.f, min(j + R, j1), A.n, A.P, c.i0, c.vin);
        }
    }
    if (A.partials != nullptr) {
        const double s = wave_sum(s2);
        const double m2 = wave_max(mx);
        if (lane == 0) {
            A.partials[2 * tile] = s;
            A.partials[2 * tile + 1] = m2;
        }
    }
}

// ---------------------------------------------------- FP64 defect correction
template <int V>
__device__ __forceinline__ void defect_tile(const DefectArgs& A, int tile, int lane) {
    const int win = tile % A.tl.nwin, chunk = tile / A.tl.nwin;
    const Cols<V> c(win, lane, A.m, A.P, A.tl.H);
    const int j0 = 1 + chunk * A.tl.ty;
    const int j1 = min(j0 + A.tl.ty - 1, A.n - 2);

    // The ring of residual_tile: row q of psi (and of the FP32 correction e)
    // in slot (q - j0 + 1) % R, of f in slot (q - j0) % R.  e is added to a
    // row when the row first enters the stencil (one iteration before it is
    // the centre row), not right after its load, so the loads ahead are not
    // waited for.
    constexpr int R = kResRing;
    double u[R][V], fq[R][V], r[V];
    float ev[R][V], r32[V];
    double s2 = 0.0, mx = 0.0;
    auto load_u = [&](int k, int q) {
        load_row<double, V>(u[k], A.psi_in, q, A.n, A.P, c.i0, c.vin);
        load_row<float, V>(ev[k], A.e, q, A.n, A.P, c.i0, c.vin);
    };
    auto add_e = [&](int k) {
        if (A.e != nullptr) {
#pragma unroll
            for (int e = 0; e < V; ++e) u[k][e] = u[k][e] + (double)ev[k][e];
        }
    };
#pragma unroll
    for (int k = 0; k < R; ++k) load_u(k, min(j0 - 1 + k, j1 + 1));
#pragma unroll
    for (int k = 0; k < R; ++k) load_row<double, V>(fq[k], A.f, min(j0 + k, j1), A.n, A.P, c.i0, c.vin);
    add_e(0);
    add_e(1);
    for (int jb = j0; jb <= j1; jb += R) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int j = jb + k;
            if (j <= j1) {
                add_e((k + 2) % R);
                const double (&uc)[V] = u[(k + 1) % R];
                residual_row<double, V>(r, u[k], uc, u[(k + 2) % R], fq[k], true, c, A.cx, A.cy, A.d);
                if (A.psi_out != A.psi_in || A.e != nullptr) store_row<double, V>(A.psi_out, uc, j, A.P, c);
#pragma unroll
                for (int e = 0; e < V; ++e) r32[e] = (float)r[e];
                store_row<float, V>(A.rhs, r32, j, A.P, c);
                if (A.ezero != nullptr) {
                    float z[V];
                    zero<float, V>(z);
                    store_row<float, V>(A.ezero, z, j, A.P, c);
                }
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    if (!c.cout[e]) continue;
                    s2 = fma(r[e], r[e], s2);
                    mx = fmax(mx, fabs(r[e]));
                }
            }
            // slot k of psi (row j - 1) and of f (row j) are free now
            load_u(k, min(j - 1 + R, j1 + 1));
            load_row<double, V>(fq[k], A.f, min(j + R, j1), A.n, A.P, c.i0, c.vin);
        }
    }
    const double s = wave_sum(s2);
    const double m2 = wave_max(mx);
    if (lane == 0) {
        A.partials[2 * tile] = s;
        A.partials[2 * tile + 1] = m2;
    }
}

// ---------------------------------------------------------- coarsest level
template <typename T>
__device__ __forceinline__ void coarse_block(const CoarseArgs<T>& A, double* rhs) {
    const int mi = A.m - 2, ni = A.n - 2, N = mi * ni;
    // right-hand side of the interior system; Dirichlet values of the
    // perimeter (level 0 only) move to the right-hand side
    auto rhs_at = [&](int i, int j) {
        double v = A.b != nullptr ? (double)A.b[(size_t)j * A.P + i] : 0.0;
        if (A.u != nullptr) {
            if (i == 1) v -= A.cx * (double)A.u[(size_t)j * A.P];
            if (i == A.m - 2) v -= A.cx * (double)A.u[(size_t)j * A.P + A.m - 1];
            if (j == 1) v -= A.cy * (double)A.u[i];
            if (j == A.n - 2) v -= A.cy * (double)A.u[(size_t)(A.n - 1) * A.P + i];
        }
        return v;
    };
    if (A.bw == 0) {
        for (int k = threadIdx.x; k < N; k += blockDim.x) rhs[k] = rhs_at(1 + k % mi, 1 + k / mi);
        __syncthreads();
        for (int k = threadIdx.x; k < N; k += blockDim.x) {
            double x = 0.0;
            for (int l = 0; l < N; ++l) x = fma(A.minv[(size_t)l * N + k], rhs[l], x);
            const int i = 1 + k % mi, j = 1 + k / mi;
            A.out[(size_t)j * A.P + i] = (T)x;
        }
        return;
    }
    // separable solve (all threads of the block): sine transform along the
    // short side, one Thomas solve per mode along the long side, inverse
    // transform.  R (A.work) holds the p x q mode coefficients.
    const int p = A.bw, q = N / p;
    const double* Q = A.minv;
    const double* fac = A.minv + (size_t)p * p;
    const double off = -(A.ifast ? A.cy : A.cx);   // long-side coupling of -L_h
    double* R = A.work;
    auto node = [&](int sidx, int l, int& i, int& j) {
        i = 1 + (A.ifast ? sidx : l);
        j = 1 + (A.ifast ? l : sidx);
    };
    for (int t = threadIdx.x; t < p * q; t += blockDim.x) {
        const int k = t / q, l = t - k * q;
        double acc = 0.0;
        for (int sidx = 0; sidx < p; ++sidx) {
            int i, j;
            node(sidx, l, i, j);
            acc = fma(Q[(size_t)k * p + sidx], -rhs_at(i, j), acc);
        }
        R[t] = acc;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < p; k += blockDim.x) {
        const double* cpr = fac + 2 * (size_t)k * q;
        const double* ipv = cpr + q;
        double* r = R + (size_t)k * q;
        double prev = 0.0;
        for (int l = 0; l < q; ++l) {
            prev = fma(-off, prev, r[l]) * ipv[l];
            r[l] = prev;
        }
        double x = 0.0;
        for (int l = q - 1; l >= 0; --l) {
            x = fma(-cpr[l], x, r[l]);
            r[l] = x;
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < p * q; t += blockDim.x) {
        const int sidx = t / q, l = t - sidx * q;
        double acc = 0.0;
        for (int k = 0; k < p; ++k) acc = fma(Q[(size_t)k * p + sidx], R[(size_t)k * q + l], acc);
        int i, j;
        node(sidx, l, i, j);
        A.out[(size_t)j * A.P + i] = (T)acc;
    }
}

// ------------------------------------------------------- small-level subtree
// One workgroup, every level in LDS (pitch m), a barrier between passes.
// Each node value is produced by the same expression, on the same operands,
// as in the streaming kernels, so the top level's result is bitwise the one
// of the multi-launch schedule.  Levels that are smoothed have odd m, so the
// interior index t = (j-1)(m-2) + (i-1) has the parity of i + j: colour c is
// exactly the nodes t = 2h + c.
template <typename T>
__device__ __forceinline__ void sub_colour(T* s, const SubLevel<T>& L, int colour, T om) {
    const int mi = L.m - 2, N = mi * (L.n - 2), m = L.m;
    T* u = s + L.ou;
    const T* b = s + L.ob;
    for (int h = threadIdx.x; 2 * h + colour < N; h += blockDim.x) {
        const int t = 2 * h + colour;
        const int c = (1 + t / mi) * m + 1 + t % mi;
        const T x = (fma(L.cy, u[c - m] + u[c + m], L.cx * (u[c - 1] + u[c + 1])) - b[c]) * L.inv_d;
        u[c] = fma(om, x - u[c], u[c]);
    }
}

template <typename T>
__device__ __forceinline__ void sub_sweep(T* s, const SubLevel<T>& L, T om) {
    sub_colour<T>(s, L, 0, om);
    __syncthreads();
    sub_colour<T>(s, L, 1, om);
    __syncthreads();
}

// residual b - L u at an interior node
template <typename T>
__device__ __forceinline__ T sub_res(const T* u, const T* b, const SubLevel<T>& L, int c) {
    const int m = L.m;
    const T Lu = fma(-L.d, u[c], fma(L.cy, u[c - m] + u[c + m], L.cx * (u[c - 1] + u[c + 1])));
    return b[c] - Lu;
}

// full weighting of the residual of level F onto the right-hand side of C
// (the nine fine nodes of an interior coarse node are interior)
template <typename T>
__device__ __forceinline__ void sub_restrict(T* s, const SubLevel<T>& F, const SubLevel<T>& C) {
    const int mi = C.m - 2, N = mi * (C.n - 2), m = F.m;
    const T* u = s + F.ou;
    const T* b = s + F.ob;
    T* bc = s + C.ob;
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        const int I = 1 + k % mi, J = 1 + k / mi;
        const int c = 2 * J * m + 2 * I;
        const T Cc = sub_res(u, b, F, c), W = sub_res(u, b, F, c - 1), E = sub_res(u, b, F, c + 1);
        const T S = sub_res(u, b, F, c - m), Nn = sub_res(u, b, F, c + m);
        const T SW = sub_res(u, b, F, c - m - 1), SE = sub_res(u, b, F, c - m + 1);
        const T NW = sub_res(u, b, F, c + m - 1), NE = sub_res(u, b, F, c + m + 1);
        bc[J * C.m + I] = (fma(T(4), Cc, T(2) * ((W + E) + (S + Nn))) + ((SW + SE) + (NW + NE))) * T(0.0625);
    }
}

// u_F += P(u_C) on the interior of F (bilinear interpolation)
template <typename T>
__device__ __forceinline__ void sub_prolong_add(T* s, const SubLevel<T>& F, const SubLevel<T>& C) {
    const int mi = F.m - 2, N = mi * (F.n - 2);
    T* u = s + F.ou;
    const T* ec = s + C.ou;
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        const int i = 1 + k % mi, j = 1 + k / mi;
        const int I = i >> 1, J = j >> 1;
        const bool sx = (i & 1) != 0, ty = (j & 1) != 0;
        const T* r0 = ec + J * C.m + I;
        const T e00 = r0[0];
        const T e10 = sx ? r0[1] : T(0);
        const T e01 = ty ? r0[C.m] : T(0);
        const T e11 = (sx && ty) ? r0[C.m + 1] : T(0);
        const T p_even = ty ? (e00 + e01) * T(0.5) : e00;
        const T p_odd = ty ? ((e00 + e10) + (e01 + e11)) * T(0.25) : (e00 + e10) * T(0.5);
        const T p = sx ? p_odd : p_even;
        const int c = j * F.m + i;
        u[c] = u[c] + p;
    }
}

template <typename T>
__device__ void subtree_block(const SubtreeArgs<T>& S, T* s, double* rhs) {
    const int L = S.nlev;
    const SubLevel<T>& top = S.lv[0];
    // zero every level (zero start, homogeneous boundary), then the top
    // level's right-hand side from HBM
    const int tb0 = top.ob, tb1 = top.ob + top.m * top.n;
    for (int k = threadIdx.x; k < S.lds_elems; k += blockDim.x)
        if (k < tb0 || k >= tb1) s[k] = T(0);
    for (int k = threadIdx.x; k < top.m * top.n; k += blockDim.x) {
        const int i = k % top.m, j = k / top.m;
        s[tb0 + k] = S.b != nullptr ? S.b[(size_t)j * S.P + i] : T(0);
    }
    __syncthreads();
    for (int k = 0; k + 1 < L; ++k) {
        for (int q = 0; q < S.nu1; ++q) sub_sweep<T>(s, S.lv[k], S.omega);
        sub_restrict<T>(s, S.lv[k], S.lv[k + 1]);
        __syncthreads();
    }
    {
        const SubLevel<T>& C = S.lv[L - 1];
        CoarseArgs<T> A{};
        A.u = nullptr;
        A.b = s + C.ob;
        A.out = s + C.ou;
        A.minv = S.minv;
        A.work = S.work;
        A.bw = S.bw;
        A.ifast = S.ifast;
        A.m = C.m;
        A.n = C.n;
        A.P = C.m;
        A.cx = S.ccx;
        A.cy = S.ccy;
        coarse_block<T>(A, rhs);
        __syncthreads();
    }
    for (int k = L - 2; k >= 0; --k) {
        sub_prolong_add<T>(s, S.lv[k], S.lv[k + 1]);
        __syncthreads();
        for (int q = 0; q < S.nu2; ++q) sub_sweep<T>(s, S.lv[k], S.omega);
    }
    for (int k = threadIdx.x; k < top.m * top.n; k += blockDim.x) {
        const int i = k % top.m, j = k / top.m;
        S.out[(size_t)j * S.P + i] = s[top.ou + k];
    }
}

// ------------------------------------------------------------ norm finalise
// One workgroup of kFinBlock threads: thread t sums partials t, t + kFinBlock,
// ... in that order (loads issued four at a time), the waves reduce with a
// fixed butterfly, and thread 0 adds the wave results in order, so the norm
// does not depend on timing.
constexpr int kFinBlock = 1024;

__device__ __forceinline__ void finalize_block(const double* partials, int ntiles, Ctrl* ctrl, double* out2,
                                               int mode, double* ss, double* sm) {
    double s = 0.0, mx = 0.0;
    const double2* p2 = reinterpret_cast<const double2*>(partials);
    int t = threadIdx.x;
    // each thread adds partials t, t + kFinBlock, t + 2 kFinBlock, ... in that
    // order; sixteen loads in flight per round trip
    for (; t < ntiles; t += 16 * kFinBlock) {
        double2 a[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) a[k] = t + k * kFinBlock < ntiles ? p2[t + k * kFinBlock] : double2{0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 16; ++k)
            if (t + k * kFinBlock < ntiles) {
                s += a[k].x;
                mx = fmax(mx, a[k].y);
            }
    }
    s = wave_sum(s);
    mx = wave_max(mx);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        ss[w] = s;
        sm[w] = mx;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double sum = 0.0, m = 0.0;
    for (int k = 0; k < kFinBlock / 64; ++k) {
        sum += ss[k];
        m = fmax(m, sm[k]);
    }

    if (mode == 1) {
        out2[0] = sum;
        out2[1] = m;
        return;
    }
    const double res = sqrt(sum);
    const double r0 = ctrl->checks == 0 ? res : ctrl->r0;
    const double rel = r0 > 0.0 ? res / r0 : 0.0;
    const double q = ctrl->stop == 0 ? rel : m;
    int status = 1;   // 1: the solve goes on
    if (!isfinite(res) || !isfinite(m) || (r0 > 0.0 && res > 1e6 * r0))
        status = -4;   // LAP_EDIVERGED
    else if (q < ctrl->tol || res == 0.0)
        status = 0;
    else if (ctrl->iters >= ctrl->max_iter)
        status = -3;   // LAP_ENOTCONV
    // mode 2 (a probe of the test the next step opens with): only a test
    // that ends the solve is recorded; otherwise that step repeats it
    if (mode == 2 && status == 1) return;
    ctrl->r0 = r0;
    ctrl->res_l2 = res;
    ctrl->res_inf = m;
    ctrl->rel = rel;
    ctrl->checks += 1;
    if (status == 1) {
        ctrl->iters += ctrl->step > 0 ? ctrl->step : 1;
    } else {
        ctrl->done = 1;
        ctrl->status = status;
    }
}

// Safety factor of the one-cycle prediction of a mixed step (the factor of a
// cycle grows by about 10-15% between steps as the FP32 rounding floor nears).
constexpr double kOneCycleMargin = 1.5;

// After the test of a mixed step (thread 0; ctrl already updated): the FP32
// cycles the step runs, as the gate pair cyc[2 p], cyc[2 p + 1].  q_prev,
// checks0 and ran are the control block's test quantity, finalisation count
// and cycle count before this test.
__device__ __forceinline__ void choose_cycles(Ctrl* ctrl, Ctrl* cyc, int cycles, double q_prev, int checks0, int ran) {
    if (ctrl->done) {
#pragma unroll
        for (int k = 0; k < 4; ++k) cyc[k].done = 1;
        return;
    }
    const int inner = cycles & 255, p = (cycles >> 8) & 1;
    bool one = false;
    if (checks0 >= 1 && q_prev > 0.0) {
        // 1.5 q (q / q_prev)^(1 / ran) < tol, as q / q_prev < (tol / (1.5 q))^ran
        const double q = ctrl->stop == 0 ? ctrl->rel : ctrl->res_inf;
        const double x = ctrl->tol / (kOneCycleMargin * q);
        double pw = 1.0;
        for (int k = 0; k < ran; ++k) pw *= x;
        one = q / q_prev < pw;
    }
    cyc[2 * p].done = one ? 1 : 0;
    cyc[2 * p + 1].done = one ? 0 : 1;
    ctrl->cycles = one ? 1 : inner;
}

// The stopping test, followed (cyc not null, mode 0) by the cycle choice of
// a mixed step of several FP32 cycles.
__device__ __forceinline__ void finalize_step(const double* partials, int ntiles, Ctrl* ctrl, double* out2, int mode,
                                              Ctrl* cyc, int cycles, double* ss, double* sm) {
    double q_prev = 0.0;
    int checks0 = 0, ran = 0;
    if (cyc != nullptr && threadIdx.x == 0) {
        q_prev = ctrl->stop == 0 ? ctrl->rel : ctrl->res_inf;
        checks0 = ctrl->checks;
        ran = ctrl->cycles;
    }
    finalize_block(partials, ntiles, ctrl, out2, mode, ss, sm);
    if (cyc != nullptr && mode == 0 && threadIdx.x == 0) choose_cycles(ctrl, cyc, cycles, q_prev, checks0, ran);
}

}  // namespace lap
