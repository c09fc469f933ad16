// Fused streaming passes: several operations of a V-cycle level in one read
// of the level.  A wavefront walks its window down the rows once; the loaded
// rows go through a pipeline of red-black sweep stages held in registers
// (each stage lags the previous one by two rows), and the rows leaving the
// last stage are stored and, optionally, turned into residual rows that are
// full-weighted onto the coarse right-hand side.  Per node every stage
// evaluates exactly the expressions of the one-sweep kernel on the same
// operands, so a fused pass is bitwise the sequence of separate launches.
//
// Valid columns shrink by two per sweep and by two more for residual + full
// weighting, so windows overlap by the tiling's halo H on each side
// (H = 2 * sweeps, + 2 with the restriction); valid rows shrink the same
// way, so a chunk reads 2 * sweeps (+ 1 or 2) rows beyond its own above and
// below.
#pragma once

#include "stencil_tiles.hpp"

namespace lap {

// One sweep stage: rows j-2 (final), j-1 (colour 0 done), j (input) and the
// right-hand side of rows j-1, j.
template <typename T, int V>
struct RBStage {
    T a[V], b[V], c[V];
    T fb[V], fc[V];
};

template <typename T, int V>
__device__ __forceinline__ void stage_zero(RBStage<T, V>& S) {
    zero<T, V>(S.a);
    zero<T, V>(S.b);
    zero<T, V>(S.c);
    zero<T, V>(S.fb);
    zero<T, V>(S.fc);
}

// Push input row j+1 (d, fd) into a stage positioned at row j: colour 0 on
// row j (its colour-1 neighbours still hold input values), then colour 1 on
// row j-1 (its colour-0 neighbours are new).  Row j-1 is then final for this
// sweep and is handed on in (out, fout); the stage moves to row j+1.
template <typename T, int V, int JP>
__device__ __forceinline__ void rb_push(RBStage<T, V>& S, const T (&d)[V], const T (&fd)[V], T (&out)[V],
                                        T (&fout)[V], int j, int n, const OmegaMask<T, V>& wm, T cx, T cy,
                                        T inv_d) {
    const T cW = lane_prev(S.c[V - 1]);
    const T cE = lane_next(S.c[0]);
    if (j >= 1 && j <= n - 2) {
#pragma unroll
        for (int e = 0; e < V; ++e) {
            if (colour_skip<V, JP>(e)) continue;
            const T W = e > 0 ? S.c[e - 1] : cW;
            const T E = e < V - 1 ? S.c[e + 1] : cE;
            const T t = (fma(cy, S.b[e] + d[e], cx * (W + E)) - S.fc[e]) * inv_d;
            S.c[e] = fma(wm.w[JP][e], t - S.c[e], S.c[e]);
        }
    }
    const T bW = lane_prev(S.b[V - 1]);
    const T bE = lane_next(S.b[0]);
    if (j - 1 >= 1 && j - 1 <= n - 2) {
#pragma unroll
        for (int e = 0; e < V; ++e) {
            if (colour_skip<V, JP>(e)) continue;
            const T W = e > 0 ? S.b[e - 1] : bW;
            const T E = e < V - 1 ? S.b[e + 1] : bE;
            const T t = (fma(cy, S.a[e] + S.c[e], cx * (W + E)) - S.fb[e]) * inv_d;
            S.b[e] = fma(wm.w[JP][e], t - S.b[e], S.b[e]);
        }
    }
    copy<T, V>(out, S.b);
    copy<T, V>(fout, S.fb);
    copy<T, V>(S.a, S.b);
    copy<T, V>(S.b, S.c);
    copy<T, V>(S.c, d);
    copy<T, V>(S.fb, S.fc);
    copy<T, V>(S.fc, fd);
}

// Input rows in flight per wavefront: a ring of PF rows, each issued PF
// steps before it enters the pipeline.  Measured on MI355X (8193^2 V-cycle
// passes): FP64 gains up to six rows, FP32 (half the bytes per row, the
// registers better spent on occupancy) is fastest with two.
// FP64 passes that also stream a right-hand side carry a second ring (6 rows
// measured best there too; 4 and 2 were slower).  The FP32 post-smoothing +
// FP64 defect pass (five input streams, two rings of FP64 rows besides the
// FP32 ones) is fastest with two rows (4 and 6 were 2-4% slower per solve).
constexpr int kPfF64WithF = 6;
template <typename T, int FL>
constexpr int fused_pf() {
    if constexpr ((FL & SW_DEF) != 0) return 2;
    if constexpr (sizeof(T) == 4 && (FL & SW_PROLONG) != 0) return 4;
    return sizeof(T) == 8 ? ((FL & SW_F) ? kPfF64WithF : 6) : 2;
}

// Whole ring turns as straight-line code (the tail turn keeps its per-step
// row test) save the register copies of the rotating pipeline: 14% fewer
// VALU instructions in the FP64 restricting pass.  Passes that prolong hold
// the coarse rows as well and would need more registers, costing a wave of
// occupancy, so they keep the tested turn; the four-sweep pass, bound by
// vector issue (its four stages rotate 20 rows per step), takes the whole
// turns anyway (8193^2 FP32: 132 instead of 118 registers, 242 instead of
// 265 us as tuned).
template <typename T, int FL>
constexpr bool fused_full_turns() {
    return (FL & SW_PROLONG) == 0 || (FL & SW_FOUR) != 0;
}

template <typename T, int V, int NS, bool RS, int PF>
struct FusedRegs {
    RBStage<T, V> st[NS];
    T ring[PF][V], fring[PF][V];        // input rows j+1 .. j+PF (slot = step phase)
    T bo[V];                            // input row j-1 (norm of the input)
    T ru0[V], ru1[V], rf1[V];           // final rows q-2, q-1 and f of row q-1
    T r2[V], r1[V];                     // residual rows q-3, q-2
    double pring[PF][V], qring[PF][V];  // SW_DEF: FP64 iterate and source rows q .. q+PF-1
    double pm[V], pc[V], fm[V];         // SW_DEF: updated rows q-2, q-1 and the source of row q-1
    double s2, mx;
    Prolong<T, V> pr;
};

// One step (ring phase PH): input row j+1 enters from its ring slot, the
// slot is refilled with row j+1+PF, and the last stage emits final row
// q = j + 1 - 2 * NS.
template <typename T, int V, int FL, int NS, bool RS, int JP, int PH>
__device__ __forceinline__ void fused_step(const SweepArgs<T>& A, FusedRegs<T, V, NS, RS, fused_pf<T, FL>()>& R,
                                           const Cols<V>& c, int j, int j0, int j1, int Lend,
                                           const OmegaMask<T, V>& wm) {
    constexpr int PF = fused_pf<T, FL>();
    T d[V], fd[V];
    copy<T, V>(d, R.ring[PH]);
    // the ring holds rows as stored; the correction is added as a row enters,
    // so the loads in flight are not waited for until then
    if constexpr (adds_correction<FL>()) R.pr.add(d, A.ec, j + 1, A.n, A.nc, A.Pc, A.Pcs, c.i0, A.m);
    copy<T, V>(fd, R.fring[PH]);
    if (j + 1 + PF <= Lend) {
        sweep_load_raw<T, V, FL>(R.ring[PH], A, j + 1 + PF, c);
        sweep_loadf<T, V, FL>(R.fring[PH], A, j + 1 + PF, c);
    }
    const T cx = A.cx, cy = A.cy, inv_d = A.inv_d;

    if constexpr (FL & SW_NORM) {
        // residual of the input at row j (rows j-1, j, j+1 are input values)
        const T cW = lane_prev(R.st[0].c[V - 1]);
        const T cE = lane_next(R.st[0].c[0]);
        if (j >= j0 && j <= j1) {
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const T W = e > 0 ? R.st[0].c[e - 1] : cW;
                const T E = e < V - 1 ? R.st[0].c[e + 1] : cE;
                const T L = fma(-A.d, R.st[0].c[e], fma(cy, R.bo[e] + d[e], cx * (W + E)));
                const double r = c.cout[e] ? (double)(R.st[0].fc[e] - L) : 0.0;
                R.s2 = fma(r, r, R.s2);
                R.mx = fmax(R.mx, fabs(r));
            }
        }
        copy<T, V>(R.bo, R.st[0].c);
    }
    if constexpr ((FL & SW_PROBE) != 0) {
        // norms only: move the input rows the norm reads, no stage work
        copy<T, V>(R.st[0].c, d);
        copy<T, V>(R.st[0].fc, fd);
        return;
    }

    T o[V], fo[V];
    rb_push<T, V, JP>(R.st[0], d, fd, o, fo, j, A.n, wm, cx, cy, inv_d);
#pragma unroll
    for (int s = 1; s < NS; ++s) {
        // stage s works two rows behind stage s - 1 (same row parity)
        T o2[V], fo2[V];
        rb_push<T, V, JP>(R.st[s], o, fo, o2, fo2, j - 2 * s, A.n, wm, cx, cy, inv_d);
        copy<T, V>(o, o2);
        copy<T, V>(fo, fo2);
    }
    const int q = j + 1 - 2 * NS;
    if constexpr (FL & SW_DEF) {
        // o is row q of the final correction: psi_out = psi_in + e there, and
        // the FP64 residual of the updated iterate at row q - 1
        double ps[V], fq[V], pn[V];
        copy<double, V>(ps, R.pring[PH]);
        copy<double, V>(fq, R.qring[PH]);
        load_row<double, V>(R.pring[PH], A.psi_in, q + PF, A.n, A.Ps, c.i0, c.vin);
        load_row<double, V>(R.qring[PH], A.f64, q + PF, A.n, A.Ps, c.i0, c.vin);
#pragma unroll
        for (int e = 0; e < V; ++e) pn[e] = ps[e] + (double)o[e];
        if (q >= j0 && q <= j1) store_row_nt<double, V>(A.nt != 0, A.psi_out, pn, q, A.Ps, c);
        if (q - 1 >= j0 && q - 1 <= j1) {
            double r[V];
            T r32[V];
            residual_row<double, V>(r, R.pm, R.pc, pn, R.fm, true, c, A.dcx, A.dcy, A.dd);
#pragma unroll
            for (int e = 0; e < V; ++e) {
                r32[e] = (T)r[e];
                const double rr = c.cout[e] ? r[e] : 0.0;
                R.s2 = fma(rr, rr, R.s2);
                R.mx = fmax(R.mx, fabs(rr));
            }
            if (A.rowpart && ((q - 1) % kRowBlock == 0 || q - 1 == j1)) {
                // end of a block of kRowBlock rows (wave-uniform): its
                // partials, summed in row order whatever chunk holds it
                const double s = wave_sum(R.s2), m = wave_max(R.mx);
                if ((threadIdx.x & 63) == 0) {
                    const int b = A.rp_off + (q - 2) / kRowBlock;
                    A.partials[2 * b] = s;
                    A.partials[2 * b + 1] = m;
                }
                R.s2 = 0.0;
                R.mx = 0.0;
            }
            store_row_nt<T, V>(A.nt != 0, A.rhs_out, r32, q - 1, A.Ps, c);
        }
        copy<double, V>(R.pm, R.pc);
        copy<double, V>(R.pc, pn);
        copy<double, V>(R.fm, fq);
    } else if (q >= j0 && q <= j1) {
        store_row_nt<T, V>(A.nt != 0, A.uout, o, q, A.Ps, c);
    }

    if constexpr (RS) {
        // residual of the result at row q-1 (SW_RDIFF: in difference form), then
        // full weighting at the even row q-2
        T r0[V];
        if constexpr ((FL & SW_RDIFF) != 0)
            residual_row_diff<T, V>(r0, R.ru0, R.ru1, o, R.rf1, (q - 1 >= 1) && (q - 1 <= A.n - 2), c, cx, cy);
        else
            residual_row<T, V>(r0, R.ru0, R.ru1, o, R.rf1, (q - 1 >= 1) && (q - 1 <= A.n - 2), c, cx, cy, A.d);
        // q - 2 is even exactly on steps with j odd
        if (JP == 1 && q - 2 >= j0 && q - 2 <= j1) {
            const int J = (q - 2) >> 1;
            const T w2 = lane_prev(R.r2[V - 1]), w1 = lane_prev(R.r1[V - 1]), w0 = lane_prev(r0[V - 1]);
            const T e2 = lane_next(R.r2[0]), e1 = lane_next(R.r1[0]), e0 = lane_next(r0[0]);
            if (J >= 1 && J <= A.nc - 2) {
                T* brow = A.bc + (ptrdiff_t)J * A.Pcs;
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const int i = c.i0 + e;
                    if ((i & 1) || !c.cout[e]) continue;
                    const int I = i >> 1;
                    if (I < 1 || I > A.mc - 2) continue;
                    const T C = R.r1[e];
                    const T W = e > 0 ? R.r1[e - 1] : w1;
                    const T E = e < V - 1 ? R.r1[e + 1] : e1;
                    const T S = R.r2[e], N = r0[e];
                    const T SW = e > 0 ? R.r2[e - 1] : w2;
                    const T SE = e < V - 1 ? R.r2[e + 1] : e2;
                    const T NW = e > 0 ? r0[e - 1] : w0;
                    const T NE = e < V - 1 ? r0[e + 1] : e0;
                    brow[I] = (fma(T(4), C, T(2) * ((W + E) + (S + N))) + ((SW + SE) + (NW + NE))) * T(0.0625);
                }
            }
        }
        copy<T, V>(R.r2, R.r1);
        copy<T, V>(R.r1, r0);
        copy<T, V>(R.ru0, R.ru1);
        copy<T, V>(R.ru1, o);
        copy<T, V>(R.rf1, fo);
    }
}

// Steps PH, PH+1, ... of one turn of the ring, starting at row j + PH.
template <typename T, int V, int FL, int NS, bool RS, int JP0, int PH>
__device__ __forceinline__ void fused_turn(const SweepArgs<T>& A, FusedRegs<T, V, NS, RS, fused_pf<T, FL>()>& R,
                                           const Cols<V>& c, int j, int j0, int j1, int Lend,
                                           const OmegaMask<T, V>& wm) {
    if constexpr (PH < fused_pf<T, FL>()) {
        if (j + PH <= Lend - 1) {
            fused_step<T, V, FL, NS, RS, (JP0 + PH) & 1, PH>(A, R, c, j + PH, j0, j1, Lend, wm);
            fused_turn<T, V, FL, NS, RS, JP0, PH + 1>(A, R, c, j, j0, j1, Lend, wm);
        }
    }
}

// A whole turn of the ring, every step taken (the caller knows all PF rows
// exist): straight-line code, so the pipeline's register roles rotate by
// renaming instead of copies.
template <typename T, int V, int FL, int NS, bool RS, int JP0, int PH>
__device__ __forceinline__ void fused_turn_full(const SweepArgs<T>& A,
                                                FusedRegs<T, V, NS, RS, fused_pf<T, FL>()>& R, const Cols<V>& c,
                                                int j, int j0, int j1, int Lend, const OmegaMask<T, V>& wm) {
    if constexpr (PH < fused_pf<T, FL>()) {
        fused_step<T, V, FL, NS, RS, (JP0 + PH) & 1, PH>(A, R, c, j + PH, j0, j1, Lend, wm);
        fused_turn_full<T, V, FL, NS, RS, JP0, PH + 1>(A, R, c, j, j0, j1, Lend, wm);
    }
}

// Odd row chunks walk upwards, through a vertically flipped view of the
// level (base at the last row, negative row strides; the coarse arrays
// likewise).  Neighbouring chunks then reach their common boundary at the
// same time, both at the start or both at the end of their walks, so the
// halo rows one of them re-reads are still in L2.  With an odd number of
// rows the flip keeps every node's colour (n - 1 is even), fine row 2J
// stays over coarse row J, and each expression only sees its north and
// south operands swapped in a commutative sum: the values are unchanged.
template <typename T, int V, int FL>
__device__ __forceinline__ void fused_tile(const SweepArgs<T>& A0, int tile, int lane) {
    constexpr int NS = (FL & SW_FOUR) ? 4 : (FL & SW_TWO) ? 2 : 1;
    constexpr bool RS = (FL & SW_RESTRICT) != 0;
    SweepArgs<T> A = A0;
    const int win = tile % A.tl.nwin, chunk = tile / A.tl.nwin;
    const Cols<V> c(win, lane, A.m, A.P, A.tl.H);
    int j0 = 1 + chunk * A.tl.ty;
    int j1 = min(j0 + A.tl.ty - 1, A.n - 2);
    A.Ps = A.P;
    A.Pcs = A.Pc;
    if ((chunk & 1) && (A.n & 1) && !((FL & SW_DEF) && A.rowpart)) {
        const ptrdiff_t last = (ptrdiff_t)(A.n - 1) * A.P, clast = (ptrdiff_t)(A.nc - 1) * A.Pc;
        if (A.uin) A.uin += last;
        if (A.uout) A.uout += last;
        if (A.f) A.f += last;
        if constexpr (FL & SW_DEF) {
            A.psi_in += last;
            A.psi_out += last;
            if (A.f64) A.f64 += last;
            A.rhs_out += last;
        }
        if (A.ec) A.ec += clast;
        if (A.bc) A.bc += clast;
        A.Ps = -A.P;
        A.Pcs = -A.Pc;
        const int t0 = A.n - 1 - j1;
        j1 = A.n - 1 - j0;
        j0 = t0;
    }
    const int ipar = c.i0 & 1;
    const OmegaMask<T, V> wm(c, ipar, A.omega);
    if constexpr ((FL & SW_DEF) != 0) A.rp_off = win * row_blocks(A.n);
    // input rows [L0, Lend]: the last stage must be exact on the chunk's rows
    // and, with the restriction, two rows around its first and last even row;
    // L0 is moved up one row if needed so the first step has parity JP0
    // (SW_DEF: the residual needs the final rows j0 - 1 .. j1 + 1)
    constexpr int JP0 = RS ? 1 : 0;
    constexpr int DX = (FL & SW_DEF) ? 1 : 0;
    const int e0 = j0 + (j0 & 1), e1 = j1 - (j1 & 1);
    int L0 = (RS ? e0 - 2 : j0 - DX) - 2 * NS;
    if (((L0 + 1) & 1) != JP0) --L0;
    const int Lend = (RS ? e1 + 2 : j1 + DX) + 2 * NS;

    FusedRegs<T, V, NS, RS, fused_pf<T, FL>()> R;
    R.s2 = 0.0;
    R.mx = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) stage_zero<T, V>(R.st[s]);
    if constexpr (RS) {
        zero<T, V>(R.ru0);
        zero<T, V>(R.ru1);
        zero<T, V>(R.rf1);
        zero<T, V>(R.r2);
        zero<T, V>(R.r1);
    }
    if constexpr (FL & SW_PROLONG) R.pr.init(A.ec, L0, A.nc, A.Pc, A.Pcs, c.i0);
    sweep_load<T, V, FL>(R.st[0].b, A, L0, c, R.pr);
    sweep_load<T, V, FL>(R.st[0].c, A, L0 + 1, c, R.pr);
    sweep_loadf<T, V, FL>(R.st[0].fc, A, L0 + 1, c);
    constexpr int PF = fused_pf<T, FL>();
#pragma unroll
    for (int k = 0; k < PF; ++k) {
        sweep_load_raw<T, V, FL>(R.ring[k], A, L0 + 2 + k, c);
        sweep_loadf<T, V, FL>(R.fring[k], A, L0 + 2 + k, c);
    }
    if constexpr (FL & SW_NORM) copy<T, V>(R.bo, R.st[0].b);
    if constexpr (FL & SW_DEF) {
        // the first step emits final row L0 + 2 - 2 * NS
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            load_row<double, V>(R.pring[k], A.psi_in, L0 + 2 - 2 * NS + k, A.n, A.Ps, c.i0, c.vin);
            load_row<double, V>(R.qring[k], A.f64, L0 + 2 - 2 * NS + k, A.n, A.Ps, c.i0, c.vin);
        }
        zero<double, V>(R.pm);
        zero<double, V>(R.pc);
        zero<double, V>(R.fm);
    }

    // the loop is unrolled over one turn of the ring (PF is even, so every
    // turn starts on the row parity JP0)
    static_assert(PF % 2 == 0, "the ring turn must keep the row parity");
    int j = L0 + 1;
    if constexpr (fused_full_turns<T, FL>())
        for (; j + PF - 1 <= Lend - 1; j += PF) fused_turn_full<T, V, FL, NS, RS, JP0, 0>(A, R, c, j, j0, j1, Lend, wm);
    for (; j <= Lend - 1; j += PF) fused_turn<T, V, FL, NS, RS, JP0, 0>(A, R, c, j, j0, j1, Lend, wm);
    if constexpr ((FL & (SW_NORM | SW_DEF)) != 0) {
        if ((FL & SW_DEF) && A.rowpart) return;
        const double s = wave_sum(R.s2);
        const double mx = wave_max(R.mx);
        if (lane == 0) {
            A.partials[2 * tile] = s;
            A.partials[2 * tile + 1] = mx;
        }
    }
}

}  // namespace lap
