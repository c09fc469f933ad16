// liblap runtime: device arena, grid hierarchies, solve drivers, hipGraph
// replay of multigrid cycles, kernel timing, and the C ABI of include/lap.h.
//
// Stopping is decided on the device: the norm kernels feed a one-block
// finalise kernel that updates a control block (Ctrl) and sets `done`; every
// later kernel of the solve reads `done` first and exits at once.  The host
// therefore enqueues cycles ahead and only polls the control block (copied
// to pinned memory after each cycle) one cycle behind.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "lap_kernels.hpp"
#include "../../include/lap.h"

using namespace lap;

// ====================================================================== errors
namespace {
thread_local std::string g_err;

lap_status fail(lap_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

#define HIPCHK(expr)                                                                           \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return fail(LAP_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define HIPERR(expr)                              \
    do {                                          \
        hipError_t e_ = (expr);                   \
        if (e_ != hipSuccess) return e_;          \
    } while (0)

constexpr size_t kAlign = 256;
size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
int pitch_of(int m) { return (int)round_up((size_t)m, 64); }

// ======================================================================= arena
// First-fit sub-allocator over the caller's device buffer; adjacent free
// blocks are merged on release.
struct Arena {
    char* base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free_;   // offset -> bytes
    std::map<size_t, size_t> used_;   // offset -> bytes
    size_t in_use = 0;

    void init(void* p, size_t bytes) {
        base = (char*)p;
        size = bytes / kAlign * kAlign;
        free_.clear();
        used_.clear();
        free_[0] = size;
        in_use = 0;
    }
    void* alloc(size_t bytes) {
        bytes = round_up(std::max<size_t>(bytes, 1), kAlign);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const size_t off = it->first, sz = it->second;
                free_.erase(it);
                if (sz > bytes) free_[off + bytes] = sz - bytes;
                used_[off] = bytes;
                in_use += bytes;
                return base + off;
            }
        }
        return nullptr;
    }
    void release(void* p) {
        if (p == nullptr) return;
        const size_t off = (size_t)((char*)p - base);
        auto it = used_.find(off);
        if (it == used_.end()) return;
        size_t sz = it->second;
        used_.erase(it);
        in_use -= sz;
        size_t start = off;
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && nx->first == off + sz) {
            sz += nx->second;
            free_.erase(nx);
        }
        auto pv = free_.lower_bound(off);
        if (pv != free_.begin()) {
            --pv;
            if (pv->first + pv->second == off) {
                start = pv->first;
                sz += pv->second;
                free_.erase(pv);
            }
        }
        free_[start] = sz;
    }
    size_t largest_free() const {
        size_t b = 0;
        for (auto& kv : free_) b = std::max(b, kv.second);
        return b;
    }
};

struct LevelGeo {
    int m, n, P;
    double dx, dy;
    size_t interior() const { return (size_t)(m - 2) * (size_t)(n - 2); }
};

template <typename T>
struct LevelBufs {
    T* u[2] = {nullptr, nullptr};
    T* b = nullptr;
};

struct Coef {
    double cx, cy, d, inv_d;
};
Coef coef(double dx, double dy) {
    Coef c;
    c.cx = 1.0 / (dx * dx);
    c.cy = 1.0 / (dy * dy);
    c.d = 2.0 * (c.cx + c.cy);
    c.inv_d = 1.0 / c.d;
    return c;
}

// Hierarchy plan: vertex coarsening while both sides are odd and stay >= 5.
std::vector<LevelGeo> plan_levels(int m, int n, double dx, double dy) {
    std::vector<LevelGeo> lv;
    lv.push_back({m, n, pitch_of(m), dx, dy});
    while (true) {
        const LevelGeo& L = lv.back();
        if ((L.m - 1) % 2 || (L.n - 1) % 2) break;
        const int mc = (L.m - 1) / 2 + 1, nc = (L.n - 1) / 2 + 1;
        if (mc < 5 || nc < 5) break;
        lv.push_back({mc, nc, pitch_of(mc), 2.0 * L.dx, 2.0 * L.dy});
    }
    return lv;
}

// Inverse of L_h restricted to the interior unknowns (k = (j-1)(m-2)+(i-1))
// of a small level, in FP64, by separation of variables: with Q the
// orthonormal sine transform across the short side (p unknowns, symmetric,
// Q^2 = I) and T_k the tridiagonal mode-k operator of -L_h along the long
// side (q unknowns), -L_h = (Q x I) diag_k(T_k) (Q x I), so
//   L_h^{-1}[(s,l),(s0,l0)] = - sum_k Q[s][k] Q[k][s0] T_k^{-1}[l][l0].
// T_k^{-1} comes from q Thomas solves; the whole inverse costs O(p N^2)
// (a dense factorisation took O(N^3), milliseconds per new level shape).
bool coarse_inverse(int m, int n, double dx, double dy, std::vector<double>& out) {
    const Coef c = coef(dx, dy);
    const int mi = m - 2, ni = n - 2, N = mi * ni;
    if (mi < 1 || ni < 1) return false;
    const bool xs = mi <= ni;                  // the short side runs along x
    const int p = xs ? mi : ni, q = xs ? ni : mi;
    const double cs = xs ? c.cx : c.cy, cl = xs ? c.cy : c.cx;
    const double pi = std::acos(-1.0), nrm = std::sqrt(2.0 / (p + 1));
    std::vector<double> Q((size_t)p * p), G((size_t)p * q * q);
    for (int k = 0; k < p; ++k)
        for (int s = 0; s < p; ++s) Q[(size_t)k * p + s] = nrm * std::sin(pi * (k + 1) * (s + 1) / (p + 1));
    std::vector<double> cp(q), z(q);
    for (int k = 0; k < p; ++k) {
        const double mu = 2.0 - 2.0 * std::cos(pi * (k + 1) / (p + 1));
        const double diag = cs * mu + 2.0 * cl, off = -cl;
        // factor once: pivots and c'
        std::vector<double> ipv(q);
        double prev = 0.0;
        for (int l = 0; l < q; ++l) {
            const double piv = diag - off * prev;
            if (!(piv > 0.0)) return false;
            ipv[l] = 1.0 / piv;
            cp[l] = off * ipv[l];
            prev = cp[l];
        }
        double* Gk = G.data() + (size_t)k * q * q;
        for (int l0 = 0; l0 < q; ++l0) {           // column l0 of T_k^{-1}
            double zp = 0.0;
            for (int l = 0; l < q; ++l) {
                zp = ((l == l0 ? 1.0 : 0.0) - off * zp) * ipv[l];
                z[l] = zp;
            }
            double x = 0.0;
            for (int l = q - 1; l >= 0; --l) {
                x = z[l] - cp[l] * x;
                Gk[(size_t)l * q + l0] = x;
            }
        }
    }
    out.assign((size_t)N * N, 0.0);
    std::vector<double> w(p);
    for (int s = 0; s < p; ++s)
        for (int s0 = 0; s0 < p; ++s0) {
            for (int k = 0; k < p; ++k) w[k] = Q[(size_t)s * p + k] * Q[(size_t)k * p + s0];
            for (int l = 0; l < q; ++l)
                for (int l0 = 0; l0 < q; ++l0) {
                    double v = 0.0;
                    for (int k = 0; k < p; ++k) v += w[k] * G[((size_t)k * q + l) * q + l0];
                    const size_t r = xs ? (size_t)l * mi + s : (size_t)s * mi + l;
                    const size_t col = xs ? (size_t)l0 * mi + s0 : (size_t)s0 * mi + l0;
                    out[r * N + col] = -v;
                }
        }
    return true;
}

// Coarsest levels above kDenseCoarseMax unknowns (long thin grids) are
// solved by separation of variables: the 5-point operator on a rectangle
// with constant coefficients is diagonalised along the short side by the
// orthonormal sine transform Q (p x p, p = short interior side), leaving one
// tridiagonal system along the long side per mode (q = long interior side).
// Factor layout: Q (p*p), then per mode k the Thomas factors of
// -L restricted to that mode, c'_l (q) and 1/pivot_l (q).
constexpr int kLineMax = 128;
constexpr size_t kLineStorageMax = (size_t)8 << 20;   // doubles

bool coarse_lines(int m, int n, double dx, double dy, std::vector<double>& out, int& p, int& ifast) {
    const Coef c = coef(dx, dy);
    const int mi = m - 2, ni = n - 2;
    ifast = mi <= ni ? 1 : 0;                // 1: the short side runs along x
    p = ifast ? mi : ni;
    const int q = ifast ? ni : mi;
    if (p < 1 || p > kLineMax || (size_t)p * p + 2 * (size_t)p * q > kLineStorageMax) return false;
    const double cs = ifast ? c.cx : c.cy, cl = ifast ? c.cy : c.cx;
    out.assign((size_t)p * p + 2 * (size_t)p * q, 0.0);
    const double pi = std::acos(-1.0), nrm = std::sqrt(2.0 / (p + 1));
    for (int k = 0; k < p; ++k)
        for (int s = 0; s < p; ++s) out[(size_t)k * p + s] = nrm * std::sin(pi * (k + 1) * (s + 1) / (p + 1));
    for (int k = 0; k < p; ++k) {
        // mode k of -L_h along the long side: diagonal cs*mu_k + 2 cl, off-diagonal -cl
        const double mu = 2.0 - 2.0 * std::cos(pi * (k + 1) / (p + 1));
        const double diag = cs * mu + 2.0 * cl, off = -cl;
        double* cpr = out.data() + (size_t)p * p + 2 * (size_t)k * q;
        double* ipv = cpr + q;
        double prev = 0.0;
        for (int l = 0; l < q; ++l) {
            const double piv = diag - off * prev;
            if (!(piv > 0.0)) return false;
            ipv[l] = 1.0 / piv;
            cpr[l] = off / piv;
            prev = cpr[l];
        }
    }
    return true;
}

bool coarse_ok(const LevelGeo& C) {
    const size_t N = C.interior();
    if (N <= (size_t)kDenseCoarseMax) return true;
    const size_t p = std::min(C.m, C.n) - 2, q = std::max(C.m, C.n) - 2;
    return p <= (size_t)kLineMax && p * p + 2 * p * q <= kLineStorageMax;
}

size_t coarse_bytes(const LevelGeo& C) {
    const size_t N = C.interior();
    if (N <= (size_t)kDenseCoarseMax) return N * N * 8;
    const size_t p = std::min(C.m, C.n) - 2, q = std::max(C.m, C.n) - 2;
    return (p * p + 2 * p * q) * 8;
}

enum Part { PART_ALL = 0, PART_HEAD = 1, PART_TAIL = 2 };

enum KClass { KC_SWEEP = 0, KC_SWEEP_PROLONG, KC_RESTRICT, KC_DEFECT, KC_COARSE, KC_FINALIZE,
              KC_ADI_ROWS, KC_ADI_COLS, KC_RESIDUAL, KC_SUBTREE, KC_PRE, KC_TWO, KC_TWO_PLAIN, KC_PAPER, KC_FOUR,
              KC_COUNT };

// Size classes for tilings, by interior node count.
// One class per factor 4 of interior nodes from 2^12 to 2^24, so each level
// of a power-of-two hierarchy (65, 129, ..., 8193 nodes a side) has a class
// of its own: 0 below 2^12, k below 2^(12 + 2k), 7 from 2^24 up.
constexpr int kSizeClasses = 8;
int size_class(size_t nint) {
    int k = 0;
    while (k < kSizeClasses - 1 && nint >= ((size_t)1 << (12 + 2 * k))) ++k;
    return k;
}

}  // namespace

// ====================================================================== context
struct lap_ctx {
    Arena arena;
    hipStream_t stream = nullptr;
    // kernel timing: 0 off, 1 HIP events around every launch, 2 events around
    // finest-level launches only (the others are counted, untimed)
    int timing = 0;
    struct Rec {
        int cls;
        bool fine;
        double bytes;
        hipEvent_t a, b;       // null: counted, not timed
        int solve, step;       // solve serial number and its outer step
        bool head;             // launched by the step's stopping test
    };
    // tags of the launches being enqueued (single-grid solves); solve -1 = untagged
    int rec_solve = -1, rec_step = 0, solve_serial = 0;
    bool rec_head = false;
    int safe_step = 0;         // steps below this of solve rec_solve are known to have done full work
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    int64_t launches[KC_COUNT][2] = {};
    double ms[KC_COUNT][2] = {};
    double bytes[KC_COUNT][2] = {};
    // tiling table: [size class][kernel class][dtype 0=f64,1=f32] -> (V, ty)
    int tileV[kSizeClasses][KC_COUNT][2];
    int tileTY[kSizeClasses][KC_COUNT][2];     // 0: auto (chunks sized for tileT waves)
    int tileT[kSizeClasses][KC_COUNT][2];
    int wave_cap = 8192;            // CUs x 32 wavefronts (read from the device)
    // small-level subtree: LDS the device grants one workgroup, and the
    // largest top level (nodes m*n) a subtree may start at (0: never)
    int lds_max = 65536;
    int64_t sub_max_nodes = -1;     // -1: any level whose subtree fits in LDS
    bool fuse = true;               // fused smoothing passes (two sweeps, + restriction, + prolongation)
    std::vector<lap_grid*> grids;
    std::map<std::string, std::vector<double>> inv_cache;
    Ctrl* pinned = nullptr;        // 4 host slots
    // batch readback: device pointer table, gathered control blocks, pinned copy
    int batch_cap = 0;
    Ctrl** batch_ptrs = nullptr;
    Ctrl* batch_ctrl = nullptr;
    Ctrl* batch_host = nullptr;      // pinned, 2 * batch_cap (two rounds in flight)
    CopyItem* copy_dev = nullptr;    // batch_cap end-of-solve buffer copies
    std::vector<Ctrl*> batch_ptrs_host;
    std::vector<CopyItem> copy_host;
    // merged-launch plans of batches, by composition key (grid set, step parity, options)
    struct Plan;
    std::vector<std::pair<std::string, Plan*>> plans;
    hipEvent_t poll_ev[2] = {nullptr, nullptr};

    hipEvent_t ev() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    void recycle(Rec& r) {
        if (r.a) pool.push_back(r.a);
        if (r.b) pool.push_back(r.b);
    }
    // Accumulate the records into the statistics.  all = false keeps the
    // records of the running solve that may still turn out speculative.
    hipError_t flush_recs(bool all = true) {
        if (recs.empty()) return hipSuccess;
        HIPERR(hipStreamSynchronize(stream));
        std::vector<Rec> keep;
        for (auto& r : recs) {
            if (!all && r.solve == rec_solve && r.solve >= 0 && r.step >= safe_step) {
                keep.push_back(r);
                continue;
            }
            float t = 0.f;
            if (r.a) HIPERR(hipEventElapsedTime(&t, r.a, r.b));
            for (int f = 0; f < 2; ++f) {
                if (f == 1 && !r.fine) continue;
                launches[r.cls][f] += 1;
                ms[r.cls][f] += t;
                bytes[r.cls][f] += r.bytes;
            }
            recycle(r);
        }
        recs.swap(keep);
        return hipSuccess;
    }
    // Forget the launches of solve `solve` that came after its stopping test
    // in step `last` (they exited at once on the device's done flag).
    void drop_speculative(int solve, int last) {
        std::vector<Rec> keep;
        for (auto& r : recs) {
            if (r.solve == solve && (r.step > last || (r.step == last && !r.head)))
                recycle(r);
            else
                keep.push_back(r);
        }
        recs.swap(keep);
    }
    template <typename F>
    hipError_t timed(int cls, bool fine, double nbytes, F&& launch) {
        if (!timing) return launch();
        if (timing == 2 && !fine) {
            HIPERR(launch());
            recs.push_back({cls, fine, nbytes, nullptr, nullptr, rec_solve, rec_step, rec_head});
        } else {
            hipEvent_t a = ev(), b = ev();
            if (a == nullptr || b == nullptr) return hipErrorOutOfMemory;
            HIPERR(hipEventRecord(a, stream));
            HIPERR(launch());
            HIPERR(hipEventRecord(b, stream));
            recs.push_back({cls, fine, nbytes, a, b, rec_solve, rec_step, rec_head});
        }
        if (recs.size() > 8192) return flush_recs(false);
        return hipSuccess;
    }
    Tiling tiling(int m, int n, int cls, int dt, int H = 2) const {
        const int sc = size_class((size_t)(m - 2) * (size_t)(n - 2));
        return make_tiling(m, n, tileV[sc][cls][dt], tileTY[sc][cls][dt], tileT[sc][cls][dt], H);
    }
};

namespace {
void plans_clear(lap_ctx* c);   // batch plans (defined with the batch executor)
}

// ========================================================================= grid
struct lap_grid {
    lap_ctx* ctx = nullptr;
    int m = 0, n = 0, P = 0;
    double dx = 0, dy = 0;
    int flags = 0;
    bool has_f = false;
    std::vector<LevelGeo> geo;
    double* psi[2] = {nullptr, nullptr};
    double* f64 = nullptr;
    std::vector<LevelBufs<double>> l64;
    std::vector<LevelBufs<float>> l32;
    float* rhs2 = nullptr;           // second level-0 FP32 right-hand side (mixed: steps alternate)
    double* minv = nullptr;          // dense inverse or separable factor of the coarsest level
    double* coarse_work = nullptr;   // separable solve scratch
    int coarse_bw = 0, coarse_ifast = 1;
    double* adi_scratch = nullptr;
    double* adi_tab = nullptr;       // rows cprime, rows piv, cols cprime, cols piv (each maxK), then
                                     // the rows and the columns segment tables (kSegTab each)
    int adi_maxk = 0;
    std::vector<double> adi_host;
    double adi_omega = -1.0;         // (omega, form) the uploaded tables were made for
    int adi_form = -1;
    bool psi1_stale = false;         // psi[1]'s interior lags psi[0] (after ADI, which works in place)
    Ctrl* ctrl = nullptr;
    Ctrl* cyc = nullptr;             // four gates of mixed steps with several FP32 cycles (two per step parity)
    Ctrl* op_ctrl = nullptr;         // while an operation is launched: the control block its kernels test
    double* partials = nullptr;
    int max_partials = 0;
    double* norm_out = nullptr;
    double last_r0 = -1.0;
    double tol = 1e-10;
    double batch_omega = 1.0;        // smoother relaxation of batched steps (lap_grid_set_omega)
    bool batch_started = false;
    bool batch_done = false;
    double batch_t0 = 0.0;
    int step_idx = 0;                // next outer step of the running solve
    int e_idx = 0;                   // buffer of the last FP32 correction (mixed)
    int e1_idx = 0;                  // buffer of the first cycle's correction (mixed, several cycles)
    // zebra line smoothing: segment tables of every smoothed level, rows then
    // columns (2 * kSegTab values per level), FP64 and FP32
    double* ztab64 = nullptr;
    float* ztab32 = nullptr;
    std::vector<double> zhost64;     // host copies (the uploads read them asynchronously)
    std::vector<float> zhost32;
    bool zebra_ok = false;
    bool pdef = false;               // the running mixed solve uses the post-smoothing + defect pass
    lap_opts batch_opts{};
    // graph cache
    hipGraphExec_t graph = nullptr;
    std::string graph_key;
    std::vector<std::string> graph_seen;   // options of recent solves (a repeat captures the graph)
    std::string graph_run_key;             // options of the running solve
    bool graph_on = false;           // the running solve replays the graph
    std::vector<void*> allocs;
};

namespace {

// The control block whose done flag the kernels of the operation being
// launched test: a gate of a mixed step while one is set, else the solve's.
inline Ctrl* kctrl(const lap_grid* g) { return g->op_ctrl != nullptr ? g->op_ctrl : g->ctrl; }

void* galloc(lap_grid* g, size_t bytes) {
    void* p = g->ctx->arena.alloc(bytes);
    if (p) g->allocs.push_back(p);
    return p;
}

struct Footprint {
    size_t bytes = 0;
    void add(size_t b) { bytes += round_up(std::max<size_t>(b, 1), kAlign); }
};

size_t max_tiles(int m, int n) {
    // the finest tiling any table entry may pick: V = 1, ty = 16
    int t = make_tiling(m, n, 1, 16).ntiles;
    for (int k : {(int)NORM_PASS, (int)NORM_DEFECT, (int)NORM_POSTDEF}) t = std::max(t, norm_partials(m, n, k));
    return (size_t)t;
}

// Whether every smoothed level's row and column lines fit the segmented line
// solver (zebra line smoothing needs it).
bool zebra_fits(const std::vector<LevelGeo>& lv) {
    for (size_t l = 0; l + 1 < lv.size(); ++l)
        if (!seg_fits(0, lv[l].m - 2) || !seg_fits(1, lv[l].n - 2)) return false;
    return true;
}

// Mirrors the allocations of lap_grid_create_ex.
Footprint footprint(int m, int n, bool has_f, int flags) {
    Footprint fp;
    const auto lv = plan_levels(m, n, 1.0, 1.0);
    const LevelGeo& L0 = lv[0];
    const size_t f0 = (size_t)L0.n * L0.P;
    fp.add(f0 * 8);
    fp.add(f0 * 8);
    if (has_f) fp.add(f0 * 8);
    if (flags & LAP_ALLOC_FP64)
        for (size_t l = 1; l < lv.size(); ++l)
            for (int k = 0; k < 3; ++k) fp.add((size_t)lv[l].n * lv[l].P * 8);
    if (flags & LAP_ALLOC_MIXED) {
        for (size_t l = 0; l < lv.size(); ++l)
            for (int k = 0; k < 3; ++k) fp.add((size_t)lv[l].n * lv[l].P * 4);
        fp.add(f0 * 4);
    }
    if (flags & (LAP_ALLOC_FP64 | LAP_ALLOC_MIXED)) {
        fp.add(coarse_bytes(lv.back()));
        if (lv.back().interior() > (size_t)kDenseCoarseMax) fp.add(lv.back().interior() * 8);
        if (zebra_fits(lv)) {
            if (flags & LAP_ALLOC_FP64) fp.add(lv.size() * 2 * kSegTab * 8);
            if (flags & LAP_ALLOC_MIXED) fp.add(lv.size() * 2 * kSegTab * 4);
        }
    }
    if (flags & LAP_ALLOC_ADI) {
        fp.add(f0 * 8);
        fp.add(((size_t)4 * std::max(m, n) + 2 * kSegTab) * 8);
    }
    fp.add(5 * sizeof(Ctrl));
    fp.add(max_tiles(m, n) * 16);
    fp.add(16);
    return fp;
}

lap_status check_ptr(const void* p, const char* what) {
    if (p == nullptr) return fail(LAP_EINVAL, std::string(what) + " is NULL");
    return LAP_OK;
}

// ------------------------------------------------------------- kernel enqueue
double nint(const LevelGeo& L) { return (double)L.interior(); }

template <typename T>
struct HierView {
    std::vector<T*> u0, u1, b;
    bool zero_start0 = false;  // level 0 starts from zero (error equation) or holds the iterate
    int root = 0;              // level of the cycle's root (full multigrid roots cycles on coarse levels)
    int sub_root = -1;         // level whose whole sub-V-cycle runs as one LDS-resident launch
};

// LDS bytes of a subtree rooted at level l: u and b of every level l..L-1
// (pitch m), then the coarsest right-hand side in FP64 (dense coarsest solve)
template <typename T>
size_t subtree_lds(const std::vector<LevelGeo>& geo, int l) {
    size_t e = 0;
    for (size_t k = (size_t)l; k < geo.size(); ++k) e += 2 * (size_t)geo[k].m * (size_t)geo[k].n;
    size_t bytes = (e * sizeof(T) + 7) / 8 * 8;
    const size_t N = geo.back().interior();
    if (N <= (size_t)kDenseCoarseMax) bytes += N * sizeof(double);
    return bytes;
}

// First level at or below `lmin` from which the rest of the V-cycle fits one
// workgroup's LDS (and the context's node limit); -1 if none.  The root must
// have a level below it, and at most kMaxSub levels may take part.
template <typename T>
int subtree_root(const lap_grid* g, int lmin) {
    const lap_ctx* c = g->ctx;
    const int L = (int)g->geo.size();
    if (c->sub_max_nodes == 0) return -1;
    for (int l = std::max(lmin, L - kMaxSub); l < L - 1; ++l) {
        const LevelGeo& G = g->geo[l];
        if (c->sub_max_nodes > 0 && (int64_t)G.m * G.n > c->sub_max_nodes) continue;
        if (subtree_lds<T>(g->geo, l) <= (size_t)c->lds_max) return l;
    }
    return -1;
}

// Arguments of the subtree rooted at level l (u -> out, right-hand side b).
template <typename T>
SubtreeArgs<T> subtree_args(const lap_grid* g, int l, T* out, const T* b, double omega, int nus) {
    SubtreeArgs<T> a{};
    const int L = (int)g->geo.size();
    a.out = out;
    a.b = b;
    a.P = g->geo[l].P;
    a.nlev = L - l;
    a.nu1 = nus & 255;
    a.nu2 = nus >> 8;
    a.omega = (T)omega;
    int off = 0;
    for (int k = 0; k < a.nlev; ++k) {
        const LevelGeo& G = g->geo[l + k];
        const Coef c = coef(G.dx, G.dy);
        SubLevel<T>& v = a.lv[k];
        v.m = G.m;
        v.n = G.n;
        v.ou = off;
        off += G.m * G.n;
        v.ob = off;
        off += G.m * G.n;
        v.cx = (T)c.cx;
        v.cy = (T)c.cy;
        v.d = (T)c.d;
        v.inv_d = (T)c.inv_d;
    }
    a.lds_elems = off;
    a.lds_bytes = (int)subtree_lds<T>(g->geo, l);
    a.minv = g->minv;
    a.work = g->coarse_work;
    a.bw = g->coarse_bw;
    a.ifast = g->coarse_ifast;
    const Coef cc = coef(g->geo.back().dx, g->geo.back().dy);
    a.ccx = cc.cx;
    a.ccy = cc.cy;
    a.ctrl = kctrl(g);
    return a;
}

template <typename T>
hipError_t enq_subtree(lap_grid* g, int l, T* out, const T* b, double omega, int nus) {
    const SubtreeArgs<T> a = subtree_args<T>(g, l, out, b, omega, nus);
    const double bytes = 2.0 * sizeof(T) * g->geo[l].m * (double)g->geo[l].n;
    return g->ctx->timed(KC_SUBTREE, false, bytes, [&]() { return launch_subtree<T>(a, g->ctx->stream); });
}

template <typename T> constexpr int dt_of() { return sizeof(T) == 8 ? 0 : 1; }

template <typename T>
SweepArgs<T> sweep_args(lap_grid* g, int l, const T* in, T* out, const T* f, const T* ec, double omega,
                        bool norm) {
    const LevelGeo& L = g->geo[l];
    const Coef c = coef(L.dx, L.dy);
    SweepArgs<T> a{};
    a.uin = in;
    a.uout = out;
    a.f = f;
    a.ec = ec;
    a.partials = norm ? g->partials : nullptr;
    a.ctrl = kctrl(g);
    a.m = L.m;
    a.n = L.n;
    a.P = L.P;
    if ((size_t)l + 1 < g->geo.size()) {
        a.mc = g->geo[l + 1].m;
        a.nc = g->geo[l + 1].n;
        a.Pc = g->geo[l + 1].P;
    }
    a.cx = (T)c.cx;
    a.cy = (T)c.cy;
    a.d = (T)c.d;
    a.inv_d = (T)c.inv_d;
    a.omega = (T)omega;
    a.tl = norm ? norm_tiling(L.m, L.n) : g->ctx->tiling(L.m, L.n, ec ? KC_SWEEP_PROLONG : KC_SWEEP, dt_of<T>());
    return a;
}

template <typename T>
hipError_t enq_sweep(lap_grid* g, int l, const T* in, T* out, const T* f, const T* ec, double omega, int flags) {
    SweepArgs<T> a = sweep_args<T>(g, l, in, out, f, ec, omega, (flags & SW_NORM) != 0);
    const LevelGeo& L = g->geo[l];
    double per = (flags & SW_ZERO) ? 1.0 : 2.0;
    if (flags & SW_F) per += 1.0;
    if (flags & SW_PROLONG) per += 0.25;
    const int cls = (flags & SW_PROLONG) ? KC_SWEEP_PROLONG : KC_SWEEP;
    return g->ctx->timed(cls, l == 0, per * sizeof(T) * nint(L),
                         [&]() { return launch_sweep<T>(a, flags, g->ctx->stream); });
}

// Halo, kernel class and tiling of a fused pass with these flags.
int fused_halo(int flags) {
    return ((flags & SW_FOUR) ? 8 : (flags & SW_TWO) ? 4 : 2) + ((flags & SW_RESTRICT) ? 2 : 0);
}
// (two-sweep passes with the prolongation and without any transfer, as red-black
// SOR runs them, are tuned apart: their best tilings differ)
int fused_class(int flags) {
    if (flags & SW_PROBE) return KC_RESIDUAL;   // norms only: timed with the residual-norm kernels
    if (flags & SW_FOUR) return KC_FOUR;
    if (flags & SW_RESTRICT) return KC_PRE;
    return (flags & SW_PROLONG) ? KC_TWO : KC_TWO_PLAIN;
}
bool is_fused(int flags) { return (flags & (SW_TWO | SW_FOUR | SW_RESTRICT)) != 0; }

// Algorithmic bytes per interior node of a sweep or fused pass.
double sweep_bytes_per_node(int flags, int sz) {
    if (flags & SW_PROBE) return ((flags & SW_F) ? 2.0 : 1.0) * sz;   // reads u (and f) only
    double per = (flags & SW_ZERO) ? 1.0 : 2.0;
    if (flags & SW_F) per += 1.0;
    if (flags & SW_PROLONG) per += 0.25;
    if (flags & SW_RESTRICT) per += 0.25;
    return per * sz;
}

// Whether a fused pass stores its rows nontemporally (past L2 and the
// Infinity Cache).  Measured on an 8193^2 solve: for the FP64 multigrid
// passes of every level it saves ~15 us per cycle on the coarser levels and
// is even on the finest (7.00 -> 6.85 ms); the FP32 passes of the mixed loop
// and the SOR passes (whose output the next pass reads at once) gain
// nothing or lose, and keep ordinary stores, as do merged batch launches of
// small grids.
bool fused_nt(int dt, int flags) {
    return dt == 0 && (flags & (SW_RESTRICT | SW_PROLONG)) != 0;
}

template <typename T>
hipError_t enq_fused(lap_grid* g, int l, const T* in, T* out, const T* f, const T* ec, T* bc, double omega,
                     int flags) {
    SweepArgs<T> a = sweep_args<T>(g, l, in, out, f, ec, omega, (flags & SW_NORM) != 0);
    const LevelGeo& L = g->geo[l];
    a.bc = bc;
    a.nt = fused_nt(dt_of<T>(), flags) ? 1 : 0;
    if (!(flags & SW_NORM)) a.tl = g->ctx->tiling(L.m, L.n, fused_class(flags), dt_of<T>(), fused_halo(flags));
    return g->ctx->timed(fused_class(flags), l == 0, sweep_bytes_per_node(flags, sizeof(T)) * nint(L),
                         [&]() { return launch_fused<T>(a, flags, g->ctx->stream); });
}

hipError_t enq_finalize(lap_grid* g, int ntiles, int mode = 0, const Ctrl* gate = nullptr, int cycles = -1) {
    return g->ctx->timed(KC_FINALIZE, false, 16.0 * ntiles, [&]() {
        return launch_finalize(g->partials, ntiles, g->ctrl, nullptr, mode, g->ctx->stream, gate,
                               cycles >= 0 ? g->cyc : nullptr, cycles >= 0 ? cycles : 0);
    });
}

template <typename T>
hipError_t enq_restrict(lap_grid* g, int l, const T* u, const T* f, T* bc, T* uc0 = nullptr, bool rdiff = false) {
    const LevelGeo& L = g->geo[l];
    const LevelGeo& C = g->geo[l + 1];
    const Coef c = coef(L.dx, L.dy);
    RestrictArgs<T> a{};
    a.u = u;
    a.f = f;
    a.bc = bc;
    a.uc0 = uc0;
    a.ctrl = kctrl(g);
    a.m = L.m;
    a.n = L.n;
    a.P = L.P;
    a.mc = C.m;
    a.nc = C.n;
    a.Pc = C.P;
    a.cx = (T)c.cx;
    a.cy = (T)c.cy;
    a.d = (T)c.d;
    a.rdiff = rdiff ? 1 : 0;
    a.tl = g->ctx->tiling(L.m, L.n, KC_RESTRICT, dt_of<T>());
    const double per = (u ? 1.0 : 0.0) + (f ? 1.0 : 0.0) + (uc0 ? 0.5 : 0.25);
    return g->ctx->timed(KC_RESTRICT, l == 0, per * sizeof(T) * nint(L),
                         [&]() { return launch_restrict<T>(a, g->ctx->stream); });
}

template <typename T>
hipError_t enq_coarse(lap_grid* g, int l, const T* ubnd, const T* b, T* out) {
    const LevelGeo& L = g->geo[l];
    const Coef c = coef(L.dx, L.dy);
    CoarseArgs<T> a{};
    a.u = ubnd;
    a.b = b;
    a.out = out;
    a.minv = g->minv;
    a.work = g->coarse_work;
    a.bw = g->coarse_bw;
    a.ifast = g->coarse_ifast;
    a.ctrl = kctrl(g);
    a.m = L.m;
    a.n = L.n;
    a.P = L.P;
    a.cx = c.cx;
    a.cy = c.cy;
    return g->ctx->timed(KC_COARSE, l == 0, 2.0 * sizeof(T) * nint(L),
                         [&]() { return launch_coarse<T>(a, g->ctx->stream); });
}

template <typename T>
hipError_t enq_residual_norm(lap_grid* g, int l, const T* u, const T* f) {
    const LevelGeo& L = g->geo[l];
    const Coef c = coef(L.dx, L.dy);
    ResidualArgs<T> a{};
    a.u = u;
    a.f = f;
    a.r = nullptr;
    a.partials = g->partials;
    a.ctrl = kctrl(g);
    a.m = L.m;
    a.n = L.n;
    a.P = L.P;
    a.cx = (T)c.cx;
    a.cy = (T)c.cy;
    a.d = (T)c.d;
    a.tl = norm_tiling(L.m, L.n);
    return g->ctx->timed(KC_RESIDUAL, l == 0, (f ? 2.0 : 1.0) * sizeof(T) * nint(L),
                         [&]() { return launch_residual<T>(a, g->ctx->stream); });
}

// ---------------------------------------------------------------- op plans
// A step of a method is first recorded as a list of operations, each with a
// merge key; the single-grid executor launches them in order, and the batch
// executor launches all grids' operations of one key as one merged launch.
// Keys order a V-cycle top-aligned across grids of different depth: the
// pre-smoothing and restriction of level l, then every grid's coarsest
// solve, then the post-smoothing of level l from coarse to fine.
enum OpKind { OP_SWEEP, OP_RESTRICT, OP_COARSE, OP_FINALIZE, OP_RESNORM, OP_DEFECT, OP_ADI_ROWS, OP_ADI_COLS,
              OP_SUBTREE, OP_POSTDEF, OP_BOUNDARY };

struct Op {
    long key;
    int kind;
    int dt;          // 0 FP64, 1 FP32
    int level;
    int flags;       // sweep flags; subtree: nu1 | nu2 << 8
    const void* in;  // sweep input, restrict / residual u, defect psi_in, coarse boundary source
    void* out;       // sweep / coarse output, defect psi_out
    const void* f;   // right-hand side
    const void* ec;  // sweep: coarse correction; defect: FP32 correction
    void* bc;        // restrict: coarse right-hand side; post + defect: the new FP32 right-hand side
    double omega;
    int parity;      // ADI line parity; post + defect: buffer of the level-0 pre-smoothing result
    void* zbuf = nullptr;   // defect: FP32 buffer to set to zero (the next zebra cycle's start)
    Ctrl* gate = nullptr;   // its kernels do nothing while gate->done is set (mixed steps of several cycles)
    int cycles = -1;        // finalisation of a mixed step of several cycles: inner | parity << 8
};

constexpr long KEY_HEAD = 10;
// Op.parity of a finalisation that probes the test the next step opens with
constexpr int kProbeFinalize = 2;
// (the stopping test's finalise must sit between the first and the second
// pre-smoothing sweep: keys of a grid increase along its own operation order)
inline long key_pre(int l, int k) { return 1000 + 100L * l + 2L * k; }
inline long key_norm_fin(int l) { return 1000 + 100L * l + 1; }
inline long key_restrict(int l) { return 1000 + 100L * l + 99; }
constexpr long KEY_COARSE = 20000;
inline long key_post(int l, int k) { return 30000 + 100L * (99 - l) + k; }
// the keys of a mixed step's FP32 cycle c (one V-cycle's keys lie below it)
// are offset by c * KEY_CYCLE
constexpr long KEY_CYCLE = 40000;

template <typename T>
void push_op(std::vector<Op>& ops, long key, int kind, int level, int flags, const void* in, void* out,
             const void* f, const void* ec, void* bc, double omega, int parity = 0) {
    Op op;
    op.key = key;
    op.kind = kind;
    op.dt = dt_of<T>();
    op.level = level;
    op.flags = flags;
    op.in = in;
    op.out = out;
    op.f = f;
    op.ec = ec;
    op.bc = bc;
    op.omega = omega;
    op.parity = parity;
    ops.push_back(op);
}

// Sweeps per pass of the pre- and post-smoothing of one level.  Without
// fusion every sweep is a pass of its own; with fusion passes take up to two
// sweeps (an odd pre-smoothing count puts the single sweep first, so the
// restriction rides on a two-sweep pass; an odd post count puts it last).
// A level that carries the iterate (not a zero start) must end in the buffer
// it started in: if the number of passes is odd, the first two-sweep pass is
// split (one exists, as nu1 + nu2 is even).
struct PassPlan {
    std::vector<int> pre, post;
};

PassPlan pass_plan(const lap_ctx* c, const lap_opts& o, bool keep_parity) {
    PassPlan p;
    if (!c->fuse) {
        p.pre.assign(o.nu1, 1);
        p.post.assign(o.nu2, 1);
        return p;
    }
    int k = o.nu1;
    if (k % 2) {
        p.pre.push_back(1);
        --k;
    }
    for (; k > 0; k -= 2) p.pre.push_back(2);
    for (k = o.nu2; k >= 2; k -= 2) p.post.push_back(2);
    if (k) p.post.push_back(1);
    if (keep_parity && (p.pre.size() + p.post.size()) % 2) {
        for (std::vector<int>* v : {&p.pre, &p.post}) {
            auto it = std::find(v->begin(), v->end(), 2);
            if (it != v->end()) {
                *it = 1;
                v->insert(it, 1);
                break;
            }
        }
    }
    return p;
}

// Sweeps per pass of one red-black SOR check block of `ce` sweeps: pairs
// with fusion (an odd count ends with a single sweep), else single sweeps.
std::vector<int> sor_passes(const lap_ctx* c, int ce) {
    std::vector<int> p;
    if (!c->fuse) {
        p.assign(ce, 1);
        return p;
    }
    p.assign(ce / 2, 2);
    if (ce % 2) p.push_back(1);
    return p;
}

// Buffer (0/1) in which a zero-start V-cycle leaves its level result: the
// first pre-smoothing pass writes buffer 0, every further pass flips.
int vcycle_result_index(const lap_ctx* c, const lap_opts& o) {
    const PassPlan p = pass_plan(c, o, false);
    const int npre = (int)p.pre.size(), npost = (int)p.post.size();
    return (npre >= 1 ? npre - 1 + npost : npost - 1) % 2;
}

// The first post-smoothing pass of level 0, left out of a cycle's plan (the
// next outer step runs it fused with its defect correction): the buffer it
// starts from and the coarse correction it adds.
struct DeferredPost {
    int in = -1;
    const void* ec = nullptr;
};

// One V-cycle on level l of hierarchy H.  Level 0 either holds the iterate in
// u0[0] (FP64 multigrid: the result returns to u0[0] since nu1+nu2 is even)
// or starts from zero (error equation).  Returns the buffer index (0/1)
// that holds the level's result.  `part` (level 0 with a norm only):
// PART_HEAD records the stopping test of the incoming iterate, PART_TAIL the rest.
// With dp, level 0 stops before its post-smoothing and describes it in *dp.
int adi_kernel_flags(int dir, int K);

// Zebra line smoothing of level l: `steps` alternating steps (odd rows, even
// rows, odd columns, even columns), in place on u, keys k0, k0+1, ...
template <typename T>
void push_zebra(lap_grid* g, int l, T* u, const T* b, double omega, int steps, long k0, std::vector<Op>& ops) {
    const LevelGeo& G = g->geo[l];
    for (int k = 0; k < steps; ++k)
        for (int q = 0; q < 4; ++q) {
            const int dir = q < 2 ? 0 : 1;
            push_op<T>(ops, k0 + 4L * k + q, dir == 0 ? OP_ADI_ROWS : OP_ADI_COLS, l,
                       ADI_MG | adi_kernel_flags(dir, dir == 0 ? G.m - 2 : G.n - 2), nullptr, u, b, nullptr,
                       nullptr, omega, (q % 2) ? 0 : 1);
        }
}

// V-cycle with zebra line smoothing (LAP_SMOOTH_ZEBRA).  Every level works
// in place on its first buffer: the smoothing steps, then r = b - L u and
// its full weighting onto the coarse right-hand side (the same launch sets
// the coarse iterate to zero), the coarse cycle, u += P(e_c), the smoothing
// steps.  A zero-start level 0 (error equation) was zeroed by the defect
// correction that formed its right-hand side.  The stopping test's norms of
// the incoming iterate come from the residual-norm kernel.  Returns 0 (the
// buffer holding the result).
template <typename T>
int plan_vcycle_zebra(lap_grid* g, HierView<T>& H, int l, const lap_opts& o, bool norm, int part,
                      std::vector<Op>& ops) {
    const int L = (int)g->geo.size();
    const bool zero_start = (l > 0) || H.zero_start0;
    const bool split = norm && !zero_start;
    const bool head = !split || part != PART_TAIL;
    const bool tail = !split || part != PART_HEAD;
    T* U = H.u0[l];
    const T* b = H.b[l];
    if (split && head) {
        push_op<T>(ops, KEY_HEAD, OP_RESNORM, l, 0, U, nullptr, b, nullptr, nullptr, 0.0);
        push_op<T>(ops, KEY_HEAD + 1, OP_FINALIZE, l, 0, nullptr, nullptr, nullptr, nullptr, nullptr, 0.0);
    }
    if (!tail) return 0;
    if (l == L - 1) {
        push_op<T>(ops, KEY_COARSE, OP_COARSE, l, 0, zero_start ? nullptr : U, U, b, nullptr, nullptr, 0.0);
        return 0;
    }
    push_zebra<T>(g, l, U, b, o.omega, o.nu1, key_pre(l, 0), ops);
    push_op<T>(ops, key_restrict(l), OP_RESTRICT, l, 0, U, H.u0[l + 1], b, nullptr, H.b[l + 1], 0.0);
    plan_vcycle_zebra<T>(g, H, l + 1, o, false, PART_ALL, ops);
    push_op<T>(ops, key_post(l, 0), OP_SWEEP, l, SW_PROLONG | SW_PONLY, U, U, nullptr, H.u0[l + 1], nullptr, 0.0);
    push_zebra<T>(g, l, U, b, o.omega, o.nu2, key_post(l, 1), ops);
    return 0;
}

template <typename T>
int plan_vcycle(lap_grid* g, HierView<T>& H, int l, const lap_opts& o, bool norm, int part, std::vector<Op>& ops,
                DeferredPost* dp = nullptr) {
    if (o.smoother == LAP_SMOOTH_ZEBRA) return plan_vcycle_zebra<T>(g, H, l, o, norm, part, ops);
    const int L = (int)g->geo.size();
    const bool zero_start = (l > H.root) || (l == H.root && H.zero_start0);
    const bool split = norm && !zero_start;
    const bool head = !split || part != PART_TAIL;
    const bool tail = !split || part != PART_HEAD;
    T* U[2] = {H.u0[l], H.u1[l]};
    const T* b = H.b[l];
    if (zero_start && l == H.sub_root && l < L - 1) {
        // the whole sub-V-cycle in one launch; its result lands where the
        // multi-launch schedule would leave it
        const int ri = vcycle_result_index(g->ctx, o);
        push_op<T>(ops, KEY_COARSE, OP_SUBTREE, l, o.nu1 | (o.nu2 << 8), nullptr, U[ri], b, nullptr, nullptr,
                   o.omega);
        return ri;
    }
    if (l == L - 1) {
        if (split && head) {
            push_op<T>(ops, KEY_HEAD, OP_RESNORM, l, 0, U[0], nullptr, b, nullptr, nullptr, 0.0);
            push_op<T>(ops, KEY_HEAD + 1, OP_FINALIZE, l, 0, nullptr, nullptr, nullptr, nullptr, nullptr, 0.0);
        }
        if (tail) push_op<T>(ops, KEY_COARSE, OP_COARSE, l, 0, zero_start ? nullptr : U[0], U[0], b, nullptr,
                             nullptr, 0.0);
        return 0;
    }
    const int fb = b ? SW_F : 0;
    int cur = 0;
    bool have_u = !zero_start;
    if (split && o.nu1 == 0) {
        if (head) {
            push_op<T>(ops, KEY_HEAD, OP_RESNORM, l, 0, U[0], nullptr, b, nullptr, nullptr, 0.0);
            push_op<T>(ops, KEY_HEAD + 1, OP_FINALIZE, l, 0, nullptr, nullptr, nullptr, nullptr, nullptr, 0.0);
        }
        if (!tail) return 0;
    }
    const PassPlan pp = pass_plan(g->ctx, o, !zero_start);
    const int npre = (int)pp.pre.size(), npost = (int)pp.post.size();
    const bool fused_restrict = g->ctx->fuse && npre > 0;
    for (int k = 0; k < npre; ++k) {
        int fl = fb | (pp.pre[k] == 2 ? SW_TWO : 0);
        void* bc = nullptr;
        if (fused_restrict && k == npre - 1) {
            fl |= SW_RESTRICT;
            bc = H.b[l + 1];
        }
        if (!have_u) {
            push_op<T>(ops, key_pre(l, k), OP_SWEEP, l, SW_ZERO | fl, nullptr, U[0], b, nullptr, bc, o.omega);
            cur = 0;
            have_u = true;
        } else {
            const bool nk = split && k == 0;
            if (!nk || head) {
                push_op<T>(ops, key_pre(l, k), OP_SWEEP, l, fl | (nk ? SW_NORM : 0), U[cur], U[1 - cur], b, nullptr,
                           bc, o.omega);
                if (nk)
                    push_op<T>(ops, key_norm_fin(l), OP_FINALIZE, l, 0, nullptr, nullptr, nullptr, nullptr, nullptr,
                               0.0);
            }
            cur = 1 - cur;
            if (nk && !tail) return 0;
        }
    }
    if (!fused_restrict)
        push_op<T>(ops, key_restrict(l), OP_RESTRICT, l, 0, have_u ? U[cur] : nullptr, nullptr, b, nullptr, H.b[l + 1],
                   0.0);
    const int cres = plan_vcycle<T>(g, H, l + 1, o, false, PART_ALL, ops);
    const T* ec = (cres == 0 ? H.u0[l + 1] : H.u1[l + 1]);
    if (dp != nullptr && l == 0) {
        dp->in = have_u ? cur : -1;
        dp->ec = ec;
        return cur;
    }
    for (int k = 0; k < npost; ++k) {
        const int fl = fb | (pp.post[k] == 2 ? SW_TWO : 0);
        if (k == 0) {
            push_op<T>(ops, key_post(l, k), OP_SWEEP, l, SW_PROLONG | fl, have_u ? U[cur] : nullptr,
                       U[have_u ? 1 - cur : 0], b, ec, nullptr, o.omega);
            cur = have_u ? 1 - cur : 0;
            have_u = true;
        } else {
            push_op<T>(ops, key_post(l, k), OP_SWEEP, l, fl, U[cur], U[1 - cur], b, nullptr, nullptr, o.omega);
            cur = 1 - cur;
        }
    }
    return cur;
}

HierView<double> view64(lap_grid* g) {
    HierView<double> H;
    const int L = (int)g->geo.size();
    H.u0.resize(L);
    H.u1.resize(L);
    H.b.resize(L);
    H.u0[0] = g->psi[0];
    H.u1[0] = g->psi[1];
    H.b[0] = g->f64;
    for (int l = 1; l < L; ++l) {
        H.u0[l] = g->l64[l].u[0];
        H.u1[l] = g->l64[l].u[1];
        H.b[l] = g->l64[l].b;
    }
    H.zero_start0 = false;
    H.sub_root = subtree_root<double>(g, 1);
    return H;
}

HierView<float> view32(lap_grid* g) {
    HierView<float> H;
    const int L = (int)g->geo.size();
    H.u0.resize(L);
    H.u1.resize(L);
    H.b.resize(L);
    for (int l = 0; l < L; ++l) {
        H.u0[l] = g->l32[l].u[0];
        H.u1[l] = g->l32[l].u[1];
        H.b[l] = g->l32[l].b;
    }
    H.zero_start0 = true;
    H.sub_root = subtree_root<float>(g, 0);
    return H;
}

hipError_t enq_defect(lap_grid* g, const double* psi_in, double* psi_out, const float* e, float* rhs,
                      float* ezero = nullptr) {
    const LevelGeo& L = g->geo[0];
    const Coef c = coef(L.dx, L.dy);
    DefectArgs a{};
    a.psi_in = psi_in;
    a.psi_out = psi_out;
    a.e = e;
    a.f = g->f64;
    a.rhs = rhs;
    a.ezero = ezero;
    a.partials = g->partials;
    a.ctrl = kctrl(g);
    a.m = L.m;
    a.n = L.n;
    a.P = L.P;
    a.cx = c.cx;
    a.cy = c.cy;
    a.d = c.d;
    a.tl = norm_tiling(L.m, L.n, NORM_DEFECT);
    // psi and e (and f) read, psi written unless in place, the FP32 right-hand side written
    const double per = 8.0 + (e ? 4.0 : 0.0) + (g->f64 ? 8.0 : 0.0) + (psi_out != psi_in || e ? 8.0 : 0.0) + 4.0 +
                       (ezero ? 4.0 : 0.0);
    return g->ctx->timed(KC_DEFECT, true, per * nint(L), [&]() { return launch_defect(a, g->ctx->stream); });
}

// The previous step's level-0 post-smoothing (two sweeps after the bilinear
// correction, FP32) fused with this step's defect correction: psi_out =
// psi_in + e, the FP64 residual of psi_out, its norms, and its FP32 copy as
// the next right-hand side, in one pass.  e itself is never stored.
constexpr int kPostDefFlags = SW_DEF | SW_PROLONG | SW_TWO | SW_F;
// Algorithmic bytes per interior node: e, a quarter node of coarse correction
// and f (FP32), psi in and out, the next right-hand side (FP32), f (FP64).
double postdef_bytes_per_node(bool with_f) { return 4.0 + 1.0 + 4.0 + 8.0 + 8.0 + 4.0 + (with_f ? 8.0 : 0.0); }

hipError_t enq_postdef(lap_grid* g, const Op& op, double omega) {
    if ((op.parity != 0 && op.parity != 1) || g->geo.size() < 2) return hipErrorInvalidValue;
    const LevelGeo& L = g->geo[0];
    const LevelGeo& C = g->geo[1];
    const Coef c = coef(L.dx, L.dy);
    SweepArgs<float> a{};
    a.uin = g->l32[0].u[op.parity];
    a.uout = nullptr;
    a.f = (const float*)op.f;
    a.ec = (const float*)op.ec;
    a.partials = g->partials;
    a.ctrl = kctrl(g);
    a.m = L.m;
    a.n = L.n;
    a.P = L.P;
    a.mc = C.m;
    a.nc = C.n;
    a.Pc = C.P;
    a.cx = (float)c.cx;
    a.cy = (float)c.cy;
    a.d = (float)c.d;
    a.inv_d = (float)c.inv_d;
    a.omega = (float)omega;
    a.tl = postdef_tiling(L.m, L.n, false);
    a.rowpart = postdef_rowpart(L.n) ? 1 : 0;
    a.psi_in = (const double*)op.in;
    a.psi_out = (double*)op.out;
    a.f64 = g->f64;
    a.rhs_out = (float*)op.bc;
    a.dcx = c.cx;
    a.dcy = c.cy;
    a.dd = c.d;
    a.nt = fused_nt(1, kPostDefFlags) ? 1 : 0;
    return g->ctx->timed(KC_DEFECT, true, postdef_bytes_per_node(g->f64 != nullptr) * nint(L), [&]() {
        return launch_fused<float>(a, kPostDefFlags, g->ctx->stream);
    });
}

// Whether a mixed solve of g with o runs its steps through the post-smoothing
// + defect pass: fusion on, level 0 of the FP32 cycle smoothed by the
// streaming kernels with one two-sweep post-smoothing pass (nu2 = 2) from a
// smoothed start (nu1 >= 2).
bool postdef_ok(lap_grid* g, const lap_opts& o) {
    if (o.method != LAP_MG || o.precision != LAP_MIXED || !g->ctx->fuse || !g->rhs2) return false;
    if (o.smoother != LAP_SMOOTH_RB) return false;
    if (o.nu2 != 2 || o.nu1 < 2 || g->geo.size() < 2) return false;
    return subtree_root<float>(g, 0) != 0;
}

// One outer step of the mixed loop: defect correction (adds the previous
// FP32 correction, forms the FP64 residual, tests it), then one FP32
// V-cycle on the error equation.  With g->pdef, step s >= 1 starts with the
// fused pass that finishes step s - 1's cycle (its level-0 post-smoothing)
// and does the defect correction; the FP32 right-hand sides of consecutive
// steps alternate between l32[0].b and rhs2.  Step 0 corrects nothing yet
// and works in place on psi[0] (no copy of the iterate); step s >= 1 reads
// psi[(s + 1) % 2] and writes psi[s % 2].
// The FP32 cycles of a mixed step on the error equation of H (level 0's
// right-hand side set): o.inner V-cycles, the first from zero, each next from
// the previous correction (level 0 then carries an iterate, in whichever of
// its two buffers the previous cycle left it).  With dp the last cycle stops
// before its level-0 post-smoothing, described in *dp.  The operations of
// the cycles after the first are gated by `later` (a step that runs one
// cycle skips them); `one` is the complementary gate (set when all cycles
// run).  With fusion, a cycle's level-0 post-smoothing pass and the next
// cycle's level-0 pre-smoothing pass (one two-sweep pass each) run as one
// four-sweep pass that reads the post pass's input and writes the other
// buffer; the next cycle is planned on the buffers swapped so that its
// pre pass reads and writes exactly those.  The post pass it replaces stays,
// gated by `one`, when it belongs to the first cycle.  Returns the level-0
// buffer (0/1 of g->l32[0].u) holding the correction; dp->in is given the
// same way, and *first the buffer holding the first cycle's correction.
int plan_inner_cycles(lap_grid* g, const lap_opts& o, HierView<float> H, std::vector<Op>& ops,
                      DeferredPost* dp = nullptr, Ctrl* later = nullptr, Ctrl* one = nullptr,
                      int* first = nullptr) {
    float* B[2] = {g->l32[0].u[0], g->l32[0].u[1]};
    const int fb = H.b[0] ? SW_F : 0;
    int base = 0;   // buffer of g->l32[0].u that H.u0[0] is
    int res = 0;
    long post_at = -1;   // index in ops of the previous cycle's level-0 post pass (a fusable one)
    for (int c = 0; c < o.inner; ++c) {
        const bool last = c == o.inner - 1;
        std::vector<Op> cyc;
        int r = 0;
        bool four = false;
        if (c > 0) {
            H.zero_start0 = false;
            if (post_at >= 0) {
                // on the swapped buffers the cycle's first pass must be the level-0
                // two-sweep pre pass on exactly the post pass's input and output
                HierView<float> Hs = H;
                Hs.u0[0] = B[1 - res];
                Hs.u1[0] = B[res];
                r = plan_vcycle<float>(g, Hs, 0, o, false, PART_ALL, cyc, last ? dp : nullptr);
                const Op& post = ops[(size_t)post_at];
                four = !cyc.empty() && cyc[0].kind == OP_SWEEP && cyc[0].level == 0 &&
                       cyc[0].flags == (SW_TWO | SW_RESTRICT | fb) && cyc[0].in == post.in && cyc[0].out == post.out;
                if (!four) cyc.clear();
            }
            base = four ? 1 - res : res;
            H.u0[0] = B[base];
            H.u1[0] = B[1 - base];
        }
        if (!four) r = plan_vcycle<float>(g, H, 0, o, false, PART_ALL, cyc, last ? dp : nullptr);
        if (c > 0)
            for (Op& op : cyc) {
                op.key += c * KEY_CYCLE;
                op.gate = later;
                // the residual of level 0's correction in difference form: in the standard
                // form it adds terms of size 8|e|/h^2 whose FP32 rounding swamps its smooth
                // part (the part the coarse levels must see)
                if (op.level == 0 && ((op.kind == OP_SWEEP && (op.flags & SW_RESTRICT)) || op.kind == OP_RESTRICT))
                    op.flags |= SW_RDIFF;
            }
        if (four) {
            Op& pre = cyc[0];
            pre.flags |= SW_FOUR | SW_PROLONG;
            pre.flags &= ~SW_TWO;
            pre.ec = ops[(size_t)post_at].ec;
            if (c == 1)
                ops[(size_t)post_at].gate = one;   // the first cycle's post pass, when only it runs
            else
                ops.erase(ops.begin() + post_at);  // gated by `later` as the four-sweep pass is
        }
        ops.insert(ops.end(), cyc.begin(), cyc.end());
        post_at = -1;
        if (!last && g->ctx->fuse && !ops.empty()) {
            const Op& q = ops.back();
            if (q.kind == OP_SWEEP && q.level == 0 && q.dt == 1 && q.flags == (SW_PROLONG | SW_TWO | fb) && o.nu1 == 2)
                post_at = (long)ops.size() - 1;
        }
        res = r == 0 ? base : 1 - base;
        if (c == 0 && first != nullptr) *first = res;
        if (last && dp != nullptr && dp->in >= 0) dp->in = dp->in == 0 ? base : 1 - base;
    }
    return res;
}

// Gates of a mixed step s with several FP32 cycles: its opening after a step
// of all cycles / after a one-cycle step (chosen by step s - 1's test), the
// gate of its own later cycles (chosen by its test), and the cycle word of
// its test's finalisation.
struct StepGates {
    Ctrl* after_all = nullptr;
    Ctrl* after_one = nullptr;
    Ctrl* later = nullptr;
    Ctrl* one = nullptr;
    int cycles = -1;
};
StepGates step_gates(lap_grid* g, const lap_opts& o, int s) {
    StepGates G;
    if (o.inner <= 1) return G;
    const int p = s % 2, q = (s + 1) % 2;
    G.after_all = g->cyc + 2 * p;
    G.after_one = g->cyc + 2 * p + 1;
    G.later = g->cyc + 2 * q;
    G.one = g->cyc + 2 * q + 1;
    G.cycles = o.inner | (q << 8);
    return G;
}

void plan_mixed_step(lap_grid* g, const lap_opts& o, int s, int e_idx, int part, std::vector<Op>& ops) {
    const bool first = s == 0;
    const int in_idx = first ? 0 : (s + 1) % 2;
    double* pin = g->psi[in_idx];
    double* pout = first ? g->psi[0] : g->psi[1 - in_idx];
    const StepGates G = step_gates(g, o, s);
    if (g->pdef) {
        float* R[2] = {g->l32[0].b, g->rhs2};
        const int par = s % 2;
        HierView<float> H = view32(g);
        DeferredPost dp;
        if (part != PART_TAIL) {
            if (first) {
                push_op<double>(ops, KEY_HEAD, OP_DEFECT, 0, 0, pin, pout, g->f64, nullptr, R[0], 0.0);
                push_op<double>(ops, KEY_HEAD + 1, OP_FINALIZE, 0, NORM_DEFECT, nullptr, nullptr, nullptr, nullptr,
                                nullptr, 0.0);
                ops.back().cycles = G.cycles;
            } else {
                // the previous step's cycles, planned again only to find its deferred pass
                std::vector<Op> prev;
                H.b[0] = R[1 - par];
                int e1 = 0;
                plan_inner_cycles(g, o, H, prev, &dp, nullptr, nullptr, &e1);
                push_op<float>(ops, KEY_HEAD, OP_POSTDEF, 0, kPostDefFlags, pin, pout, R[1 - par], dp.ec, R[par],
                               o.omega, dp.in);
                ops.back().gate = G.after_all;
                push_op<double>(ops, KEY_HEAD + 1, OP_FINALIZE, 0, NORM_POSTDEF, nullptr, nullptr, nullptr, nullptr,
                                nullptr, 0.0);
                ops.back().gate = G.after_all;
                ops.back().cycles = G.cycles;
                if (o.inner > 1) {
                    // after a one-cycle step: its correction is complete (its level-0
                    // post-smoothing ran), a plain defect correction adds it
                    push_op<double>(ops, KEY_HEAD + 2, OP_DEFECT, 0, 0, pin, pout, g->f64, g->l32[0].u[e1], R[par],
                                    0.0);
                    ops.back().gate = G.after_one;
                    push_op<double>(ops, KEY_HEAD + 3, OP_FINALIZE, 0, NORM_DEFECT, nullptr, nullptr, nullptr,
                                    nullptr, nullptr, 0.0);
                    ops.back().gate = G.after_one;
                    ops.back().cycles = G.cycles;
                }
            }
        }
        if (part == PART_HEAD) return;
        H.b[0] = R[par];
        plan_inner_cycles(g, o, H, ops, &dp, G.later, G.one);
        return;
    }
    if (o.smoother == LAP_SMOOTH_ZEBRA) {
        // step s's FP32 cycle works in place on level-0 buffer s % 2, which
        // the step's defect correction sets to zero while it adds the previous
        // correction (buffer (s - 1) % 2)
        float* z = g->l32[0].u[s % 2];
        if (part != PART_TAIL) {
            const float* e = first ? nullptr : g->l32[0].u[(s + 1) % 2];
            push_op<double>(ops, KEY_HEAD, OP_DEFECT, 0, 0, pin, pout, g->f64, e, g->l32[0].b, 0.0);
            ops.back().zbuf = z;
            push_op<double>(ops, KEY_HEAD + 1, OP_FINALIZE, 0, NORM_DEFECT, nullptr, nullptr, nullptr, nullptr,
                            nullptr, 0.0);
        }
        if (part == PART_HEAD) return;
        HierView<float> H = view32(g);
        H.u0[0] = z;
        plan_vcycle<float>(g, H, 0, o, false, PART_ALL, ops);
        return;
    }
    if (part != PART_TAIL) {
        const float* e = first ? nullptr : (e_idx == 0 ? g->l32[0].u[0] : g->l32[0].u[1]);
        push_op<double>(ops, KEY_HEAD, OP_DEFECT, 0, 0, pin, pout, g->f64, e, g->l32[0].b, 0.0);
        const bool alt = !first && o.inner > 1;
        if (alt) {
            // after a step of all cycles its last correction, after a one-cycle step its first
            ops.back().gate = G.after_all;
            push_op<double>(ops, KEY_HEAD + 1, OP_DEFECT, 0, 0, pin, pout, g->f64, g->l32[0].u[g->e1_idx],
                            g->l32[0].b, 0.0);
            ops.back().gate = G.after_one;
        }
        push_op<double>(ops, KEY_HEAD + (alt ? 2 : 1), OP_FINALIZE, 0, NORM_DEFECT, nullptr, nullptr, nullptr, nullptr,
                        nullptr, 0.0);
        ops.back().cycles = G.cycles;
    }
    if (part == PART_HEAD) return;
    HierView<float> H = view32(g);
    plan_inner_cycles(g, o, H, ops, nullptr, G.later, G.one);
}

// Full multigrid start (FP64): the source full-weighted down the hierarchy
// into the levels' right-hand sides, every level's boundary nodes set from
// the finest level's Dirichlet data, the coarsest problem solved exactly;
// then, level by level upwards, the interior starts from the bilinear
// interpolation of the coarser solution (boundary included), the coarser
// level's boundary goes back to zero (it serves the next cycle as an error
// level) and one V-cycle rooted at this level runs.  Ends with the FMG field
// in psi[0].
void plan_fmg(lap_grid* g, const lap_opts& o, std::vector<Op>& ops) {
    const int L = (int)g->geo.size();
    HierView<double> H = view64(g);
    long key = 50000;   // single-grid schedule: keys only need to increase
    auto boundary = [&](int l, bool set) {
        Op op{};
        op.key = key++;
        op.kind = OP_BOUNDARY;
        op.dt = 0;
        op.level = l;
        op.flags = set ? 1 : 0;
        op.out = H.u0[l];
        op.bc = H.u1[l];
        ops.push_back(op);
    };
    for (int l = 1; l < L; ++l)
        push_op<double>(ops, key++, OP_RESTRICT, l - 1, 0, nullptr, nullptr, H.b[l - 1], nullptr, H.b[l], 0.0);
    for (int l = 1; l < L; ++l) boundary(l, true);
    push_op<double>(ops, key++, OP_COARSE, L - 1, 0, H.u0[L - 1], H.u0[L - 1], H.b[L - 1], nullptr, nullptr, 0.0);
    for (int l = L - 2; l >= 0; --l) {
        push_op<double>(ops, key++, OP_SWEEP, l, SW_ZERO | SW_PROLONG | SW_PONLY, nullptr, H.u0[l], nullptr,
                        H.u0[l + 1], nullptr, 0.0);
        boundary(l + 1, false);
        HierView<double> R = H;
        R.root = l;
        R.sub_root = subtree_root<double>(g, l + 1);
        plan_vcycle<double>(g, R, l, o, false, PART_ALL, ops);
    }
}

// ------------------------------------------------------------------ ADI
// Algorithmic bytes of one zebra half (all lines of one parity) per interior
// node of the grid: half the nodes are updated, each reading its own old
// value and f and writing the new one, and the other half are read once as
// the neighbours across the lines (FP64).
double adi_bytes_per_node(bool with_f) { return 0.5 * (8.0 + 8.0 + 8.0 + (with_f ? 8.0 : 0.0)); }

// Which line solver (and workgroup size) a half of lines of length K takes;
// merged launches group operations by these flags.
int adi_kernel_flags(int dir, int K) {
    if (!seg_fits(dir, K)) return 0;
    return ADI_SEG | (seg_code(dir, K) << ADI_CODE_SHIFT);
}

void adi_factor(double b, double a, double c, int K, double* cp, double* piv) {
    if (K <= 0) return;
    cp[0] = c / b;
    piv[0] = b;
    for (int k = 1; k < K; ++k) {
        piv[k] = b - a * cp[k - 1];
        cp[k] = c / piv[k];
    }
}

LineArgs adi_args(lap_grid* g, double omega, int form, int dir, int parity) {
    const LevelGeo& L = g->geo[0];
    const Coef c = coef(L.dx, L.dy);
    const int mk = g->adi_maxk;
    LineArgs a{};
    a.u = g->psi[0];
    a.f = g->f64;
    a.scratch = g->adi_scratch;
    a.ctrl = kctrl(g);
    a.m = L.m;
    a.n = L.n;
    a.P = L.P;
    a.cx = c.cx;
    a.cy = c.cy;
    a.d = c.d;
    a.omega = omega;
    a.form = form & 1;
    a.parity = parity;
    a.seg = g->adi_tab + 4 * mk + dir * kSegTab;
    if (dir == 0) {
        a.cprime = g->adi_tab;
        a.piv = g->adi_tab + mk;
        a.a_off = (form & 1) == 0 ? -c.cx : -omega * c.cx;
    } else {
        a.cprime = g->adi_tab + 2 * mk;
        a.piv = g->adi_tab + 3 * mk;
        a.a_off = (form & 1) == 0 ? -c.cy : -omega * c.cy;
    }
    return a;
}

hipError_t enq_adi_half(lap_grid* g, double omega, int form, int dir, int parity) {
    const LineArgs a = adi_args(g, omega, form, dir, parity);
    const double per = adi_bytes_per_node(g->f64 != nullptr) * nint(g->geo[0]);
    if (dir == 0)
        return g->ctx->timed(KC_ADI_ROWS, true, per, [&]() { return launch_adi_rows(a, g->ctx->stream); });
    return g->ctx->timed(KC_ADI_COLS, true, per, [&]() { return launch_adi_cols(a, g->ctx->stream); });
}

// Arguments of a zebra line-smoothing half on level l (relaxation after the
// line solve with omega; the level's own segment table).
template <typename T>
LineArgsT<T> zebra_args(lap_grid* g, int l, T* u, const T* b, double omega, int dir, int parity) {
    const LevelGeo& L = g->geo[l];
    const Coef c = coef(L.dx, L.dy);
    LineArgsT<T> a{};
    a.u = u;
    a.f = b;
    a.ctrl = kctrl(g);
    a.m = L.m;
    a.n = L.n;
    a.P = L.P;
    a.cx = c.cx;
    a.cy = c.cy;
    a.d = c.d;
    a.omega = omega;
    a.form = LAP_ADI_RELAX_AFTER;
    a.parity = parity;
    const size_t off = ((size_t)2 * l + dir) * kSegTab;
    if constexpr (sizeof(T) == 8)
        a.seg = g->ztab64 + off;
    else
        a.seg = g->ztab32 + off;
    return a;
}

template <typename T>
hipError_t enq_zebra(lap_grid* g, const Op& op, int dir) {
    const LineArgsT<T> a = zebra_args<T>(g, op.level, (T*)op.out, (const T*)op.f, op.omega, dir, op.parity);
    const double per = adi_bytes_per_node(op.f != nullptr) * sizeof(T) / 8.0 * nint(g->geo[op.level]);
    return g->ctx->timed(dir == 0 ? KC_ADI_ROWS : KC_ADI_COLS, op.level == 0, per,
                         [&]() { return launch_zebra_lines<T>(a, dir, g->ctx->stream); });
}

// Launch one recorded operation of grid g.
hipError_t exec_op_body(lap_grid* g, const Op& op) {
    const int l = op.level;
    switch (op.kind) {
        case OP_SWEEP:
            if (is_fused(op.flags)) {
                if (op.dt == 0)
                    return enq_fused<double>(g, l, (const double*)op.in, (double*)op.out, (const double*)op.f,
                                             (const double*)op.ec, (double*)op.bc, op.omega, op.flags);
                return enq_fused<float>(g, l, (const float*)op.in, (float*)op.out, (const float*)op.f,
                                        (const float*)op.ec, (float*)op.bc, op.omega, op.flags);
            }
            if (op.dt == 0)
                return enq_sweep<double>(g, l, (const double*)op.in, (double*)op.out, (const double*)op.f,
                                         (const double*)op.ec, op.omega, op.flags);
            return enq_sweep<float>(g, l, (const float*)op.in, (float*)op.out, (const float*)op.f,
                                    (const float*)op.ec, op.omega, op.flags);
        case OP_RESTRICT:
            if (op.dt == 0)
                return enq_restrict<double>(g, l, (const double*)op.in, (const double*)op.f, (double*)op.bc,
                                            (double*)op.out);
            return enq_restrict<float>(g, l, (const float*)op.in, (const float*)op.f, (float*)op.bc, (float*)op.out,
                                       (op.flags & SW_RDIFF) != 0);
        case OP_COARSE:
            if (op.dt == 0)
                return enq_coarse<double>(g, l, (const double*)op.in, (const double*)op.f, (double*)op.out);
            return enq_coarse<float>(g, l, (const float*)op.in, (const float*)op.f, (float*)op.out);
        case OP_FINALIZE:
            return enq_finalize(g, norm_partials(g->geo[0].m, g->geo[0].n, op.flags),
                                op.parity == kProbeFinalize ? 2 : 0, op.gate, op.cycles);
        case OP_RESNORM:
            return enq_residual_norm<double>(g, l, (const double*)op.in, (const double*)op.f);
        case OP_DEFECT:
            return enq_defect(g, (const double*)op.in, (double*)op.out, (const float*)op.ec, (float*)op.bc,
                              (float*)op.zbuf);
        case OP_POSTDEF:
            return enq_postdef(g, op, op.omega);
        case OP_ADI_ROWS:
        case OP_ADI_COLS: {
            const int dir = op.kind == OP_ADI_ROWS ? 0 : 1;
            if (op.flags & ADI_MG) return op.dt == 0 ? enq_zebra<double>(g, op, dir) : enq_zebra<float>(g, op, dir);
            return enq_adi_half(g, op.omega, op.flags, dir, op.parity);
        }
        case OP_SUBTREE:
            if (op.dt == 0)
                return enq_subtree<double>(g, l, (double*)op.out, (const double*)op.f, op.omega, op.flags);
            return enq_subtree<float>(g, l, (float*)op.out, (const float*)op.f, op.omega, op.flags);
        case OP_BOUNDARY: {
            const LevelGeo& G = g->geo[l];
            return launch_level_boundary((double*)op.out, (double*)op.bc, op.flags ? g->psi[0] : nullptr, G.m, G.n,
                                         G.P, g->P, 1 << l, kctrl(g), g->ctx->stream);
        }
    }
    return hipErrorInvalidValue;
}

hipError_t exec_op(lap_grid* g, const Op& op) {
    g->op_ctrl = op.kind == OP_FINALIZE ? nullptr : op.gate;
    const hipError_t e = exec_op_body(g, op);
    g->op_ctrl = nullptr;
    return e;
}

// Launch a step's operations in order; for the timing records, the
// operations up to and including the step's first norm finalisation form
// its stopping test (its head).
hipError_t exec_ops(lap_grid* g, const std::vector<Op>& ops) {
    lap_ctx* c = g->ctx;
    size_t fin = ops.size();
    for (size_t k = 0; k < ops.size(); ++k)
        if (ops[k].kind == OP_FINALIZE) {
            fin = k;
            break;
        }
    for (size_t k = 0; k < ops.size(); ++k) {
        c->rec_head = k <= fin && fin < ops.size();
        HIPERR(exec_op(g, ops[k]));
    }
    c->rec_head = false;
    return hipSuccess;
}

// ---------------------------------------------------------------- driver
lap_status init_ctrl(lap_grid* g, const lap_opts& o, int step) {
    HIPCHK(launch_ctrl_init(g->ctrl, o.tol, o.stop, o.max_iter, step, g->ctx->stream));
    return LAP_OK;
}

// Enqueue steps until the device says done; poll one step behind.  Once
// the last two tests predict (by their ratio) that the step in flight will
// stop the solve with a margin of 2, the next step is enqueued only after
// that step's test has been read: a converged solve then does not drain a
// whole speculative step of launches that exit at once (about 0.1 ms for a
// multigrid cycle of an 8193^2 grid); a wrong prediction costs one host
// round trip.
//
// A solve that can probe (FP64 multigrid) does more once the tests predict,
// two steps ahead of the last one read, that the test step s opens with
// will end the solve: it first enqueues that test alone (the norms-only
// version of the step's first pass and a finalisation that records the test
// only if it ends the solve) and reads it.  If it ends the solve, the step's
// sweeps, its restriction and the rest of its cycle are never enqueued;
// otherwise the full step follows and repeats the same test (same norms,
// same control block), so results and counts do not depend on probing.
lap_status drive(lap_grid* g, int max_steps, const std::function<hipError_t(int)>& step, Ctrl& out,
                 const std::function<hipError_t(int, bool*)>* probe = nullptr) {
    lap_ctx* c = g->ctx;
    int polled = -1;                 // last step whose control block was read
    double q_prev = -1.0, q_last = -1.0, tol = 0.0;
    bool stop = false;
    auto poll = [&](int k) -> hipError_t {
        const hipError_t e = hipEventSynchronize(c->poll_ev[k & 1]);
        if (e != hipSuccess) return e;
        const Ctrl& h = c->pinned[k & 1];
        polled = k;
        stop = h.done != 0;
        tol = h.tol;
        q_prev = q_last;
        q_last = h.stop == 0 ? h.rel : h.res_inf;
        if (!stop) c->safe_step = k + 1;   // step k did not stop: steps up to k did full work
        return hipSuccess;
    };
    c->safe_step = 0;
    for (int s = 0; s < max_steps && !stop; ++s) {
        if (s >= 2 && polled == s - 2 && q_prev > 0.0 && q_last > 0.0 && q_last < q_prev &&
            q_last * (q_last / q_prev) < 0.5 * tol) {
            HIPCHK(poll(s - 1));
            if (stop) break;
        }
        if (probe != nullptr && s >= 2 && polled >= s - 2 && q_prev > 0.0 && q_last > 0.0 && q_last < q_prev) {
            double qs = q_last;
            for (int k = polled; k < s; ++k) qs *= q_last / q_prev;
            bool did = false;
            if (qs < 0.5 * tol) {
                c->rec_step = s;
                hipError_t e = (*probe)(s, &did);
                if (e != hipSuccess) return fail(LAP_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
            }
            if (did) {
                HIPCHK(hipMemcpyAsync(&c->pinned[s & 1], g->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, c->stream));
                HIPCHK(hipEventRecord(c->poll_ev[s & 1], c->stream));
                if (polled < s - 1) HIPCHK(poll(s - 1));
                if (stop) break;
                HIPCHK(hipEventSynchronize(c->poll_ev[s & 1]));
                if (c->pinned[s & 1].done) break;   // the probe ended the solve
            }
        }
        c->rec_step = s;
        hipError_t e = step(s);
        if (e != hipSuccess) return fail(LAP_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
        HIPCHK(hipMemcpyAsync(&c->pinned[s & 1], g->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipEventRecord(c->poll_ev[s & 1], c->stream));
        if (s >= 1 && polled < s - 1) HIPCHK(poll(s - 1));
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(&c->pinned[2], g->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
    out = c->pinned[2];
    return LAP_OK;
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

lap_status finish(lap_grid* g, const lap_opts& o, const Ctrl& h, double t0, lap_info* info) {
    lap_status st = (lap_status)h.status;
    if (!h.done) st = LAP_ENOTCONV;
    if (o.tol <= 0.0 && st == LAP_ENOTCONV) st = LAP_OK;
    g->last_r0 = h.r0;
    if (info) {
        info->iterations = h.iters;
        info->status = st;
        info->rel_res_l2 = h.rel;
        info->res_l2 = h.res_l2;
        info->res_linf = h.res_inf;
        info->res0_l2 = h.r0;
        info->seconds = now_s() - t0;
        info->monitor = 0.0;
    }
    if (st == LAP_ENOTCONV) g_err = "max_iter reached before the stopping rule held";
    if (st == LAP_EDIVERGED) g_err = "residual diverged (NaN/Inf or growth by 1e6)";
    return st;
}

bool is_paper_method(int method) {
    return method == LAP_JACOBI || method == LAP_SOR_LEX || method == LAP_SLOR_LEX || method == LAP_ADI_LEX;
}

lap_status validate_opts(lap_grid* g, const lap_opts& o) {
    if (!(o.omega > 0.0 && o.omega < 2.0)) return fail(LAP_EINVAL, "omega must lie in (0, 2)");
    if (o.max_iter < 0) return fail(LAP_EINVAL, "max_iter must be >= 0");
    if (!(o.tol >= 0.0)) return fail(LAP_EINVAL, "tol must be >= 0");
    if (o.inner < 1 || o.inner > 8) return fail(LAP_EINVAL, "inner must lie in 1..8");
    if (o.inner > 1 && (o.precision != LAP_MIXED || o.smoother != LAP_SMOOTH_RB))
        return fail(LAP_EINVAL, "inner > 1 needs LAP_MIXED and the red-black smoother");
    if (is_paper_method(o.method)) {
        if (o.stop != LAP_STOP_REL_L2 && o.stop != LAP_STOP_RES_INF && o.stop != LAP_STOP_DELTA)
            return fail(LAP_EINVAL, "unknown stopping rule");
        if (o.precision != LAP_FP64) return fail(LAP_EINVAL, "the paper-order methods run in FP64");
        if (paper_lds_bytes(g->m, g->n) > (size_t)g->ctx->lds_max)
            return fail(LAP_EINVAL, "the paper-order methods need the grid in one workgroup's LDS "
                                    "(2 m n + 3 max(m, n) doubles)");
        if ((o.method == LAP_SLOR_LEX || o.method == LAP_ADI_LEX) && o.adi_form != 0 && o.adi_form != 1)
            return fail(LAP_EINVAL, "unknown line relaxation form");
        if ((o.method == LAP_SLOR_LEX || o.method == LAP_ADI_LEX) && o.adi_form == 1) {
            const Coef c = coef(g->dx, g->dy);
            const double lim = o.method == LAP_SLOR_LEX ? 1.0 + c.cy / c.cx : 1.0 + std::min(c.cy / c.cx, c.cx / c.cy);
            if (o.omega >= lim)
                return fail(LAP_EINVAL, "relaxation inside the line system needs omega < 1 + beta^2");
        }
        if (o.max_iter < 0 || !(o.tol >= 0.0) || !(o.omega > 0.0 && o.omega < 2.0))
            return fail(LAP_EINVAL, "bad omega, tol or max_iter");
        return LAP_OK;
    }
    if (o.stop != LAP_STOP_REL_L2 && o.stop != LAP_STOP_RES_INF) return fail(LAP_EINVAL, "unknown stopping rule");
    if (o.method != LAP_SOR_RB && o.method != LAP_ADI && o.method != LAP_MG)
        return fail(LAP_EINVAL, "unknown method");
    if (o.precision != LAP_FP64 && o.precision != LAP_MIXED) return fail(LAP_EINVAL, "unknown precision");
    if (o.precision == LAP_MIXED && o.method != LAP_MG) return fail(LAP_EINVAL, "LAP_MIXED needs LAP_MG");
    if (o.smoother != LAP_SMOOTH_RB && o.smoother != LAP_SMOOTH_ZEBRA) return fail(LAP_EINVAL, "unknown smoother");
    if (o.fmg != 0 && o.fmg != 1) return fail(LAP_EINVAL, "fmg must be 0 or 1");
    if (o.fmg && (o.method != LAP_MG || o.precision != LAP_FP64 || o.smoother != LAP_SMOOTH_RB))
        return fail(LAP_EINVAL, "the full multigrid start needs LAP_MG, LAP_FP64 and the red-black smoother");
    if (o.method == LAP_MG && o.smoother == LAP_SMOOTH_ZEBRA) {
        if (!g->zebra_ok)
            return fail(LAP_EINVAL, "zebra smoothing needs every level's lines in the segmented line solver "
                                    "(sides of at most 4097)");
        if (o.nu1 < 0 || o.nu2 < 0 || o.nu1 + o.nu2 < 1 || o.nu1 > 8 || o.nu2 > 8)
            return fail(LAP_EINVAL, "zebra smoothing needs 0 <= nu1, nu2 <= 8 and nu1 + nu2 >= 1");
        if (o.precision == LAP_FP64 && !(g->flags & LAP_ALLOC_FP64)) return fail(LAP_EINVAL, "grid has no FP64 hierarchy");
        if (o.precision == LAP_MIXED && !(g->flags & LAP_ALLOC_MIXED)) return fail(LAP_EINVAL, "grid has no mixed hierarchy");
    } else if (o.method == LAP_MG) {
        if (o.nu1 < 0 || o.nu2 < 1) return fail(LAP_EINVAL, "multigrid needs nu1 >= 0 and nu2 >= 1");
        if ((o.nu1 + o.nu2) % 2) return fail(LAP_EINVAL, "multigrid needs nu1 + nu2 even");
        if (o.precision == LAP_FP64 && !(g->flags & LAP_ALLOC_FP64)) return fail(LAP_EINVAL, "grid has no FP64 hierarchy");
        if (o.precision == LAP_MIXED && !(g->flags & LAP_ALLOC_MIXED)) return fail(LAP_EINVAL, "grid has no mixed hierarchy");
    }
    if (o.method == LAP_ADI) {
        if (!(g->flags & LAP_ALLOC_ADI)) return fail(LAP_EINVAL, "grid has no ADI scratch");
        if (o.adi_form != 0 && o.adi_form != 1) return fail(LAP_EINVAL, "unknown ADI form");
        if (o.adi_form == 1) {
            const Coef c = coef(g->dx, g->dy);
            if (o.omega >= 1.0 + std::min(c.cy / c.cx, c.cx / c.cy))
                return fail(LAP_EINVAL, "relaxation inside the line system needs omega < 1 + beta^2 in both directions");
        }
    }
    if (o.check_every < 1) return fail(LAP_EINVAL, "check_every must be >= 1");
    return LAP_OK;
}

// ------------------------------------------------------------------ methods
// Every method is (prepare, step, fixup): prepare resets the control block
// and builds per-solve tables / graphs; step s enqueues one outer iteration
// whose first kernels test the current iterate; fixup moves the tested
// iterate (the solution) into psi[0] once the device reports done.

int max_steps(const lap_opts& o) {
    switch (o.method) {
        case LAP_MG: return o.max_iter + 1;
        default: return (o.max_iter + o.check_every - 1) / o.check_every + 1;
    }
}

hipError_t capture(lap_grid* g, const char* key, const std::function<hipError_t()>& body) {
    lap_ctx* c = g->ctx;
    if (g->graph != nullptr && g->graph_key == key) return hipSuccess;
    if (g->graph) {
        HIPERR(hipGraphExecDestroy(g->graph));
        g->graph = nullptr;
    }
    HIPERR(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = body();
    hipGraph_t tmp = nullptr;
    hipError_t e2 = hipStreamEndCapture(c->stream, &tmp);
    if (e != hipSuccess) return e;
    if (e2 != hipSuccess) return e2;
    e = hipGraphInstantiate(&g->graph, tmp, nullptr, nullptr, 0);
    hipGraphDestroy(tmp);
    if (e == hipSuccess) g->graph_key = key;
    return e;
}

bool use_graph(lap_grid* g, const lap_opts& o) {
    return o.use_graph && g->ctx->stream != nullptr && !g->ctx->timing && o.method == LAP_MG;
}

int ctrl_step(const lap_opts& o) { return (o.method == LAP_MG) ? 1 : o.check_every; }

// Per-solve set-up of one grid; init = false leaves the control block to the
// caller (a batch resets all of them in one launch).
lap_status prepare(lap_grid* g, const lap_opts& o, bool init = true) {
    if (init) {
        lap_status st = init_ctrl(g, o, ctrl_step(o));
        if (st != LAP_OK) return st;
    }
    g->step_idx = 0;
    g->pdef = postdef_ok(g, o);   // fixed for the whole solve
    g->e_idx = vcycle_result_index(g->ctx, o);
    if (o.method == LAP_MG && o.precision == LAP_MIXED && o.inner > 1 && !g->l32.empty()) {
        std::vector<Op> dry;   // where the step's first and last FP32 cycles leave the correction
        g->e_idx = plan_inner_cycles(g, o, view32(g), dry, nullptr, nullptr, nullptr, &g->e1_idx);
    }
    // the two-buffer methods need both buffers equal when they start
    if (g->psi1_stale && o.method != LAP_ADI) {
        HIPCHK(hipMemcpyAsync(g->psi[1], g->psi[0], (size_t)g->n * g->P * 8, hipMemcpyDeviceToDevice,
                              g->ctx->stream));
        g->psi1_stale = false;
    }
    if (o.method == LAP_ADI && (g->adi_omega != o.omega || g->adi_form != o.adi_form)) {
        g->adi_omega = o.omega;
        g->adi_form = o.adi_form;
        const Coef c = coef(g->dx, g->dy);
        const int mk = g->adi_maxk;
        g->adi_host.assign((size_t)4 * mk, 0.0);
        const double wx = o.adi_form == 0 ? c.cx : o.omega * c.cx;
        const double wy = o.adi_form == 0 ? c.cy : o.omega * c.cy;
        adi_factor(c.d, -wx, -wx, g->m - 2, g->adi_host.data(), g->adi_host.data() + mk);
        adi_factor(c.d, -wy, -wy, g->n - 2, g->adi_host.data() + 2 * mk, g->adi_host.data() + 3 * mk);
        g->adi_host.resize((size_t)4 * mk + 2 * kSegTab);
        adi_seg_table(c.d, wx, g->m - 2, g->adi_host.data() + 4 * mk);
        adi_seg_table(c.d, wy, g->n - 2, g->adi_host.data() + 4 * mk + kSegTab);
        HIPCHK(hipMemcpyAsync(g->adi_tab, g->adi_host.data(), g->adi_host.size() * 8, hipMemcpyHostToDevice,
                              g->ctx->stream));
    }
    // A grid's cycle graph is captured on its second solve with the same
    // options: capturing and instantiating costs more than one solve of a
    // small or medium grid saves by replaying (a request solved once, as in
    // serving, never pays for it).
    g->graph_on = false;
    if (use_graph(g, o)) {
        char key[128];
        if (o.precision == LAP_FP64)
            snprintf(key, sizeof key, "mg64:%d:%d:%d:%.17g", o.smoother, o.nu1, o.nu2, o.omega);
        else
            snprintf(key, sizeof key, "mixed%s:%d:%d:%d:%d:%.17g", g->pdef ? "+pd" : "", o.smoother, o.nu1, o.nu2,
                     o.inner, o.omega);
        const bool have = g->graph != nullptr && g->graph_key == key;
        auto& seen = g->graph_seen;
        const bool again = std::find(seen.begin(), seen.end(), std::string(key)) != seen.end();
        g->graph_on = have || again;
        if (!again) {
            if (seen.size() >= 8) seen.erase(seen.begin());
            seen.push_back(key);
        }
        g->graph_run_key = key;
    }
    if (g->graph_on) {
        const std::string key = g->graph_run_key;
        hipError_t e;
        if (o.precision == LAP_FP64) {
            e = capture(g, key.c_str(), [&]() {
                HierView<double> H = view64(g);
                std::vector<Op> ops;
                plan_vcycle<double>(g, H, 0, o, true, PART_ALL, ops);
                return exec_ops(g, ops);
            });
        } else {
            // two outer steps, an odd one (psi[0] -> psi[1]) and the next (psi[1] -> psi[0]);
            // step 0 runs without the graph
            e = capture(g, key.c_str(), [&]() {
                std::vector<Op> ops;
                plan_mixed_step(g, o, 1, g->e_idx, PART_ALL, ops);
                plan_mixed_step(g, o, 2, g->e_idx, PART_ALL, ops);
                return exec_ops(g, ops);
            });
        }
        if (e != hipSuccess) return fail(LAP_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    }
    return LAP_OK;
}

// Record outer step s of grid g (SOR / ADI: one check block; MG: one cycle;
// mixed: one defect correction + FP32 cycle).  PART_ALL records the whole
// step, PART_HEAD only its stopping test of the incoming iterate, PART_TAIL
// the rest.
void plan_step(lap_grid* g, const lap_opts& o, int s, int part, std::vector<Op>& ops) {
    switch (o.method) {
        case LAP_MG:
            if (o.precision == LAP_FP64 && o.fmg && s == 0) {
                // the stopping test of the incoming field, then the full multigrid pass
                if (part != PART_TAIL) {
                    push_op<double>(ops, KEY_HEAD, OP_RESNORM, 0, 0, g->psi[0], nullptr, g->f64, nullptr, nullptr, 0.0);
                    push_op<double>(ops, KEY_HEAD + 1, OP_FINALIZE, 0, 0, nullptr, nullptr, nullptr, nullptr,
                                    nullptr, 0.0);
                }
                if (part != PART_HEAD) plan_fmg(g, o, ops);
            } else if (o.precision == LAP_FP64) {
                HierView<double> H = view64(g);
                plan_vcycle<double>(g, H, 0, o, true, part, ops);
            } else {
                plan_mixed_step(g, o, s, g->e_idx, part, ops);
            }
            return;
        case LAP_SOR_RB: {
            // one check block: the first pass also forms the residual norms
            // of the incoming iterate (the stopping test)
            const int fb = g->f64 ? SW_F : 0;
            const std::vector<int> pp = sor_passes(g->ctx, o.check_every);
            const int np = (int)pp.size();
            int cur = (s % 2) * (np % 2);   // parity of the passes of steps 0..s-1
            for (int k = 0; k < np; ++k) {
                if ((part == PART_TAIL && k == 0) || (part == PART_HEAD && k > 0)) {
                    cur = 1 - cur;
                    continue;
                }
                const int fl = fb | (k == 0 ? SW_NORM : 0) | (pp[k] == 2 ? SW_TWO : 0);
                push_op<double>(ops, key_pre(0, 0) + 2L * k, OP_SWEEP, 0, fl, g->psi[cur], g->psi[1 - cur], g->f64,
                                nullptr, nullptr, o.omega);
                if (k == 0)
                    push_op<double>(ops, key_pre(0, 0) + 1, OP_FINALIZE, 0, 0, nullptr, nullptr, nullptr, nullptr,
                                    nullptr, 0.0);
                cur = 1 - cur;
            }
            return;
        }
        case LAP_ADI:
            if (part != PART_TAIL) {
                push_op<double>(ops, KEY_HEAD, OP_RESNORM, 0, 0, g->psi[0], nullptr, g->f64, nullptr, nullptr, 0.0);
                push_op<double>(ops, KEY_HEAD + 1, OP_FINALIZE, 0, 0, nullptr, nullptr, nullptr, nullptr, nullptr,
                                0.0);
            }
            if (part != PART_HEAD)
                for (int k = 0; k < o.check_every; ++k)
                    for (int q = 0; q < 4; ++q)
                        push_op<double>(ops, 1000 + 4L * k + q, q < 2 ? OP_ADI_ROWS : OP_ADI_COLS, 0,
                                        o.adi_form | adi_kernel_flags(q < 2 ? 0 : 1, q < 2 ? g->m - 2 : g->n - 2),
                                        nullptr, nullptr, nullptr, nullptr, nullptr, o.omega, (q % 2) ? 0 : 1);
            return;
    }
}

// Enqueue outer step number g->step_idx (single grid).  PART_HEAD does not
// advance step_idx; PART_ALL and PART_TAIL do.
hipError_t step(lap_grid* g, const lap_opts& o, int part = PART_ALL) {
    const int s = g->step_idx;
    if (part != PART_HEAD) g->step_idx++;
    lap_ctx* c = g->ctx;
    const bool graph = g->graph_on && part == PART_ALL && !(o.fmg && s == 0);
    if (graph && o.method == LAP_MG) {
        if (o.precision == LAP_FP64) return hipGraphLaunch(g->graph, c->stream);
        if (s % 2 == 1) {               // the mixed graph covers steps s (odd) and s + 1
            g->step_idx++;
            return hipGraphLaunch(g->graph, c->stream);
        }
    }
    std::vector<Op> ops;
    plan_step(g, o, s, part, ops);
    return exec_ops(g, ops);
}

// The test FP64 multigrid step s opens with, as a probe: the step's first
// (fused) pre-smoothing pass with SW_PROBE, which computes the norms of the
// incoming iterate exactly as that pass does and stores nothing, and a
// finalisation that records the test only if it ends the solve.  Empty when
// the step does not open with such a pass (nothing to save then).
std::vector<Op> probe_ops(lap_grid* g, const lap_opts& o, int s) {
    std::vector<Op> ops;
    if (o.method != LAP_MG || o.precision != LAP_FP64 || o.smoother != LAP_SMOOTH_RB || (o.fmg && s == 0))
        return ops;
    plan_step(g, o, s, PART_HEAD, ops);
    if (ops.size() != 2 || ops[0].kind != OP_SWEEP || !(ops[0].flags & SW_NORM) || !is_fused(ops[0].flags) ||
        ops[1].kind != OP_FINALIZE) {
        ops.clear();
        return ops;
    }
    ops[0].flags |= SW_PROBE;
    ops[0].out = nullptr;
    ops[0].bc = nullptr;
    ops[1].parity = kProbeFinalize;
    return ops;
}

// The buffer holding the tested iterate (the solution) at the end of a solve.
int result_buffer(lap_grid* g, const lap_opts& o, const Ctrl& h) {
    if (o.method == LAP_SOR_RB) return ((h.checks - 1) % 2) * ((int)sor_passes(g->ctx, o.check_every).size() % 2);
    if (o.method == LAP_MG && o.precision == LAP_MIXED) return h.checks > 0 ? (h.checks - 1) % 2 : 0;
    return 0;
}

// The tested iterate is the solution; bring it to psi[0] and make psi[1] equal.
lap_status fixup(lap_grid* g, const lap_opts& o, const Ctrl& h) {
    lap_ctx* c = g->ctx;
    const size_t bytes = (size_t)g->n * g->P * 8;
    if (result_buffer(g, o, h) == 1)
        HIPCHK(hipMemcpyAsync(g->psi[0], g->psi[1], bytes, hipMemcpyDeviceToDevice, c->stream));
    if (o.method == LAP_ADI) g->psi1_stale = true;   // copied when a two-buffer method next starts
    return LAP_OK;
}

// With kernel timing on, the solve runs as without (steps enqueued one
// ahead of the poll, no graph replay) and every launch is tagged with its
// step; once the device has stopped, the records of the launches that came
// after the deciding stopping test (they exited at once) are dropped, so
// the statistics hold only launches that did their full work.
lap_status residual_norms(lap_grid* g, double* l2, double* linf);

// The paper's sequential orderings: the whole solve in one launch of one
// workgroup (the grid in LDS); FP64 residual norms before and after.
lap_status solve_paper(lap_grid* g, const lap_opts& o, lap_info* info) {
    const double t0 = now_s();
    double r0 = 0.0, r0inf = 0.0;
    lap_status st = residual_norms(g, &r0, &r0inf);
    if (st != LAP_OK) return st;
    const LevelGeo& L = g->geo[0];
    const Coef c = coef(L.dx, L.dy);
    PaperArgs a{};
    a.u = g->psi[0];
    a.f = g->f64;
    a.ctrl = g->ctrl;
    a.m = L.m;
    a.n = L.n;
    a.P = L.P;
    a.cx = c.cx;
    a.cy = c.cy;
    a.d = c.d;
    a.inv_d = c.inv_d;
    a.omega = o.omega;
    a.method = o.method;
    a.form = o.adi_form;
    a.stop = o.stop;
    a.tol = o.tol;
    a.max_iter = o.max_iter;
    lap_ctx* cx = g->ctx;
    HIPCHK(cx->timed(KC_PAPER, true, 0.0, [&]() { return launch_paper(a, cx->stream); }));
    Ctrl h{};
    HIPCHK(hipMemcpyAsync(&h, g->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, cx->stream));
    HIPCHK(hipStreamSynchronize(cx->stream));
    g->psi1_stale = true;   // psi[0] changed alone
    double l2 = 0.0, linf = 0.0;
    st = residual_norms(g, &l2, &linf);
    if (st != LAP_OK) return st;
    lap_status res = (lap_status)h.status;
    if (res == LAP_OK && !h.done) res = o.tol > 0.0 ? LAP_ENOTCONV : LAP_OK;
    if (info) {
        info->iterations = h.iters;
        info->status = res;
        info->rel_res_l2 = r0 > 0.0 ? l2 / r0 : 0.0;
        info->res_l2 = l2;
        info->res_linf = linf;
        info->res0_l2 = r0;
        info->monitor = h.rel;
        info->seconds = now_s() - t0;
    }
    if (res == LAP_ENOTCONV) g_err = "max_iter reached before the stopping rule held";
    if (res == LAP_EDIVERGED) g_err = "iterate diverged (NaN/Inf or beyond 1e30)";
    return res;
}

lap_status solve_one(lap_grid* g, const lap_opts& o, lap_info* info) {
    if (is_paper_method(o.method)) return solve_paper(g, o, info);
    const double t0 = now_s();
    lap_status st = prepare(g, o);
    if (st != LAP_OK) return st;
    lap_ctx* c = g->ctx;
    c->rec_solve = c->timing ? c->solve_serial++ : -1;
    Ctrl h{};
    const std::function<hipError_t(int, bool*)> probe = [&](int s, bool* did) -> hipError_t {
        const std::vector<Op> ops = probe_ops(g, o, s);
        *did = !ops.empty();
        return ops.empty() ? hipSuccess : exec_ops(g, ops);
    };
    st = drive(g, max_steps(o) + 1, [&](int) -> hipError_t { return step(g, o); }, h, &probe);
    if (c->timing && st == LAP_OK) c->drop_speculative(c->rec_solve, h.checks - 1);
    c->rec_solve = -1;
    if (st != LAP_OK) return st;
    st = fixup(g, o, h);
    if (st != LAP_OK) return st;
    HIPCHK(hipStreamSynchronize(g->ctx->stream));
    return finish(g, o, h, t0, info);
}

void default_tilings(lap_ctx* c) {
    for (int sc = 0; sc < kSizeClasses; ++sc)
        for (int k = 0; k < KC_COUNT; ++k) {
            c->tileV[sc][k][0] = 2;
            c->tileTY[sc][k][0] = 0;
            c->tileT[sc][k][0] = c->wave_cap;
            c->tileV[sc][k][1] = 4;
            c->tileTY[sc][k][1] = 0;
            c->tileT[sc][k][1] = c->wave_cap;
        }
}

}  // namespace

// =========================================================================== ABI
extern "C" {

const char* lap_last_error(void) { return g_err.c_str(); }
const char* lap_version(void) { return "liblap 0.1 (gfx950)"; }

void lap_opts_default(lap_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->method = LAP_MG;
    o->precision = LAP_FP64;
    o->omega = 1.0;
    o->tol = 1e-10;
    o->max_iter = 100;
    o->stop = LAP_STOP_REL_L2;
    o->nu1 = 2;
    o->nu2 = 2;
    o->check_every = 1;
    o->adi_form = LAP_ADI_RELAX_AFTER;
    o->use_graph = 1;
    o->smoother = LAP_SMOOTH_RB;
    o->inner = 1;
}

lap_status lap_ctx_create(void* dev_arena, size_t arena_bytes, void* hip_stream, lap_ctx** out) {
    if (!out) return fail(LAP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!dev_arena) return fail(LAP_EINVAL, "arena is NULL");
    if (((uintptr_t)dev_arena) % kAlign) return fail(LAP_EINVAL, "arena must be 256-byte aligned");
    if (arena_bytes < (1u << 20)) return fail(LAP_EINVAL, "arena must hold at least 1 MiB");
    lap_ctx* c = new (std::nothrow) lap_ctx();
    if (!c) return fail(LAP_ENOMEM, "host allocation failed");
    c->arena.init(dev_arena, arena_bytes);
    c->stream = (hipStream_t)hip_stream;
    {
        int dev = 0, cus = 0, tpm = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            hipDeviceGetAttribute(&tpm, hipDeviceAttributeMaxThreadsPerMultiProcessor, dev) == hipSuccess &&
            cus > 0 && tpm > 0)
            c->wave_cap = cus * (tpm / kWave);
        int lds = 0, optin = 0;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) lds = 0;
        if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess) optin = 0;
        lds = std::max(lds, optin);
        if (lds > 0) {
            if (subtree_set_lds_limit(lds) == hipSuccess && paper_set_lds_limit(lds) == hipSuccess) {
                c->lds_max = lds;
            } else {
                (void)hipGetLastError();
                c->lds_max = std::min(lds, 65536);
            }
        }
    }
    default_tilings(c);
    if (hipHostMalloc((void**)&c->pinned, 4 * sizeof(Ctrl), hipHostMallocDefault) != hipSuccess) {
        delete c;
        return fail(LAP_EHIP, "hipHostMalloc of the control slots failed");
    }
    for (int k = 0; k < 2; ++k)
        if (hipEventCreateWithFlags(&c->poll_ev[k], hipEventDisableTiming) != hipSuccess) {
            delete c;
            return fail(LAP_EHIP, "hipEventCreate failed");
        }
    *out = c;
    return LAP_OK;
}

lap_status lap_grid_destroy(lap_grid* g);

lap_status lap_ctx_destroy(lap_ctx* c) {
    if (!c) return LAP_OK;
    hipStreamSynchronize(c->stream);
    while (!c->grids.empty()) lap_grid_destroy(c->grids.back());
    plans_clear(c);
    for (auto& r : c->recs) {
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    for (auto e : c->pool) hipEventDestroy(e);
    for (int k = 0; k < 2; ++k)
        if (c->poll_ev[k]) hipEventDestroy(c->poll_ev[k]);
    if (c->pinned) hipHostFree(c->pinned);
    if (c->batch_host) hipHostFree(c->batch_host);
    delete c;
    return LAP_OK;
}

lap_status lap_ctx_usage(lap_ctx* c, size_t* used, size_t* largest_free) {
    if (!c) return fail(LAP_EINVAL, "ctx is NULL");
    if (used) *used = c->arena.in_use;
    if (largest_free) *largest_free = c->arena.largest_free();
    return LAP_OK;
}

lap_status lap_ctx_set_timing(lap_ctx* c, int32_t on) {
    if (!c) return fail(LAP_EINVAL, "ctx is NULL");
    if (on < 0 || on > 2) return fail(LAP_EINVAL, "timing must be 0 (off), 1 (every launch) or 2 (finest level)");
    HIPCHK(c->flush_recs());
    c->timing = on;
    return LAP_OK;
}

lap_status lap_ctx_reset_stats(lap_ctx* c) {
    if (!c) return fail(LAP_EINVAL, "ctx is NULL");
    HIPCHK(c->flush_recs());
    std::memset(c->launches, 0, sizeof c->launches);
    std::memset(c->ms, 0, sizeof c->ms);
    std::memset(c->bytes, 0, sizeof c->bytes);
    return LAP_OK;
}

lap_status lap_ctx_kernel_stats(lap_ctx* c, int32_t cls, int32_t fine_only, int64_t* launches, double* ms,
                                double* bytes) {
    if (!c) return fail(LAP_EINVAL, "ctx is NULL");
    if (cls < 0 || cls >= KC_COUNT) return fail(LAP_EINVAL, "unknown kernel class");
    HIPCHK(c->flush_recs());
    const int f = fine_only ? 1 : 0;
    if (launches) *launches = c->launches[cls][f];
    if (ms) *ms = c->ms[cls][f];
    if (bytes) *bytes = c->bytes[cls][f];
    return LAP_OK;
}

size_t lap_grid_footprint(int32_t m, int32_t n, int32_t flags) {
    if (m < 3 || n < 3) return 0;
    return footprint(m, n, true, flags).bytes;
}

lap_status lap_grid_create_ex(lap_ctx* c, int32_t m, int32_t n, double dx, double dy, const double* psi0,
                              const double* source, int32_t flags, lap_grid** out) {
    if (!out) return fail(LAP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c) return fail(LAP_EINVAL, "ctx is NULL");
    if (m < 3 || n < 3) return fail(LAP_EINVAL, "m and n must be >= 3");
    if (!(dx > 0.0) || !(dy > 0.0) || !std::isfinite(dx) || !std::isfinite(dy))
        return fail(LAP_EINVAL, "dx and dy must be positive and finite");
    if (check_ptr(psi0, "psi0") != LAP_OK) return LAP_EINVAL;
    if (flags <= 0 || flags > LAP_ALLOC_ALL) return fail(LAP_EINVAL, "bad allocation flags");
    auto lv = plan_levels(m, n, dx, dy);
    if (flags == LAP_ALLOC_ALL && !coarse_ok(lv.back()))
        flags = LAP_ALLOC_ADI;   // "everything the grid supports": no multigrid on this size
    const bool mg = (flags & (LAP_ALLOC_FP64 | LAP_ALLOC_MIXED)) != 0;
    if (mg && !coarse_ok(lv.back()))
        return fail(LAP_EINVAL, "coarsest multigrid level too large for its direct solve; use sizes c*2^k+1");
    const Footprint fp = footprint(m, n, source != nullptr, flags);
    if (fp.bytes > c->arena.largest_free()) return fail(LAP_ENOMEM, "arena cannot hold the grid");

    lap_grid* g = new (std::nothrow) lap_grid();
    if (!g) return fail(LAP_ENOMEM, "host allocation failed");
    g->ctx = c;
    g->m = m;
    g->n = n;
    g->dx = dx;
    g->dy = dy;
    g->flags = flags;
    g->geo = lv;
    g->P = lv[0].P;
    g->has_f = source != nullptr;
    const size_t f0 = (size_t)n * g->P;
    const int L = (int)lv.size();
    bool ok = true;
    auto A = [&](size_t bytes) -> void* {
        void* p = galloc(g, bytes);
        if (!p) ok = false;
        return p;
    };
    g->psi[0] = (double*)A(f0 * 8);
    g->psi[1] = (double*)A(f0 * 8);
    if (source) g->f64 = (double*)A(f0 * 8);
    g->l64.resize(L);
    g->l32.resize(L);
    if (flags & LAP_ALLOC_FP64)
        for (int l = 1; l < L; ++l) {
            const size_t sz = (size_t)lv[l].n * lv[l].P * 8;
            g->l64[l].u[0] = (double*)A(sz);
            g->l64[l].u[1] = (double*)A(sz);
            g->l64[l].b = (double*)A(sz);
        }
    if (flags & LAP_ALLOC_MIXED)
        for (int l = 0; l < L; ++l) {
            const size_t sz = (size_t)lv[l].n * lv[l].P * 4;
            g->l32[l].u[0] = (float*)A(sz);
            g->l32[l].u[1] = (float*)A(sz);
            g->l32[l].b = (float*)A(sz);
        }
    if (flags & LAP_ALLOC_MIXED) g->rhs2 = (float*)A(f0 * 4);
    std::vector<double> inv;
    const std::vector<double>* factor = nullptr;   // lives in the context's cache
    if (mg) {
        const LevelGeo& C = lv.back();
        char key[96];
        snprintf(key, sizeof key, "%d:%d:%.17g:%.17g", C.m, C.n, C.dx, C.dy);
        auto it = c->inv_cache.find(key);
        int bw = 0, ifast = 1;
        if (it == c->inv_cache.end()) {
            const bool okf = C.interior() <= (size_t)kDenseCoarseMax ? coarse_inverse(C.m, C.n, C.dx, C.dy, inv)
                                                                     : coarse_lines(C.m, C.n, C.dx, C.dy, inv, bw, ifast);
            if (!okf) {
                lap_grid_destroy(g);
                return fail(LAP_EINVAL, "coarse operator factorisation failed");
            }
            c->inv_cache[key] = inv;
        } else {
            if (C.interior() > (size_t)kDenseCoarseMax) {
                ifast = C.m <= C.n ? 1 : 0;
                bw = std::min(C.m, C.n) - 2;
            }
        }
        g->coarse_bw = bw;
        g->coarse_ifast = ifast;
        if (bw > 0) g->coarse_work = (double*)A(C.interior() * 8);
        factor = &c->inv_cache[key];
        g->minv = (double*)A(factor->size() * 8);
    }
    std::vector<double>& z64 = g->zhost64;
    std::vector<float>& z32 = g->zhost32;
    if (mg && zebra_fits(lv)) {
        g->zebra_ok = true;
        z64.assign((size_t)L * 2 * kSegTab, 0.0);
        z32.assign((size_t)L * 2 * kSegTab, 0.0f);
        for (int l = 0; l + 1 < L; ++l) {
            const Coef k = coef(lv[l].dx, lv[l].dy);
            adi_seg_table(k.d, k.cx, lv[l].m - 2, z64.data() + (size_t)2 * l * kSegTab);
            adi_seg_table(k.d, k.cy, lv[l].n - 2, z64.data() + ((size_t)2 * l + 1) * kSegTab);
            adi_seg_table(k.d, k.cx, lv[l].m - 2, z32.data() + (size_t)2 * l * kSegTab);
            adi_seg_table(k.d, k.cy, lv[l].n - 2, z32.data() + ((size_t)2 * l + 1) * kSegTab);
        }
        if (flags & LAP_ALLOC_FP64) g->ztab64 = (double*)A(z64.size() * 8);
        if (flags & LAP_ALLOC_MIXED) g->ztab32 = (float*)A(z32.size() * 4);
    }
    if (flags & LAP_ALLOC_ADI) {
        g->adi_scratch = (double*)A(f0 * 8);
        g->adi_maxk = std::max(m, n);
        g->adi_tab = (double*)A(((size_t)4 * g->adi_maxk + 2 * kSegTab) * 8);
    }
    g->ctrl = (Ctrl*)A(5 * sizeof(Ctrl));
    g->cyc = g->ctrl + 1;
    g->max_partials = (int)max_tiles(m, n);
    g->partials = (double*)A((size_t)g->max_partials * 16);
    g->norm_out = (double*)A(16);
    if (!ok) {
        for (void* p : g->allocs) c->arena.release(p);
        delete g;
        return fail(LAP_ENOMEM, "arena exhausted");
    }
    hipStream_t s = c->stream;
    for (void* p : g->allocs) {
        // zero every buffer (padding included) so no kernel ever reads garbage
        const size_t off = (size_t)((char*)p - c->arena.base);
        const size_t sz = c->arena.used_[off];
        if (hipMemsetAsync(p, 0, sz, s) != hipSuccess) {
            lap_grid_destroy(g);
            return fail(LAP_EHIP, "hipMemsetAsync failed");
        }
    }
    hipError_t e = launch_write_field(psi0, g->psi[0], g->psi[1], m, n, g->P, s);
    if (e == hipSuccess && source) e = launch_write_field(source, g->f64, nullptr, m, n, g->P, s);
    if (e == hipSuccess && mg)
        e = hipMemcpyAsync(g->minv, factor->data(), factor->size() * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && g->ztab64) e = hipMemcpyAsync(g->ztab64, z64.data(), z64.size() * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && g->ztab32) e = hipMemcpyAsync(g->ztab32, z32.data(), z32.size() * 4, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
        lap_grid_destroy(g);
        return fail(LAP_EHIP, std::string("grid upload: ") + hipGetErrorString(e));
    }
    c->grids.push_back(g);
    *out = g;
    return LAP_OK;
}

lap_status lap_grid_create(lap_ctx* c, int32_t m, int32_t n, double dx, double dy, const double* psi0,
                           const double* source, lap_grid** out) {
    return lap_grid_create_ex(c, m, n, dx, dy, psi0, source, LAP_ALLOC_ALL, out);
}

lap_status lap_grid_destroy(lap_grid* g) {
    if (!g) return LAP_OK;
    lap_ctx* c = g->ctx;
    hipStreamSynchronize(c->stream);
    plans_clear(c);   // cached batch plans may point into this grid
    if (g->graph) hipGraphExecDestroy(g->graph);
    for (void* p : g->allocs) c->arena.release(p);
    auto it = std::find(c->grids.begin(), c->grids.end(), g);
    if (it != c->grids.end()) c->grids.erase(it);
    delete g;
    return LAP_OK;
}

lap_status lap_grid_read(lap_grid* g, double* dst) {
    if (!g) return fail(LAP_EINVAL, "grid is NULL");
    if (!dst) return fail(LAP_EINVAL, "dst is NULL");
    HIPCHK(hipMemcpy2DAsync(dst, (size_t)g->m * 8, g->psi[0], (size_t)g->P * 8, (size_t)g->m * 8, g->n,
                            hipMemcpyDeviceToDevice, g->ctx->stream));
    return LAP_OK;
}

lap_status lap_grid_write(lap_grid* g, const double* src) {
    if (!g) return fail(LAP_EINVAL, "grid is NULL");
    if (!src) return fail(LAP_EINVAL, "src is NULL");
    HIPCHK(launch_write_field(src, g->psi[0], g->psi[1], g->m, g->n, g->P, g->ctx->stream));
    g->psi1_stale = false;
    g->batch_started = false;
    return LAP_OK;
}

lap_status lap_grid_levels(lap_grid* g, int32_t* nl) {
    if (!g || !nl) return fail(LAP_EINVAL, "NULL argument");
    *nl = (int32_t)g->geo.size();
    return LAP_OK;
}

lap_status lap_grid_level_shape(lap_grid* g, int32_t l, int32_t* m, int32_t* n) {
    if (!g || !m || !n) return fail(LAP_EINVAL, "NULL argument");
    if (l < 0 || l >= (int)g->geo.size()) return fail(LAP_EINVAL, "level out of range");
    *m = g->geo[l].m;
    *n = g->geo[l].n;
    return LAP_OK;
}

lap_status lap_solve_ex(lap_grid* g, const lap_opts* o, lap_info* info) {
    if (!g || !o) return fail(LAP_EINVAL, "NULL argument");
    lap_status st = validate_opts(g, *o);
    if (st != LAP_OK) return st;
    return solve_one(g, *o, info);
}

lap_status lap_solve(lap_grid* g, int32_t method, double omega, double tol, int32_t max_iter, int32_t precision,
                     lap_info* info) {
    lap_opts o;
    lap_opts_default(&o);
    o.method = method;
    o.omega = omega;
    o.tol = tol;
    o.max_iter = max_iter;
    o.precision = precision;
    return lap_solve_ex(g, &o, info);
}

lap_status lap_residual_ex(lap_grid* g, double* l2, double* linf) {
    if (!g) return fail(LAP_EINVAL, "grid is NULL");
    return residual_norms(g, l2, linf);
}
}  // extern "C"

namespace {
lap_status residual_norms(lap_grid* g, double* l2, double* linf) {
    const LevelGeo& L = g->geo[0];
    const Coef c = coef(L.dx, L.dy);
    ResidualArgs<double> a{};
    a.u = g->psi[0];
    a.f = g->f64;
    a.partials = g->partials;
    a.m = L.m;
    a.n = L.n;
    a.P = L.P;
    a.cx = c.cx;
    a.cy = c.cy;
    a.d = c.d;
    a.tl = norm_tiling(L.m, L.n);
    const double bytes = (g->f64 ? 16.0 : 8.0) * nint(L);   // u (and f) read once
    HIPCHK(g->ctx->timed(KC_RESIDUAL, true, bytes, [&]() { return launch_residual<double>(a, g->ctx->stream); }));
    HIPCHK(launch_finalize(g->partials, a.tl.ntiles, nullptr, g->norm_out, 1, g->ctx->stream));
    double h[2];
    HIPCHK(hipMemcpyAsync(h, g->norm_out, 16, hipMemcpyDeviceToHost, g->ctx->stream));
    HIPCHK(hipStreamSynchronize(g->ctx->stream));
    if (l2) *l2 = std::sqrt(h[0]);
    if (linf) *linf = h[1];
    return LAP_OK;
}
}  // namespace

extern "C" {

lap_status lap_residual(lap_grid* g, double* l2_rel, double* linf) {
    double l2 = 0.0;
    lap_status st = lap_residual_ex(g, &l2, linf);
    if (st != LAP_OK) return st;
    if (l2_rel) *l2_rel = (g->last_r0 > 0.0) ? l2 / g->last_r0 : (l2 > 0.0 ? 1.0 : 0.0);
    return LAP_OK;
}

lap_status lap_grid_set_tol(lap_grid* g, double tol) {
    if (!g) return fail(LAP_EINVAL, "grid is NULL");
    if (!(tol >= 0.0)) return fail(LAP_EINVAL, "tol must be >= 0");
    g->tol = tol;
    return LAP_OK;
}

lap_status lap_grid_set_omega(lap_grid* g, double omega) {
    if (!g) return fail(LAP_EINVAL, "grid is NULL");
    if (!(omega > 0.0 && omega < 2.0)) return fail(LAP_EINVAL, "omega must lie in (0, 2)");
    g->batch_omega = omega;
    return LAP_OK;
}

lap_status lap_grid_reset(lap_grid* g) {
    if (!g) return fail(LAP_EINVAL, "grid is NULL");
    g->batch_started = false;
    return LAP_OK;
}

}  // extern "C"

// ------------------------------------------------------------------- op level
static lap_status op_check(int32_t dtype, int32_t m, int32_t n, int32_t ld, double dx, double dy) {
    if (dtype != 0 && dtype != 1) return fail(LAP_EINVAL, "dtype must be 0 (FP64) or 1 (FP32)");
    if (m < 3 || n < 3) return fail(LAP_EINVAL, "m and n must be >= 3");
    if (ld < m || ld % 64) return fail(LAP_EINVAL, "ld must be >= m and a multiple of 64");
    if (!(dx > 0.0) || !(dy > 0.0)) return fail(LAP_EINVAL, "dx and dy must be positive");
    return LAP_OK;
}
static bool aligned(const void* p) { return ((uintptr_t)p % kAlign) == 0; }

static const int kOpV[2] = {2, 4};
static const int kOpTY = 32;

template <typename T>
static lap_status op_sweep(int32_t m, int32_t n, int32_t ld, double dx, double dy, double omega, const void* u_in,
                           const void* f, const void* ec, int32_t ldc, void* u_out, hipStream_t s) {
    const Coef c = coef(dx, dy);
    SweepArgs<T> a{};
    a.uin = (const T*)u_in;
    a.uout = (T*)u_out;
    a.f = (const T*)f;
    a.ec = (const T*)ec;
    a.m = m;
    a.n = n;
    a.P = ld;
    a.mc = (m - 1) / 2 + 1;
    a.nc = (n - 1) / 2 + 1;
    a.Pc = ldc;
    a.cx = (T)c.cx;
    a.cy = (T)c.cy;
    a.d = (T)c.d;
    a.inv_d = (T)c.inv_d;
    a.omega = (T)omega;
    a.tl = make_tiling(m, n, kOpV[dt_of<T>()], kOpTY);
    int flags = (f ? SW_F : 0);
    if (!u_in && !ec) flags |= SW_ZERO;
    if (ec) flags |= SW_PROLONG;
    HIPCHK(launch_sweep<T>(a, flags, s));
    return LAP_OK;
}

extern "C" lap_status lap_op_rb_sweep(int32_t dtype, int32_t m, int32_t n, int32_t ld, double dx, double dy, double omega,
                           const void* u_in, const void* f, const void* ec, int32_t ldc, void* u_out, void* stream) {
    lap_status st = op_check(dtype, m, n, ld, dx, dy);
    if (st != LAP_OK) return st;
    if (!(omega > 0.0 && omega < 2.0)) return fail(LAP_EINVAL, "omega must lie in (0, 2)");
    if (!u_out) return fail(LAP_EINVAL, "u_out is NULL");
    if (!aligned(u_out) || (u_in && !aligned(u_in)) || (f && !aligned(f)) || (ec && !aligned(ec)))
        return fail(LAP_EINVAL, "pointers must be 256-byte aligned");
    if (ec) {
        if (m % 2 == 0 || n % 2 == 0) return fail(LAP_EINVAL, "prolongation needs odd m and n");
        if (ldc < (m - 1) / 2 + 1 || ldc % 64) return fail(LAP_EINVAL, "bad ldc");
    }
    hipStream_t s = (hipStream_t)stream;
    return dtype == 0 ? op_sweep<double>(m, n, ld, dx, dy, omega, u_in, f, ec, ldc, u_out, s)
                      : op_sweep<float>(m, n, ld, dx, dy, omega, u_in, f, ec, ldc, u_out, s);
}

extern "C" size_t lap_op_work_bytes(int32_t m, int32_t n) {
    if (m < 3 || n < 3) return 0;
    const size_t part = round_up((size_t)make_tiling(m, n, 1, 16).ntiles * 16, kAlign);
    const size_t line = round_up((size_t)n * pitch_of(m) * 8, kAlign) +
                        round_up(((size_t)2 * std::max(m, n) + kSegTab) * 8, kAlign);
    return std::max(part, line);
}

template <typename T>
static lap_status op_residual(int32_t m, int32_t n, int32_t ld, double dx, double dy, const void* u, const void* f,
                              void* r, double* norms, void* work, hipStream_t s) {
    const Coef c = coef(dx, dy);
    ResidualArgs<T> a{};
    a.u = (const T*)u;
    a.f = (const T*)f;
    a.r = (T*)r;
    a.partials = norms ? (double*)work : nullptr;
    a.m = m;
    a.n = n;
    a.P = ld;
    a.cx = (T)c.cx;
    a.cy = (T)c.cy;
    a.d = (T)c.d;
    a.tl = make_tiling(m, n, kOpV[dt_of<T>()], kOpTY);
    HIPCHK(launch_residual<T>(a, s));
    if (norms) HIPCHK(launch_finalize((double*)work, a.tl.ntiles, nullptr, norms, 1, s));
    return LAP_OK;
}

extern "C" lap_status lap_op_residual(int32_t dtype, int32_t m, int32_t n, int32_t ld, double dx, double dy, const void* u,
                           const void* f, void* r, double* norms, void* work, void* stream) {
    lap_status st = op_check(dtype, m, n, ld, dx, dy);
    if (st != LAP_OK) return st;
    if (!u) return fail(LAP_EINVAL, "u is NULL");
    if (norms && !work) return fail(LAP_EINVAL, "norms need a work buffer");
    if (!aligned(u) || (f && !aligned(f)) || (r && !aligned(r))) return fail(LAP_EINVAL, "pointers must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    return dtype == 0 ? op_residual<double>(m, n, ld, dx, dy, u, f, r, norms, work, s)
                      : op_residual<float>(m, n, ld, dx, dy, u, f, r, norms, work, s);
}

// ------------------------------------------- residual without a workspace
// The per-tile norm partials of lap_op_residual_static live in this fixed
// device array instead of a caller's work buffer.  Every GPU the library runs
// on holds its own copy, at its own address, until the process ends.  Host
// code never passes the array's name to a kernel (on the host it is only a
// stand-in symbol): it looks up the device address once per device and
// passes that.
constexpr int kStaticNormTiles = 65536;                 // 1 MiB of partials
static __device__ __align__(256) double scratch[2 * kStaticNormTiles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// The address of `scratch` on the device of `s` (the current device for the
// default stream); looked up on the first call per device.
lap_status static_scratch(hipStream_t s, double** out) {
    int cur = 0, dev = 0;
    HIPCHK(hipGetDevice(&cur));
    dev = cur;
    if (s != nullptr) HIPCHK(hipStreamGetDevice(s, &dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(LAP_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_dev[dev] == nullptr) {
        if (dev != cur) HIPCHK(hipSetDevice(dev));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (dev != cur) HIPCHK(hipSetDevice(cur));
        if (e != hipSuccess || p == nullptr)
            return fail(LAP_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[dev] = (double*)p;
    }
    *out = g_scratch_dev[dev];
    return LAP_OK;
}
}  // namespace

extern "C" lap_status lap_op_residual_static(int32_t dtype, int32_t m, int32_t n, int32_t ld, double dx, double dy,
                                             const void* u, const void* f, void* r, double* norms, void* stream) {
    lap_status st = op_check(dtype, m, n, ld, dx, dy);
    if (st != LAP_OK) return st;
    if (!u) return fail(LAP_EINVAL, "u is NULL");
    if (!aligned(u) || (f && !aligned(f)) || (r && !aligned(r))) return fail(LAP_EINVAL, "pointers must be 256-byte aligned");
    const int ntiles = make_tiling(m, n, kOpV[dtype == 0 ? 0 : 1], kOpTY).ntiles;
    if (norms && ntiles > kStaticNormTiles)
        return fail(LAP_EINVAL, "grid too large for lap_op_residual_static: " + std::to_string(ntiles) +
                                    " norm tiles, at most " + std::to_string(kStaticNormTiles) +
                                    " (use lap_op_residual with a work buffer)");
    hipStream_t s = (hipStream_t)stream;
    double* work = nullptr;
    if (norms) {
        st = static_scratch(s, &work);
        if (st != LAP_OK) return st;
    }
    // every tile overwrites its two partials, so nothing is cleared first
    return dtype == 0 ? op_residual<double>(m, n, ld, dx, dy, u, f, r, norms, work, s)
                      : op_residual<float>(m, n, ld, dx, dy, u, f, r, norms, work, s);
}

template <typename T>
static lap_status op_restrict(int32_t m, int32_t n, int32_t ld, double dx, double dy, const void* u, const void* f,
                              void* bc, int32_t ldc, hipStream_t s) {
    const Coef c = coef(dx, dy);
    RestrictArgs<T> a{};
    a.u = (const T*)u;
    a.f = (const T*)f;
    a.bc = (T*)bc;
    a.m = m;
    a.n = n;
    a.P = ld;
    a.mc = (m - 1) / 2 + 1;
    a.nc = (n - 1) / 2 + 1;
    a.Pc = ldc;
    a.cx = (T)c.cx;
    a.cy = (T)c.cy;
    a.d = (T)c.d;
    a.tl = make_tiling(m, n, kOpV[dt_of<T>()], kOpTY);
    HIPCHK(launch_restrict<T>(a, s));
    return LAP_OK;
}

extern "C" lap_status lap_op_restrict(int32_t dtype, int32_t m, int32_t n, int32_t ld, double dx, double dy, const void* u,
                           const void* f, void* bc, int32_t ldc, void* stream) {
    lap_status st = op_check(dtype, m, n, ld, dx, dy);
    if (st != LAP_OK) return st;
    if (m % 2 == 0 || n % 2 == 0 || m < 5 || n < 5) return fail(LAP_EINVAL, "restriction needs odd m, n >= 5");
    if (!bc) return fail(LAP_EINVAL, "bc is NULL");
    if (ldc < (m - 1) / 2 + 1 || ldc % 64) return fail(LAP_EINVAL, "bad ldc");
    if ((u && !aligned(u)) || (f && !aligned(f)) || !aligned(bc)) return fail(LAP_EINVAL, "pointers must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    return dtype == 0 ? op_restrict<double>(m, n, ld, dx, dy, u, f, bc, ldc, s)
                      : op_restrict<float>(m, n, ld, dx, dy, u, f, bc, ldc, s);
}

extern "C" lap_status lap_op_adi_half(int32_t dtype, int32_t m, int32_t n, int32_t ld, double dx, double dy, double omega,
                           int32_t dir, int32_t form, void* u, const void* f, void* work, void* stream) {
    lap_status st = op_check(dtype, m, n, ld, dx, dy);
    if (st != LAP_OK) return st;
    if (dtype != 0) return fail(LAP_EINVAL, "ADI lines are FP64 only");
    if (!(omega > 0.0 && omega < 2.0)) return fail(LAP_EINVAL, "omega must lie in (0, 2)");
    if (dir != 0 && dir != 1) return fail(LAP_EINVAL, "dir must be 0 (rows) or 1 (columns)");
    if (form != 0 && form != 1) return fail(LAP_EINVAL, "unknown form");
    if (!u || !work) return fail(LAP_EINVAL, "u and work are required");
    if (!aligned(u) || (f && !aligned(f)) || !aligned(work)) return fail(LAP_EINVAL, "pointers must be 256-byte aligned");
    if (ld != pitch_of(m)) return fail(LAP_EINVAL, "ADI needs ld = m rounded up to 64");
    const Coef c = coef(dx, dy);
    const double cl = dir == 0 ? c.cx : c.cy;
    if (form == 1 && omega >= 1.0 + (dir == 0 ? c.cy / c.cx : c.cx / c.cy))
        return fail(LAP_EINVAL, "relaxation inside the line system needs omega < 1 + beta^2");
    const int K = dir == 0 ? m - 2 : n - 2;
    std::vector<double> tab(2 * (size_t)K + kSegTab);
    const double wl = form == 0 ? cl : omega * cl;
    adi_factor(c.d, -wl, -wl, K, tab.data(), tab.data() + K);
    adi_seg_table(c.d, wl, K, tab.data() + 2 * (size_t)K);
    // tables live at the end of the work buffer
    char* wbase = (char*)work;
    double* scratch = (double*)wbase;
    double* dtab = (double*)(wbase + round_up((size_t)n * ld * 8, kAlign));
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipMemcpyAsync(dtab, tab.data(), tab.size() * 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    LineArgs a{};
    a.u = (double*)u;
    a.f = (const double*)f;
    a.scratch = scratch;
    a.cprime = dtab;
    a.piv = dtab + K;
    a.seg = dtab + 2 * (size_t)K;
    a.m = m;
    a.n = n;
    a.P = ld;
    a.cx = c.cx;
    a.cy = c.cy;
    a.d = c.d;
    a.omega = omega;
    a.form = form;
    a.a_off = -wl;
    for (int par : {1, 0}) {
        a.parity = par;
        HIPCHK(dir == 0 ? launch_adi_rows(a, s) : launch_adi_cols(a, s));
    }
    return LAP_OK;
}

// ------------------------------------------------------------------ batches
struct MergedLaunch {
    int kind, dt, flags;     // BatchKind, dtype, step flags of a sweep
    int V;                   // fused passes: columns per lane of every item
    int cls;                 // kernel class for timing
    bool fine;
    int count, total, blocks;
    int lds;                 // subtree: dynamic LDS bytes (largest item)
    size_t off;              // first item in the plan's item array
    size_t toff;             // first entry in the plan's tile map
    double bytes;            // algorithmic bytes of the launch
};

struct lap_ctx::Plan {
    std::vector<MergedLaunch> launches;
    std::vector<BatchItem> items;
    std::vector<unsigned char> subs;                 // SubtreeArgs of subtree items
    std::vector<std::pair<size_t, size_t>> sub_of;   // (item, byte offset in subs)
    std::vector<int32_t> tmap;                       // item (within its launch) of every tile
    BatchItem* dev = nullptr;
    const int32_t* tmap_dev = nullptr;
    hipGraphExec_t graph = nullptr;
    int uses = 0;
};

namespace {

void plan_free(lap_ctx* c, lap_ctx::Plan* p) {
    if (!p) return;
    if (p->graph) hipGraphExecDestroy(p->graph);
    if (p->dev) c->arena.release(p->dev);
    delete p;
}

void plans_clear(lap_ctx* c) {
    hipStreamSynchronize(c->stream);
    for (auto& kv : c->plans) plan_free(c, kv.second);
    c->plans.clear();
}

// Batch plans and captured per-grid graphs bake in tilings and the subtree
// split: drop them when either changes.
void invalidate_cached(lap_ctx* c) {
    plans_clear(c);
    for (lap_grid* g : c->grids)
        if (g->graph) {
            hipGraphExecDestroy(g->graph);
            g->graph = nullptr;
            g->graph_key.clear();
        }
}

int batch_kind(const Op& op) {
    switch (op.kind) {
        case OP_SWEEP: return is_fused(op.flags) ? BK_FUSED : BK_SWEEP;
        case OP_RESTRICT: return BK_RESTRICT;
        case OP_COARSE: return BK_COARSE;
        case OP_FINALIZE: return BK_FINALIZE;
        case OP_RESNORM: return BK_RESNORM;
        case OP_DEFECT: return BK_DEFECT;
        case OP_ADI_ROWS: return BK_ADI_ROWS;
        case OP_ADI_COLS: return BK_ADI_COLS;
        case OP_SUBTREE: return BK_SUBTREE;
        case OP_POSTDEF: return BK_FUSED;
    }
    return -1;
}

constexpr int kBatchMinRows = 32;
// Four-sweep passes (halo 10) in plans of many grids: chunks of >= 64 rows
// (512-grid ragged batch, four FP32 cycles per correction: 12.3 ms with 32,
// 11.0 with 64, 11.2 with 128; four columns per lane 11.1-11.3)
constexpr int kBatchFourMinRows = 64;
constexpr size_t kBatchManyGrids = 4;
constexpr int kBatchV = 2;

// Fill the item of grid g for operation op (tiling, geometry, coefficients).
BatchItem make_item(lap_grid* g, const Op& op, const lap_opts& o, size_t nplan) {
    lap_ctx* c = g->ctx;
    const LevelGeo& L = g->geo[op.level];
    const Coef k = coef(L.dx, L.dy);
    BatchItem it{};
    it.in = op.in;
    it.out = op.out;
    it.f = op.f;
    it.ec = op.ec;
    it.bc = op.bc;
    it.minv = g->minv;
    it.cwork = g->coarse_work;
    it.cbw = g->coarse_bw;
    it.cifast = g->coarse_ifast;
    it.partials = g->partials;
    // a gated operation's items skip at its gate (set, like the control
    // block's done flag, once the solve has ended)
    it.ctrl = op.gate != nullptr && op.kind != OP_FINALIZE ? op.gate : g->ctrl;
    it.m = L.m;
    it.n = L.n;
    it.P = L.P;
    if ((size_t)op.level + 1 < g->geo.size()) {
        it.mc = g->geo[op.level + 1].m;
        it.nc = g->geo[op.level + 1].n;
        it.Pc = g->geo[op.level + 1].P;
    }
    it.cx = k.cx;
    it.cy = k.cy;
    it.d = k.d;
    it.inv_d = k.inv_d;
    it.omega = op.omega;
    it.flags = (op.kind == OP_SWEEP) ? (op.flags & SW_F) : 0;
    Tiling t{};
    switch (op.kind) {
        case OP_SWEEP:
            if (op.flags & SW_NORM)
                t = norm_tiling(L.m, L.n);
            else if (is_fused(op.flags))
                t = c->tiling(L.m, L.n, fused_class(op.flags), op.dt, fused_halo(op.flags));
            else
                t = c->tiling(L.m, L.n, (op.flags & SW_PROLONG) ? KC_SWEEP_PROLONG : KC_SWEEP, op.dt);
            break;
        case OP_RESTRICT:
            t = c->tiling(L.m, L.n, KC_RESTRICT, op.dt);
            it.flags = op.flags & SW_RDIFF;
            break;
        case OP_RESNORM: t = norm_tiling(g->geo[0].m, g->geo[0].n); break;
        case OP_DEFECT:
            t = norm_tiling(g->geo[0].m, g->geo[0].n, NORM_DEFECT);
            it.e = op.zbuf;   // the FP32 buffer the defect correction sets to zero (zebra cycles)
            break;
        case OP_POSTDEF:
            t = postdef_tiling(L.m, L.n, true);
            it.rowpart = postdef_rowpart(L.n) ? 1 : 0;
            it.e = (op.parity == 0 || op.parity == 1) ? g->l32[0].u[op.parity] : nullptr;
            it.f64 = g->f64;
            it.flags = SW_F;
            break;
        case OP_FINALIZE:
            t.ntiles = norm_partials(g->geo[0].m, g->geo[0].n, op.flags);
            it.gate = op.gate;
            if (op.cycles >= 0) {
                it.cyc = g->cyc;
                it.cycles = op.cycles;
            }
            break;
        case OP_ADI_ROWS:
        case OP_ADI_COLS: {
            const int dir = op.kind == OP_ADI_ROWS ? 0 : 1;
            if (op.flags & ADI_MG) {
                // zebra smoothing of a multigrid level: the level's buffers and table
                it.out = op.out;
                it.f = op.f;
                it.seg = op.dt == 0 ? (const void*)zebra_args<double>(g, op.level, (double*)op.out,
                                                                      (const double*)op.f, op.omega, dir, op.parity).seg
                                    : (const void*)zebra_args<float>(g, op.level, (float*)op.out, (const float*)op.f,
                                                                     op.omega, dir, op.parity).seg;
                it.flags = LAP_ADI_RELAX_AFTER;
            } else {
                const LineArgs la = adi_args(g, op.omega, op.flags, dir, op.parity);
                it.out = la.u;
                it.f = la.f;
                it.scratch = la.scratch;
                it.cprime = la.cprime;
                it.piv = la.piv;
                it.seg = la.seg;
                it.a_off = la.a_off;
                it.flags = op.flags & 1;
            }
            it.parity = op.parity;
            const int first = op.parity ? 1 : 2;
            const int span = op.kind == OP_ADI_ROWS ? L.n - 2 : L.m - 2;
            const int lines = span >= first ? (span - first) / 2 + 1 : 0;
            int per = op.kind == OP_ADI_ROWS ? kRowTile : kBlock;
            if (op.flags & ADI_SEG) per = op.kind == OP_ADI_ROWS ? seg_lines(0, L.m - 2) : seg_lines(1, L.n - 2);
            t.ntiles = (lines + per - 1) / per;
            break;
        }
        case OP_COARSE:
        case OP_SUBTREE: t.ntiles = 1; break;
    }
    // The table's short row chunks (down to 2 rows) and narrow windows
    // minimise the latency of one grid's small level.  Inside a merged launch
    // over several grids a chunk's halo rows (up to 11 for a fused pass)
    // weigh more, so plans of 4 or more grids use chunks of >= 32 rows (>= 64
    // for four-sweep passes), and every plan of 2 or more grids 2 columns per
    // lane (one launch per key; a 512-grid ragged batch of 33..1025 points a
    // side: 13.8 ms with 4 columns per lane and >= 64 rows, 11.7 ms with 2 and
    // >= 32; 15.4 ms with the table's chunks).
    const bool tile_op = (op.kind == OP_SWEEP || op.kind == OP_RESTRICT) && !(op.flags & SW_NORM);
    if (tile_op && nplan >= kBatchManyGrids) {
        const bool four = (op.flags & SW_FOUR) != 0;
        t = make_tiling(L.m, L.n, kBatchV, std::max(t.ty, four ? kBatchFourMinRows : kBatchMinRows), 0, t.H);
    } else if (tile_op && nplan >= 2) {
        t = make_tiling(L.m, L.n, kBatchV, t.ty, 0, t.H);
    }
    it.V = t.V;
    it.ty = t.ty;
    it.nwin = t.nwin;
    it.nchunk = t.nchunk;
    it.ntiles = t.ntiles;
    it.H = t.H;
    return it;
}

double item_bytes(const Op& op, const BatchItem& it) {
    const double n = (double)(it.m - 2) * (double)(it.n - 2);
    const double sz = op.dt == 0 ? 8.0 : 4.0;
    switch (op.kind) {
        case OP_SWEEP: return sweep_bytes_per_node(op.flags, (int)sz) * n;
        case OP_RESTRICT: return ((op.in ? 1.0 : 0.0) + (op.f ? 1.0 : 0.0) + (op.out ? 0.5 : 0.25)) * sz * n;
        case OP_RESNORM: return (op.f ? 16.0 : 8.0) * n;
        case OP_DEFECT:
            return (8.0 + (op.ec ? 4.0 : 0.0) + (op.f ? 8.0 : 0.0) + (op.out != op.in || op.ec ? 8.0 : 0.0) + 4.0 +
                    (op.zbuf ? 4.0 : 0.0)) * n;
        case OP_POSTDEF: return postdef_bytes_per_node(it.f64 != nullptr) * n;
        case OP_ADI_ROWS:
        case OP_ADI_COLS: return adi_bytes_per_node(op.f != nullptr) * sz / 8.0 * n;
        case OP_SUBTREE: return 2.0 * sz * (double)it.m * (double)it.n;
        default: return 0.0;
    }
}

int kclass_of(const Op& op) {
    switch (op.kind) {
        case OP_SWEEP:
            if (is_fused(op.flags)) return fused_class(op.flags);
            return (op.flags & SW_PROLONG) ? KC_SWEEP_PROLONG : KC_SWEEP;
        case OP_RESTRICT: return KC_RESTRICT;
        case OP_COARSE: return KC_COARSE;
        case OP_FINALIZE: return KC_FINALIZE;
        case OP_RESNORM: return KC_RESIDUAL;
        case OP_DEFECT: return KC_DEFECT;
        case OP_ADI_ROWS: return KC_ADI_ROWS;
        case OP_ADI_COLS: return KC_ADI_COLS;
        case OP_SUBTREE: return KC_SUBTREE;
        case OP_POSTDEF: return KC_DEFECT;
    }
    return KC_SWEEP;
}

// Build (or fetch) the merged-launch plan of one step of `gs`; steps[k] is
// grid k's step number (its buffer parity).
// grid_omega: each grid's smoother relaxation is its own (lap_grid_set_omega)
// instead of o.omega.
lap_status get_plan(lap_ctx* c, const std::vector<lap_grid*>& gs, const std::vector<int>& steps, const lap_opts& o,
                    lap_ctx::Plan** out, bool grid_omega = false) {
    std::string key;
    {
        char buf[96];
        snprintf(buf, sizeof buf, "%d:%d:%d:%d:%d:%d:%d:%d:%.17g|", o.method, o.precision, o.smoother, o.nu1, o.nu2,
                 o.check_every, o.adi_form, o.inner, o.omega);
        key = buf;
        for (size_t k = 0; k < gs.size(); ++k) {
            const int par = (o.method == LAP_MG && o.precision == LAP_MIXED)
                                ? (steps[k] == 0 ? 2 : steps[k] % 2)
                                : (o.method == LAP_SOR_RB ? (steps[k] % 2) * ((int)sor_passes(c, o.check_every).size() % 2)
                                                          : 0);
            snprintf(buf, sizeof buf, "%p:%d%s,", (void*)gs[k], par, gs[k]->pdef ? "d" : "");
            key += buf;
            if (grid_omega) {
                snprintf(buf, sizeof buf, "w%.17g,", gs[k]->batch_omega);
                key += buf;
            }
        }
    }
    for (size_t k = 0; k < c->plans.size(); ++k)
        if (c->plans[k].first == key) {
            *out = c->plans[k].second;
            return LAP_OK;
        }
    // group every grid's operations by merge key
    std::map<long, std::vector<std::pair<lap_grid*, Op>>> groups;
    for (size_t k = 0; k < gs.size(); ++k) {
        std::vector<Op> ops;
        lap_opts ok = o;
        if (grid_omega) ok.omega = gs[k]->batch_omega;
        plan_step(gs[k], ok, steps[k], PART_ALL, ops);
        for (size_t q = 1; q < ops.size(); ++q)
            if (ops[q].key <= ops[q - 1].key)   // merging by key must keep each grid's own order
                return fail(LAP_EINVAL, "internal error: operation keys out of order");
        for (const Op& op : ops) groups[op.key].push_back({gs[k], op});
    }
    lap_ctx::Plan* p = new lap_ctx::Plan();
    for (auto& kv : groups) {
        auto& v = kv.second;
        // one merged launch per (kind, dtype, step flags) inside a key (normally
        // exactly one), fused passes also per columns-per-lane V: each V is a
        // kernel of its own, so a launch occupies the registers of its own V
        // only (one kernel for all three ran at the V = 4 variant's occupancy)
        using GoIt = std::pair<std::pair<lap_grid*, Op>, BatchItem>;
        std::map<std::tuple<int, int, int, int>, std::vector<GoIt>> sub;
        for (auto& go : v) {
            const BatchItem it = make_item(go.first, go.second, o, gs.size());
            const int bk = batch_kind(go.second);
            const int vkey = bk == BK_FUSED ? it.V : 0;
            // the merged residual-norm and defect kernels are built for the canonical V only
            if ((bk == BK_RESNORM && it.V != kNormPassV) || (bk == BK_DEFECT && it.V != kNormDefectV) ||
                (go.second.kind == OP_POSTDEF && it.e == nullptr)) {
                delete p;
                return fail(LAP_EINVAL, "internal error: a norm item without its canonical tiling or input");
            }
            sub[std::make_tuple(go.second.kind, go.second.dt, go.second.flags & ~SW_F, vkey)].push_back({go, it});
        }
        for (auto& skv : sub) {
            if (batch_kind(skv.second[0].first.second) == BK_SUBTREE) {
                // one workgroup per grid, all with the largest grid's LDS: the
                // largest sub-V-cycles go first so the last round holds the short ones
                auto nodes = [](const GoIt& gi) {
                    const LevelGeo& L = gi.first.first->geo[gi.first.second.level];
                    return (size_t)L.m * (size_t)L.n;
                };
                std::stable_sort(skv.second.begin(), skv.second.end(),
                                 [&](const GoIt& a, const GoIt& b) { return nodes(a) > nodes(b); });
            }
            MergedLaunch L{};
            const Op& op0 = skv.second[0].first.second;
            L.kind = batch_kind(op0);
            L.dt = std::get<1>(skv.first);
            L.flags = std::get<2>(skv.first);
            L.V = std::get<3>(skv.first);
            L.off = p->items.size();
            L.toff = p->tmap.size();
            L.cls = kclass_of(op0);
            L.fine = op0.level == 0;
            int tile0 = 0;
            for (auto& gi : skv.second) {
                const auto& go = gi.first;
                BatchItem it = gi.second;
                it.tile0 = tile0;
                if (L.kind == BK_SUBTREE) {
                    const Op& op = go.second;
                    const size_t off = p->subs.size();
                    int lds = 0;
                    if (op.dt == 0) {
                        const auto a = subtree_args<double>(go.first, op.level, (double*)op.out,
                                                            (const double*)op.f, op.omega, op.flags);
                        p->subs.resize(off + round_up(sizeof(a), 64));
                        std::memcpy(p->subs.data() + off, &a, sizeof(a));
                        lds = a.lds_bytes;
                    } else {
                        const auto a = subtree_args<float>(go.first, op.level, (float*)op.out, (const float*)op.f,
                                                           op.omega, op.flags);
                        p->subs.resize(off + round_up(sizeof(a), 64));
                        std::memcpy(p->subs.data() + off, &a, sizeof(a));
                        lds = a.lds_bytes;
                    }
                    L.lds = std::max(L.lds, lds);
                    p->sub_of.push_back({p->items.size(), off});
                }
                if (L.kind != BK_COARSE && L.kind != BK_FINALIZE && L.kind != BK_SUBTREE) {
                    p->tmap.insert(p->tmap.end(), (size_t)it.ntiles, (int32_t)(p->items.size() - L.off));
                    tile0 += it.ntiles;
                }
                L.bytes += item_bytes(go.second, it);
                p->items.push_back(it);
            }
            L.count = (int)skv.second.size();
            L.total = tile0;
            if (L.kind == BK_SUBTREE) {
                L.blocks = L.count;
            } else if (L.kind == BK_COARSE || L.kind == BK_FINALIZE) {
                L.blocks = std::min(L.count, 2048);
            } else if (L.kind == BK_ADI_ROWS || L.kind == BK_ADI_COLS) {
                L.blocks = std::max(1, L.total);   // one workgroup per line tile
            } else {
                int nb = (L.total + kWavesPerBlock - 1) / kWavesPerBlock;
                nb = std::min(nb, 2 * c->wave_cap / kWavesPerBlock);
                L.blocks = std::max(kXcds, (nb + kXcds - 1) / kXcds * kXcds);
            }
            p->launches.push_back(L);
        }
    }
    const size_t ibytes = round_up(p->items.size() * sizeof(BatchItem), kAlign);
    const size_t sbytes = round_up(p->subs.size(), kAlign);
    const size_t pbytes = ibytes + sbytes + p->tmap.size() * sizeof(int32_t);
    p->dev = (BatchItem*)c->arena.alloc(pbytes);
    if (!p->dev && !c->plans.empty()) {
        // the grids filled the arena: drop the cached plans (after the work
        // that may still read them) and try once more
        plans_clear(c);
        p->dev = (BatchItem*)c->arena.alloc(pbytes);
    }
    if (!p->dev) {
        delete p;
        return fail(LAP_ENOMEM, "arena cannot hold the batch plan");
    }
    unsigned char* sub_dev = (unsigned char*)p->dev + ibytes;
    p->tmap_dev = (const int32_t*)(sub_dev + sbytes);
    for (const auto& so : p->sub_of) p->items[so.first].sub = sub_dev + so.second;
    if (hipMemcpyAsync(p->dev, p->items.data(), p->items.size() * sizeof(BatchItem), hipMemcpyHostToDevice,
                       c->stream) != hipSuccess ||
        (!p->subs.empty() &&
         hipMemcpyAsync(sub_dev, p->subs.data(), p->subs.size(), hipMemcpyHostToDevice, c->stream) != hipSuccess) ||
        (!p->tmap.empty() && hipMemcpyAsync((void*)p->tmap_dev, p->tmap.data(), p->tmap.size() * sizeof(int32_t),
                                            hipMemcpyHostToDevice, c->stream) != hipSuccess)) {
        plan_free(c, p);
        return fail(LAP_EHIP, "plan upload failed");
    }
    if (c->plans.size() >= 8) {
        hipStreamSynchronize(c->stream);
        plan_free(c, c->plans.front().second);
        c->plans.erase(c->plans.begin());
    }
    c->plans.push_back({key, p});
    *out = p;
    return LAP_OK;
}

hipError_t run_plan_launches(lap_ctx* c, lap_ctx::Plan* p) {
    // launches up to and including the first norm finalisation are the
    // step's stopping test (its head)
    size_t fin = p->launches.size();
    for (size_t k = 0; k < p->launches.size(); ++k)
        if (p->launches[k].kind == BK_FINALIZE) {
            fin = k;
            break;
        }
    for (size_t k = 0; k < p->launches.size(); ++k) {
        const MergedLaunch& L = p->launches[k];
        c->rec_head = k <= fin && fin < p->launches.size();
        HIPERR(c->timed(L.cls, L.fine, L.bytes, [&]() {
            if (L.kind == BK_SUBTREE) return launch_batch_subtree(L.dt, p->dev + L.off, L.count, L.lds, c->stream);
            const int32_t* tm = p->tmap_dev + L.toff;
            if (L.kind == BK_FUSED)
                return launch_batch_fused(L.dt, L.flags, L.V, p->dev + L.off, tm, L.total, L.blocks, c->stream);
            return launch_batch(L.kind, L.dt, L.flags, p->dev + L.off, tm, L.count, L.total, L.blocks, c->stream);
        }));
    }
    c->rec_head = false;
    return hipSuccess;
}

// Enqueue a plan: replay its captured graph (captured on first use) or launch.
hipError_t run_plan(lap_ctx* c, lap_ctx::Plan* p, bool graph) {
    // capture a plan only once it is reused (a serving tick's active set
    // changes often; a fixed batch replays the same plans every cycle)
    if (graph && ++p->uses >= 2 && c->stream != nullptr && !c->timing) {
        if (!p->graph) {
            HIPERR(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            hipError_t e = run_plan_launches(c, p);
            hipGraph_t tmp = nullptr;
            hipError_t e2 = hipStreamEndCapture(c->stream, &tmp);
            if (e != hipSuccess) return e;
            if (e2 != hipSuccess) return e2;
            e = hipGraphInstantiate(&p->graph, tmp, nullptr, nullptr, 0);
            hipGraphDestroy(tmp);
            HIPERR(e);
        }
        return hipGraphLaunch(p->graph, c->stream);
    }
    return run_plan_launches(c, p);
}

lap_status batch_reserve(lap_ctx* c, int count) {
    if (count <= c->batch_cap) return LAP_OK;
    int cap = std::max(count, 2 * c->batch_cap);
    hipStreamSynchronize(c->stream);   // the old tables may still be in use by queued work
    if (c->batch_ptrs) c->arena.release(c->batch_ptrs);
    if (c->batch_ctrl) c->arena.release(c->batch_ctrl);
    if (c->copy_dev) c->arena.release(c->copy_dev);
    if (c->batch_host) hipHostFree(c->batch_host);
    c->batch_ptrs = (Ctrl**)c->arena.alloc((size_t)cap * sizeof(Ctrl*));
    c->batch_ctrl = (Ctrl*)c->arena.alloc((size_t)cap * sizeof(Ctrl));
    c->copy_dev = (CopyItem*)c->arena.alloc((size_t)cap * sizeof(CopyItem));
    c->batch_host = nullptr;
    c->batch_cap = 0;
    if (!c->batch_ptrs || !c->batch_ctrl || !c->copy_dev) return fail(LAP_ENOMEM, "arena cannot hold the batch tables");
    HIPCHK(hipHostMalloc((void**)&c->batch_host, (size_t)2 * cap * sizeof(Ctrl), hipHostMallocDefault));
    c->batch_cap = cap;
    return LAP_OK;
}

// Read the control blocks of `gs` (one gather kernel, one copy, one sync).
lap_status batch_read(lap_ctx* c, const std::vector<lap_grid*>& gs, std::vector<Ctrl>& out) {
    const int n = (int)gs.size();
    out.resize(n);
    if (n == 0) return LAP_OK;
    lap_status st = batch_reserve(c, n);
    if (st != LAP_OK) return st;
    c->batch_ptrs_host.resize(n);
    for (int k = 0; k < n; ++k) c->batch_ptrs_host[k] = gs[k]->ctrl;
    HIPCHK(hipMemcpyAsync(c->batch_ptrs, c->batch_ptrs_host.data(), (size_t)n * sizeof(Ctrl*),
                          hipMemcpyHostToDevice, c->stream));
    HIPCHK(launch_gather_ctrl(c->batch_ptrs, c->batch_ctrl, n, c->stream));
    HIPCHK(hipMemcpyAsync(c->batch_host, c->batch_ctrl, (size_t)n * sizeof(Ctrl), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    std::memcpy(out.data(), c->batch_host, (size_t)n * sizeof(Ctrl));
    return LAP_OK;
}

}  // namespace

extern "C" lap_status lap_solve_batch(lap_ctx* c, lap_grid* const* grids, int32_t count, const lap_opts* o,
                                      lap_info* infos) {
    if (!c || !o || (count > 0 && !grids)) return fail(LAP_EINVAL, "NULL argument");
    if (count < 0) return fail(LAP_EINVAL, "count must be >= 0");
    if (is_paper_method(o->method))
        return fail(LAP_EINVAL, "the paper-order methods solve one grid at a time (lap_solve)");
    if (o->fmg) return fail(LAP_EINVAL, "the full multigrid start runs on one grid at a time (lap_solve)");
    const double t0 = now_s();
    for (int k = 0; k < count; ++k) {
        if (!grids[k] || grids[k]->ctx != c) return fail(LAP_EINVAL, "grid does not belong to this context");
        for (int q = 0; q < k; ++q)
            if (grids[q] == grids[k]) return fail(LAP_EINVAL, "a grid appears twice in the batch");
        lap_status st = validate_opts(grids[k], *o);
        if (st != LAP_OK) return st;
    }
    lap_opts po = *o;
    po.use_graph = 0;   // per-grid graphs are not used; the merged plans have their own
    for (int k = 0; k < count; ++k) {
        lap_status st = prepare(grids[k], po, false);
        if (st != LAP_OK) return st;
    }
    if (count > 0) {   // all control blocks reset in one launch
        lap_status st = batch_reserve(c, count);
        if (st != LAP_OK) return st;
        c->batch_ptrs_host.resize(count);
        for (int k = 0; k < count; ++k) c->batch_ptrs_host[k] = grids[k]->ctrl;
        HIPCHK(hipMemcpyAsync(c->batch_ptrs, c->batch_ptrs_host.data(), (size_t)count * sizeof(Ctrl*),
                              hipMemcpyHostToDevice, c->stream));
        HIPCHK(launch_ctrl_init_many(c->batch_ptrs, count, o->tol, o->stop, o->max_iter, ctrl_step(*o), c->stream));
    }
    // every grid stays in the plan until all are done (a finished grid's
    // tiles exit at its control block), so the plans and graphs are reused.
    // Rounds are enqueued one ahead: after enqueueing round r the host reads
    // the control blocks as they stood after round r-1 (gathered into pinned
    // memory behind it), so the device never waits for the host.
    std::vector<lap_grid*> all(grids, grids + count);
    std::vector<int> steps(count, 0);
    std::vector<char> known(count, 0);
    std::vector<Ctrl> final_ctrl(count);
    int remaining = count;
    const int rounds = max_steps(*o) + 1;
    // kernel timing: each round is a step of one timed solve; the launches
    // after the stopping tests that ended the last grids exited at once and
    // are dropped from the statistics
    c->rec_solve = c->timing ? c->solve_serial++ : -1;
    c->safe_step = 0;
    int decided = -1;   // the round after which every grid was done
    auto absorb = [&](int r) -> lap_status {
        HIPCHK(hipEventSynchronize(c->poll_ev[r & 1]));
        const Ctrl* hs = c->batch_host + (size_t)(r & 1) * c->batch_cap;
        for (int k = 0; k < count; ++k)
            if (!known[k]) {
                final_ctrl[k] = hs[k];   // the last state seen, final once done
                if (hs[k].done) {
                    known[k] = 1;
                    --remaining;
                }
            }
        if (remaining == 0 && decided < 0) decided = r;
        if (remaining > 0) c->safe_step = r + 1;
        return LAP_OK;
    };
    int r = 0;
    for (; r < rounds && remaining > 0 && decided < 0; ++r) {
        lap_ctx::Plan* p = nullptr;
        c->rec_step = r;
        for (int k = 0; k < count; ++k) steps[k] = r;
        lap_status st = get_plan(c, all, steps, *o, &p);
        if (st != LAP_OK) return st;
        hipError_t e = run_plan(c, p, o->use_graph != 0);
        if (e != hipSuccess) return fail(LAP_EHIP, std::string("batch launch: ") + hipGetErrorString(e));
        for (lap_grid* g : all) g->step_idx = r + 1;
        HIPCHK(launch_gather_ctrl(c->batch_ptrs, c->batch_ctrl, count, c->stream));
        HIPCHK(hipMemcpyAsync(c->batch_host + (size_t)(r & 1) * c->batch_cap, c->batch_ctrl,
                              (size_t)count * sizeof(Ctrl), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipEventRecord(c->poll_ev[r & 1], c->stream));
        if (r >= 1) {
            st = absorb(r - 1);
            if (st != LAP_OK) return st;
        }
    }
    if (r >= 1 && decided < 0) {
        lap_status st = absorb(r - 1);
        if (st != LAP_OK) return st;
    }
    if (c->timing && decided >= 0) c->drop_speculative(c->rec_solve, decided);
    c->rec_solve = -1;
    // results that ended in the second buffer come back in one launch
    c->copy_host.clear();
    for (int k = 0; k < count; ++k) {
        lap_grid* g = grids[k];
        const Ctrl& h = final_ctrl[k];
        if (result_buffer(g, *o, h) == 1)
            c->copy_host.push_back({(const double2*)g->psi[1], (double2*)g->psi[0], (size_t)g->n * g->P / 2});
        if (o->method == LAP_ADI) g->psi1_stale = true;
    }
    if (!c->copy_host.empty()) {
        HIPCHK(hipMemcpyAsync(c->copy_dev, c->copy_host.data(), c->copy_host.size() * sizeof(CopyItem),
                              hipMemcpyHostToDevice, c->stream));
        HIPCHK(launch_copy_many(c->copy_dev, (int)c->copy_host.size(), c->stream));
    }
    lap_status worst = LAP_OK;
    for (int k = 0; k < count; ++k) {
        lap_status st = finish(grids[k], *o, final_ctrl[k], t0, infos ? &infos[k] : nullptr);
        if (st != LAP_OK && worst == LAP_OK) worst = st;
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    return worst;
}

extern "C" lap_status lap_batch_step(lap_ctx* c, lap_grid* const* grids, int32_t count, int32_t precision,
                                     int32_t nsteps, int32_t* done_host, lap_info* infos) {
    if (!c || (count > 0 && (!grids || !done_host))) return fail(LAP_EINVAL, "NULL argument");
    if (precision != LAP_FP64 && precision != LAP_MIXED) return fail(LAP_EINVAL, "unknown precision");
    if (nsteps < 1) return fail(LAP_EINVAL, "steps must be >= 1");
    const double t0 = now_s();
    std::vector<lap_grid*> active;
    std::vector<int> steps;
    lap_opts o;
    lap_opts_default(&o);
    o.method = LAP_MG;
    o.precision = precision;
    o.max_iter = 1000;
    o.use_graph = 1;
    for (int k = 0; k < count; ++k) {
        lap_grid* g = grids[k];
        if (!g || g->ctx != c) return fail(LAP_EINVAL, "grid does not belong to this context");
        for (int q = 0; q < k; ++q)
            if (grids[q] == g) return fail(LAP_EINVAL, "a grid appears twice in the batch");
        done_host[k] = 0;
        if (g->batch_started && g->batch_done) {
            done_host[k] = 1;
            continue;
        }
        if (!g->batch_started) {
            lap_opts go = o;
            go.tol = g->tol;
            go.omega = g->batch_omega;
            go.use_graph = 0;
            lap_status st = validate_opts(g, go);
            if (st != LAP_OK) return st;
            st = prepare(g, go);
            if (st != LAP_OK) return st;
            g->batch_opts = go;
            g->batch_started = true;
            g->batch_done = false;
            g->batch_t0 = t0;
        }
        active.push_back(g);
        steps.push_back(g->step_idx);
    }
    for (int t = 0; t < nsteps && !active.empty(); ++t) {
        // the stopping tolerance lives in each grid's control block, so grids
        // with different tolerances share one plan
        lap_ctx::Plan* p = nullptr;
        lap_status st = get_plan(c, active, steps, o, &p, true);
        if (st != LAP_OK) return st;
        hipError_t e = run_plan(c, p, true);
        if (e != hipSuccess) return fail(LAP_EHIP, std::string("batch launch: ") + hipGetErrorString(e));
        for (size_t k = 0; k < active.size(); ++k) steps[k] = ++active[k]->step_idx;
    }
    std::vector<Ctrl> hs;
    lap_status st = batch_read(c, active, hs);
    if (st != LAP_OK) return st;
    lap_status worst = LAP_OK;
    for (size_t k = 0; k < active.size(); ++k) {
        lap_grid* g = active[k];
        const int idx = (int)(std::find(grids, grids + count, g) - grids);
        if (hs[k].done) {
            g->batch_done = true;
            done_host[idx] = 1;
            st = fixup(g, g->batch_opts, hs[k]);
            if (st != LAP_OK) return st;
            st = finish(g, g->batch_opts, hs[k], g->batch_t0, infos ? &infos[idx] : nullptr);
            if (st != LAP_OK && worst == LAP_OK) worst = st;
        } else if (infos) {
            infos[idx].iterations = hs[k].iters;
            infos[idx].status = LAP_ENOTCONV;
            infos[idx].rel_res_l2 = hs[k].rel;
            infos[idx].res_l2 = hs[k].res_l2;
            infos[idx].res_linf = hs[k].res_inf;
            infos[idx].res0_l2 = hs[k].r0;
            infos[idx].seconds = now_s() - g->batch_t0;
        }
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    return worst;
}

// ------------------------------------------------------------------ autotuner
extern "C" int32_t lap_size_class(int32_t m, int32_t n) {
    if (m < 3 || n < 3) return -1;
    return size_class((size_t)(m - 2) * (size_t)(n - 2));
}

static lap_status tiling_args_ok(lap_ctx* c, int32_t cls, int32_t dtype, int32_t sc) {
    if (!c) return fail(LAP_EINVAL, "ctx is NULL");
    if (cls < 0 || cls >= KC_COUNT) return fail(LAP_EINVAL, "unknown kernel class");
    if (dtype != 0 && dtype != 1) return fail(LAP_EINVAL, "dtype must be 0 or 1");
    if (sc < 0 || sc >= kSizeClasses) return fail(LAP_EINVAL, "size class must be 0..7");
    return LAP_OK;
}

extern "C" lap_status lap_ctx_set_tiling(lap_ctx* c, int32_t cls, int32_t dtype, int32_t sc, int32_t V, int32_t ty,
                                         int32_t target) {
    lap_status st = tiling_args_ok(c, cls, dtype, sc);
    if (st != LAP_OK) return st;
    if (V != 1 && V != 2 && V != 4) return fail(LAP_EINVAL, "V must be 1, 2 or 4");
    if (ty != 0 && (ty < 2 || ty % 2)) return fail(LAP_EINVAL, "ty must be 0 (auto) or an even number >= 2");
    if (ty == 0 && target < 64) return fail(LAP_EINVAL, "auto tiling needs target_waves >= 64");
    c->tileV[sc][cls][dtype] = V;
    c->tileTY[sc][cls][dtype] = ty;
    c->tileT[sc][cls][dtype] = ty == 0 ? target : 0;
    invalidate_cached(c);
    return LAP_OK;
}

extern "C" lap_status lap_ctx_set_subtree(lap_ctx* c, int64_t max_nodes) {
    if (!c) return fail(LAP_EINVAL, "ctx is NULL");
    if (max_nodes < -1) return fail(LAP_EINVAL, "max_nodes must be -1, 0 or a node count");
    c->sub_max_nodes = max_nodes;
    invalidate_cached(c);
    return LAP_OK;
}

extern "C" lap_status lap_ctx_set_fusion(lap_ctx* c, int32_t on) {
    if (!c) return fail(LAP_EINVAL, "ctx is NULL");
    c->fuse = on != 0;
    invalidate_cached(c);
    return LAP_OK;
}

extern "C" lap_status lap_ctx_get_fusion(lap_ctx* c, int32_t* on) {
    if (!c) return fail(LAP_EINVAL, "ctx is NULL");
    if (on) *on = c->fuse ? 1 : 0;
    return LAP_OK;
}

extern "C" lap_status lap_ctx_get_subtree(lap_ctx* c, int64_t* max_nodes, int32_t* lds_bytes) {
    if (!c) return fail(LAP_EINVAL, "ctx is NULL");
    if (max_nodes) *max_nodes = c->sub_max_nodes;
    if (lds_bytes) *lds_bytes = c->lds_max;
    return LAP_OK;
}

extern "C" lap_status lap_ctx_get_tiling(lap_ctx* c, int32_t cls, int32_t dtype, int32_t sc, int32_t* V, int32_t* ty,
                                         int32_t* target) {
    lap_status st = tiling_args_ok(c, cls, dtype, sc);
    if (st != LAP_OK) return st;
    if (V) *V = c->tileV[sc][cls][dtype];
    if (ty) *ty = c->tileTY[sc][cls][dtype];
    if (target) *target = c->tileT[sc][cls][dtype];
    return LAP_OK;
}

namespace {
struct TuneBufs {
    void* u[2];
    void* f;
    void* ec;
    void* bc;
    void* rhs32;
    void* e32;
    double* partials;
};

template <typename T>
hipError_t tune_launch(lap_ctx* c, int cls, const Tiling& t, int m, int n, int P, int Pc, const TuneBufs& B,
                       int flags) {
    const Coef k = coef(1.0 / (m - 1), 1.0 / (n - 1));
    const int mc = (m - 1) / 2 + 1, nc = (n - 1) / 2 + 1;
    if (cls == KC_SWEEP || cls == KC_SWEEP_PROLONG) {
        SweepArgs<T> a{};
        a.uin = (const T*)B.u[0];
        a.uout = (T*)B.u[1];
        a.f = (flags & SW_F) ? (const T*)B.f : nullptr;
        a.ec = (const T*)B.ec;
        a.partials = B.partials;
        a.m = m; a.n = n; a.P = P; a.mc = mc; a.nc = nc; a.Pc = Pc;
        a.cx = (T)k.cx; a.cy = (T)k.cy; a.d = (T)k.d; a.inv_d = (T)k.inv_d; a.omega = (T)1.0;
        a.tl = t;
        return launch_sweep<T>(a, flags | (cls == KC_SWEEP_PROLONG ? SW_PROLONG : 0), c->stream);
    }
    if (cls == KC_PRE || cls == KC_TWO || cls == KC_TWO_PLAIN || cls == KC_FOUR) {
        SweepArgs<T> a{};
        a.uin = (const T*)B.u[0];
        a.uout = (T*)B.u[1];
        a.f = (flags & SW_F) ? (const T*)B.f : nullptr;
        a.ec = (const T*)B.ec;
        a.bc = (T*)B.bc;
        a.m = m; a.n = n; a.P = P; a.mc = mc; a.nc = nc; a.Pc = Pc;
        a.cx = (T)k.cx; a.cy = (T)k.cy; a.d = (T)k.d; a.inv_d = (T)k.inv_d; a.omega = (T)1.0;
        a.tl = t;
        return launch_fused<T>(a, flags, c->stream);
    }
    if (cls == KC_RESTRICT) {
        RestrictArgs<T> a{};
        a.u = (const T*)B.u[0]; a.f = (const T*)B.f; a.bc = (T*)B.bc;
        a.m = m; a.n = n; a.P = P; a.mc = mc; a.nc = nc; a.Pc = Pc;
        a.cx = (T)k.cx; a.cy = (T)k.cy; a.d = (T)k.d; a.tl = t;
        return launch_restrict<T>(a, c->stream);
    }
    if (cls == KC_RESIDUAL) {
        ResidualArgs<T> a{};
        a.u = (const T*)B.u[0]; a.f = (const T*)B.f; a.partials = B.partials;
        a.m = m; a.n = n; a.P = P; a.cx = (T)k.cx; a.cy = (T)k.cy; a.d = (T)k.d; a.tl = t;
        return launch_residual<T>(a, c->stream);
    }
    if (cls == KC_DEFECT) {
        DefectArgs a{};
        a.psi_in = (const double*)B.u[0]; a.psi_out = (double*)B.u[1]; a.e = (const float*)B.e32;
        a.f = (const double*)B.f; a.rhs = (float*)B.rhs32; a.partials = B.partials;
        a.m = m; a.n = n; a.P = P; a.cx = k.cx; a.cy = k.cy; a.d = k.d; a.tl = t;
        return launch_defect(a, c->stream);
    }
    return hipErrorInvalidValue;
}
}  // namespace

extern "C" lap_status lap_autotune(lap_ctx* c, int32_t m, int32_t n, int32_t reps, char* report, size_t report_bytes) {
    if (!c) return fail(LAP_EINVAL, "ctx is NULL");
    if (m < 5 || n < 5 || m % 2 == 0 || n % 2 == 0) return fail(LAP_EINVAL, "autotune needs odd m, n >= 5");
    if (reps < 1) reps = 1;
    const int sc = size_class((size_t)(m - 2) * (size_t)(n - 2));
    const int P = pitch_of(m);
    const int mc = (m - 1) / 2 + 1, nc = (n - 1) / 2 + 1, Pc = pitch_of(mc);
    const size_t fine = (size_t)n * P * 8, coarse = (size_t)nc * Pc * 8;
    std::vector<void*> held;
    auto A = [&](size_t b) -> void* {
        void* p = c->arena.alloc(b);
        if (p) held.push_back(p);
        return p;
    };
    TuneBufs B{};
    B.u[0] = A(fine);
    B.u[1] = A(fine);
    B.f = A(fine);
    B.ec = A(coarse);
    B.bc = A(coarse);
    B.rhs32 = A(fine / 2);
    B.e32 = A(fine / 2);
    B.partials = (double*)A(max_tiles(m, n) * 16);
    auto release = [&]() {
        hipStreamSynchronize(c->stream);
        for (void* p : held) c->arena.release(p);
    };
    if (held.size() != 8) {
        release();
        return fail(LAP_ENOMEM, "arena cannot hold the autotune buffers");
    }
    for (void* p : held) {
        const size_t off = (size_t)((char*)p - c->arena.base);
        if (hipMemsetAsync(p, 0, c->arena.used_[off], c->stream) != hipSuccess) {
            release();
            return fail(LAP_EHIP, "hipMemsetAsync failed");
        }
    }
    // Levels whose arrays are large enough to live in HBM during a V-cycle
    // are timed from a cold cache: before every timed launch a copy through
    // a buffer of twice the 256 MB Infinity Cache evicts the candidate's
    // data, so halo re-reads cost what they cost in the solver.  (Timed warm,
    // back to back, a 4097^2 level stays in that cache and thin row chunks
    // look free.)  Skipped when the arena cannot hold the buffer.
    constexpr size_t kFlushBytes = (size_t)512 << 20;
    void* flush = fine >= ((size_t)16 << 20) ? c->arena.alloc(kFlushBytes) : nullptr;
    auto release_flush = [&]() {
        if (flush) {
            hipStreamSynchronize(c->stream);
            c->arena.release(flush);
            flush = nullptr;
        }
    };
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        release_flush();
        release();
        return fail(LAP_EHIP, "hipEventCreate failed");
    }
    struct Cand { int V, ty, tgt; };
    std::vector<Cand> cands;
    for (int V : {1, 2, 4}) {
        for (int ty : {2, 4, 8, 16, 32, 64, 128}) cands.push_back({V, ty, 0});
        // one round of waves at 2 to 6 and 8 waves per SIMD, and two at 8
        // (a pass whose waves fill the device exactly once avoids a partly
        // occupied last round: 8193^2 post pass 276 -> 270 us at 5 per SIMD;
        // passes of 129 to 156 registers hold at most 3 waves per SIMD)
        for (int q : {2, 3, 4, 5, 6}) cands.push_back({V, 0, c->wave_cap * q / 8});
        cands.push_back({V, 0, c->wave_cap});
        cands.push_back({V, 0, 2 * c->wave_cap});
    }
    std::string js = "{\"m\": " + std::to_string(m) + ", \"n\": " + std::to_string(n) + ", \"size_class\": " +
                     std::to_string(sc) + ", \"wave_cap\": " + std::to_string(c->wave_cap) + ", \"best\": [";
    const char* names[KC_COUNT] = {"sweep",    "sweep_prolong", "restrict", "defect", "coarse",    "finalize",
                                   "adi_rows", "adi_cols",      "residual", "subtree", "pre",      "two",
                                   "two_plain", "paper",        "four"};
    // the variant each class is timed on: pre-smoothing from zero with the
    // restriction (coarse levels, FP32 level 0), post-smoothing with the
    // prolongation (with and without a right-hand side, as the one-sweep kernel)
    auto base_flags = [](int cls) {
        if (cls == KC_PRE) return (int)(SW_RESTRICT | SW_TWO | SW_ZERO);
        if (cls == KC_TWO) return (int)(SW_TWO | SW_PROLONG);
        if (cls == KC_TWO_PLAIN) return (int)SW_TWO;
        if (cls == KC_FOUR) return (int)(SW_FOUR | SW_PROLONG | SW_RESTRICT | SW_RDIFF);
        return 0;
    };
    bool first = true;
    lap_status result = LAP_OK;
    for (int cls : {(int)KC_SWEEP, (int)KC_SWEEP_PROLONG, (int)KC_RESTRICT, (int)KC_RESIDUAL, (int)KC_DEFECT,
                    (int)KC_PRE, (int)KC_TWO, (int)KC_TWO_PLAIN, (int)KC_FOUR}) {
        for (int dt = 0; dt < 2; ++dt) {
            if ((cls == KC_DEFECT || cls == KC_TWO_PLAIN) && dt == 1) continue;   // FP64 only
            if (cls == KC_FOUR && dt == 0) continue;                              // FP32 only
            double best = 1e30;
            Cand bc{2, 0, c->wave_cap};
            for (const Cand& cd : cands) {
                const int H = (cls == KC_PRE || cls == KC_TWO || cls == KC_TWO_PLAIN || cls == KC_FOUR)
                                  ? fused_halo(base_flags(cls))
                                  : 2;
                const Tiling t = make_tiling(m, n, cd.V, cd.ty, cd.tgt, H);
                double total = 0.0;
                for (int fl0 : {0, (int)SW_F}) {
                    if (fl0 == 0 && cls != KC_SWEEP && cls != KC_TWO && cls != KC_TWO_PLAIN) continue;
                    if (fl0 == 0 && (cls == KC_PRE || cls == KC_FOUR)) continue;
                    const int fl = fl0 | base_flags(cls);
                    auto go = [&]() {
                        return dt == 0 ? tune_launch<double>(c, cls, t, m, n, P, Pc, B, fl)
                                       : tune_launch<float>(c, cls, t, m, n, P, Pc, B, fl);
                    };
                    hipError_t e = go();
                    double sum = 0.0;
                    if (flush) {
                        for (int r = 0; r < reps && e == hipSuccess; ++r) {
                            e = launch_stream_copy(flush, (char*)flush + kFlushBytes / 2, kFlushBytes / 2, 4096,
                                                   c->stream);
                            if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
                            if (e == hipSuccess) e = go();
                            if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
                            if (e == hipSuccess) e = hipEventSynchronize(e1);
                            float ms = 0.f;
                            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                            sum += ms;
                        }
                    } else {
                        if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
                        for (int r = 0; r < reps && e == hipSuccess; ++r) e = go();
                        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
                        if (e == hipSuccess) e = hipEventSynchronize(e1);
                        float ms = 0.f;
                        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                        sum = ms;
                    }
                    if (e != hipSuccess) {
                        result = fail(LAP_EHIP, std::string("autotune launch: ") + hipGetErrorString(e));
                        break;
                    }
                    total += sum / reps;
                }
                if (result != LAP_OK) break;
                if (total < best) {
                    best = total;
                    bc = cd;
                }
            }
            if (result != LAP_OK) break;
            c->tileV[sc][cls][dt] = bc.V;
            c->tileTY[sc][cls][dt] = bc.ty;
            c->tileT[sc][cls][dt] = bc.tgt;
            char buf[256];
            snprintf(buf, sizeof buf,
                     "%s{\"kernel\": \"%s\", \"class\": %d, \"dtype\": \"%s\", \"V\": %d, \"ty\": %d, \"target_waves\": %d, "
                     "\"ms\": %.5f}",
                     first ? "" : ", ", names[cls], cls, dt == 0 ? "f64" : "f32", bc.V, bc.ty, bc.tgt, best);
            js += buf;
            first = false;
        }
        if (result != LAP_OK) break;
    }
    js += "], \"cold_cache\": ";
    js += flush ? "true}" : "false}";
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    release_flush();
    release();
    if (result != LAP_OK) return result;
    // cached graphs and batch plans hold the old tilings
    invalidate_cached(c);
    if (report && report_bytes > 0) {
        std::strncpy(report, js.c_str(), report_bytes - 1);
        report[report_bytes - 1] = 0;
    }
    return LAP_OK;
}

// ------------------------------------------------------------- stream copy
extern "C" lap_status lap_op_stream_copy(const void* src, void* dst, size_t bytes, int32_t blocks, void* stream) {
    if (!src || !dst) return fail(LAP_EINVAL, "NULL pointer");
    if (bytes % 16 || ((uintptr_t)src % 16) || ((uintptr_t)dst % 16))
        return fail(LAP_EINVAL, "bytes and pointers must be multiples of 16");
    if (blocks < 1) return fail(LAP_EINVAL, "blocks must be >= 1");
    HIPCHK(launch_stream_copy(src, dst, bytes, blocks, (hipStream_t)stream));
    return LAP_OK;
}
