// Host side of the C ABI declared in include/fbsde.h, per-point path: validation, workspace carving and
// the launch sequence of Algorithm 1 (forward sweep, then the backward level loop) and of its adjoint.
// The shared-increment form and the persistent batched launch live in their own translation units.
#include "fbsde_host.hpp"
#include "fbsde_kernels.hpp"
#include "fbsde_adjoint.hpp"
#include "fbsde_cgloop.hpp"
#include "fbsde_dual.hpp"
#include "fbsde_coef_adjoint.hpp"

#include <atomic>
#include <cstdlib>
#include <cstring>
#include <map>
#include <functional>
#include <vector>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

using namespace fbsde;
using namespace fbsde::host;

namespace {

// ------------------------------------------------------------------ autotuned launch shapes
using TuneKey = std::tuple<int, int64_t, int64_t, int64_t>;
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int, int>> g_tune;
TuneKey tune_key(const fbsde_problem* pb, int64_t P) { return TuneKey{pb->prec, pb->d, pb->M, P}; }

// ------------------------------------------------------------------ launch timer
// While on, every timed launch (the CG product; the Gram and anchor launches of the literal scheme) is
// bracketed by two events on its own stream (not inside a stream capture).  The events are created on
// first use and reused after each restart.
struct TimedLaunch {
    hipEvent_t a, b;
    bool ok;
    double work;    // algorithmic work of the launch: bytes (CG product) or FP64 flops (literal scheme)
    int kind;       // FBSDE_TIMED_*
};
std::mutex g_lt_mu;
std::atomic<bool> g_lt_on{false};   // read without the lock on every launch, so a stopped timer costs nothing
std::vector<TimedLaunch> g_lt;
size_t g_lt_used = 0;

long lt_begin(hipStream_t st, double work, int kind = FBSDE_TIMED_CG_PRODUCT) {
    if (!g_lt_on.load(std::memory_order_relaxed)) return -1;
    std::lock_guard<std::mutex> lk(g_lt_mu);
    if (!g_lt_on.load(std::memory_order_relaxed)) return -1;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return -1;
    if (g_lt_used == g_lt.size()) {
        TimedLaunch t{nullptr, nullptr, false, 0.0, 0};
        if (hipEventCreate(&t.a) != hipSuccess) return -1;
        if (hipEventCreate(&t.b) != hipSuccess) { (void)hipEventDestroy(t.a); return -1; }
        g_lt.push_back(t);
    }
    const size_t i = g_lt_used++;
    g_lt[i].ok = false;
    g_lt[i].work = work;
    g_lt[i].kind = kind;
    if (hipEventRecord(g_lt[i].a, st) != hipSuccess) return -1;
    return (long)i;
}

void lt_end(long i, hipStream_t st) {
    if (i < 0) return;
    std::lock_guard<std::mutex> lk(g_lt_mu);
    g_lt[(size_t)i].ok = hipEventRecord(g_lt[(size_t)i].b, st) == hipSuccess;
}

}  // namespace

namespace fbsde {
namespace host {
// The share of the chip one CG loop launch asks for: 1 (all of it) unless the calling thread runs one of
// several streams of a batched call (run_tiled sets it for the duration of its worker), where a loop
// sized for the whole chip would keep the other streams' loops out until its level ends.
thread_local int loop_share = 1;

long timer_begin(hipStream_t st, double work, int kind) { return lt_begin(st, work, kind); }
void timer_end(long i, hipStream_t st) { lt_end(i, st); }

bool tuned_shape(const fbsde_problem* pb, int64_t P, int& team, int& nchunk) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const auto it = g_tune.find(tune_key(pb, P));
    if (it == g_tune.end()) return false;
    team = it->second.first;
    nchunk = it->second.second;
    return true;
}
}  // namespace host
}  // namespace fbsde

namespace {

// Buffers of the reverse mode under x-dependent coefficients (after the per-point workspace): the tape
// of the reversal per level (1 / F', |Z|^2, sum Z per particle), the tangent state J (as the state), and
// per particle the Newton adjoint's Z weight, the design adjoint's coefficients and row dots; the x0
// accumulator [P][ld]; Vbar [P][N + 1].
struct CoefAdj {
    void* J;
    double *dydc, *zz, *zs;
    double *zw, *c1, *c2, *c3, *pd, *qd, *n2;
    double *x0acc, *Vbar;
};

struct WS {
    CgCtl* ctl;     // device-side CG loop control (offset 0 of the workspace)
    void* W;
    double *Ya, *Yb, *rn2, *w, *c2;
    double *x, *r, *pv, *qv, *Wbar;
    double *part1, *part2, *part3, *psc, *scal;
    int *iscal, *active;
    double *dK, *drhs;   // the direct dual solve's M x M systems and right-hand sides (plan.dual)
    int* cnt;       // CG arrival counters [P][ncnt]
    int ncnt;
    unsigned long long* queue;   // CG work queues [nq][qcap]
    int nq;
    int64_t qcap;
    bool fixed_buffer;           // the allocation-free entry point: no timer events, device CG loop only
    // x-dependent coefficients (fbsde_solve_coef): the family, V[p][k] of the moment recursion and the
    // mean path's m_k = x0 A[k] + B[k]; null for the constant-coefficient solve
    const CoefArgs* coef = nullptr;
    const double* coefV = nullptr;
    const double* coefA = nullptr;
    const double* coefB = nullptr;
    // a step after the forward sweep that rewrites the terminal values (constant matrix sigma)
    const host::TerminalStep* terminal = nullptr;
    const host::AdjTerminalHooks* adjh = nullptr;   // the same for the reverse mode
    // x-dependent coefficients with a tape: the per-particle tape of the reversal and the reverse mode's
    // buffers (tangent state, design adjoint, variance adjoint); tag_salt tells such a tape apart
    const CoefAdj* cadj = nullptr;
    int tag_salt = 0;
    // tape for the adjoint: per level k (cloud t_{k+1})
    double *tY, *tw, *tax, *tWbar, *tscal;
    int* tag;
    // adjoint work
    double *G, *cbar, *adj;
};

// Carve the workspace (base == nullptr: only count).  Returns bytes.  The loop control comes first and
// the buffers whose size depends on the chunk count (partials, arrival counters) last, so that the tape
// keeps its place whatever launch shape a later call takes.
size_t carve(const Plan& pl, int64_t P, int flags, char* base, WS& ws) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        char* p = base ? base + off : nullptr;
        off += round_up((int64_t)bytes, 256);
        return p;
    };
    const size_t PM = (size_t)P * pl.M, PL = (size_t)P * pl.ld;
    const size_t parts = (size_t)P * pl.nchunk * pl.ld;
    ws.fixed_buffer = false;
    ws.ctl = (CgCtl*)take(sizeof(CgCtl));
    ws.W = take(PM * pl.ld * pl.esz);
    ws.Ya = (double*)take(PM * 8);
    ws.Yb = (double*)take(PM * 8);
    ws.rn2 = (double*)take(PM * 8);
    ws.w = (double*)take(PM * 8);
    ws.c2 = (double*)take(PM * 8);
    ws.x = (double*)take(PL * 8);
    ws.r = (double*)take(PL * 8);
    ws.pv = (double*)take(PL * 8);
    ws.qv = (double*)take(PL * 8);
    ws.Wbar = (double*)take(PL * 8);
    ws.scal = (double*)take((size_t)P * NS * 8);
    ws.iscal = (int*)take((size_t)P * 4 * 4);
    ws.active = (int*)take(64);
    ws.dK = ws.drhs = nullptr;
    if (pl.dual) {
        ws.dK = (double*)take((size_t)P * pl.M * pl.M * 8);
        ws.drhs = (double*)take((size_t)P * pl.M * 8);
    }
    ws.tY = ws.tw = ws.tax = ws.tWbar = ws.tscal = nullptr;
    ws.tag = nullptr;
    ws.G = ws.cbar = ws.adj = nullptr;
    if (flags & FBSDE_WS_TAPE) {
        ws.tY = (double*)take((size_t)pl.N * PM * 8);
        ws.tw = (double*)take((size_t)pl.N * PM * 8);
        ws.tax = (double*)take((size_t)pl.N * PL * 8);
        ws.tWbar = (double*)take((size_t)pl.N * PL * 8);
        ws.tscal = (double*)take((size_t)pl.N * P * NS * 8);
        ws.tag = (int*)take(64);
        ws.G = (double*)take(PM * 8);
        ws.cbar = (double*)take(PM * 8);
        ws.adj = (double*)take((size_t)P * 16 * 8);
    }
    ws.part1 = (double*)take(parts * 8);
    ws.part2 = (double*)take(parts * 8);
    ws.part3 = (double*)take(parts * 8);
    ws.psc = (double*)take((size_t)P * pl.nchunk * 4 * 8);
    ws.ncnt = std::max(1, cg_tree_counters(pl.nchunk));
    ws.cnt = (int*)take((size_t)P * ws.ncnt * 4);
    ws.nq = (int)std::min<int64_t>(CG_MAXQ, std::max<int64_t>(P, 1));
    // a slot for every item the level can produce (its points x chunks x iterations): no slot is reused
    // within a launch, so a producer never waits for a taker
    ws.qcap = (P + ws.nq - 1) / ws.nq * (int64_t)pl.nchunk * (int64_t)pl.maxit;
    ws.queue = (unsigned long long*)take((size_t)ws.nq * ws.qcap * 8);
    return off;
}

// -------------------------------------------------------------------- launch sequences
template <typename S>
void launch_forward(const fbsde_problem* pb, const Plan& pl, int64_t P, const double* x0, S* W, int64_t ldw,
                    double* Y, double* rn2, uint32_t* status, hipStream_t st, const WS* ws = nullptr) {
    const Keys ky = keys_of(pb);
    const double dt = pb->T / (double)pb->N;
    dispatch<S>(pl.Q, pl.TEAM, [&](auto qc, auto tc) {
        constexpr int QQ = decltype(qc)::value, TT = decltype(tc)::value;
        if (ws && ws->coef) {   // x-dependent coefficients: Euler-Maruyama positions, state D_N = X_N - m_N
            CoefArgs cf = *ws->coef;
            cf.Aa = ws->coefA[pl.N];
            cf.Ba = ws->coefB[pl.N];
            hipLaunchKernelGGL((k_forward<S, QQ, TT, true>), dim3(pl.nchunk, (unsigned)P), dim3(Geo<QQ, TT>::BS), 0, st,
                               W, ldw, (int)pl.M, pl.rows_per_chunk, x0, nullptr, pb->gvec, (int)pl.d, pl.ld,
                               (int)pl.N, std::sqrt(dt), pb->s, pb->T, pb->g_kind, pb->gp[0], pb->gp[1], ky.k0, ky.k1,
                               pb->point_base, 0, Y, rn2, status, cf);
        } else {
            hipLaunchKernelGGL((k_forward<S, QQ, TT>), dim3(pl.nchunk, (unsigned)P), dim3(Geo<QQ, TT>::BS), 0, st, W,
                               ldw, (int)pl.M, pl.rows_per_chunk, x0, pb->mu, pb->gvec, (int)pl.d, pl.ld, (int)pl.N,
                               std::sqrt(dt), pb->s, pb->T, pb->g_kind, pb->gp[0], pb->gp[1], ky.k0, ky.k1,
                               pb->point_base, 0, Y, rn2, status, CoefArgs{});
        }
    });
}

template <typename S>
void launch_rownorm(const Plan& pl, int64_t P, const S* W, int64_t ldw, double* rn2, hipStream_t st) {
    dispatch<S>(pl.Q, pl.TEAM, [&](auto qc, auto tc) {
        constexpr int QQ = decltype(qc)::value, TT = decltype(tc)::value;
        hipLaunchKernelGGL((k_rownorm<S, QQ, TT>), dim3(pl.nchunk, (unsigned)P), dim3(Geo<QQ, TT>::BS), 0, st, W,
                           ldw, (int)pl.M, pl.rows_per_chunk, pl.ld, rn2);
    });
}

// Run CG on the per-point systems prepared in ws (x, r, pv, Wbar, scal, iscal, active).
// Returns the number of matvec launches.
// Folds the per-chunk partial vectors of each point into chunk 0 when a point is split over more
// than four chunks; returns how many chunk vectors the per-point finish kernel then sums.
int fold_parts(const Plan& pl, int64_t P, double* a, double* b, double* c, hipStream_t st) {
    if (pl.nchunk <= 4) return pl.nchunk;
    hipLaunchKernelGGL(k_fold_chunks, dim3((unsigned)((pl.ld + 63) / 64), (unsigned)P), dim3(256), 0, st, a, b, c,
                       pl.nchunk, pl.ld);
    return 1;
}

// The CG solve of a level as one launch of the device-side loop (fbsde_cgloop.hpp): every iteration of
// every point, no host round trip.  The loop's grid is what the chip holds at once, or the calling
// thread's share of it (more blocks would only take tickets later); the wait bound is two seconds of the
// device's wall clock.
template <typename S, typename R>
int run_cg_device(const fbsde_problem* pb, const Plan& pl, int64_t P, const S* W, int64_t ldw, const double* w,
                  const double* Wbar, WS& ws, uint32_t* status, hipStream_t st, int& err) {
    const int fixed = pb->cg_fixed_iters;
    const int cap = (fixed > 0) ? fixed : pb->cg_maxit;
    int dev = 0, ncu = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) !=
        hipSuccess || hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) {
        err = FBSDE_EHIP;
        return 0;
    }
    const uint64_t wait_ticks = (uint64_t)std::max(khz, 1000) * 2000ull;
    const int64_t ncnt_total = P * (int64_t)ws.ncnt, nitems = P * (int64_t)pl.nchunk;
    const int64_t nslots = ws.nq * ws.qcap;
    hipLaunchKernelGGL(k_cg_arm,
                       dim3((unsigned)std::min<int64_t>((std::max({ncnt_total, nslots, P}) + 255) / 256, 1024)),
                       dim3(256), 0, st, ws.ctl, ws.queue, ws.nq, ws.qcap, pl.nchunk, ws.cnt, ncnt_total, ws.iscal, P,
                       0);
    dispatch<S>(pl.Q, pl.TEAM, [&](auto qc, auto tc) {
        constexpr int QQ = decltype(qc)::value, TT = decltype(tc)::value;
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_cg_loop<S, R, QQ, TT>),
                                                         Geo<QQ, TT>::BS, 0) != hipSuccess)
            per_cu = 1;
        const int64_t slots = std::max<int64_t>(1, (int64_t)std::max(per_cu, 1) * ncu / std::max(loop_share, 1));
        const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(nitems, slots));
        const long tl = ws.fixed_buffer ? -1 : lt_begin(st, 0.0, FBSDE_TIMED_CG_LOOP);
        hipLaunchKernelGGL((k_cg_loop<S, R, QQ, TT>), dim3((unsigned)grid), dim3(Geo<QQ, TT>::BS), 0, st, W, ldw,
                           (int)pl.M, pl.rows_per_chunk, pl.nchunk, pl.ld, pb->s, w, Wbar, ws.x, ws.r, ws.pv, ws.qv,
                           ws.scal, NS, ws.iscal, ws.part1, ws.psc, ws.ctl, ws.queue, ws.nq, ws.qcap, ws.active,
                           ws.cnt, ws.ncnt, cg_rtol_of(pb) * cg_rtol_of(pb), std::min(cap, pb->cg_maxit), status,
                           wait_ticks);
        lt_end(tl, st);
    });
    hipLaunchKernelGGL(k_cg_check, dim3((unsigned)std::min<int64_t>((P + 255) / 256, 1024)), dim3(256), 0, st,
                       ws.ctl, ws.iscal, P, (int64_t)pl.M, (int64_t)pl.d * (int64_t)pl.esz, status);
    err = last_error();
    return cap;
}

// The host-driven loop: three launches per iteration and a poll of the active-point count every eight
// (kept as a diagnostic alternative, selected by the environment variable FBSDE_CG_HOST_LOOP=1).
bool host_cg_loop() {
    const char* e = std::getenv("FBSDE_CG_HOST_LOOP");
    return e && e[0] == '1';
}

template <typename S, typename R = S>
int run_cg(const fbsde_problem* pb, const Plan& pl, int64_t P, const S* W, int64_t ldw, const double* w,
           const double* Wbar, WS& ws, uint32_t* status, hipStream_t st, int& err) {
    if (ws.fixed_buffer || !host_cg_loop()) return run_cg_device<S, R>(pb, pl, P, W, ldw, w, Wbar, ws, status, st, err);
    const int fixed = pb->cg_fixed_iters;
    const int cap = (fixed > 0) ? fixed : pb->cg_maxit;
    const int poll = 8;
    int it = 0;
    for (; it < cap; ++it) {
        const long tl = lt_begin(st, (double)P * (double)pl.M * (double)pl.d * (double)sizeof(S));
        dispatch<S>(pl.Q, pl.TEAM, [&](auto qc, auto tc) {
            constexpr int QQ = decltype(qc)::value, TT = decltype(tc)::value;
            hipLaunchKernelGGL((k_matvec<S, R, QQ, TT>), dim3(pl.nchunk, (unsigned)P), dim3(Geo<QQ, TT>::BS), 0, st,
                               W, ldw, (int)pl.M, pl.rows_per_chunk, pl.nchunk, pl.ld, pb->s, w, ws.pv, ws.scal, NS,
                               ws.iscal, ws.part1, ws.psc);
        });
        lt_end(tl, st);
        const int vc = fold_parts(pl, P, ws.part1, nullptr, nullptr, st);
        hipLaunchKernelGGL(k_cg_update, dim3((unsigned)P), dim3(256), 0, st, ws.part1, ws.psc, pl.nchunk, vc, pl.ld,
                           pb->s, Wbar, ws.x, ws.r, ws.pv, ws.qv, ws.scal, NS, ws.iscal,
                           cg_rtol_of(pb) * cg_rtol_of(pb), std::min(cap, pb->cg_maxit), ws.active, status);
        if (fixed <= 0 && (it + 1) % poll == 0) {
            int active = 0;
            if (hipMemcpyAsync(&active, ws.active, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess) {
                err = FBSDE_EHIP;
                return it + 1;
            }
            if (active <= 0) { ++it; break; }
        }
    }
    err = last_error();
    return it;
}

// The largest CG iteration count over the points of the level just solved (iscal[p][0]); the
// launches after the last point converged exit at once and are not counted.  Synchronises.
int point_iters_max(const WS& ws, int64_t P, hipStream_t st, int& err) {
    std::vector<int> h((size_t)P * 4);
    if (hipMemcpyAsync(h.data(), ws.iscal, h.size() * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        err = FBSDE_EHIP;
        return 0;
    }
    int m = 0;
    for (int64_t p = 0; p < P; ++p) m = std::max(m, h[(size_t)p * 4]);
    return m;
}

// One backward level: regression of Y_next on the cloud W (at t_{k+1}); leaves alpha_x in ws.x,
// alpha / zz in ws.scal, and returns the number of CG iterations.
template <typename S>
int run_level(const fbsde_problem* pb, const Plan& pl, int64_t P, int k, const S* W, int64_t ldw,
              const double* Y_next, const double* rn2, double* w_out, double* Wbar_out, WS& ws,
              double* alpha_out, double* alpha_x_out, uint32_t* status, hipStream_t st, int& err, int warm = 0) {
    const double dt = pb->T / (double)pb->N;
    const double t_next = (double)(k + 1) * dt;
    const double s2 = pb->s * pb->s;
    const double eps2 = (pb->eps_h > 0.0) ? pb->eps_h * pb->eps_h * s2 * t_next * (double)pl.d : 0.0;
    const double lam = pb->ridge_rel * s2 * t_next;
    // x-dependent coefficients: the point's own bandwidth h^2 V_{k+1} and ridge ridge_rel V_{k+1} / d
    const double* vt = ws.coef ? ws.coefV + (k + 1) : nullptr;
    const int vstride = (int)pl.N + 1;
    hipLaunchKernelGGL(k_weights, dim3((unsigned)P), dim3(256), 0, st, rn2, Y_next, (int)pl.M, s2, eps2, w_out,
                       ws.c2, ws.scal, NS, ws.active, (int)P, warm, vt, vstride, pb->eps_h * pb->eps_h);
    // a rank-deficient design (M <= d + 1) in FP32C: FP64 arithmetic on the FP32 state in the moments and
    // the CG product, whose FP32 rounding would otherwise reach the ridge-only null space of the design
    // (where the solution carries it with weight 1/lam)
    const bool r64 = !std::is_same<S, double>::value && pl.M <= pl.d + 1;
    dispatch<S>(pl.Q, pl.TEAM, [&](auto qc, auto tc) {
        constexpr int QQ = decltype(qc)::value, TT = decltype(tc)::value;
        if (r64)
            hipLaunchKernelGGL((k_moments<S, double, QQ, TT>), dim3(pl.nchunk, (unsigned)P), dim3(Geo<QQ, TT>::BS), 0,
                               st, W, ldw, (int)pl.M, pl.rows_per_chunk, pl.nchunk, pl.ld, w_out, ws.c2, ws.x, ws.scal,
                               NS, warm, ws.part1, ws.part2, ws.part3, ws.psc);
        else
            hipLaunchKernelGGL((k_moments<S, S, QQ, TT>), dim3(pl.nchunk, (unsigned)P), dim3(Geo<QQ, TT>::BS), 0, st,
                               W, ldw, (int)pl.M, pl.rows_per_chunk, pl.nchunk, pl.ld, w_out, ws.c2, ws.x, ws.scal, NS,
                               warm, ws.part1, ws.part2, ws.part3, ws.psc);
    });
    const int vc = fold_parts(pl, P, ws.part1, ws.part2, warm ? ws.part3 : nullptr, st);
    hipLaunchKernelGGL(k_moments_finish, dim3((unsigned)P), dim3(256), 0, st, ws.part1, ws.part2, ws.part3, ws.psc,
                       pl.nchunk, vc, pl.ld, pb->s, lam, warm, Wbar_out, ws.x, ws.r, ws.pv, ws.scal, NS, ws.iscal,
                       ws.active, vt, vstride, pb->ridge_rel / (double)pl.d);
    int iters = 0;
    if (pl.dual) {   // small rank-deficient cloud: the M x M dual system, factored
        hipLaunchKernelGGL((k_dual_gram<S>), dim3((unsigned)P), dim3(256), 0, st, W, ldw, (int)pl.M, (int)pl.d, pl.ld,
                           pb->s, Wbar_out, w_out, Y_next, ws.scal, NS, ws.dK, ws.drhs);
        hipLaunchKernelGGL((k_dual_solve<S>), dim3((unsigned)P), dim3(256), 0, st, ws.dK, ws.drhs, (int)pl.M, W, ldw,
                           (int)pl.d, pl.ld, pb->s, Wbar_out, w_out, ws.x, ws.iscal, status);
        err = last_error();
    } else {
        iters = r64 ? run_cg<S, double>(pb, pl, P, W, ldw, w_out, Wbar_out, ws, status, st, err)
                    : run_cg<S, S>(pb, pl, P, W, ldw, w_out, Wbar_out, ws, status, st, err);
    }
    if (err) return iters;
    hipLaunchKernelGGL(k_level_finish, dim3((unsigned)P), dim3(256), 0, st, ws.x, Wbar_out, pl.ld, (int)pl.d, pb->s,
                       ws.scal, NS, alpha_out, alpha_x_out);
    err = last_error();
    return iters;
}

template <typename S>
void launch_reverse(const fbsde_problem* pb, const Plan& pl, int64_t P, int k, S* W, int64_t ldw, const double* ax,
                    WS& ws, double* Y, double* rn2, uint32_t* status, hipStream_t st, double* dydc = nullptr,
                    const double* scal = nullptr, int shared = 0, const double* x0 = nullptr) {
    const Keys ky = keys_of(pb);
    const double dt = pb->T / (double)pb->N;
    dispatch<S>(pl.Q, pl.TEAM, [&](auto qc, auto tc) {
        constexpr int QQ = decltype(qc)::value, TT = decltype(tc)::value;
        // the particles' positions x0 + t_k mu + s W_k enter f
        if (ws.coef) {   // x-dependent coefficients: the Euler-Maruyama step inverted, per-particle Z
            CoefArgs cf = *ws.coef;
            cf.Aa = ws.coefA[k];
            cf.Ba = ws.coefB[k];
            cf.Ab = ws.coefA[k + 1];
            cf.Bb = ws.coefB[k + 1];
            const int64_t PM = P * pl.M;
            double* zz_t = ws.cadj ? ws.cadj->zz + (size_t)k * PM : nullptr;
            double* zs_t = ws.cadj ? ws.cadj->zs + (size_t)k * PM : nullptr;
            hipLaunchKernelGGL((k_reverse<S, QQ, TT, 3>), dim3(pl.nchunk, (unsigned)P), dim3(Geo<QQ, TT>::BS), 0,
                               st, W, ldw, (int)pl.M, pl.rows_per_chunk, (int)pl.d, pl.ld, k, (k == 0) ? 1 : 0,
                               std::sqrt(dt), pb->s, dt, ax, scal ? scal : ws.scal, NS, fspec_of(pb), pb->newton_iters,
                               ky.k0, ky.k1, pb->point_base, Y, rn2, dydc, status, shared, x0, nullptr, 0.0, cf,
                               zz_t, zs_t);
        } else if (pb->f_kind == FBSDE_F_HJ_SINK)
            hipLaunchKernelGGL((k_reverse<S, QQ, TT, 1>), dim3(pl.nchunk, (unsigned)P), dim3(Geo<QQ, TT>::BS), 0,
                               st, W, ldw, (int)pl.M, pl.rows_per_chunk, (int)pl.d, pl.ld, k, (k == 0) ? 1 : 0,
                               std::sqrt(dt), pb->s, dt, ax, scal ? scal : ws.scal, NS, fspec_of(pb), pb->newton_iters,
                               ky.k0, ky.k1, pb->point_base, Y, rn2, dydc, status, shared, x0, pb->mu, (double)k * dt);
        else if (pb->f_kind == FBSDE_F_LOG_POT)
            hipLaunchKernelGGL((k_reverse<S, QQ, TT, 2>), dim3(pl.nchunk, (unsigned)P), dim3(Geo<QQ, TT>::BS), 0,
                               st, W, ldw, (int)pl.M, pl.rows_per_chunk, (int)pl.d, pl.ld, k, (k == 0) ? 1 : 0,
                               std::sqrt(dt), pb->s, dt, ax, scal ? scal : ws.scal, NS, fspec_of(pb), pb->newton_iters,
                               ky.k0, ky.k1, pb->point_base, Y, rn2, dydc, status, shared, x0, pb->mu, (double)k * dt);
        else
            hipLaunchKernelGGL((k_reverse<S, QQ, TT>), dim3(pl.nchunk, (unsigned)P), dim3(Geo<QQ, TT>::BS), 0, st, W,
                               ldw, (int)pl.M, pl.rows_per_chunk, (int)pl.d, pl.ld, k, (k == 0) ? 1 : 0, std::sqrt(dt),
                               pb->s, dt, ax, scal ? scal : ws.scal, NS, fspec_of(pb), pb->newton_iters, ky.k0, ky.k1,
                               pb->point_base, Y, rn2, dydc, status, shared, nullptr, nullptr, 0.0);
    });
}

int tape_tag(const fbsde_problem* pb, int64_t P) {
    uint64_t h = 1469598103934665603ull;
    const uint64_t v[6] = {(uint64_t)pb->d, (uint64_t)pb->M, (uint64_t)pb->N, (uint64_t)P, (uint64_t)pb->prec,
                           pb->seed ^ ((uint64_t)pb->instance << 32) ^ pb->point_base};
    for (uint64_t x : v) { h ^= x; h *= 1099511628211ull; }
    return (int)(h & 0x7FFFFFFF) | 1;
}

void clear_status_impl(uint32_t* status, int64_t P, hipStream_t st) {
    if (P > 0) hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::min<int64_t>((P + 255) / 256, 1024)), dim3(256), 0,
                                  st, status, P, 0u);
}

template <typename S>
int solve_impl(const fbsde_problem* pb, const Plan& pl, int64_t P, const double* x0, double* u, double* grad,
               uint32_t* status, WS& ws, bool tape, int32_t* cg_iters_out, hipStream_t st, bool reset_counts = true) {
    S* W = (S*)ws.W;
    const int64_t ldw = pl.ld;
    const int64_t PM = P * pl.M, PL = P * (int64_t)pl.ld;
    clear_status(status, P, st);
    // the count of particle rows streamed by CG products starts again with every solve (a batched tile
    // after the first on its arena adds to the count instead)
    hipLaunchKernelGGL(k_cg_arm, dim3(1), dim3(64), 0, st, ws.ctl, nullptr, 0, (int64_t)0, 1, nullptr, (int64_t)0,
                       nullptr, (int64_t)0, reset_counts ? 1 : 0);
    double* Ycur = ws.Ya;
    double* Yk = ws.Yb;
    if (ws.coef)   // x-dependent coefficients: V[p][k] and the mean path's coordinates (r, pv as scratch)
        hipLaunchKernelGGL(k_coef_moments, dim3((unsigned)P), dim3(256), 0, st, x0, (int)pl.d, pl.ld, (int)pl.N,
                           *ws.coef, ws.r, ws.pv, (double*)ws.coefV);
    launch_forward<S>(pb, pl, P, x0, W, ldw, Ycur, ws.rn2, status, st, &ws);
    int err = last_error();
    if (err) return err;
    if (ws.terminal && (err = (*ws.terminal)(W, ldw, Ycur, st))) return err;
    for (int k = (int)pl.N - 1; k >= 0; --k) {
        double* w_k = tape ? ws.tw + (size_t)k * PM : ws.w;
        double* Wbar_k = tape ? ws.tWbar + (size_t)k * PL : ws.Wbar;
        // Warm start from the previous level's slope (Y_{k+1} is the Newton image of a linear model),
        // only when the centred design has full rank (M > d + 1): otherwise A has a (d - M + 1)-fold
        // eigenvalue lam whose eigenspace a cold start never enters, while the previous slope does,
        // and the residual test would then bound the error there only up to a factor 1 / lam.
        const int warm = (k < (int)pl.N - 1 && pl.M > pl.d + 1) ? 1 : 0;
        const int iters = run_level<S>(pb, pl, P, k, W, ldw, Ycur, ws.rn2, w_k, Wbar_k, ws, nullptr, nullptr, status,
                                       st, err, warm);
        if (err) return err;
        if (cg_iters_out) {
            cg_iters_out[k] = point_iters_max(ws, P, st, err);
            if (err) return err;
        }
        (void)iters;
        if (tape) {
            if (hipMemcpyAsync(ws.tax + (size_t)k * PL, ws.x, PL * 8, hipMemcpyDeviceToDevice, st) != hipSuccess ||
                hipMemcpyAsync(ws.tscal + (size_t)k * P * NS, ws.scal, (size_t)P * NS * 8, hipMemcpyDeviceToDevice,
                               st) != hipSuccess)
                return FBSDE_EHIP;
        }
        if (k > 0) {
            double* Yout = tape ? ws.tY + (size_t)k * PM : Yk;
            launch_reverse<S>(pb, pl, P, k, W, ldw, ws.x, ws, Yout, ws.rn2, status, st, ws.c2, nullptr, 0, x0);
            // the coefficient family's tape keeps 1 / F' per particle (c2 itself feeds the next warm start)
            if (tape && ws.cadj &&
                hipMemcpyAsync(ws.cadj->dydc + (size_t)k * PM, ws.c2, PM * 8, hipMemcpyDeviceToDevice, st) != hipSuccess)
                return FBSDE_EHIP;
            if (!tape) std::swap(Ycur, Yk);
            else Ycur = Yout;
        } else {
            hipLaunchKernelGGL(k_outputs, dim3((unsigned)P), dim3(256), 0, st, ws.x, pl.ld, (int)pl.d, ws.scal, NS,
                               fspec_of(pb), pb->T / (double)pb->N, pb->newton_iters, u, grad, status, x0, pb->s,
                               ws.coef ? 1 : 0, ws.coef ? *ws.coef : CoefArgs{});
        }
        err = last_error();
        if (err) return err;
    }
    if (tape) hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, ws.tag, tape_tag(pb, P) ^ ws.tag_salt);
    return last_error();
}

template <typename S>
int backward_impl(const fbsde_problem* pb, const Plan& pl, int64_t P, const double* x0, const double* u_bar,
                  double* x0_bar, double* gp_bar, double* fp_bar, uint32_t* status, WS& ws, int32_t* cg_iters_out,
                  hipStream_t st) {
    S* W = (S*)ws.W;
    const int64_t ldw = pl.ld;
    const int64_t PM = P * pl.M, PL = P * (int64_t)pl.ld;
    const double dt = pb->T / (double)pb->N, sqdt = std::sqrt(dt), s2 = pb->s * pb->s;
    const Keys ky = keys_of(pb);
    const FSpec fs = fspec_of(pb);
    int err = FBSDE_OK;
    for (int k = 0; k < (int)pl.N; ++k) {
        const double lam = pb->ridge_rel * s2 * (double)(k + 1) * dt;
        hipLaunchKernelGGL(k_adj_newton, dim3((unsigned)P), dim3(256), 0, st, ws.G,
                           k > 0 ? ws.tw + (size_t)(k - 1) * PM : nullptr, (int64_t)pl.M, ws.psc, pl.nchunk,
                           k > 0 ? ws.tY + (size_t)k * PM : nullptr, ws.tscal + (size_t)k * P * NS, NS, fs, dt,
                           pb->newton_iters, (int)pl.M, u_bar, ws.cbar, ws.adj, k == 0 ? 1 : 0, 0, status);
        dispatch<S>(pl.Q, pl.TEAM, [&](auto qc, auto tc) {
            constexpr int QQ = decltype(qc)::value, TT = decltype(tc)::value;
            hipLaunchKernelGGL((k_adj_advance<S, QQ, TT>), dim3(pl.nchunk, (unsigned)P), dim3(Geo<QQ, TT>::BS), 0,
                               st, W, ldw, (int)pl.M, pl.rows_per_chunk, pl.nchunk, (int)pl.d, pl.ld, k,
                               k == 0 ? 1 : 0, sqdt, ws.cbar, ky.k0, ky.k1, pb->point_base, ws.part1);
        });
        const double* w_k = ws.tw + (size_t)k * PM;
        const double* Wbar_k = ws.tWbar + (size_t)k * PL;
        hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, ws.active, (int)P);
        const int vc = fold_parts(pl, P, ws.part1, nullptr, nullptr, st);
        // warm start from the previous level's bbar (full-rank designs, as in the forward)
        const int warm = (k > 0 && pl.M > pl.d + 1) ? 1 : 0;
        hipLaunchKernelGGL(k_adj_rhs_finish, dim3((unsigned)P), dim3(256), 0, st, ws.part1, pl.nchunk, vc, pl.ld,
                           (int)pl.d, pb->s, lam, Wbar_k, ws.tax + (size_t)k * PL, ws.adj, ws.x, ws.r, ws.pv, ws.scal, NS, ws.iscal,
                           ws.active, warm);
        if (warm) {
            dispatch<S>(pl.Q, pl.TEAM, [&](auto qc, auto tc) {
                constexpr int QQ = decltype(qc)::value, TT = decltype(tc)::value;
                hipLaunchKernelGGL((k_matvec<S, S, QQ, TT>), dim3(pl.nchunk, (unsigned)P), dim3(Geo<QQ, TT>::BS), 0,
                                   st, W, ldw, (int)pl.M, pl.rows_per_chunk, pl.nchunk, pl.ld, pb->s, w_k, ws.pv,
                                   ws.scal, NS, ws.iscal, ws.part1, ws.psc);
            });
            const int vw = fold_parts(pl, P, ws.part1, nullptr, nullptr, st);
            hipLaunchKernelGGL(k_adj_warm_start, dim3((unsigned)P), dim3(256), 0, st, ws.part1, ws.psc, pl.nchunk, vw,
                               pl.ld, pb->s, Wbar_k, ws.x, ws.r, ws.pv, ws.qv, ws.scal, NS, ws.iscal, ws.active);
        }
        // rank-deficient design: FP64 arithmetic in the CG product (the right-hand side has a
        // large component in the ridge-only null space, carried by the iterate with weight 1/lam)
        const int iters = (pl.M > pl.d + 1) ? run_cg<S, S>(pb, pl, P, W, ldw, w_k, Wbar_k, ws, status, st, err)
                                            : run_cg<S, double>(pb, pl, P, W, ldw, w_k, Wbar_k, ws, status, st, err);
        (void)iters;
        if (cg_iters_out) {
            cg_iters_out[k] = point_iters_max(ws, P, st, err);
            if (err) return err;
        }
        if (err) return err;
        hipLaunchKernelGGL(k_adj_bbar, dim3((unsigned)P), dim3(256), 0, st, ws.x, Wbar_k, pl.ld, ws.adj);
        dispatch<S>(pl.Q, pl.TEAM, [&](auto qc, auto tc) {
            constexpr int QQ = decltype(qc)::value, TT = decltype(tc)::value;
            hipLaunchKernelGGL((k_adj_rowdot<S, QQ, TT>), dim3(pl.nchunk, (unsigned)P), dim3(Geo<QQ, TT>::BS), 0,
                               st, W, ldw, (int)pl.M, pl.rows_per_chunk, pl.nchunk, pl.ld, pb->s, w_k, ws.x, ws.adj,
                               ws.G, ws.psc);
        });
        if ((err = last_error())) return err;
    }
    hipLaunchKernelGGL(k_adj_newton, dim3((unsigned)P), dim3(256), 0, st, ws.G, ws.tw + (size_t)(pl.N - 1) * PM,
                       (int64_t)pl.M, ws.psc, pl.nchunk, nullptr, ws.tscal, NS, fs, dt, pb->newton_iters, (int)pl.M, u_bar, ws.cbar,
                       ws.adj, 0, 1, status);
    if (ws.adjh && (err = ws.adjh->before(W, ldw, st))) return err;
    dispatch<S>(pl.Q, pl.TEAM, [&](auto qc, auto tc) {
        constexpr int QQ = decltype(qc)::value, TT = decltype(tc)::value;
        hipLaunchKernelGGL((k_adj_terminal<S, QQ, TT>), dim3(pl.nchunk, (unsigned)P), dim3(Geo<QQ, TT>::BS), 0, st, W,
                           ldw, (int)pl.M, pl.rows_per_chunk, pl.nchunk, (int)pl.d, pl.ld, x0, pb->mu, pb->gvec, pb->s,
                           pb->T, pb->g_kind, pb->gp[0], ws.G, ws.part1, ws.psc, ws.adjh ? ws.adjh->qpre : nullptr);
    });
    const int vc = fold_parts(pl, P, ws.part1, nullptr, nullptr, st);
    // with the caller's terminal stage the W-column term is added by its `after` step (s = 0 leaves it out)
    hipLaunchKernelGGL(k_adj_x0bar, dim3((unsigned)P), dim3(256), 0, st, ws.part1, ws.psc, pl.nchunk, vc, (int)pl.d,
                       pl.ld, x0, pb->mu, pb->gvec, ws.adjh ? 0.0 : pb->s, pb->T, pb->g_kind, ws.adj, x0_bar);
    if (ws.adjh && (err = ws.adjh->after(ws.part1, pl.nchunk, vc, pl.ld, x0_bar, st))) return err;
    hipLaunchKernelGGL(k_adj_params, dim3(1), dim3(64), 0, st, ws.adj, P, gp_bar, fp_bar);
    // the tape is consumed: the state no longer holds W_1 of the primal pass
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, ws.tag, 0);
    return last_error();
}

// The reverse mode under the affine diagonal coefficients (fbsde_coef_adjoint.hpp), after a taped
// fbsde_solve_coef on the same workspace: the state holds D_0 = 0 again.  cf: the family with dt; A, B: the
// mean path's m_k = x0 A_k + B_k.
template <typename S>
int coef_backward_impl(const fbsde_problem* pb, const Plan& pl, int64_t P, const double* x0, const double* u_bar,
                       double* x0_bar, double* gp_bar, double* fp_bar, uint32_t* status, WS& ws, const CoefArgs& cf,
                       const double* A, const double* B, int32_t* cg_iters_out, hipStream_t st) {
    S* W = (S*)ws.W;
    S* J = (S*)ws.cadj->J;
    const CoefAdj& ca = *ws.cadj;
    const int64_t ldw = pl.ld;
    const int64_t PM = P * pl.M, PL = P * (int64_t)pl.ld;
    const double dt = pb->T / (double)pb->N, sqdt = std::sqrt(dt);
    const Keys ky = keys_of(pb);
    const FSpec fs = fspec_of(pb);
    const int vstride = (int)pl.N + 1;
    const double rho_d = pb->ridge_rel / (double)pl.d, h2 = pb->eps_h * pb->eps_h;
    int err = FBSDE_OK;
    for (int k = 0; k < (int)pl.N; ++k) {
        const double* ax_k = ws.tax + (size_t)k * PL;
        const double* w_k = ws.tw + (size_t)k * PM;
        const double* Dbar_k = ws.tWbar + (size_t)k * PL;
        const double* ts_k = ws.tscal + (size_t)k * P * NS;
        CoefArgs ck = cf;
        ck.Aa = A[k];
        ck.Ba = B[k];
        hipLaunchKernelGGL(k_cadj_newton, dim3((unsigned)P), dim3(256), 0, st, ws.G,
                           k > 0 ? ws.tY + (size_t)k * PM : nullptr, ca.dydc + (size_t)k * PM, ca.zz + (size_t)k * PM,
                           ca.zs + (size_t)k * PM, ts_k, NS, x0, ax_k, (int)pl.d, pl.ld, ck, fs, dt,
                           pb->newton_iters, (int)pl.M, u_bar, ws.cbar, ca.zw, ws.adj, k == 0 ? 1 : 0, status);
        // the previous level's design adjoint (mu = its CG solution, still in x) acts on this state
        dispatch<S>(pl.Q, pl.TEAM, [&](auto qc, auto tc) {
            constexpr int QQ = decltype(qc)::value, TT = decltype(tc)::value;
            hipLaunchKernelGGL((k_cadj_advance<S, QQ, TT>), dim3(pl.nchunk, (unsigned)P), dim3(Geo<QQ, TT>::BS), 0,
                               st, W, J, ldw, (int)pl.M, pl.rows_per_chunk, pl.nchunk, (int)pl.d, pl.ld, k,
                               k == 0 ? 1 : 0, sqdt, ck, fs.kind, x0, ax_k,
                               k > 0 ? ws.tax + (size_t)(k - 1) * PL : nullptr, ws.x, ws.cbar, ca.zw, ca.c1, ca.c2,
                               ca.c3, ky.k0, ky.k1, pb->point_base, ws.part1, ws.part2);
        });
        hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, ws.active, (int)P);
        const int vc = fold_parts(pl, P, ws.part1, ws.part2, nullptr, st);
        hipLaunchKernelGGL(k_cadj_rhs, dim3((unsigned)P), dim3(256), 0, st, ws.part1, ws.part2, pl.nchunk, vc, pl.ld,
                           Dbar_k, ws.adj, ws.coefV + (k + 1), vstride, rho_d, ws.x, ws.r, ws.pv, ws.scal, NS,
                           ws.iscal, ws.active, ca.x0acc, k == 0 ? 1 : 0);
        // a rank-deficient design keeps FP64 arithmetic in the CG product, as the constant-coefficient adjoint
        if (pl.M > pl.d + 1) run_cg<S, S>(pb, pl, P, W, ldw, w_k, Dbar_k, ws, status, st, err);
        else run_cg<S, double>(pb, pl, P, W, ldw, w_k, Dbar_k, ws, status, st, err);
        if (err) return err;
        if (cg_iters_out) {
            cg_iters_out[k] = point_iters_max(ws, P, st, err);
            if (err) return err;
        }
        dispatch<S>(pl.Q, pl.TEAM, [&](auto qc, auto tc) {
            constexpr int QQ = decltype(qc)::value, TT = decltype(tc)::value;
            hipLaunchKernelGGL((k_cadj_rowdot<S, QQ, TT>), dim3(pl.nchunk, (unsigned)P), dim3(Geo<QQ, TT>::BS), 0,
                               st, W, ldw, (int)pl.M, pl.rows_per_chunk, pl.ld, ws.x, ax_k, ca.pd, ca.qd, ca.n2);
        });
        const double* Ynext = (k + 1 < (int)pl.N) ? ws.tY + (size_t)(k + 1) * PM : ws.Ya;
        hipLaunchKernelGGL(k_cadj_design, dim3((unsigned)P), dim3(256), 0, st, ca.pd, ca.qd, ca.n2, w_k, Ynext, ts_k,
                           NS, ws.x, ax_k, Dbar_k, pl.ld, ws.adj, ws.coefV + (k + 1), ca.Vbar + (k + 1), vstride, h2,
                           rho_d, (int)pl.M, ws.G, ca.c1, ca.c2, ca.c3);
        if ((err = last_error())) return err;
    }
    CoefArgs cN = cf;
    cN.Aa = A[pl.N];
    cN.Ba = B[pl.N];
    dispatch<S>(pl.Q, pl.TEAM, [&](auto qc, auto tc) {
        constexpr int QQ = decltype(qc)::value, TT = decltype(tc)::value;
        hipLaunchKernelGGL((k_cadj_terminal<S, QQ, TT>), dim3(pl.nchunk, (unsigned)P), dim3(Geo<QQ, TT>::BS), 0, st,
                           W, J, ldw, (int)pl.M, pl.rows_per_chunk, pl.nchunk, (int)pl.d, pl.ld, x0, pb->gvec, cN,
                           pb->g_kind, pb->gp[0], ws.G, ws.x, ws.tax + (size_t)(pl.N - 1) * PL, ca.c1, ca.c2, ca.c3,
                           ws.part1, ws.psc);
    });
    const int vc = fold_parts(pl, P, ws.part1, nullptr, nullptr, st);
    hipLaunchKernelGGL(k_cadj_x0bar, dim3((unsigned)P), dim3(256), 0, st, ws.part1, ws.psc, pl.nchunk, vc, (int)pl.d,
                       pl.ld, ca.x0acc, x0, cf, (int)pl.N, ca.Vbar, vstride, ws.adj, x0_bar);
    hipLaunchKernelGGL(k_adj_params, dim3(1), dim3(64), 0, st, ws.adj, P, gp_bar, fp_bar);
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, ws.tag, 0);
    return last_error();
}

// Box-Muller normals of caller-given Philox words, exactly as the hot-path kernels form them.
template <typename R>
__global__ void k_box_muller(int64_t n, const uint32_t* __restrict__ words, double* __restrict__ out) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const Words4 w = {words[4 * t], words[4 * t + 1], words[4 * t + 2], words[4 * t + 3]};
        R z[4];
        box_muller4<R>(w, z);
#pragma unroll
        for (int e = 0; e < 4; ++e) out[4 * t + e] = (double)z[e];
    }
}

// Read ceiling of a buffer: a plain grid-stride stream over n16 16-byte words with four non-temporal
// loads in flight per lane, XOR-reduced to one word per block (nothing but the loads costs time).  It
// measures the read bandwidth the hardware delivers on the same bytes the CG product reads.
__global__ void __launch_bounds__(256) k_stream_read(const uint4* __restrict__ a, int64_t n16, uint32_t* __restrict__ out) {
    typedef uint32_t u4v __attribute__((ext_vector_type(4)));
    const u4v* v = reinterpret_cast<const u4v*>(a);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    uint32_t x = 0;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const u4v a0 = __builtin_nontemporal_load(v + i), a1 = __builtin_nontemporal_load(v + i + stride);
        const u4v a2 = __builtin_nontemporal_load(v + i + 2 * stride), a3 = __builtin_nontemporal_load(v + i + 3 * stride);
        const u4v t = a0 ^ a1 ^ a2 ^ a3;
        x ^= t.x ^ t.y ^ t.z ^ t.w;
    }
    for (; i < n16; i += stride) {
        const u4v t = __builtin_nontemporal_load(v + i);
        x ^= t.x ^ t.y ^ t.z ^ t.w;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x ^= (uint32_t)__shfl_xor((int)x, off, 64);
    __shared__ uint32_t red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = red[0] ^ red[1] ^ red[2] ^ red[3];
}

}  // namespace

namespace fbsde {
namespace host {

void clear_status(uint32_t* status, int64_t P, hipStream_t st) { clear_status_impl(status, P, st); }
void set_int(int* a, int v, hipStream_t st) { hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, a, v); }

template <typename S>
void shared_forward(const fbsde_problem* pb, const Plan& pl1, S* W, double* Yscratch, double* rn2, uint32_t* status,
                    hipStream_t st) {
    const Keys ky = keys_of(pb);
    const double dt = pb->T / (double)pb->N;
    dispatch<S>(pl1.Q, pl1.TEAM, [&](auto qc, auto tc) {
        constexpr int QQ = decltype(qc)::value, TT = decltype(tc)::value;
        hipLaunchKernelGGL((k_forward<S, QQ, TT>), dim3(pl1.nchunk, 1), dim3(Geo<QQ, TT>::BS), 0, st, W,
                           (int64_t)pl1.ld, (int)pl1.M, pl1.rows_per_chunk, nullptr, nullptr, nullptr, (int)pl1.d,
                           pl1.ld, (int)pl1.N, std::sqrt(dt), pb->s, pb->T, G_QUAD, 1.0, 0.0, ky.k0, ky.k1, 0u, 1,
                           Yscratch, rn2, status);
    });
}

template <typename S>
void shared_reverse(const fbsde_problem* pb, const Plan& pl1, int k, S* W, const double* ax_dummy, const double* scal,
                    double* Yscratch, double* rn2, uint32_t* status, hipStream_t st) {
    const Keys ky = keys_of(pb);
    const double dt = pb->T / (double)pb->N;
    dispatch<S>(pl1.Q, pl1.TEAM, [&](auto qc, auto tc) {
        constexpr int QQ = decltype(qc)::value, TT = decltype(tc)::value;
        hipLaunchKernelGGL((k_reverse<S, QQ, TT>), dim3(pl1.nchunk, 1), dim3(Geo<QQ, TT>::BS), 0, st, W,
                           (int64_t)pl1.ld, (int)pl1.M, pl1.rows_per_chunk, (int)pl1.d, pl1.ld, k, 0, std::sqrt(dt),
                           pb->s, dt, ax_dummy, scal, NS, fspec_of(pb), 1, ky.k0, ky.k1, 0u, Yscratch, rn2, nullptr,
                           status, 1);
    });
}

template <typename S>
void shared_advance(const fbsde_problem* pb, const Plan& pl1, int k, S* W, hipStream_t st) {
    const Keys ky = keys_of(pb);
    const double dt = pb->T / (double)pb->N;
    dispatch<S>(pl1.Q, pl1.TEAM, [&](auto qc, auto tc) {
        constexpr int QQ = decltype(qc)::value, TT = decltype(tc)::value;
        hipLaunchKernelGGL((k_adj_advance<S, QQ, TT>), dim3(pl1.nchunk, 1), dim3(Geo<QQ, TT>::BS), 0, st, W,
                           (int64_t)pl1.ld, (int)pl1.M, pl1.rows_per_chunk, pl1.nchunk, (int)pl1.d, pl1.ld, k,
                           k == 0 ? 1 : 0, std::sqrt(dt), nullptr, ky.k0, ky.k1, 0xFFFFFFFFu, nullptr);
    });
}

void adj_newton(const fbsde_problem* pb, int64_t P, double* G, const double* w_prev, int64_t w_stride,
                const double* psc, int nchunk, const double* Yk, const double* tscal_k, const double* u_bar,
                double* cbar, double* adj, int init, int terminal, uint32_t* status, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_newton, dim3((unsigned)P), dim3(256), 0, st, G, w_prev, w_stride, psc, nchunk, Yk,
                       tscal_k, NS, fspec_of(pb), pb->T / (double)pb->N, pb->newton_iters, (int)pb->M, u_bar, cbar,
                       adj, init, terminal, status);
}

void adj_params(const double* adj, int64_t P, double* gp_bar, double* fp_bar, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_params, dim3(1), dim3(64), 0, st, adj, P, gp_bar, fp_bar);
}

int tape_tag_of(const fbsde_problem* pb, int64_t P) { return tape_tag(pb, P); }

template void shared_advance<double>(const fbsde_problem*, const Plan&, int, double*, hipStream_t);
template void shared_advance<float>(const fbsde_problem*, const Plan&, int, float*, hipStream_t);
template void shared_forward<double>(const fbsde_problem*, const Plan&, double*, double*, double*, uint32_t*,
                                     hipStream_t);
template void shared_forward<float>(const fbsde_problem*, const Plan&, float*, double*, double*, uint32_t*,
                                    hipStream_t);
template void shared_reverse<double>(const fbsde_problem*, const Plan&, int, double*, const double*, const double*,
                                     double*, double*, uint32_t*, hipStream_t);
template void shared_reverse<float>(const fbsde_problem*, const Plan&, int, float*, const double*, const double*,
                                    double*, double*, uint32_t*, hipStream_t);

}  // namespace host
}  // namespace fbsde

// ============================================================================ C ABI
extern "C" {

int64_t fbsde_state_ld(const fbsde_problem* pb) {
    Plan pl;
    if (check_problem(pb, 1) != FBSDE_OK || make_plan(pb, 1, pl) != FBSDE_OK) return 0;
    return pl.ld;
}

int fbsde_workspace_size(const fbsde_problem* pb, int64_t P, int32_t flags, size_t* bytes) {
    if (!bytes) return FBSDE_EINVAL;
    int rc = check_problem(pb, P);
    if (rc) return rc;
    Plan pl;
    if ((rc = make_plan(pb, P, pl))) return rc;
    if (pb->shared_dw) {
        *bytes = shared_workspace_bytes(pb, P, flags);
        return FBSDE_OK;
    }
    WS ws;
    *bytes = carve(pl, P, flags, nullptr, ws);
    return FBSDE_OK;
}

int fbsde_terminal(const fbsde_problem* pb, int64_t P, const double* x0, void* W, int64_t ldw, double* Y,
                   uint32_t* status, fbsde_stream stream) {
    int rc = check_problem(pb, P);
    if (rc) return rc;
    if (pb->shared_dw) return FBSDE_EINVAL;   // the shared form runs only as a whole solve
    Plan pl;
    if ((rc = make_plan(pb, P, pl))) return rc;
    if (ldw < pl.ld || ldw % 4 != 0) return FBSDE_EINVAL;
    if (P == 0) return FBSDE_OK;   // nothing is read or written; the pointers may be null
    if (!x0 || !W || !Y || !status) return FBSDE_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    clear_status(status, P, st);
    if (pb->prec == FBSDE_F64) launch_forward<double>(pb, pl, P, x0, (double*)W, ldw, Y, nullptr, status, st);
    else launch_forward<float>(pb, pl, P, x0, (float*)W, ldw, Y, nullptr, status, st);
    return last_error();
}

int fbsde_solve_step(const fbsde_problem* pb, int64_t P, int32_t k, const double* x0, void* W, int64_t ldw,
                     const double* Y_next, double* Y, double* alpha, double* alpha_x, uint32_t* status, void* wsp,
                     size_t ws_bytes, fbsde_stream stream) {
    int rc = check_problem(pb, P);
    if (rc) return rc;
    if (pb->shared_dw) return FBSDE_EINVAL;   // the shared form runs only as a whole solve
    Plan pl;
    if ((rc = make_plan(pb, P, pl))) return rc;
    if (k < 0 || k >= pb->N || ldw < pl.ld || ldw % 4 != 0) return FBSDE_EINVAL;
    if (P == 0) return FBSDE_OK;   // nothing is read or written; the pointers may be null
    if (!W || !Y_next || !Y || Y == Y_next || !status || !wsp) return FBSDE_EINVAL;
    WS ws;
    if (carve(pl, P, 0, nullptr, ws) > ws_bytes) return FBSDE_ENOSPC;
    carve(pl, P, 0, (char*)wsp, ws);
    hipStream_t st = (hipStream_t)stream;
    int err = FBSDE_OK;
    if (pb->prec == FBSDE_F64) {
        double* Ws = (double*)W;
        launch_rownorm<double>(pl, P, Ws, ldw, ws.rn2, st);
        run_level<double>(pb, pl, P, k, Ws, ldw, Y_next, ws.rn2, ws.w, ws.Wbar, ws, alpha, alpha_x, status, st, err);
        if (err) return err;
        launch_reverse<double>(pb, pl, P, k, Ws, ldw, ws.x, ws, Y, ws.rn2, status, st, nullptr, nullptr, 0, x0);
    } else {
        float* Ws = (float*)W;
        launch_rownorm<float>(pl, P, Ws, ldw, ws.rn2, st);
        run_level<float>(pb, pl, P, k, Ws, ldw, Y_next, ws.rn2, ws.w, ws.Wbar, ws, alpha, alpha_x, status, st, err);
        if (err) return err;
        launch_reverse<float>(pb, pl, P, k, Ws, ldw, ws.x, ws, Y, ws.rn2, status, st, nullptr, nullptr, 0, x0);
    }
    return last_error();
}

int fbsde_solve(const fbsde_problem* pb, int64_t P, const double* x0, double* u, double* grad, uint32_t* status,
                void* wsp, size_t ws_bytes, int32_t flags, int32_t* cg_iters_out, fbsde_stream stream) {
    int rc = check_problem(pb, P);
    if (rc) return rc;
    Plan pl;
    if ((rc = make_plan(pb, P, pl))) return rc;
    if (P == 0) {   // nothing is read or written but the per-level counts; the pointers may be null
        if (cg_iters_out)
            for (int64_t k = 0; k < pb->N; ++k) cg_iters_out[k] = 0;
        return FBSDE_OK;
    }
    if (!x0 || !u || !status || !wsp) return FBSDE_EINVAL;
    if (pb->shared_dw) {
        if (per_point_forward_only(pb)) return FBSDE_EINVAL;   // evaluated by the per-point form only
        if (cg_iters_out)
            for (int64_t k = 0; k < pb->N; ++k) cg_iters_out[k] = 0;   // direct (Cholesky) solve
        return solve_shared(pb, P, x0, u, grad, status, wsp, ws_bytes, flags, (hipStream_t)stream);
    }
    WS ws;
    if (carve(pl, P, flags, nullptr, ws) > ws_bytes) return FBSDE_ENOSPC;
    carve(pl, P, flags, (char*)wsp, ws);
    const bool tape = (flags & FBSDE_WS_TAPE) != 0;
    hipStream_t st = (hipStream_t)stream;
    if (pb->prec == FBSDE_F64) return solve_impl<double>(pb, pl, P, x0, u, grad, status, ws, tape, cg_iters_out, st);
    return solve_impl<float>(pb, pl, P, x0, u, grad, status, ws, tape, cg_iters_out, st);
}

}  // extern "C"

namespace {
// The per-point scheme under the affine diagonal coefficients: the problem as the kernels see it (s = 1:
// the state is the displacement from the mean path itself), the plan and the family.
int coef_r_check(const fbsde_problem* pb, const fbsde_coef* coef, int64_t P, fbsde_problem& pbc, Plan& pl,
                 CoefArgs& cf, int32_t flags = 0) {
    int rc = check_problem(pb, P);
    if (rc) return rc;
    if (!coef || coef->reserved != 0) return FBSDE_EINVAL;
    if (coef->kind != FBSDE_COEF_GEOMETRIC && coef->kind != FBSDE_COEF_AFFINE_DIAG) return FBSDE_EINVAL;
    if (coef->kind == FBSDE_COEF_GEOMETRIC && (coef->mu1 != 0.0 || coef->sigma1 != 0.0)) return FBSDE_EINVAL;
    const double v[4] = {coef->mu0, coef->sigma0, coef->mu1, coef->sigma1};
    for (double x : v)
        if (!std::isfinite(x)) return FBSDE_EINVAL;
    if (!(coef->sigma0 * coef->sigma0 + coef->sigma1 * coef->sigma1 > 0.0)) return FBSDE_EINVAL;
    // the family's drift replaces the constant one; one cloud per point; sources that read x are not covered
    if (pb->mu || pb->shared_dw || per_point_forward_only(pb)) return FBSDE_EINVAL;
    pbc = *pb;
    pbc.s = 1.0;
    // The reverse mode on a rank-deficient design (M <= d + 1) keeps the state in FP64: its adjoint
    // right-hand side reaches the ridge-only null space, whose component the solve scales by 1 / lam and
    // the sums over the cloud then cancel, so FP32 rounding of the state would come back amplified by the
    // ridge's inverse (measured 1.6e-5 against the FP64 oracle at ridge_rel = 1e-3, d = 80, M = 64)
    if ((flags & FBSDE_WS_TAPE) && pbc.prec == FBSDE_F32C && pb->M <= pb->d + 1) pbc.prec = FBSDE_F64;
    if ((rc = make_plan(&pbc, P, pl))) return rc;
    cf = CoefArgs{coef->mu0, coef->sigma0, coef->mu1, coef->sigma1, pb->T / (double)pb->N, 0.0, 0.0, 0.0, 0.0};
    return FBSDE_OK;
}

}  // namespace

namespace fbsde {
namespace host {
size_t per_point_workspace_bytes(const fbsde_problem* pb, int64_t P, int32_t flags) {
    Plan pl;
    if (check_problem(pb, P) != FBSDE_OK || make_plan(pb, P, pl) != FBSDE_OK) return 0;
    WS ws;
    return carve(pl, P, flags, nullptr, ws);
}

int solve_per_point_terminal(const fbsde_problem* pb, int64_t P, const double* x0, double* u, double* grad,
                             uint32_t* status, void* wsp, size_t ws_bytes, int32_t flags, int32_t* cg_iters_out,
                             hipStream_t st, const TerminalStep& terminal) {
    int rc = check_problem(pb, P);
    if (rc) return rc;
    if (pb->shared_dw) return FBSDE_EINVAL;
    Plan pl;
    if ((rc = make_plan(pb, P, pl))) return rc;
    if (P == 0) return FBSDE_OK;
    if (!x0 || !u || !status || !wsp) return FBSDE_EINVAL;
    WS ws;
    if (carve(pl, P, flags, nullptr, ws) > ws_bytes) return FBSDE_ENOSPC;
    carve(pl, P, flags, (char*)wsp, ws);
    ws.terminal = &terminal;
    const bool tape = (flags & FBSDE_WS_TAPE) != 0;
    if (pb->prec == FBSDE_F64) return solve_impl<double>(pb, pl, P, x0, u, grad, status, ws, tape, cg_iters_out, st);
    return solve_impl<float>(pb, pl, P, x0, u, grad, status, ws, tape, cg_iters_out, st);
}

}  // namespace host
}  // namespace fbsde

namespace {
// After the per-point workspace: the table V[p][k], k = 0..N, and with the tape the reverse mode's buffers
// (CoefAdj).  base == nullptr: only count.  Returns bytes.
size_t coef_r_extra(const Plan& pl, int64_t P, int32_t flags, char* base, double** V, CoefAdj* ca) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        char* q = base ? base + off : nullptr;
        off += round_up((int64_t)bytes, 256);
        return q;
    };
    const size_t PM = (size_t)P * pl.M, PL = (size_t)P * pl.ld;
    *V = (double*)take((size_t)P * (pl.N + 1) * 8);
    if (flags & FBSDE_WS_TAPE) {
        ca->Vbar = (double*)take((size_t)P * (pl.N + 1) * 8);
        ca->dydc = (double*)take((size_t)pl.N * PM * 8);
        ca->zz = (double*)take((size_t)pl.N * PM * 8);
        ca->zs = (double*)take((size_t)pl.N * PM * 8);
        ca->J = take(PM * pl.ld * pl.esz);
        ca->zw = (double*)take(PM * 8);
        ca->c1 = (double*)take(PM * 8);
        ca->c2 = (double*)take(PM * 8);
        ca->c3 = (double*)take(PM * 8);
        ca->pd = (double*)take(PM * 8);
        ca->qd = (double*)take(PM * 8);
        ca->n2 = (double*)take(PM * 8);
        ca->x0acc = (double*)take(PL * 8);
    }
    return off;
}

// The mean path m_k = x0 A[k] + B[k] of the Euler-Maruyama step, per coordinate.
void coef_mean_path(const Plan& pl, const CoefArgs& cf, std::vector<double>& A, std::vector<double>& B) {
    A.assign((size_t)pl.N + 1, 0.0);
    B.assign((size_t)pl.N + 1, 0.0);
    A[0] = 1.0;
    for (int64_t k = 0; k < pl.N; ++k) {
        A[k + 1] = A[k] * (1.0 + cf.mu0 * cf.dt);
        B[k + 1] = B[k] * (1.0 + cf.mu0 * cf.dt) + cf.mu1 * cf.dt;
    }
}

// Sets a coefficient family's tape apart from the constant-coefficient one (even: tape tags are odd).
int coef_salt(const CoefArgs& cf) {
    uint64_t h = 1469598103934665603ull;
    const double v[4] = {cf.mu0, cf.s0, cf.mu1, cf.s1};
    for (double x : v) {
        uint64_t b;
        std::memcpy(&b, &x, 8);
        h ^= b;
        h *= 1099511628211ull;
    }
    return (int)((h >> 17) & 0x7FFFFFFE) | 2;
}
}  // namespace

extern "C" {

int fbsde_coef_workspace_size(const fbsde_problem* pb, const fbsde_coef* coef, int64_t P, int32_t flags,
                              size_t* bytes) {
    if (!bytes || (flags & ~FBSDE_WS_TAPE)) return FBSDE_EINVAL;
    fbsde_problem pbc;
    Plan pl;
    CoefArgs cf;
    const int rc = coef_r_check(pb, coef, P, pbc, pl, cf, flags);
    if (rc) return rc;
    WS ws;
    double* V = nullptr;
    CoefAdj ca{};
    *bytes = carve(pl, P, flags, nullptr, ws) + coef_r_extra(pl, P, flags, nullptr, &V, &ca);
    return FBSDE_OK;
}

int fbsde_solve_coef(const fbsde_problem* pb, const fbsde_coef* coef, int64_t P, const double* x0, double* u,
                     double* grad, uint32_t* status, void* wsp, size_t ws_bytes, int32_t flags,
                     int32_t* cg_iters_out, fbsde_stream stream) {
    if (flags & ~FBSDE_WS_TAPE) return FBSDE_EINVAL;
    fbsde_problem pbc;
    Plan pl;
    CoefArgs cf;
    const int rc = coef_r_check(pb, coef, P, pbc, pl, cf, flags);
    if (rc) return rc;
    if (P == 0) {
        if (cg_iters_out)
            for (int64_t k = 0; k < pb->N; ++k) cg_iters_out[k] = 0;
        return FBSDE_OK;
    }
    if (!x0 || !u || !status || !wsp) return FBSDE_EINVAL;
    WS ws;
    double* V = nullptr;
    CoefAdj ca{};
    const size_t base = carve(pl, P, flags, nullptr, ws);
    if (base + coef_r_extra(pl, P, flags, nullptr, &V, &ca) > ws_bytes) return FBSDE_ENOSPC;
    carve(pl, P, flags, (char*)wsp, ws);
    coef_r_extra(pl, P, flags, (char*)wsp + base, &V, &ca);
    std::vector<double> A, B;
    coef_mean_path(pl, cf, A, B);
    const bool tape = (flags & FBSDE_WS_TAPE) != 0;
    ws.coef = &cf;
    ws.coefV = V;
    ws.coefA = A.data();
    ws.coefB = B.data();
    if (tape) {
        ws.cadj = &ca;
        ws.tag_salt = coef_salt(cf);
    }
    hipStream_t st = (hipStream_t)stream;
    if (pbc.prec == FBSDE_F64)
        return solve_impl<double>(&pbc, pl, P, x0, u, grad, status, ws, tape, cg_iters_out, st);
    return solve_impl<float>(&pbc, pl, P, x0, u, grad, status, ws, tape, cg_iters_out, st);
}

int fbsde_solve_coef_backward(const fbsde_problem* pb, const fbsde_coef* coef, int64_t P, const double* x0,
                              const double* u_bar, double* x0_bar, double* gp_bar, double* fp_bar, uint32_t* status,
                              void* wsp, size_t ws_bytes, int32_t* cg_iters_out, fbsde_stream stream) {
    fbsde_problem pbc;
    Plan pl;
    CoefArgs cf;
    const int rc = coef_r_check(pb, coef, P, pbc, pl, cf, FBSDE_WS_TAPE);
    if (rc) return rc;
    if (!gp_bar || !fp_bar) return FBSDE_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (P == 0) {   // an empty sum: zero parameter adjoints
        if (cg_iters_out)
            for (int64_t k = 0; k < pb->N; ++k) cg_iters_out[k] = 0;
        adj_params(nullptr, 0, gp_bar, fp_bar, st);
        return last_error();
    }
    if (!x0 || !u_bar || !x0_bar || !status || !wsp) return FBSDE_EINVAL;
    WS ws;
    double* V = nullptr;
    CoefAdj ca{};
    const size_t base = carve(pl, P, FBSDE_WS_TAPE, nullptr, ws);
    if (base + coef_r_extra(pl, P, FBSDE_WS_TAPE, nullptr, &V, &ca) > ws_bytes) return FBSDE_ENOSPC;
    carve(pl, P, FBSDE_WS_TAPE, (char*)wsp, ws);
    coef_r_extra(pl, P, FBSDE_WS_TAPE, (char*)wsp + base, &V, &ca);
    int tag = 0;
    if (hipMemcpyAsync(&tag, ws.tag, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return FBSDE_EHIP;
    if (tag != (tape_tag(&pbc, P) ^ coef_salt(cf))) return FBSDE_ESTATE;
    std::vector<double> A, B;
    coef_mean_path(pl, cf, A, B);
    ws.coef = &cf;
    ws.coefV = V;
    ws.coefA = A.data();
    ws.coefB = B.data();
    ws.cadj = &ca;
    if (pbc.prec == FBSDE_F64)
        return coef_backward_impl<double>(&pbc, pl, P, x0, u_bar, x0_bar, gp_bar, fp_bar, status, ws, cf, A.data(),
                                          B.data(), cg_iters_out, st);
    return coef_backward_impl<float>(&pbc, pl, P, x0, u_bar, x0_bar, gp_bar, fp_bar, status, ws, cf, A.data(),
                                     B.data(), cg_iters_out, st);
}

}  // extern "C"

namespace {
// The reverse mode; check_tape: read the tape's tag back first (one stream wait) and refuse a workspace
// whose tape does not belong to this problem.
int backward_entry(const fbsde_problem* pb, int64_t P, const double* x0, const double* u_bar, double* x0_bar,
                   double* gp_bar, double* fp_bar, uint32_t* status, void* wsp, size_t ws_bytes,
                   int32_t* cg_iters_out, fbsde_stream stream, bool check_tape,
                   const host::AdjTerminalHooks* hooks = nullptr) {
    int rc = check_problem(pb, P);
    if (rc) return rc;
    if (per_point_forward_only(pb)) return FBSDE_EINVAL;   // the reverse mode covers neither family
    Plan pl;
    if ((rc = make_plan(pb, P, pl))) return rc;
    if (!gp_bar || !fp_bar) return FBSDE_EINVAL;
    if (P == 0) {   // the loss is an empty sum: zero parameter adjoints; the other pointers may be null
        if (cg_iters_out)
            for (int64_t k = 0; k < pb->N; ++k) cg_iters_out[k] = 0;
        adj_params(nullptr, 0, gp_bar, fp_bar, (hipStream_t)stream);
        return last_error();
    }
    if (!x0 || !u_bar || !x0_bar || !status || !wsp) return FBSDE_EINVAL;
    if (pb->shared_dw) {
        if (per_point_forward_only(pb)) return FBSDE_EINVAL;   // evaluated by the per-point form only
        if (cg_iters_out)
            for (int64_t k = 0; k < pb->N; ++k) cg_iters_out[k] = 0;   // direct (Cholesky) solves
        return backward_shared(pb, P, x0, u_bar, x0_bar, gp_bar, fp_bar, status, wsp, ws_bytes, (hipStream_t)stream);
    }
    WS ws;
    if (carve(pl, P, FBSDE_WS_TAPE, nullptr, ws) > ws_bytes) return FBSDE_ENOSPC;
    carve(pl, P, FBSDE_WS_TAPE, (char*)wsp, ws);
    ws.adjh = hooks;
    hipStream_t st = (hipStream_t)stream;
    if (check_tape) {
        int tag = 0;
        if (hipMemcpyAsync(&tag, ws.tag, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return FBSDE_EHIP;
        if (tag != tape_tag(pb, P)) return FBSDE_ESTATE;
    }
    if (pb->prec == FBSDE_F64)
        return backward_impl<double>(pb, pl, P, x0, u_bar, x0_bar, gp_bar, fp_bar, status, ws, cg_iters_out, st);
    return backward_impl<float>(pb, pl, P, x0, u_bar, x0_bar, gp_bar, fp_bar, status, ws, cg_iters_out, st);
}
}  // namespace

namespace fbsde {
namespace host {
int solve_per_point_backward_terminal(const fbsde_problem* pb, int64_t P, const double* x0, const double* u_bar,
                                      double* x0_bar, double* gp_bar, double* fp_bar, uint32_t* status, void* ws,
                                      size_t ws_bytes, int32_t* cg_iters_out, hipStream_t st,
                                      const AdjTerminalHooks& hooks) {
    if (pb->shared_dw) return FBSDE_EINVAL;
    return backward_entry(pb, P, x0, u_bar, x0_bar, gp_bar, fp_bar, status, ws, ws_bytes, cg_iters_out,
                          (fbsde_stream)st, true, &hooks);
}

int solve_tile(const fbsde_problem* pb, int64_t P, const double* x0, double* u, double* grad, uint32_t* status,
               void* wsp, size_t ws_bytes, int32_t flags, bool reset_counts, hipStream_t st) {
    if (pb->shared_dw || P == 0)
        return fbsde_solve(pb, P, x0, u, grad, status, wsp, ws_bytes, flags, nullptr, (fbsde_stream)st);
    int rc = check_problem(pb, P);
    if (rc) return rc;
    Plan pl;
    if ((rc = make_plan(pb, P, pl))) return rc;
    if (!x0 || !u || !status || !wsp) return FBSDE_EINVAL;
    WS ws;
    if (carve(pl, P, flags, nullptr, ws) > ws_bytes) return FBSDE_ENOSPC;
    carve(pl, P, flags, (char*)wsp, ws);
    const bool tape = (flags & FBSDE_WS_TAPE) != 0;
    if (pb->prec == FBSDE_F64)
        return solve_impl<double>(pb, pl, P, x0, u, grad, status, ws, tape, nullptr, st, reset_counts);
    return solve_impl<float>(pb, pl, P, x0, u, grad, status, ws, tape, nullptr, st, reset_counts);
}

int solve_backward_after_forward(const fbsde_problem* pb, int64_t P, const double* x0, const double* u_bar,
                                 double* x0_bar, double* gp_bar, double* fp_bar, uint32_t* status, void* ws,
                                 size_t ws_bytes, hipStream_t st) {
    return backward_entry(pb, P, x0, u_bar, x0_bar, gp_bar, fp_bar, status, ws, ws_bytes, nullptr,
                          (fbsde_stream)st, false);
}
}  // namespace host
}  // namespace fbsde

extern "C" {

int fbsde_solve_backward(const fbsde_problem* pb, int64_t P, const double* x0, const double* u_bar, double* x0_bar,
                         double* gp_bar, double* fp_bar, uint32_t* status, void* wsp, size_t ws_bytes,
                         int32_t* cg_iters_out, fbsde_stream stream) {
    return backward_entry(pb, P, x0, u_bar, x0_bar, gp_bar, fp_bar, status, wsp, ws_bytes, cg_iters_out, stream,
                          true);
}

int fbsde_normals(const fbsde_problem* pb, int64_t p, int32_t k, int64_t j0, int64_t rows, double* out,
                  uint32_t* words, fbsde_stream stream) {
    int rc = check_problem(pb, 1);
    if (rc) return rc;
    if (p < 0 || k < 0 || j0 < 0 || rows < 0 || !out) return FBSDE_EINVAL;
    if (rows == 0) return FBSDE_OK;
    const Keys ky = keys_of(pb);
    const uint32_t q = pb->shared_dw ? 0xFFFFFFFFu : pb->point_base + (uint32_t)p;
    const int64_t n = rows * ((pb->d + 3) / 4);
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 65535);
    if (pb->prec == FBSDE_F64)
        hipLaunchKernelGGL(k_normals<double>, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (int)pb->d, j0, rows, k, q, ky.k0,
                       ky.k1, out, words);
    else
        hipLaunchKernelGGL(k_normals<float>, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (int)pb->d, j0, rows, k, q, ky.k0,
                       ky.k1, out, words);
    return last_error();
}

int fbsde_box_muller(int32_t prec, int64_t n, const uint32_t* words, double* out, fbsde_stream stream) {
    if (n < 0 || (prec != FBSDE_F64 && prec != FBSDE_F32C)) return FBSDE_EINVAL;
    if (n == 0) return FBSDE_OK;
    if (!words || !out) return FBSDE_EINVAL;
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    if (prec == FBSDE_F64)
        hipLaunchKernelGGL(k_box_muller<double>, dim3(blocks), dim3(256), 0, (hipStream_t)stream, n, words, out);
    else
        hipLaunchKernelGGL(k_box_muller<float>, dim3(blocks), dim3(256), 0, (hipStream_t)stream, n, words, out);
    return last_error();
}

int fbsde_time_kernel(const fbsde_problem* pb, int64_t P, int32_t which, int32_t reps, void* wsp, size_t ws_bytes,
                      float* avg_ms, fbsde_stream stream) {
    int rc = check_problem(pb, P);
    if (rc) return rc;
    if (pb->shared_dw) return FBSDE_EINVAL;   // the shared form runs only as a whole solve
    Plan pl;
    if ((rc = make_plan(pb, P, pl))) return rc;
    if (!wsp || !avg_ms || reps < 1 || which < 0 || which > 4 || P == 0) return FBSDE_EINVAL;
    WS ws;
    if (carve(pl, P, 0, nullptr, ws) > ws_bytes) return FBSDE_ENOSPC;
    carve(pl, P, 0, (char*)wsp, ws);
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return FBSDE_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return FBSDE_EHIP; }
    // iscal[p][1] = 0: every point iterates
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::min<int64_t>((P * 4 + 255) / 256, 1024)), dim3(256), 0, st,
                       (uint32_t*)ws.iscal, P * 4, 0u);
    auto body = [&](auto tag) {
        using S = decltype(tag);
        S* W = (S*)ws.W;
        const int64_t ldw = pl.ld;
        for (int r = 0; r < reps; ++r) {
            if (which == 0) {
                dispatch<S>(pl.Q, pl.TEAM, [&](auto qc, auto tc) {
                    constexpr int QQ = decltype(qc)::value, TT = decltype(tc)::value;
                    hipLaunchKernelGGL((k_matvec<S, S, QQ, TT>), dim3(pl.nchunk, (unsigned)P), dim3(Geo<QQ, TT>::BS),
                                       0, st, W, ldw, (int)pl.M, pl.rows_per_chunk, pl.nchunk, pl.ld, pb->s, ws.w,
                                       ws.pv, ws.scal, NS, ws.iscal, ws.part1, ws.psc);
                });
            } else if (which == 1) {
                launch_reverse<S>(pb, pl, P, 1, W, ldw, ws.x, ws, ws.Yb, ws.rn2, (uint32_t*)ws.iscal, st);
            } else if (which == 4) {
                // the state's bytes, one XOR word per block into the chunk partials (>= P ld doubles)
                const int64_t n16 = (int64_t)P * pl.M * pl.ld * (int64_t)sizeof(S) / 16;
                const int64_t cap = 2 * (int64_t)P * pl.nchunk * pl.ld;
                const unsigned blocks = (unsigned)std::max<int64_t>(
                    1, std::min<int64_t>({32768, cap, (n16 + 1023) / 1024}));
                hipLaunchKernelGGL(k_stream_read, dim3(blocks), dim3(256), 0, st, (const uint4*)W, n16,
                                   (uint32_t*)ws.part1);
            } else if (which == 2) {
                dispatch<S>(pl.Q, pl.TEAM, [&](auto qc, auto tc) {
                    constexpr int QQ = decltype(qc)::value, TT = decltype(tc)::value;
                    hipLaunchKernelGGL((k_moments<S, S, QQ, TT>), dim3(pl.nchunk, (unsigned)P), dim3(Geo<QQ, TT>::BS),
                                       0, st, W, ldw, (int)pl.M, pl.rows_per_chunk, pl.nchunk, pl.ld, ws.w, ws.c2,
                                       ws.x, ws.scal, NS, 1, ws.part1, ws.part2, ws.part3, ws.psc);
                });
            } else {
                // the evaluation points of this timing run: the [P][ld] >= [P][d] scratch vector
                launch_forward<S>(pb, pl, P, ws.Wbar, W, ldw, ws.Yb, ws.rn2, (uint32_t*)ws.iscal, st);
            }
            if (r == 0) (void)hipEventRecord(e0, st);   // the first launch warms up, the rest are timed
        }
    };
    if (reps < 2) reps = 2;
    if (pb->prec == FBSDE_F64) body(double{}); else body(float{});
    (void)hipEventRecord(e1, st);
    rc = (hipEventSynchronize(e1) == hipSuccess) ? last_error() : FBSDE_EHIP;
    float ms = 0.0f;
    if (rc == FBSDE_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = FBSDE_EHIP;
    *avg_ms = ms / (float)(reps - 1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

int fbsde_autotune(const fbsde_problem* pb, int64_t P, const double* x0, void* wsp, size_t ws_bytes,
                   fbsde_tune_result* out, fbsde_stream stream) {
    int rc = check_problem(pb, P);
    if (rc) return rc;
    if (pb->shared_dw || P < 1 || !x0 || !wsp || !out) return FBSDE_EINVAL;   // the shared form has no CG
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune.erase(tune_key(pb, P));
    }
    Plan p0;
    if ((rc = make_plan(pb, P, p0))) return rc;
    WS ws;
    if (carve(p0, P, 0, nullptr, ws) > ws_bytes) return FBSDE_ENOSPC;
    carve(p0, P, 0, (char*)wsp, ws);
    hipStream_t st = (hipStream_t)stream;
    // a state to time on: the forward sweep of these points; zero weights, direction and scalars
    // (the product's cost does not depend on the values), every point iterating
    auto fill0 = [&](void* a, size_t bytes) {
        const int64_t n = (int64_t)(bytes / 4);
        hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0, st,
                           (uint32_t*)a, n, 0u);
    };
    const int64_t PM = P * p0.M, PL = P * (int64_t)p0.ld;
    auto sweep = [&](auto tag) {
        using S = decltype(tag);
        launch_forward<S>(pb, p0, P, x0, (S*)ws.W, p0.ld, ws.Ya, ws.rn2, (uint32_t*)ws.iscal, st);
    };
    if (pb->prec == FBSDE_F64) sweep(double{}); else sweep(float{});
    fill0(ws.w, (size_t)PM * 8);
    fill0(ws.pv, (size_t)PL * 8);
    fill0(ws.scal, (size_t)P * NS * 8);
    fill0(ws.iscal, (size_t)P * 16);
    if ((rc = last_error())) return rc;
    // candidates: the row split over 1, 2 or 4 times the default team width, times the default,
    // half or a quarter of the default chunks per point
    std::vector<std::pair<int, int>> cand;
    for (int tm = p0.TEAM; tm <= std::min(16, 4 * p0.TEAM); tm *= 2)
        for (int nc : {p0.nchunk, p0.nchunk / 2, p0.nchunk / 4}) {
            Plan t = p0;
            if (nc >= 1 && shape_plan(t, tm, nc) &&
                std::find(cand.begin(), cand.end(), std::make_pair(tm, t.nchunk)) == cand.end())
                cand.emplace_back(tm, t.nchunk);
        }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return FBSDE_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return FBSDE_EHIP; }
    const int reps = 4;
    float best = 0.0f, dflt = 0.0f;
    int bi = 0;
    for (size_t ci = 0; ci < cand.size() && !rc; ++ci) {
        Plan t = p0;
        shape_plan(t, cand[ci].first, cand[ci].second);
        auto body = [&](auto tag) {
            using S = decltype(tag);
            for (int r = 0; r <= reps; ++r) {
                dispatch<S>(t.Q, t.TEAM, [&](auto qc, auto tc) {
                    constexpr int QQ = decltype(qc)::value, TT = decltype(tc)::value;
                    hipLaunchKernelGGL((k_matvec<S, S, QQ, TT>), dim3(t.nchunk, (unsigned)P), dim3(Geo<QQ, TT>::BS), 0,
                                       st, (const S*)ws.W, (int64_t)t.ld, (int)t.M, t.rows_per_chunk, t.nchunk, t.ld,
                                       pb->s, ws.w, ws.pv, ws.scal, NS, ws.iscal, ws.part1, ws.psc);
                });
                if (r == 0) (void)hipEventRecord(e0, st);
            }
        };
        if (pb->prec == FBSDE_F64) body(double{}); else body(float{});
        (void)hipEventRecord(e1, st);
        float ms = 0.0f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = FBSDE_EHIP;
        else rc = last_error();
        ms /= (float)reps;
        if (ci == 0) { best = ms; dflt = ms; }
        else if (ms < 0.98f * best) { best = ms; bi = (int)ci; }   // a new shape must win by 2 %
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[tune_key(pb, P)] = cand[(size_t)bi];
    }
    Plan t = p0;
    shape_plan(t, cand[(size_t)bi].first, cand[(size_t)bi].second);
    out->team = t.TEAM;
    out->q = t.Q;
    out->nchunk = t.nchunk;
    out->n_candidates = (int32_t)cand.size();
    out->best_ms = best;
    out->default_ms = dflt;
    return FBSDE_OK;
}

int fbsde_launch_timer(int32_t on) {
    if (on != 0 && on != 1) return FBSDE_EINVAL;
    std::lock_guard<std::mutex> lk(g_lt_mu);
    if (on) g_lt_used = 0;
    g_lt_on.store(on != 0);
    return FBSDE_OK;
}

int fbsde_launch_timer_read(float* ms, double* bytes, int64_t cap, int64_t* n) {
    if (!n || cap < 0 || (cap > 0 && !ms)) return FBSDE_EINVAL;
    std::lock_guard<std::mutex> lk(g_lt_mu);
    int64_t k = 0;
    for (size_t i = 0; i < g_lt_used; ++i) {
        if (!g_lt[i].ok) continue;
        float t = 0.0f;
        if (hipEventSynchronize(g_lt[i].b) != hipSuccess || hipEventElapsedTime(&t, g_lt[i].a, g_lt[i].b) != hipSuccess)
            return FBSDE_EHIP;
        if (k < cap) {
            ms[k] = t;
            if (bytes) bytes[k] = g_lt[i].work;
        }
        ++k;
    }
    *n = k;
    return FBSDE_OK;
}

}  // extern "C"

namespace fbsde {
namespace host {
unsigned long long* cg_bytes_counter(void* ws) { return &((CgCtl*)ws)->bytes; }
}  // namespace host
}  // namespace fbsde

struct fbsde_graph_s {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

namespace fbsde {
namespace host {
// Capture what `body` enqueues on a private stream that first waits for the caller's stream, and
// instantiate it.  Streams that body forks onto (by events) join the capture and must join back.
int capture_graph(const std::function<int(hipStream_t)>& body, hipStream_t stream, fbsde_graph* out) {
    hipStream_t cap;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return FBSDE_EHIP;
    hipEvent_t ev;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) { (void)hipStreamDestroy(cap); return FBSDE_EHIP; }
    int err = FBSDE_OK;
    if (hipEventRecord(ev, stream) != hipSuccess || hipStreamWaitEvent(cap, ev, 0) != hipSuccess) err = FBSDE_EHIP;
    hipGraph_t g = nullptr;
    if (!err && hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) err = FBSDE_EHIP;
    if (!err) {
        const int rs = body(cap);
        const hipError_t he = hipStreamEndCapture(cap, &g);
        err = rs ? rs : (he != hipSuccess ? FBSDE_EHIP : FBSDE_OK);
    }
    hipGraphExec_t exec = nullptr;
    if (!err && hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) != hipSuccess) err = FBSDE_EHIP;
    (void)hipEventDestroy(ev);
    (void)hipStreamDestroy(cap);
    if (err) {
        if (g) (void)hipGraphDestroy(g);
        return err;
    }
    fbsde_graph h = new (std::nothrow) fbsde_graph_s{g, exec};
    if (!h) {
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(g);
        return FBSDE_EINVAL;
    }
    *out = h;
    return FBSDE_OK;
}
}  // namespace host
}  // namespace fbsde

extern "C" {

int fbsde_workspace_cg_rows(const void* ws, int64_t* rows, fbsde_stream stream) {
    if (!ws || !rows) return FBSDE_EINVAL;
    unsigned long long v = 0;
    const CgCtl* ctl = (const CgCtl*)ws;   // the loop control sits at offset 0 of the per-point workspace
    if (hipMemcpyAsync(&v, &ctl->rows, sizeof(v), hipMemcpyDeviceToHost, (hipStream_t)stream) != hipSuccess ||
        hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
        return FBSDE_EHIP;
    *rows = (int64_t)v;
    return FBSDE_OK;
}

int fbsde_launch_timer_kinds(int32_t* kinds, int64_t cap, int64_t* n) {
    if (!n || cap < 0 || (cap > 0 && !kinds)) return FBSDE_EINVAL;
    std::lock_guard<std::mutex> lk(g_lt_mu);
    int64_t k = 0;
    for (size_t i = 0; i < g_lt_used; ++i) {
        if (!g_lt[i].ok) continue;
        if (k < cap) kinds[k] = g_lt[i].kind;
        ++k;
    }
    *n = k;
    return FBSDE_OK;
}

int fbsde_autotune_reset(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    return FBSDE_OK;
}



int fbsde_graph_capture(const fbsde_problem* pb, int64_t P, const double* x0, double* u, double* grad,
                        uint32_t* status, void* ws, size_t ws_bytes, int32_t flags, fbsde_graph* out,
                        fbsde_stream stream) {
    if (!out) return FBSDE_EINVAL;
    *out = nullptr;
    int rc = check_problem(pb, P);
    if (rc) return rc;
    // the host-driven CG loop (a diagnostic alternative) polls the device, which a graph cannot do
    if (!pb->shared_dw && pb->cg_fixed_iters <= 0 && host_cg_loop()) return FBSDE_EINVAL;
    if (!x0 || !u || !status || !ws || P < 1) return FBSDE_EINVAL;
    size_t need = 0;
    if ((rc = fbsde_workspace_size(pb, P, flags, &need))) return rc;
    if (need > ws_bytes) return FBSDE_ENOSPC;
    return capture_graph([&](hipStream_t cap) {
        return fbsde_solve(pb, P, x0, u, grad, status, ws, ws_bytes, flags, nullptr, (fbsde_stream)cap);
    }, (hipStream_t)stream, out);
}

int fbsde_graph_launch(fbsde_graph g, fbsde_stream stream) {
    if (!g) return FBSDE_EINVAL;
    return hipGraphLaunch(g->exec, (hipStream_t)stream) == hipSuccess ? FBSDE_OK : FBSDE_EHIP;
}

int fbsde_graph_destroy(fbsde_graph g) {
    if (!g) return FBSDE_OK;
    const bool ok = hipGraphExecDestroy(g->exec) == hipSuccess && hipGraphDestroy(g->graph) == hipSuccess;
    delete g;
    return ok ? FBSDE_OK : FBSDE_EHIP;
}

}  // extern "C"

// ------------------------------------------------------------------ allocation-free entry point
// The workspace of fbsde_solve_noalloc: a file-scope device array (each GPU that runs the library holds
// its own copy until the process ends).  Host code never passes its name to a kernel: the name is a
// host-side stand-in, so its device address is looked up once per device (hipGetSymbolAddress, with the
// device current) and that address is used everywhere.
__device__ __align__(256) unsigned char scratch[FBSDE_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (set-up on the first call on each device).
int scratch_of_current_device(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return FBSDE_EHIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return FBSDE_EHIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return FBSDE_OK;
}
}  // namespace

extern "C" {

int fbsde_solve_noalloc(const fbsde_problem* pb, int64_t P, const double* x0, double* u, double* grad,
                        uint32_t* status, fbsde_stream stream) {
    int rc = check_problem(pb, P);
    if (rc) return rc;
    if (pb->shared_dw) return FBSDE_EINVAL;   // the per-point form only
    Plan pl;
    if ((rc = make_plan(pb, P, pl))) return rc;
    if (P == 0) return FBSDE_OK;
    if (!x0 || !u || !status) return FBSDE_EINVAL;
    WS ws;
    if (carve(pl, P, 0, nullptr, ws) > (size_t)FBSDE_NOALLOC_SCRATCH_BYTES) return FBSDE_ENOSPC;
    void* base = nullptr;
    if ((rc = scratch_of_current_device(&base))) return rc;
    carve(pl, P, 0, (char*)base, ws);
    ws.fixed_buffer = true;
    hipStream_t st = (hipStream_t)stream;
    if (pb->prec == FBSDE_F64) return solve_impl<double>(pb, pl, P, x0, u, grad, status, ws, false, nullptr, st);
    return solve_impl<float>(pb, pl, P, x0, u, grad, status, ws, false, nullptr, st);
}

const char* fbsde_strerror(int code) {
    switch (code) {
        case FBSDE_OK: return "ok";
        case FBSDE_EINVAL: return "invalid argument or unsupported problem descriptor";
        case FBSDE_ENOSPC: return "workspace too small";
        case FBSDE_EHIP: return "HIP launch or runtime failure";
        case FBSDE_ESTATE: return "workspace does not hold the tape of a preceding fbsde_solve";
        default: return "unknown error";
    }
}

}  // extern "C"
