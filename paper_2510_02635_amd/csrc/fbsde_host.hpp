// Host-side helpers shared by the translation units of libfbsde (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <type_traits>

#include "fbsde.h"
#include "fbsde_device.hpp"

namespace fbsde {
namespace host {


constexpr int NS = 10;   // per-point FP64 scalars (see k_moments_finish and k_level_finish)

struct Plan {
    int64_t d, M, N;
    int ld, Q, TEAM, BS, TPW, nchunk, rows_per_chunk;
    size_t esz;
    int maxit;   // CG iterations per point and level at most (sizes the device loop's work queues)
    bool dual;   // the forward levels use the direct dual solve (M x M Cholesky) instead of CG
};

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

inline int check_problem(const fbsde_problem* pb, int64_t P) {
    if (!pb || P < 0) return FBSDE_EINVAL;
    if (pb->d < 1 || pb->M < 2 || pb->N < 1) return FBSDE_EINVAL;
    if (!(pb->T > 0.0) || !(pb->s > 0.0)) return FBSDE_EINVAL;
    if (pb->f_kind < FBSDE_F_ZERO || pb->f_kind > FBSDE_F_LOG_POT) return FBSDE_EINVAL;
    if (pb->g_kind < FBSDE_G_QUAD || pb->g_kind > FBSDE_G_CASE2) return FBSDE_EINVAL;
    if ((pb->g_kind == FBSDE_G_AFFINE || pb->g_kind == FBSDE_G_LOGISTIC) && !pb->gvec) return FBSDE_EINVAL;
    if (!(pb->eps_h >= 0.0) || !(pb->ridge_rel >= 0.0)) return FBSDE_EINVAL;
    if (pb->ridge_rel == 0.0 && pb->M <= pb->d + 1) return FBSDE_EINVAL;
    if (pb->newton_iters < 1 || pb->cg_maxit < 1 || !(pb->cg_rtol >= 0.0)) return FBSDE_EINVAL;
    if (pb->prec != FBSDE_F64 && pb->prec != FBSDE_F32C) return FBSDE_EINVAL;
    if (pb->shared_dw != 0 && pb->shared_dw != 1) return FBSDE_EINVAL;
    if (pb->solver != FBSDE_SOLVER_AUTO && pb->solver != FBSDE_SOLVER_CG) return FBSDE_EINVAL;
    // grid.y carries the point index
    if (pb->M > (int64_t)1 << 30 || pb->N > (int64_t)1 << 30 || P > 65535) return FBSDE_EINVAL;
    return FBSDE_OK;
}

// CG stopping tolerance actually used.  In FP32C with a rank-deficient centred design (M <= d + 1) the
// right-hand side carries FP32 rounding in the ridge-only null space; a test tighter than that rounding
// makes CG resolve it, scaled by 1/lam, into the slope: the tolerance is held at 1e-7 or above there.
inline double cg_rtol_of(const fbsde_problem* pb) {
    if (pb->prec == FBSDE_F32C && pb->M <= pb->d + 1) return std::max(pb->cg_rtol, 1e-7);
    return pb->cg_rtol;
}

// Launch timer records (fbsde_launch_timer): begin returns a record index or -1 when the timer is off.
long timer_begin(hipStream_t st, double work, int kind);
void timer_end(long i, hipStream_t st);

// Launch shapes recorded by fbsde_autotune (process-wide table keyed by precision, d, M and P).
bool tuned_shape(const fbsde_problem* pb, int64_t P, int& team, int& nchunk);

// Groups of four coordinates per lane for q needed: 1, 2, 4, 8, and 5 on the FP32 state (rows of
// 4097-5120 coordinates on four-wave teams, 8193-10240 on eight: no idle lane groups, and fewer registers
// than 8 groups).
inline int groups_per_lane(int q, int esz) {
    return (q <= 1) ? 1 : (q <= 2) ? 2 : (q <= 4) ? 4 : (q <= 5 && esz == 4) ? 5 : 8;
}

// Re-shape a plan: team width `team` (groups per lane recomputed) and `nchunk` chunks per point.
// Returns false if the team cannot hold the row within the per-lane register budget.
inline bool shape_plan(Plan& pl, int team, int nchunk) {
    const int groups = pl.ld / 4;
    const int qmax = (pl.esz == 8) ? 4 : 8;
    if (team < 1 || team > 16 || (team & (team - 1)) || nchunk < 1) return false;
    const int q = (groups + 64 * team - 1) / (64 * team);
    if (q > qmax) return false;
    pl.TEAM = team;
    pl.Q = groups_per_lane(q, pl.esz);
    pl.BS = 64 * std::max(pl.TEAM, 4);
    pl.TPW = pl.BS / (64 * pl.TEAM);
    pl.rows_per_chunk = (int)((pl.M + nchunk - 1) / nchunk);
    pl.nchunk = (int)((pl.M + pl.rows_per_chunk - 1) / pl.rows_per_chunk);
    return true;
}

inline int make_plan(const fbsde_problem* pb, int64_t P, Plan& pl) {
    pl.d = pb->d; pl.M = pb->M; pl.N = pb->N;
    pl.maxit = std::max(1, (int)pb->cg_maxit);
    // the direct dual solve where the cloud is small and not much thinner than d: CG iterations grow with
    // M / d towards the near-square design (measured at M = 100: 157 per level at d = 100, 34 at d = 500,
    // 14 at d = 1000, where the CG level is the faster one, 0.52 against 0.69 ms)
    pl.dual = pb->solver == FBSDE_SOLVER_AUTO && !pb->shared_dw && pb->M <= FBSDE_DUAL_MAXM &&
              pb->M <= pb->d + 1 && 8 * pb->M >= pb->d && pb->ridge_rel > 0.0 && pb->cg_fixed_iters == 0;
    pl.esz = (pb->prec == FBSDE_F64) ? 8 : 4;
    pl.ld = (int)round_up(pb->d, (pl.esz == 8) ? 16 : 32);
    const int groups = pl.ld / 4;
    const int qmax = (pl.esz == 8) ? 4 : 8;
    pl.TEAM = 0;
    for (int team = 1; team <= 16; team *= 2) {
        const int q = (groups + 64 * team - 1) / (64 * team);
        if (q <= qmax) {
            pl.TEAM = team;
            pl.Q = groups_per_lane(q, pl.esz);
            break;
        }
    }
    if (pl.TEAM == 0) return FBSDE_EINVAL;   // d beyond 16384 (FP64) / 32768 (FP32C)
    pl.BS = 64 * std::max(pl.TEAM, 4);
    pl.TPW = pl.BS / (64 * pl.TEAM);
    const int64_t target_blocks = 4096;
    int64_t nchunk = (target_blocks + std::max<int64_t>(P, 1) - 1) / std::max<int64_t>(P, 1);
    // at least 64 rows per chunk: each chunk writes one [ld] FP64 partial per pass, so the partials stay
    // within a few per cent of the state bytes the pass reads.  Short rows (ld <= 1024) take chunks of 16
    // rows: there a CG iteration of few points is bound by the time one chunk's rows take one after
    // another, and summing the extra partials costs little (measured: one point at d = 100, M = 512
    // 4.4 -> 2.7 ms per solve; 8 points at d = 1000, M = 832 20.7 -> 14.2 ms; at d >= 5000 smaller chunks
    // were slower, the deeper arrival tree adding more than the shorter chunks save).
    const int64_t min_rows = (pl.ld <= 1024) ? 16 : 64;
    nchunk = std::max<int64_t>(1, std::min<int64_t>(nchunk, std::min<int64_t>(pb->M / (2 * pl.TPW), pb->M / min_rows)));
    pl.rows_per_chunk = (int)((pb->M + nchunk - 1) / nchunk);
    pl.nchunk = (int)((pb->M + pl.rows_per_chunk - 1) / pl.rows_per_chunk);
    // a shape chosen by the autotuner: never more chunks than the default, so workspaces sized
    // before the tuning still fit
    int tt, tn;
    if (P > 0 && tuned_shape(pb, P, tt, tn)) {
        Plan t = pl;
        if (tn <= pl.nchunk && shape_plan(t, tt, tn)) pl = t;
    }
    return FBSDE_OK;
}

template <typename S, typename Fn>
void dispatch(int Q, int TEAM, Fn&& fn) {
#define FB_CASE(QQ, TT) \
    case QQ * 100 + TT: fn(std::integral_constant<int, QQ>{}, std::integral_constant<int, TT>{}); return;
    switch (Q * 100 + TEAM) {
        FB_CASE(1, 1) FB_CASE(1, 2) FB_CASE(1, 4) FB_CASE(1, 8) FB_CASE(1, 16)
        FB_CASE(2, 1) FB_CASE(2, 2) FB_CASE(2, 4) FB_CASE(2, 8) FB_CASE(2, 16)
        FB_CASE(4, 1) FB_CASE(4, 2) FB_CASE(4, 4) FB_CASE(4, 8) FB_CASE(4, 16)
        default: break;
    }
    if constexpr (std::is_same<S, float>::value) {
        switch (Q * 100 + TEAM) {
            FB_CASE(5, 1) FB_CASE(5, 2) FB_CASE(5, 4) FB_CASE(5, 8) FB_CASE(5, 16)
            FB_CASE(8, 1) FB_CASE(8, 2) FB_CASE(8, 4) FB_CASE(8, 8) FB_CASE(8, 16)
            default: break;
        }
    }
#undef FB_CASE
}

struct Keys { uint32_t k0, k1; };
inline Keys keys_of(const fbsde_problem* pb) {
    return {(uint32_t)(pb->seed & 0xFFFFFFFFull), (uint32_t)((pb->seed >> 32) ^ (uint64_t)pb->instance)};
}
inline FSpec fspec_of(const fbsde_problem* pb) {
    if (pb->f_kind == FBSDE_F_HJ_SINK) return {pb->f_kind, pb->fp[0], 1.0 / (pb->s * pb->s)};
    return {pb->f_kind, pb->fp[0], pb->fp[1], pb->fp[2]};
}
// f depends on x (a source term): only the per-point forward paths evaluate it, at the particles'
// positions.
inline bool f_depends_on_x(const fbsde_problem* pb) {
    return pb->f_kind == FBSDE_F_HJ_SINK || pb->f_kind == FBSDE_F_LOG_POT;
}
// A family only the per-point forward paths evaluate: f depends on x, or g needs the product of the
// coordinates (the Case 2 terminal value, formed in the forward sweep of the per-point form).
inline bool per_point_forward_only(const fbsde_problem* pb) {
    return f_depends_on_x(pb) || pb->g_kind == FBSDE_G_CASE2;
}

inline int last_error() { return (hipGetLastError() == hipSuccess) ? FBSDE_OK : FBSDE_EHIP; }


// Entry points of the other translation units.
size_t shared_workspace_bytes(const fbsde_problem* pb, int64_t P, int32_t flags);
int solve_shared(const fbsde_problem* pb, int64_t P, const double* x0, double* u, double* grad, uint32_t* status,
                 void* ws, size_t ws_bytes, int32_t flags, hipStream_t st);
int backward_shared(const fbsde_problem* pb, int64_t P, const double* x0, const double* u_bar, double* x0_bar,
                    double* gp_bar, double* fp_bar, uint32_t* status, void* ws, size_t ws_bytes, hipStream_t st);
// Newton adjoint of a level and the parameter sums (core translation unit owns these kernels).
void adj_newton(const fbsde_problem* pb, int64_t P, double* G, const double* w_prev, int64_t w_stride,
                const double* psc, int nchunk, const double* Yk, const double* tscal_k, const double* u_bar,
                double* cbar, double* adj, int init, int terminal, uint32_t* status, hipStream_t st);
void adj_params(const double* adj, int64_t P, double* gp_bar, double* fp_bar, hipStream_t st);
int tape_tag_of(const fbsde_problem* pb, int64_t P);
// W_{k+1} = W_k + sqrt(dt) xi_k on a single shared cloud (k = 0: from W_0 = 0).
template <typename S>
void shared_advance(const fbsde_problem* pb, const Plan& pl1, int k, S* W, hipStream_t st);
// Forward sweep / reversal of a single shared cloud (core translation unit owns these kernels).
template <typename S>
void shared_forward(const fbsde_problem* pb, const Plan& pl1, S* W, double* Yscratch, double* rn2, uint32_t* status,
                    hipStream_t st);
template <typename S>
void shared_reverse(const fbsde_problem* pb, const Plan& pl1, int k, S* W, const double* ax_dummy, const double* scal,
                    double* Yscratch, double* rn2, uint32_t* status, hipStream_t st);
void clear_status(uint32_t* status, int64_t P, hipStream_t st);
// Capture what body enqueues (on the stream it is given) into a graph, as fbsde_graph_capture does.
int capture_graph(const std::function<int(hipStream_t)>& body, hipStream_t stream, fbsde_graph* out);
// Divisor of the chip's block slots that a CG loop launch from this host thread asks for (1 by default).
extern thread_local int loop_share;
// fbsde_solve for one tile of a batched call; reset_counts = false adds its CG traffic to the count the
// arena already holds (the per-point form keeps it in the loop control at offset 0 of the workspace).
int solve_tile(const fbsde_problem* pb, int64_t P, const double* x0, double* u, double* grad, uint32_t* status,
               void* ws, size_t ws_bytes, int32_t flags, bool reset_counts, hipStream_t st);
// Device address of the algorithmic CG-product byte count in a per-point workspace.
unsigned long long* cg_bytes_counter(void* ws);
// fbsde_solve_backward without the read-back of the tape's tag, for a caller that has just enqueued the
// forward solve with the tape on the same stream and workspace (the batched schedule): no stream wait.
int solve_backward_after_forward(const fbsde_problem* pb, int64_t P, const double* x0, const double* u_bar,
                                 double* x0_bar, double* gp_bar, double* fp_bar, uint32_t* status, void* ws,
                                 size_t ws_bytes, hipStream_t st);
void set_int(int* a, int v, hipStream_t st);
// The per-point solve (fbsde_solve, no tape) with a step run after the forward sweep that may rewrite the
// terminal values Y [P][M] from the state W [P][M][ldw] (a constant diffusion matrix enters here);
// per_point_workspace_bytes is its workspace.
using TerminalStep = std::function<int(const void* W, int64_t ldw, double* Y, hipStream_t)>;
size_t per_point_workspace_bytes(const fbsde_problem* pb, int64_t P, int32_t flags);
int solve_per_point_terminal(const fbsde_problem* pb, int64_t P, const double* x0, double* u, double* grad,
                             uint32_t* status, void* ws, size_t ws_bytes, int32_t flags, int32_t* cg_iters_out,
                             hipStream_t st, const TerminalStep& terminal);
// The reverse mode of that solve with the terminal stage changed the same way: `before` fills qpre [P][M]
// (the argument of g per particle) from the state W_N, the terminal adjoint then reads it, its x0 adjoint is
// formed without the W-column term, and `after` adds that term from the W-column sums (part, summed over
// its first vchunks chunk slots of ld) to x0_bar.
struct AdjTerminalHooks {
    std::function<int(const void* W, int64_t ldw, hipStream_t)> before;
    double* qpre;
    std::function<int(const double* part, int nchunk, int vchunks, int ld, double* x0_bar, hipStream_t)> after;
};
int solve_per_point_backward_terminal(const fbsde_problem* pb, int64_t P, const double* x0, const double* u_bar,
                                      double* x0_bar, double* gp_bar, double* fp_bar, uint32_t* status, void* ws,
                                      size_t ws_bytes, int32_t* cg_iters_out, hipStream_t st,
                                      const AdjTerminalHooks& hooks);

}  // namespace host
}  // namespace fbsde
