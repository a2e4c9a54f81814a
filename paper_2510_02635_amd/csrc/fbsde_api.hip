// Host side of the C ABI declared in include/fbsde.h: validation, workspace carving and the
// launch sequence of Algorithm 1 (forward sweep, then the backward level loop) and of its
// adjoint.  All control crosses host -> device here; kernels live in fbsde_kernels.hpp /
// fbsde_adjoint.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "fbsde.h"
#include "fbsde_kernels.hpp"
#include "fbsde_adjoint.hpp"
#include "fbsde_shared.hpp"
#include "fbsde_batched.hpp"

#include <map>
#include <tuple>
#include <vector>

using namespace fbsde;

namespace {

constexpr int NS = 8;   // per-point FP64 scalars (see k_moments_finish)

struct Plan {
    int64_t d, M, N;
    int ld, Q, TEAM, BS, TPW, nchunk, rows_per_chunk;
    size_t esz;
};

int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

int check_problem(const fbsde_problem* pb, int64_t P) {
    if (!pb || P < 0) return FBSDE_EINVAL;
    if (pb->d < 1 || pb->M < 2 || pb->N < 1) return FBSDE_EINVAL;
    if (!(pb->T > 0.0) || !(pb->s > 0.0)) return FBSDE_EINVAL;
    if (pb->f_kind < FBSDE_F_ZERO || pb->f_kind > FBSDE_F_HJB) return FBSDE_EINVAL;
    if (pb->g_kind < FBSDE_G_QUAD || pb->g_kind > FBSDE_G_AFFINE) return FBSDE_EINVAL;
    if (pb->g_kind == FBSDE_G_AFFINE && !pb->gvec) return FBSDE_EINVAL;
    if (!(pb->eps_h >= 0.0) || !(pb->ridge_rel >= 0.0)) return FBSDE_EINVAL;
    if (pb->ridge_rel == 0.0 && pb->M <= pb->d + 1) return FBSDE_EINVAL;
    if (pb->newton_iters < 1 || pb->cg_maxit < 1 || !(pb->cg_rtol >= 0.0)) return FBSDE_EINVAL;
    if (pb->prec != FBSDE_F64 && pb->prec != FBSDE_F32C) return FBSDE_EINVAL;
    if (pb->shared_dw != 0 && pb->shared_dw != 1) return FBSDE_EINVAL;
    if (pb->reserved != 0) return FBSDE_EINVAL;
    // grid.y carries the point index
    if (pb->M > (int64_t)1 << 30 || pb->N > (int64_t)1 << 30 || P > 65535) return FBSDE_EINVAL;
    return FBSDE_OK;
}

int make_plan(const fbsde_problem* pb, int64_t P, Plan& pl) {
    pl.d = pb->d; pl.M = pb->M; pl.N = pb->N;
    pl.esz = (pb->prec == FBSDE_F64) ? 8 : 4;
    pl.ld = (int)round_up(pb->d, (pl.esz == 8) ? 16 : 32);
    const int groups = pl.ld / 4;
    const int qmax = (pl.esz == 8) ? 4 : 8;
    pl.TEAM = 0;
    for (int team = 1; team <= 16; team *= 2) {
        const int q = (groups + 64 * team - 1) / (64 * team);
        if (q <= qmax) {
            pl.TEAM = team;
            pl.Q = (q <= 1) ? 1 : (q <= 2) ? 2 : (q <= 4) ? 4 : 8;
            break;
        }
    }
    if (pl.TEAM == 0) return FBSDE_EINVAL;   // d beyond 16384 (FP64) / 32768 (FP32C)
    pl.BS = 64 * std::max(pl.TEAM, 4);
    pl.TPW = pl.BS / (64 * pl.TEAM);
    const int64_t target_blocks = 4096;
    int64_t nchunk = (target_blocks + std::max<int64_t>(P, 1) - 1) / std::max<int64_t>(P, 1);
    nchunk = std::max<int64_t>(1, std::min<int64_t>(nchunk, pb->M / (2 * pl.TPW)));
    pl.rows_per_chunk = (int)((pb->M + nchunk - 1) / nchunk);
    pl.nchunk = (int)((pb->M + pl.rows_per_chunk - 1) / pl.rows_per_chunk);
    return FBSDE_OK;
}

struct WS {
    void* W;
    double *Ya, *Yb, *rn2, *w, *c2;
    double *x, *r, *pv, *qv, *Wbar;
    double *part1, *part2, *part3, *psc, *scal;
    int *iscal, *active;
    // tape for the adjoint: per level k (cloud t_{k+1})
    double *tY, *tw, *tax, *tWbar, *tscal;
    int* tag;
    // adjoint work
    double *G, *cbar, *adj;
};

// Carve the workspace (base == nullptr: only count).  Returns bytes.
size_t carve(const Plan& pl, int64_t P, int flags, char* base, WS& ws) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        char* p = base ? base + off : nullptr;
        off += round_up((int64_t)bytes, 256);
        return p;
    };
    const size_t PM = (size_t)P * pl.M, PL = (size_t)P * pl.ld;
    const size_t parts = (size_t)P * pl.nchunk * pl.ld;
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
    ws.part1 = (double*)take(parts * 8);
    ws.part2 = (double*)take(parts * 8);
    ws.part3 = (double*)take(parts * 8);
    ws.psc = (double*)take((size_t)P * pl.nchunk * 4 * 8);
    ws.scal = (double*)take((size_t)P * NS * 8);
    ws.iscal = (int*)take((size_t)P * 4 * 4);
    ws.active = (int*)take(64);
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
    return off;
}

// ------------------------------------------------------------------ shared-increment workspace
struct SWS {
    void *W, *Dt, *K, *R, *ax, *xc, *DtT;
    double *Wbar, *wpart, *w, *sqw, *rn2, *Ya, *Yb, *scal, *xc2, *ysc;
    int* info;
};
constexpr int SH_RCH = 64;   // row chunks of the two-stage weighted mean

size_t carve_shared(const Plan& pl, int64_t P, char* base, SWS& ws) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        char* p = base ? base + off : nullptr;
        off += round_up((int64_t)bytes, 256);
        return p;
    };
    const size_t M = pl.M, ld = pl.ld, e = pl.esz;
    ws.W = take(M * ld * e);
    ws.Dt = take(M * ld * e);
    // dual form (M <= d): K is M x M; primal form (M > d): K is ld x ld, Dt^T [ld][M] is needed
    const bool primal = pl.M > pl.d;
    const size_t kn = primal ? ld : M;
    ws.K = take(kn * kn * e);
    ws.DtT = primal ? take(ld * M * e) : nullptr;
    ws.R = take((size_t)P * M * e);
    ws.ax = take((size_t)P * ld * e);
    ws.xc = take((size_t)P * ld * e);
    ws.Wbar = (double*)take(ld * 8);
    ws.wpart = (double*)take((size_t)SH_RCH * ld * 8);
    ws.w = (double*)take(M * 8);
    ws.sqw = (double*)take(M * 8);
    ws.rn2 = (double*)take(M * 8);
    ws.Ya = (double*)take((size_t)P * M * 8);
    ws.Yb = (double*)take((size_t)P * M * 8);
    ws.scal = (double*)take((size_t)P * NS * 8);
    ws.xc2 = (double*)take((size_t)P * 8);
    ws.ysc = (double*)take(M * 8);
    ws.info = (int*)take(64);
    return off;
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
            FB_CASE(8, 1) FB_CASE(8, 2) FB_CASE(8, 4) FB_CASE(8, 8) FB_CASE(8, 16)
            default: break;
        }
    }
#undef FB_CASE
}

struct Keys { uint32_t k0, k1; };
Keys keys_of(const fbsde_problem* pb) {
    return {(uint32_t)(pb->seed & 0xFFFFFFFFull), (uint32_t)((pb->seed >> 32) ^ (uint64_t)pb->instance)};
}
FSpec fspec_of(const fbsde_problem* pb) { return {pb->f_kind, pb->fp[0], pb->fp[1]}; }

int last_error() { return (hipGetLastError() == hipSuccess) ? FBSDE_OK : FBSDE_EHIP; }

// -------------------------------------------------------------------- launch sequences
template <typename S>
void launch_forward(const fbsde_problem* pb, const Plan& pl, int64_t P, const double* x0, S* W, int64_t ldw,
                    double* Y, double* rn2, uint32_t* status, hipStream_t st) {
    const Keys ky = keys_of(pb);
    const double dt = pb->T / (double)pb->N;
    dispatch<S>(pl.Q, pl.TEAM, [&](auto qc, auto tc) {
        constexpr int QQ = decltype(qc)::value, TT = decltype(tc)::value;
        hipLaunchKernelGGL((k_forward<S, QQ, TT>), dim3(pl.nchunk, (unsigned)P), dim3(Geo<QQ, TT>::BS), 0, st, W,
                           ldw, (int)pl.M, pl.rows_per_chunk, x0, pb->mu, pb->gvec, (int)pl.d, pl.ld, (int)pl.N,
                           std::sqrt(dt), pb->s, pb->T, pb->g_kind, pb->gp[0], pb->gp[1], ky.k0, ky.k1,
                           pb->point_base, 0, Y, rn2, status);
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
template <typename S>
int run_cg(const fbsde_problem* pb, const Plan& pl, int64_t P, const S* W, int64_t ldw, const double* w,
           const double* Wbar, WS& ws, uint32_t* status, hipStream_t st, int& err) {
    const int fixed = pb->cg_fixed_iters;
    const int cap = (fixed > 0) ? fixed : pb->cg_maxit;
    const int poll = 8;
    int it = 0;
    for (; it < cap; ++it) {
        dispatch<S>(pl.Q, pl.TEAM, [&](auto qc, auto tc) {
            constexpr int QQ = decltype(qc)::value, TT = decltype(tc)::value;
            hipLaunchKernelGGL((k_matvec<S, QQ, TT>), dim3(pl.nchunk, (unsigned)P), dim3(Geo<QQ, TT>::BS), 0, st,
                               W, ldw, (int)pl.M, pl.rows_per_chunk, pl.nchunk, pl.ld, pb->s, w, ws.pv, ws.scal, NS,
                               ws.iscal, ws.part1, ws.psc);
        });
        hipLaunchKernelGGL(k_cg_update, dim3((unsigned)P), dim3(256), 0, st, ws.part1, ws.psc, pl.nchunk, pl.ld,
                           pb->s, Wbar, ws.x, ws.r, ws.pv, ws.qv, ws.scal, NS, ws.iscal,
                           pb->cg_rtol * pb->cg_rtol, pb->cg_maxit, ws.active, status);
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
    hipLaunchKernelGGL(k_weights, dim3((unsigned)P), dim3(256), 0, st, rn2, Y_next, (int)pl.M, s2, eps2, w_out,
                       ws.c2, ws.scal, NS, ws.active, (int)P, warm);
    dispatch<S>(pl.Q, pl.TEAM, [&](auto qc, auto tc) {
        constexpr int QQ = decltype(qc)::value, TT = decltype(tc)::value;
        hipLaunchKernelGGL((k_moments<S, QQ, TT>), dim3(pl.nchunk, (unsigned)P), dim3(Geo<QQ, TT>::BS), 0, st, W,
                           ldw, (int)pl.M, pl.rows_per_chunk, pl.nchunk, pl.ld, w_out, ws.c2, ws.x, ws.scal, NS, warm,
                           ws.part1, ws.part2, ws.part3, ws.psc);
    });
    hipLaunchKernelGGL(k_moments_finish, dim3((unsigned)P), dim3(256), 0, st, ws.part1, ws.part2, ws.part3, ws.psc,
                       pl.nchunk, pl.ld, pb->s, lam, warm, Wbar_out, ws.x, ws.r, ws.pv, ws.scal, NS, ws.iscal,
                       ws.active);
    const int iters = run_cg<S>(pb, pl, P, W, ldw, w_out, Wbar_out, ws, status, st, err);
    if (err) return iters;
    hipLaunchKernelGGL(k_level_finish, dim3((unsigned)P), dim3(256), 0, st, ws.x, Wbar_out, pl.ld, (int)pl.d, pb->s,
                       ws.scal, NS, alpha_out, alpha_x_out);
    err = last_error();
    return iters;
}

template <typename S>
void launch_reverse(const fbsde_problem* pb, const Plan& pl, int64_t P, int k, S* W, int64_t ldw, const double* ax,
                    WS& ws, double* Y, double* rn2, uint32_t* status, hipStream_t st, double* dydc = nullptr,
                    const double* scal = nullptr, int shared = 0) {
    const Keys ky = keys_of(pb);
    const double dt = pb->T / (double)pb->N;
    dispatch<S>(pl.Q, pl.TEAM, [&](auto qc, auto tc) {
        constexpr int QQ = decltype(qc)::value, TT = decltype(tc)::value;
        hipLaunchKernelGGL((k_reverse<S, QQ, TT>), dim3(pl.nchunk, (unsigned)P), dim3(Geo<QQ, TT>::BS), 0, st, W,
                           ldw, (int)pl.M, pl.rows_per_chunk, (int)pl.d, pl.ld, k, (k == 0) ? 1 : 0, std::sqrt(dt),
                           pb->s, dt, ax, scal ? scal : ws.scal, NS, fspec_of(pb), pb->newton_iters, ky.k0, ky.k1,
                           pb->point_base, Y, rn2, dydc, status, shared);
    });
}

int tape_tag(const fbsde_problem* pb, int64_t P) {
    uint64_t h = 1469598103934665603ull;
    const uint64_t v[6] = {(uint64_t)pb->d, (uint64_t)pb->M, (uint64_t)pb->N, (uint64_t)P, (uint64_t)pb->prec,
                           pb->seed ^ ((uint64_t)pb->instance << 32) ^ pb->point_base};
    for (uint64_t x : v) { h ^= x; h *= 1099511628211ull; }
    return (int)(h & 0x7FFFFFFF) | 1;
}

void clear_status(uint32_t* status, int64_t P, hipStream_t st) {
    if (P > 0) hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::min<int64_t>((P + 255) / 256, 1024)), dim3(256), 0,
                                  st, status, P, 0u);
}

template <typename S>
int solve_impl(const fbsde_problem* pb, const Plan& pl, int64_t P, const double* x0, double* u, double* grad,
               uint32_t* status, WS& ws, bool tape, int32_t* cg_iters_out, hipStream_t st) {
    S* W = (S*)ws.W;
    const int64_t ldw = pl.ld;
    const int64_t PM = P * pl.M, PL = P * (int64_t)pl.ld;
    clear_status(status, P, st);
    double* Ycur = ws.Ya;
    double* Yk = ws.Yb;
    launch_forward<S>(pb, pl, P, x0, W, ldw, Ycur, ws.rn2, status, st);
    int err = last_error();
    if (err) return err;
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
        if (cg_iters_out) cg_iters_out[k] = iters;
        if (tape) {
            if (hipMemcpyAsync(ws.tax + (size_t)k * PL, ws.x, PL * 8, hipMemcpyDeviceToDevice, st) != hipSuccess ||
                hipMemcpyAsync(ws.tscal + (size_t)k * P * NS, ws.scal, (size_t)P * NS * 8, hipMemcpyDeviceToDevice,
                               st) != hipSuccess)
                return FBSDE_EHIP;
        }
        if (k > 0) {
            double* Yout = tape ? ws.tY + (size_t)k * PM : Yk;
            launch_reverse<S>(pb, pl, P, k, W, ldw, ws.x, ws, Yout, ws.rn2, status, st, ws.c2);
            if (!tape) std::swap(Ycur, Yk);
            else Ycur = Yout;
        } else {
            hipLaunchKernelGGL(k_outputs, dim3((unsigned)P), dim3(256), 0, st, ws.x, pl.ld, (int)pl.d, ws.scal, NS,
                               fspec_of(pb), pb->T / (double)pb->N, pb->newton_iters, u, grad, status);
        }
        err = last_error();
        if (err) return err;
    }
    if (tape) hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, ws.tag, tape_tag(pb, P));
    return last_error();
}

template <typename S>
int backward_impl(const fbsde_problem* pb, const Plan& pl, int64_t P, const double* x0, const double* u_bar,
                  double* x0_bar, double* gp_bar, double* fp_bar, uint32_t* status, WS& ws, hipStream_t st) {
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
                           k > 0 ? ws.tw + (size_t)(k - 1) * PM : nullptr, ws.psc, pl.nchunk,
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
        hipLaunchKernelGGL(k_adj_rhs_finish, dim3((unsigned)P), dim3(256), 0, st, ws.part1, pl.nchunk, pl.ld, pb->s,
                           lam, Wbar_k, ws.tax + (size_t)k * PL, ws.adj, ws.x, ws.r, ws.pv, ws.scal, NS, ws.iscal,
                           ws.active);
        run_cg<S>(pb, pl, P, W, ldw, w_k, Wbar_k, ws, status, st, err);
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
                       ws.psc, pl.nchunk, nullptr, ws.tscal, NS, fs, dt, pb->newton_iters, (int)pl.M, u_bar, ws.cbar,
                       ws.adj, 0, 1, status);
    dispatch<S>(pl.Q, pl.TEAM, [&](auto qc, auto tc) {
        constexpr int QQ = decltype(qc)::value, TT = decltype(tc)::value;
        hipLaunchKernelGGL((k_adj_terminal<S, QQ, TT>), dim3(pl.nchunk, (unsigned)P), dim3(Geo<QQ, TT>::BS), 0, st, W,
                           ldw, (int)pl.M, pl.rows_per_chunk, pl.nchunk, (int)pl.d, pl.ld, x0, pb->mu, pb->gvec, pb->s,
                           pb->T, pb->g_kind, pb->gp[0], ws.G, ws.part1, ws.psc);
    });
    hipLaunchKernelGGL(k_adj_x0bar, dim3((unsigned)P), dim3(256), 0, st, ws.part1, ws.psc, pl.nchunk, (int)pl.d,
                       pl.ld, x0, pb->mu, pb->gvec, pb->s, pb->T, pb->g_kind, ws.adj, x0_bar);
    hipLaunchKernelGGL(k_adj_params, dim3(1), dim3(64), 0, st, ws.adj, P, gp_bar, fp_bar);
    // the tape is consumed: the state no longer holds W_1 of the primal pass
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, ws.tag, 0);
    return last_error();
}

__global__ void k_info_to_status(const int* info, uint32_t* status, int64_t P) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p < P && *info) atomicOr(&status[p], (uint32_t)ST_NONFINITE);
}

// Algorithm 1 with increments shared by all points: one cloud, one ridge system per level, the
// regressions of all points as dense MFMA contractions (fbsde_shared.hpp).
template <typename T>
int solve_shared_impl(const fbsde_problem* pb, const Plan& pl, const Plan& pl1, int64_t P, const double* x0,
                      double* u, double* grad, uint32_t* status, SWS& ws, hipStream_t st) {
    T* W = (T*)ws.W;
    T* Dt = (T*)ws.Dt;
    T* K = (T*)ws.K;
    T* R = (T*)ws.R;
    T* ax = (T*)ws.ax;
    T* xc = (T*)ws.xc;
    const int M = (int)pl.M, ld = pl.ld, d = (int)pl.d, Pi = (int)P;
    const double dt = pb->T / (double)pb->N, s = pb->s, s2 = s * s;
    const Keys ky = keys_of(pb);
    const FSpec fs = fspec_of(pb);
    clear_status(status, P, st);
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, ws.info, 0);
    // the shared cloud at t_N (one row set, stream 0xFFFFFFFF) and its squared norms
    dispatch<T>(pl1.Q, pl1.TEAM, [&](auto qc, auto tc) {
        constexpr int QQ = decltype(qc)::value, TT = decltype(tc)::value;
        hipLaunchKernelGGL((k_forward<T, QQ, TT>), dim3(pl1.nchunk, 1), dim3(Geo<QQ, TT>::BS), 0, st, W, (int64_t)ld,
                           M, pl1.rows_per_chunk, nullptr, nullptr, nullptr, d, ld, (int)pl.N, std::sqrt(dt), s, pb->T,
                           G_QUAD, 1.0, 0.0, ky.k0, ky.k1, 0u, 1, ws.ysc, ws.rn2, status);
    });
    double* Ycur = ws.Ya;
    double* Yk = ws.Yb;
    if (pb->g_kind == FBSDE_G_AFFINE) {
        hipLaunchKernelGGL((k_sh_affine_terminal<T>), dim3((unsigned)P), dim3(256), 0, st, W, ld, M, d, pb->gvec, x0,
                           pb->mu, pb->T, s, pb->gp[0], Pi, Ycur);
    } else {
        hipLaunchKernelGGL((k_sh_xc<T>), dim3((unsigned)P), dim3(256), 0, st, x0, pb->mu, d, ld, pb->T, xc, ws.xc2);
        gemm<T, true>(Pi, M, ld, xc, ld, W, ld,
                      EpiTerminal{Ycur, ws.xc2, ws.rn2, s, pb->gp[0], pb->gp[1], pb->g_kind, M, d, status}, st);
    }
    int err = last_error();
    if (err) return err;
    const unsigned cblocks = (unsigned)((ld + 255) / 256);
    const int rch = std::min(SH_RCH, M);
    const int rpc = (M + rch - 1) / rch;
    for (int k = (int)pl.N - 1; k >= 0; --k) {
        const double t_next = (double)(k + 1) * dt;
        const double eps2 = (pb->eps_h > 0.0) ? pb->eps_h * pb->eps_h * s2 * t_next * (double)d : 0.0;
        const double lam = pb->ridge_rel * s2 * t_next;
        hipLaunchKernelGGL(k_sh_weights, dim3(1), dim3(256), 0, st, ws.rn2, M, s2, eps2, ws.w, ws.sqw);
        hipLaunchKernelGGL((k_sh_rhs<T>), dim3((unsigned)P), dim3(256), 0, st, Ycur, ws.w, ws.sqw, M, R, ws.scal, NS);
        hipLaunchKernelGGL((k_sh_colsum<T>), dim3(cblocks, (unsigned)((M + rpc - 1) / rpc)), dim3(256), 0, st, W, ld,
                           M, rpc, ws.w, ws.wpart);
        hipLaunchKernelGGL((k_sh_dtilde<T>), dim3(cblocks, 32), dim3(256), 0, st, W, ld, M, ws.wpart,
                           (M + rpc - 1) / rpc, ws.sqw, ws.Wbar, Dt);
        if (pl.M <= pl.d) {
            // dual: alpha_x[p] = s F[p] Dt with F = R (lam I + s^2 Dt Dt^T)^{-1}
            gemm<T, true>(M, M, ld, Dt, ld, Dt, ld, EpiStore<T>{K, (int64_t)M, s2, 0.0, lam}, st, 1);
            cholesky<T>(K, M, M, ws.info, st);
            cholesky_solve_rows<T>(K, M, M, R, M, Pi, st);
            gemm<T, false>(Pi, ld, M, R, M, Dt, ld, EpiStore<T>{ax, (int64_t)ld, s, 0.0, 0.0}, st);
        } else {
            // primal: alpha_x[p] = b_p (lam I + s^2 Dt^T Dt)^{-1}, b_p = s R[p] Dt (the pad rows/columns
            // of the ld x ld matrix are lam I and decouple)
            T* DtT = (T*)ws.DtT;
            hipLaunchKernelGGL((k_transpose<T>), dim3(cblocks * 8, (unsigned)((M + 31) / 32)), dim3(256), 0, st, Dt,
                               (int64_t)ld, M, ld, DtT, (int64_t)M);
            gemm<T, true>(ld, ld, M, DtT, M, DtT, M, EpiStore<T>{K, (int64_t)ld, s2, 0.0, lam, d, 1.0}, st, 1);
            cholesky<T>(K, ld, ld, ws.info, st);
            gemm<T, false>(Pi, ld, M, R, M, Dt, ld, EpiStore<T>{ax, (int64_t)ld, s, 0.0, 0.0}, st);
            cholesky_solve_rows<T>(K, ld, ld, ax, ld, Pi, st);
        }
        hipLaunchKernelGGL((k_sh_point_finish<T>), dim3((unsigned)P), dim3(256), 0, st, ax, ld, ws.Wbar, s, ws.scal, NS);
        if (k > 0) {
            // reverse the shared cloud to t_k (its Newton output goes to scratch) and |W_k|^2
            dispatch<T>(pl1.Q, pl1.TEAM, [&](auto qc, auto tc) {
                constexpr int QQ = decltype(qc)::value, TT = decltype(tc)::value;
                hipLaunchKernelGGL((k_reverse<T, QQ, TT>), dim3(pl1.nchunk, 1), dim3(Geo<QQ, TT>::BS), 0, st, W,
                                   (int64_t)ld, M, pl1.rows_per_chunk, d, ld, k, 0, std::sqrt(dt), s, dt, ws.Wbar,
                                   ws.scal, NS, fs, 1, ky.k0, ky.k1, 0u, ws.ysc, ws.rn2, nullptr, status, 1);
            });
            gemm<T, true>(Pi, M, ld, ax, ld, W, ld, EpiNewton{Yk, ws.scal, NS, M, pb->newton_iters, fs, s, dt, status},
                          st);
            std::swap(Ycur, Yk);
        } else {
            hipLaunchKernelGGL((k_sh_outputs<T>), dim3((unsigned)P), dim3(256), 0, st, ax, ld, d, ws.scal, NS, fs, dt,
                               pb->newton_iters, u, grad, status);
        }
        if ((err = last_error())) return err;
    }
    hipLaunchKernelGGL(k_info_to_status, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, ws.info, status, P);
    return last_error();
}

// ------------------------------------------------------------------ persistent batched launch
SlotLayout slot_layout(int64_t M, int ld, size_t esz) {
    SlotLayout lay;
    size_t off = (size_t)round_up((int64_t)(M * ld * esz), 256);
    lay.off_rn2 = off; off += (size_t)round_up(M * 8, 256);
    lay.off_Y = off; off += (size_t)round_up(M * 8, 256);
    lay.off_w = off; off += (size_t)round_up(M * 8, 256);
    lay.off_c2 = off; off += (size_t)round_up(M * 8, 256);
    lay.off_vec = off; off += (size_t)round_up(6 * (int64_t)ld * 8, 256);
    lay.bytes = off;
    return lay;
}

struct BatchClass {
    int prec, Q, TEAM;
    std::vector<int> insts;   // instance indices, by decreasing per-point cost
    int64_t items = 0;
    int64_t maxM = 0;
    int ld = 0;
};

int batch_classes(const fbsde_problem* pbs, int64_t n_inst, const int64_t* P, std::vector<BatchClass>& out) {
    std::map<std::tuple<int, int, int, int>, BatchClass> cls;
    for (int64_t i = 0; i < n_inst; ++i) {
        int rc = check_problem(&pbs[i], P[i]);
        if (rc) return rc;
        if (pbs[i].shared_dw) return FBSDE_EINVAL;
        Plan pl;
        if ((rc = make_plan(&pbs[i], 1, pl))) return rc;
        const auto key = std::make_tuple(pbs[i].prec, pl.Q, pl.TEAM, pl.ld);
        BatchClass& c = cls[key];
        c.prec = pbs[i].prec; c.Q = pl.Q; c.TEAM = pl.TEAM; c.ld = pl.ld;
        c.insts.push_back((int)i);
        c.items += P[i];
        c.maxM = std::max<int64_t>(c.maxM, pbs[i].M);
    }
    for (auto& kv : cls) {
        BatchClass& c = kv.second;
        std::stable_sort(c.insts.begin(), c.insts.end(), [&](int a, int b) { return pbs[a].M > pbs[b].M; });
        out.push_back(c);
    }
    return FBSDE_OK;
}

size_t batch_header_bytes(int64_t n_inst, int64_t total_items) {
    return (size_t)round_up(n_inst * (int64_t)sizeof(BatchInst), 256) +
           (size_t)round_up(total_items * (int64_t)sizeof(BatchItem), 256) + 256;
}

template <typename S>
void launch_batched_class(const BatchClass& c, const BatchInst* d_insts, const BatchItem* d_items, int n_items,
                          int* queue, char* slots, const SlotLayout& lay, int nslots, hipStream_t st) {
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, queue, 0);
    dispatch<S>(c.Q, c.TEAM, [&](auto qc, auto tc) {
        constexpr int QQ = decltype(qc)::value, TT = decltype(tc)::value;
        hipLaunchKernelGGL((k_batched<S, QQ, TT>), dim3(nslots), dim3(Geo<QQ, TT>::BS), 0, st, d_insts, d_items,
                           n_items, queue, slots, lay);
    });
}

}  // namespace

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
        if (flags & FBSDE_WS_TAPE) return FBSDE_EINVAL;   // the shared form has no adjoint tape yet
        SWS sws;
        *bytes = carve_shared(pl, P, nullptr, sws);
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
    if (ldw < pl.ld || ldw % 4 != 0 || !x0 || !W || !Y || !status) return FBSDE_EINVAL;
    if (P == 0) return FBSDE_OK;
    hipStream_t st = (hipStream_t)stream;
    clear_status(status, P, st);
    if (pb->prec == FBSDE_F64) launch_forward<double>(pb, pl, P, x0, (double*)W, ldw, Y, nullptr, status, st);
    else launch_forward<float>(pb, pl, P, x0, (float*)W, ldw, Y, nullptr, status, st);
    return last_error();
}

int fbsde_solve_step(const fbsde_problem* pb, int64_t P, int32_t k, const double* x0, void* W, int64_t ldw,
                     const double* Y_next, double* Y, double* alpha, double* alpha_x, uint32_t* status, void* wsp,
                     size_t ws_bytes, fbsde_stream stream) {
    (void)x0;
    int rc = check_problem(pb, P);
    if (rc) return rc;
    if (pb->shared_dw) return FBSDE_EINVAL;   // the shared form runs only as a whole solve
    Plan pl;
    if ((rc = make_plan(pb, P, pl))) return rc;
    if (k < 0 || k >= pb->N || ldw < pl.ld || ldw % 4 != 0 || !W || !Y_next || !Y || Y == Y_next || !status ||
        !wsp)
        return FBSDE_EINVAL;
    WS ws;
    if (carve(pl, P, 0, nullptr, ws) > ws_bytes) return FBSDE_ENOSPC;
    carve(pl, P, 0, (char*)wsp, ws);
    if (P == 0) return FBSDE_OK;
    hipStream_t st = (hipStream_t)stream;
    int err = FBSDE_OK;
    if (pb->prec == FBSDE_F64) {
        double* Ws = (double*)W;
        launch_rownorm<double>(pl, P, Ws, ldw, ws.rn2, st);
        run_level<double>(pb, pl, P, k, Ws, ldw, Y_next, ws.rn2, ws.w, ws.Wbar, ws, alpha, alpha_x, status, st, err);
        if (err) return err;
        launch_reverse<double>(pb, pl, P, k, Ws, ldw, ws.x, ws, Y, ws.rn2, status, st);
    } else {
        float* Ws = (float*)W;
        launch_rownorm<float>(pl, P, Ws, ldw, ws.rn2, st);
        run_level<float>(pb, pl, P, k, Ws, ldw, Y_next, ws.rn2, ws.w, ws.Wbar, ws, alpha, alpha_x, status, st, err);
        if (err) return err;
        launch_reverse<float>(pb, pl, P, k, Ws, ldw, ws.x, ws, Y, ws.rn2, status, st);
    }
    return last_error();
}

int fbsde_solve(const fbsde_problem* pb, int64_t P, const double* x0, double* u, double* grad, uint32_t* status,
                void* wsp, size_t ws_bytes, int32_t flags, int32_t* cg_iters_out, fbsde_stream stream) {
    int rc = check_problem(pb, P);
    if (rc) return rc;
    Plan pl;
    if ((rc = make_plan(pb, P, pl))) return rc;
    if (!x0 || !u || !status || !wsp) return FBSDE_EINVAL;
    if (pb->shared_dw) {
        if (flags & FBSDE_WS_TAPE) return FBSDE_EINVAL;
        Plan pl1;
        if ((rc = make_plan(pb, 1, pl1))) return rc;
        SWS sws;
        if (carve_shared(pl, P, nullptr, sws) > ws_bytes) return FBSDE_ENOSPC;
        carve_shared(pl, P, (char*)wsp, sws);
        if (P == 0) return FBSDE_OK;
        if (cg_iters_out)
            for (int64_t k = 0; k < pb->N; ++k) cg_iters_out[k] = 0;   // direct (Cholesky) solve
        hipStream_t st = (hipStream_t)stream;
        if (pb->prec == FBSDE_F64) return solve_shared_impl<double>(pb, pl, pl1, P, x0, u, grad, status, sws, st);
        return solve_shared_impl<float>(pb, pl, pl1, P, x0, u, grad, status, sws, st);
    }
    WS ws;
    if (carve(pl, P, flags, nullptr, ws) > ws_bytes) return FBSDE_ENOSPC;
    carve(pl, P, flags, (char*)wsp, ws);
    if (P == 0) return FBSDE_OK;
    const bool tape = (flags & FBSDE_WS_TAPE) != 0;
    hipStream_t st = (hipStream_t)stream;
    if (pb->prec == FBSDE_F64) return solve_impl<double>(pb, pl, P, x0, u, grad, status, ws, tape, cg_iters_out, st);
    return solve_impl<float>(pb, pl, P, x0, u, grad, status, ws, tape, cg_iters_out, st);
}

int fbsde_solve_backward(const fbsde_problem* pb, int64_t P, const double* x0, const double* u_bar, double* x0_bar,
                         double* gp_bar, double* fp_bar, uint32_t* status, void* wsp, size_t ws_bytes,
                         fbsde_stream stream) {
    int rc = check_problem(pb, P);
    if (rc) return rc;
    if (pb->shared_dw) return FBSDE_EINVAL;   // the shared form runs only as a whole solve
    Plan pl;
    if ((rc = make_plan(pb, P, pl))) return rc;
    if (!x0 || !u_bar || !x0_bar || !gp_bar || !fp_bar || !status || !wsp) return FBSDE_EINVAL;
    WS ws;
    if (carve(pl, P, FBSDE_WS_TAPE, nullptr, ws) > ws_bytes) return FBSDE_ENOSPC;
    carve(pl, P, FBSDE_WS_TAPE, (char*)wsp, ws);
    if (P == 0) return FBSDE_OK;
    hipStream_t st = (hipStream_t)stream;
    int tag = 0;
    if (hipMemcpyAsync(&tag, ws.tag, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return FBSDE_EHIP;
    if (tag != tape_tag(pb, P)) return FBSDE_ESTATE;
    if (pb->prec == FBSDE_F64)
        return backward_impl<double>(pb, pl, P, x0, u_bar, x0_bar, gp_bar, fp_bar, status, ws, st);
    return backward_impl<float>(pb, pl, P, x0, u_bar, x0_bar, gp_bar, fp_bar, status, ws, st);
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
    hipLaunchKernelGGL(k_normals, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (int)pb->d, j0, rows, k, q, ky.k0,
                       ky.k1, out, words);
    return last_error();
}

int fbsde_time_kernel(const fbsde_problem* pb, int64_t P, int32_t which, int32_t reps, void* wsp, size_t ws_bytes,
                      float* avg_ms, fbsde_stream stream) {
    int rc = check_problem(pb, P);
    if (rc) return rc;
    if (pb->shared_dw) return FBSDE_EINVAL;   // the shared form runs only as a whole solve
    Plan pl;
    if ((rc = make_plan(pb, P, pl))) return rc;
    if (!wsp || !avg_ms || reps < 1 || which < 0 || which > 3 || P == 0) return FBSDE_EINVAL;
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
                    hipLaunchKernelGGL((k_matvec<S, QQ, TT>), dim3(pl.nchunk, (unsigned)P), dim3(Geo<QQ, TT>::BS),
                                       0, st, W, ldw, (int)pl.M, pl.rows_per_chunk, pl.nchunk, pl.ld, pb->s, ws.w,
                                       ws.pv, ws.scal, NS, ws.iscal, ws.part1, ws.psc);
                });
            } else if (which == 1) {
                launch_reverse<S>(pb, pl, P, 1, W, ldw, ws.x, ws, ws.Yb, ws.rn2, (uint32_t*)ws.iscal, st);
            } else if (which == 2) {
                dispatch<S>(pl.Q, pl.TEAM, [&](auto qc, auto tc) {
                    constexpr int QQ = decltype(qc)::value, TT = decltype(tc)::value;
                    hipLaunchKernelGGL((k_moments<S, QQ, TT>), dim3(pl.nchunk, (unsigned)P), dim3(Geo<QQ, TT>::BS),
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

int fbsde_gemm(int32_t prec, int32_t nt, int64_t m, int64_t n, int64_t k, const void* A, int64_t lda, const void* B,
               int64_t ldb, void* C, int64_t ldc, double alpha, double beta, fbsde_stream stream) {
    if ((prec != FBSDE_F64 && prec != FBSDE_F32C) || m < 0 || n < 0 || k < 0 || !A || !B || !C) return FBSDE_EINVAL;
    if (m > INT32_MAX || n > INT32_MAX || k > INT32_MAX || lda < k * (nt ? 1 : 0) || ldc < n) return FBSDE_EINVAL;
    if (nt ? ldb < k : ldb < n) return FBSDE_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (prec == FBSDE_F64) {
        if (nt) gemm<double, true>((int)m, (int)n, (int)k, (const double*)A, lda, (const double*)B, ldb,
                                   EpiStore<double>{(double*)C, ldc, alpha, beta, 0.0}, st);
        else gemm<double, false>((int)m, (int)n, (int)k, (const double*)A, lda, (const double*)B, ldb,
                                 EpiStore<double>{(double*)C, ldc, alpha, beta, 0.0}, st);
    } else {
        if (nt) gemm<float, true>((int)m, (int)n, (int)k, (const float*)A, lda, (const float*)B, ldb,
                                  EpiStore<float>{(float*)C, ldc, alpha, beta, 0.0}, st);
        else gemm<float, false>((int)m, (int)n, (int)k, (const float*)A, lda, (const float*)B, ldb,
                                EpiStore<float>{(float*)C, ldc, alpha, beta, 0.0}, st);
    }
    return last_error();
}

size_t fbsde_cholesky_workspace(int32_t prec, int64_t n, int64_t P) {
    (void)prec; (void)n; (void)P;
    return 256;   // the status word of the factorisation
}

int fbsde_cholesky_solve(int32_t prec, int64_t n, void* K, int64_t ldk, int64_t P, void* R, int64_t ldr, void* ws,
                         size_t ws_bytes, int32_t* info, fbsde_stream stream) {
    if ((prec != FBSDE_F64 && prec != FBSDE_F32C) || n < 1 || n > INT32_MAX || P < 0 || P > INT32_MAX || !K || !ws ||
        !info || ldk < n || (P > 0 && (!R || ldr < n)))
        return FBSDE_EINVAL;
    if (fbsde_cholesky_workspace(prec, n, P) > ws_bytes) return FBSDE_ENOSPC;
    hipStream_t st = (hipStream_t)stream;
    int* dinfo = (int*)ws;
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, dinfo, 0);
    if (prec == FBSDE_F64) {
        cholesky<double>((double*)K, ldk, (int)n, dinfo, st);
        if (P > 0) cholesky_solve_rows<double>((const double*)K, ldk, (int)n, (double*)R, ldr, (int)P, st);
    } else {
        cholesky<float>((float*)K, ldk, (int)n, dinfo, st);
        if (P > 0) cholesky_solve_rows<float>((const float*)K, ldk, (int)n, (float*)R, ldr, (int)P, st);
    }
    if (hipMemcpyAsync(info, dinfo, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return FBSDE_EHIP;
    return last_error();
}

int fbsde_batched_workspace_size(const fbsde_problem* pbs, int64_t n_inst, const int64_t* P, int32_t max_slots,
                                 size_t* bytes) {
    if (!pbs || !P || !bytes || n_inst < 1 || max_slots < 1) return FBSDE_EINVAL;
    std::vector<BatchClass> cls;
    int rc = batch_classes(pbs, n_inst, P, cls);
    if (rc) return rc;
    int64_t total = 0;
    size_t slot_max = 0;
    for (const auto& c : cls) {
        total += c.items;
        const SlotLayout lay = slot_layout(c.maxM, c.ld, c.prec == FBSDE_F64 ? 8 : 4);
        slot_max = std::max(slot_max, lay.bytes * (size_t)std::min<int64_t>(c.items, max_slots));
    }
    *bytes = batch_header_bytes(n_inst, total) + slot_max;
    return FBSDE_OK;
}

int fbsde_solve_batched(const fbsde_problem* pbs, int64_t n_inst, const int64_t* P, const double* const* x0,
                        double* const* u, double* const* grad, uint32_t* const* status, int32_t max_slots, void* wsp,
                        size_t ws_bytes, fbsde_stream stream) {
    if (!pbs || !P || !x0 || !u || !status || !wsp || n_inst < 1 || max_slots < 1) return FBSDE_EINVAL;
    std::vector<BatchClass> cls;
    int rc = batch_classes(pbs, n_inst, P, cls);
    if (rc) return rc;
    size_t need = 0;
    if ((rc = fbsde_batched_workspace_size(pbs, n_inst, P, max_slots, &need))) return rc;
    if (need > ws_bytes) return FBSDE_ENOSPC;
    for (int64_t i = 0; i < n_inst; ++i)
        if (P[i] > 0 && (!x0[i] || !u[i] || !status[i])) return FBSDE_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    // descriptor table and the work items of every class (device copies in the workspace header)
    std::vector<BatchInst> hi((size_t)n_inst);
    for (int64_t i = 0; i < n_inst; ++i) {
        const fbsde_problem* pb = &pbs[i];
        Plan pl;
        make_plan(pb, 1, pl);
        const Keys ky = keys_of(pb);
        BatchInst& b = hi[(size_t)i];
        b.d = (int)pb->d; b.ld = pl.ld; b.M = (int)pb->M; b.N = (int)pb->N; b.P = (int)P[i];
        b.T = pb->T; b.s = pb->s; b.eps_h = pb->eps_h; b.ridge_rel = pb->ridge_rel;
        b.rtol2 = pb->cg_rtol * pb->cg_rtol;
        b.newton_iters = pb->newton_iters;
        b.cg_maxit = pb->cg_fixed_iters > 0 ? pb->cg_fixed_iters : pb->cg_maxit;
        b.g_kind = pb->g_kind;
        b.warm = (pb->M > pb->d + 1) ? 1 : 0;
        b.f = fspec_of(pb);
        b.ga = pb->gp[0]; b.gb = pb->gp[1];
        b.mu = pb->mu; b.gvec = pb->gvec;
        b.k0 = ky.k0; b.k1 = ky.k1; b.point_base = pb->point_base;
        b.x0 = x0[i]; b.u = u[i]; b.grad = grad ? grad[i] : nullptr; b.status = status[i];
        clear_status(status[i], P[i], st);
    }
    std::vector<BatchItem> items;
    std::vector<std::pair<int64_t, int64_t>> ranges;   // per class: [first item, count)
    for (const auto& c : cls) {
        const int64_t first = (int64_t)items.size();
        for (int i : c.insts)
            for (int64_t p = 0; p < P[i]; ++p) items.push_back(BatchItem{i, (int)p});
        ranges.emplace_back(first, (int64_t)items.size() - first);
    }
    char* base = (char*)wsp;
    BatchInst* d_insts = (BatchInst*)base;
    BatchItem* d_items = (BatchItem*)(base + round_up(n_inst * (int64_t)sizeof(BatchInst), 256));
    int* queue = (int*)(base + batch_header_bytes(n_inst, (int64_t)items.size()) - 256);
    char* slots = base + batch_header_bytes(n_inst, (int64_t)items.size());
    if (hipMemcpyAsync(d_insts, hi.data(), hi.size() * sizeof(BatchInst), hipMemcpyHostToDevice, st) != hipSuccess)
        return FBSDE_EHIP;
    if (!items.empty() &&
        hipMemcpyAsync(d_items, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice, st) != hipSuccess)
        return FBSDE_EHIP;
    // the host tables must outlive the copies
    if (hipStreamSynchronize(st) != hipSuccess) return FBSDE_EHIP;
    for (size_t ci = 0; ci < cls.size(); ++ci) {
        const BatchClass& c = cls[ci];
        if (ranges[ci].second == 0) continue;
        const SlotLayout lay = slot_layout(c.maxM, c.ld, c.prec == FBSDE_F64 ? 8 : 4);
        const int nslots = (int)std::min<int64_t>(ranges[ci].second, max_slots);
        if (c.prec == FBSDE_F64)
            launch_batched_class<double>(c, d_insts, d_items + ranges[ci].first, (int)ranges[ci].second, queue, slots,
                                         lay, nslots, st);
        else
            launch_batched_class<float>(c, d_insts, d_items + ranges[ci].first, (int)ranges[ci].second, queue, slots,
                                        lay, nslots, st);
        if ((rc = last_error())) return rc;
    }
    return FBSDE_OK;
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
