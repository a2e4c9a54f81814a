// Host side of the shared-increment form (every point uses the same increments): workspace, the dense
// level chain on the matrix cores, and the exported dense helpers (MFMA GEMM, blocked Cholesky solve).
#include "fbsde_host.hpp"
#include "fbsde_shared.hpp"

using namespace fbsde;
using namespace fbsde::host;

namespace {

// ------------------------------------------------------------------ shared-increment workspace
struct SWS {
    void *W, *Dt, *K, *R, *ax, *xc, *DtT, *Li, *Sq, *R2;
    double *Wbar, *wpart, *w, *sqw, *rn2, *Ya, *Yb, *scal, *xc2, *ysc;
    int* info;
    // tape for the reverse mode, per level k (cloud t_{k+1}): Y_k [P][M], alpha_x [P][ld], the
    // Cholesky factor, w and sqrt(w) [M], Wbar [ld], the point scalars; |X_N|^2 [P][M]
    bool tape = false;
    double *tY, *tw, *tsqw, *tWbar, *tscal, *tq;
    void *tax, *tK;
    int* tag;
    // reverse-mode work
    double *G, *cbar, *adj, *psc;
    size_t kn;
};
constexpr int SH_RCH = 64;   // row chunks of the two-stage weighted mean

size_t carve_shared(const Plan& pl, int64_t P, int32_t flags, char* base, SWS& ws) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        char* p = base ? base + off : nullptr;
        off += round_up((int64_t)bytes, 256);
        return p;
    };
    const size_t M = pl.M, ld = pl.ld, e = pl.esz, N = pl.N;
    ws.W = take(M * ld * e);
    ws.Dt = take(M * ld * e);
    // dual form (M <= d): K is M x M; primal form (M > d): K is ld x ld, Dt^T [ld][M] is needed
    const bool primal = pl.M > pl.d;
    const size_t kn = primal ? ld : M;
    ws.kn = kn;
    ws.K = take(kn * kn * e);
    ws.Li = take(kn * kn * e);
    ws.Sq = take(kn * kn * e);
    ws.DtT = primal ? take(ld * M * e) : nullptr;
    ws.R = take((size_t)P * M * e);
    ws.R2 = take((size_t)P * M * e);
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
    ws.tape = (flags & FBSDE_WS_TAPE) != 0;
    if (ws.tape) {
        ws.tY = (double*)take(N * P * M * 8);
        ws.tax = take(N * P * ld * e);
        ws.tK = take(N * kn * kn * e);
        ws.tw = (double*)take(N * M * 8);
        ws.tsqw = (double*)take(N * M * 8);
        ws.tWbar = (double*)take(N * ld * 8);
        ws.tscal = (double*)take(N * P * NS * 8);
        ws.tq = (double*)take((size_t)P * M * 8);
        ws.tag = (int*)take(64);
        ws.G = (double*)take((size_t)P * M * 8);
        ws.cbar = (double*)take((size_t)P * M * 8);
        ws.adj = (double*)take((size_t)P * A_NS * 8);
        ws.psc = (double*)take((size_t)P * 4 * 8);
    }
    return off;
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
    T* R = (T*)ws.R;
    T* xc = (T*)ws.xc;
    const int M = (int)pl.M, ld = pl.ld, d = (int)pl.d, Pi = (int)P;
    const double dt = pb->T / (double)pb->N, s = pb->s, s2 = s * s;
    const FSpec fs = fspec_of(pb);
    clear_status(status, P, st);
    set_int(ws.info, 0, st);
    // the shared cloud at t_N (one row set, stream 0xFFFFFFFF) and its squared norms
    shared_forward<T>(pb, pl1, W, ws.ysc, ws.rn2, status, st);
    double* Ycur = ws.Ya;
    double* Yk = ws.Yb;
    if (pb->g_kind == FBSDE_G_AFFINE || pb->g_kind == FBSDE_G_LOGISTIC) {
        hipLaunchKernelGGL((k_sh_affine_terminal<T>), dim3((unsigned)P), dim3(256), 0, st, W, ld, M, d, pb->gvec, x0,
                           pb->mu, pb->T, s, pb->gp[0], Pi, pb->g_kind, Ycur, ws.tape ? ws.tq : nullptr, status);
    } else {
        hipLaunchKernelGGL((k_sh_xc<T>), dim3((unsigned)P), dim3(256), 0, st, x0, pb->mu, d, ld, pb->T, xc, ws.xc2);
        gemm<T, true>(Pi, M, ld, xc, ld, W, ld,
                      EpiTerminal{Ycur, ws.xc2, ws.rn2, s, pb->gp[0], pb->gp[1], pb->g_kind, M, d, status,
                                  ws.tape ? ws.tq : nullptr}, st);
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
        // with the tape, the level's weights, mean, factor, slope and scalars are written in place
        double* w = ws.tape ? ws.tw + (size_t)k * M : ws.w;
        double* sqw = ws.tape ? ws.tsqw + (size_t)k * M : ws.sqw;
        double* Wbar = ws.tape ? ws.tWbar + (size_t)k * ld : ws.Wbar;
        double* scal = ws.tape ? ws.tscal + (size_t)k * P * NS : ws.scal;
        T* K = ws.tape ? (T*)ws.tK + (size_t)k * ws.kn * ws.kn : (T*)ws.K;
        T* ax = ws.tape ? (T*)ws.tax + (size_t)k * P * ld : (T*)ws.ax;
        hipLaunchKernelGGL(k_sh_weights, dim3(1), dim3(256), 0, st, ws.rn2, M, s2, eps2, w, sqw);
        hipLaunchKernelGGL((k_sh_rhs<T>), dim3((unsigned)P), dim3(256), 0, st, Ycur, w, sqw, M, R, scal, NS);
        hipLaunchKernelGGL((k_sh_colsum<T>), dim3(cblocks, (unsigned)((M + rpc - 1) / rpc)), dim3(256), 0, st, W, ld,
                           M, rpc, w, ws.wpart);
        hipLaunchKernelGGL((k_sh_dtilde<T>), dim3(cblocks, 32), dim3(256), 0, st, W, ld, M, ws.wpart,
                           (M + rpc - 1) / rpc, sqw, Wbar, Dt);
        if (pl.M <= pl.d) {
            // dual: alpha_x[p] = s F[p] Dt with F = R (lam I + s^2 Dt Dt^T)^{-1}
            // (K^{-1} formed once per level from the factor: every solve is then one GEMM; the Gram
            // matrix carries the lift c sqrt(w) sqrt(w)^T of its null direction, c ~ s^2 t_{k+1} d / M)
            const double lift = s2 * t_next * (double)d / (double)M;
            gemm<T, true>(M, M, ld, Dt, ld, Dt, ld, EpiGram<T>{K, (int64_t)M, s2, lam, lift, sqw}, st, 1);
            spd_inverse<T>(K, M, M, K, M, (T*)ws.Li, (T*)ws.Sq, ws.info, st);
            gemm<T, false>(Pi, M, M, R, M, K, M, EpiStore<T>{(T*)ws.R2, (int64_t)M, 1.0, 0.0, 0.0}, st);
            gemm<T, false>(Pi, ld, M, (T*)ws.R2, M, Dt, ld, EpiStore<T>{ax, (int64_t)ld, s, 0.0, 0.0}, st);
        } else {
            // primal: alpha_x[p] = b_p (lam I + s^2 Dt^T Dt)^{-1}, b_p = s R[p] Dt (the pad rows/columns
            // of the ld x ld matrix are lam I and decouple)
            T* DtT = (T*)ws.DtT;
            hipLaunchKernelGGL((k_transpose<T>), dim3(cblocks * 8, (unsigned)((M + 31) / 32)), dim3(256), 0, st, Dt,
                               (int64_t)ld, M, ld, DtT, (int64_t)M);
            gemm<T, true>(ld, ld, M, DtT, M, DtT, M, EpiStore<T>{K, (int64_t)ld, s2, 0.0, lam, d, 1.0}, st, 1);
            spd_inverse<T>(K, ld, ld, K, ld, (T*)ws.Li, (T*)ws.Sq, ws.info, st);
            gemm<T, false>(Pi, ld, M, R, M, Dt, ld, EpiStore<T>{xc, (int64_t)ld, s, 0.0, 0.0}, st);
            gemm<T, false>(Pi, ld, ld, xc, ld, K, ld, EpiStore<T>{ax, (int64_t)ld, 1.0, 0.0, 0.0}, st);
        }
        hipLaunchKernelGGL((k_sh_point_finish<T>), dim3((unsigned)P), dim3(256), 0, st, ax, ld, Wbar, s, scal, NS);
        if (k > 0) {
            // reverse the shared cloud to t_k (its Newton output goes to scratch) and |W_k|^2
            shared_reverse<T>(pb, pl1, k, W, Wbar, scal, ws.ysc, ws.rn2, status, st);
            double* Yout = ws.tape ? ws.tY + (size_t)k * P * M : Yk;
            gemm<T, true>(Pi, M, ld, ax, ld, W, ld, EpiNewton{Yout, scal, NS, M, pb->newton_iters, fs, s, dt, status},
                          st);
            if (ws.tape) Ycur = Yout;
            else std::swap(Ycur, Yk);
        } else {
            hipLaunchKernelGGL((k_sh_outputs<T>), dim3((unsigned)P), dim3(256), 0, st, ax, ld, d, scal, NS, fs, dt,
                               pb->newton_iters, u, grad, status);
        }
        if ((err = last_error())) return err;
    }
    if (ws.tape) set_int(ws.tag, tape_tag_of(pb, P), st);
    hipLaunchKernelGGL(k_info_to_status, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, ws.info, status, P);
    return last_error();
}

// Reverse mode of solve_shared_impl for L = sum_p ubar_p u_p (see fbsde_shared.hpp): the cloud is
// regenerated forward in time from W_0 = 0, every level reads its taped weights, mean, factor, slope
// and Y_k, and the contractions with the cloud are MFMA GEMMs.
template <typename T>
int backward_shared_impl(const fbsde_problem* pb, const Plan& pl, const Plan& pl1, int64_t P, const double* x0,
                         const double* u_bar, double* x0_bar, double* gp_bar, double* fp_bar, uint32_t* status,
                         SWS& ws, hipStream_t st) {
    T* W = (T*)ws.W;
    T* Dt = (T*)ws.Dt;
    T* V = (T*)ws.R;       // [P][M]: cbar, then the ridge adjoint, then 2h'G at the terminal
    T* axbar = (T*)ws.xc;  // [P][ld]
    const int M = (int)pl.M, ld = pl.ld, d = (int)pl.d, Pi = (int)P;
    const double s = pb->s;
    const unsigned cblocks = (unsigned)((ld + 255) / 256);
    const bool dual = pl.M <= pl.d;
    int err;
    for (int k = 0; k < (int)pl.N; ++k) {
        const double* tw_prev = k > 0 ? ws.tw + (size_t)(k - 1) * M : nullptr;
        const double* tscal_k = ws.tscal + (size_t)k * P * NS;
        const T* tax_k = (const T*)ws.tax + (size_t)k * P * ld;
        const double* tWbar_k = ws.tWbar + (size_t)k * ld;
        const T* tK_k = (const T*)ws.tK + (size_t)k * ws.kn * ws.kn;
        adj_newton(pb, P, ws.G, tw_prev, 0, ws.psc, 1, k > 0 ? ws.tY + (size_t)k * P * M : nullptr, tscal_k, u_bar,
                   ws.cbar, ws.adj, k == 0 ? 1 : 0, 0, status, st);
        // alpha_xbar: the cloud term needs W_k before it is advanced
        if (k == 0) {
            hipLaunchKernelGGL((k_sha_axbar0<T>), dim3((unsigned)P), dim3(256), 0, st, axbar, tax_k, tWbar_k, ws.adj,
                               ld, d, s);
        } else {
            const int64_t n = P * (int64_t)M;
            hipLaunchKernelGGL((k_sha_to_elem<T>), dim3((unsigned)std::min<int64_t>((n + 255) / 256, 8192)), dim3(256),
                               0, st, ws.cbar, n, V);
            gemm<T, false>(Pi, ld, M, V, M, W, ld, EpiAxbar<T>{axbar, tax_k, tWbar_k, ws.adj, ld, d, s}, st);
        }
        shared_advance<T>(pb, pl1, k, W, st);
        hipLaunchKernelGGL((k_sha_dtilde<T>), dim3(cblocks, 32), dim3(256), 0, st, W, ld, M, tWbar_k,
                           ws.tsqw + (size_t)k * M, Dt);
        // the tape holds K^{-1} (dual M x M, primal ld x ld): each ridge adjoint is two GEMMs
        if (dual) {
            gemm<T, true>(Pi, M, ld, axbar, ld, Dt, ld, EpiStore<T>{(T*)ws.R2, (int64_t)M, 1.0, 0.0, 0.0}, st);
            gemm<T, false>(Pi, M, M, (T*)ws.R2, M, tK_k, M, EpiStore<T>{V, (int64_t)M, 1.0, 0.0, 0.0}, st);
        } else {
            gemm<T, false>(Pi, ld, ld, axbar, ld, tK_k, ld, EpiStore<T>{(T*)ws.ax, (int64_t)ld, 1.0, 0.0, 0.0}, st);
            gemm<T, true>(Pi, M, ld, (T*)ws.ax, ld, Dt, ld, EpiStore<T>{V, (int64_t)M, 1.0, 0.0, 0.0}, st);
        }
        hipLaunchKernelGGL((k_sha_G<T>), dim3((unsigned)P), dim3(256), 0, st, V, M, ws.tsqw + (size_t)k * M, s, ws.G,
                           ws.psc);
        if ((err = last_error())) return err;
    }
    // G_N, then the terminal condition on the cloud at t_N (W now holds W_N)
    adj_newton(pb, P, ws.G, ws.tw + (size_t)(pl.N - 1) * M, 0, ws.psc, 1, nullptr, ws.tscal, u_bar, ws.cbar, ws.adj,
               0, 1, status, st);
    if (pb->g_kind == FBSDE_G_AFFINE || pb->g_kind == FBSDE_G_LOGISTIC) {
        const bool lg = pb->g_kind == FBSDE_G_LOGISTIC;
        hipLaunchKernelGGL((k_sha_terminal<T>), dim3((unsigned)P), dim3(256), 0, st, ws.G, lg ? ws.tq : nullptr, M, d,
                           pb->g_kind, pb->gp[0], nullptr, ws.adj);
        hipLaunchKernelGGL(k_sha_x0bar_affine, dim3((unsigned)P), dim3(256), 0, st, pb->gvec, d, ws.adj,
                           lg ? A_GP + 0 : A_SG, x0_bar);
    } else {
        hipLaunchKernelGGL((k_sha_terminal<T>), dim3((unsigned)P), dim3(256), 0, st, ws.G, ws.tq, M, d, pb->g_kind,
                           pb->gp[0], V, ws.adj);
        gemm<T, false>(Pi, ld, M, V, M, W, ld, EpiX0bar{x0_bar, x0, pb->mu, ws.adj, d, s, pb->T}, st);
    }
    adj_params(ws.adj, P, gp_bar, fp_bar, st);
    return last_error();
}

}  // namespace

namespace fbsde {
namespace host {

size_t shared_workspace_bytes(const fbsde_problem* pb, int64_t P, int32_t flags) {
    Plan pl;
    if (make_plan(pb, P, pl)) return 0;
    SWS sws;
    return carve_shared(pl, P, flags, nullptr, sws);
}

int solve_shared(const fbsde_problem* pb, int64_t P, const double* x0, double* u, double* grad, uint32_t* status,
                 void* wsp, size_t ws_bytes, int32_t flags, hipStream_t st) {
    Plan pl, pl1;
    int rc;
    if ((rc = make_plan(pb, P, pl)) || (rc = make_plan(pb, 1, pl1))) return rc;
    SWS sws;
    if (carve_shared(pl, P, flags, nullptr, sws) > ws_bytes) return FBSDE_ENOSPC;
    carve_shared(pl, P, flags, (char*)wsp, sws);
    if (P == 0) return FBSDE_OK;
    if (pb->prec == FBSDE_F64) return solve_shared_impl<double>(pb, pl, pl1, P, x0, u, grad, status, sws, st);
    return solve_shared_impl<float>(pb, pl, pl1, P, x0, u, grad, status, sws, st);
}

int backward_shared(const fbsde_problem* pb, int64_t P, const double* x0, const double* u_bar, double* x0_bar,
                    double* gp_bar, double* fp_bar, uint32_t* status, void* wsp, size_t ws_bytes, hipStream_t st) {
    Plan pl, pl1;
    int rc;
    if ((rc = make_plan(pb, P, pl)) || (rc = make_plan(pb, 1, pl1))) return rc;
    SWS sws;
    if (carve_shared(pl, P, FBSDE_WS_TAPE, nullptr, sws) > ws_bytes) return FBSDE_ENOSPC;
    carve_shared(pl, P, FBSDE_WS_TAPE, (char*)wsp, sws);
    if (P == 0) return FBSDE_OK;
    int tag = 0;
    if (hipMemcpyAsync(&tag, sws.tag, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return FBSDE_EHIP;
    if (tag != tape_tag_of(pb, P)) return FBSDE_ESTATE;
    if (pb->prec == FBSDE_F64)
        return backward_shared_impl<double>(pb, pl, pl1, P, x0, u_bar, x0_bar, gp_bar, fp_bar, status, sws, st);
    return backward_shared_impl<float>(pb, pl, pl1, P, x0, u_bar, x0_bar, gp_bar, fp_bar, status, sws, st);
}

}  // namespace host
}  // namespace fbsde

extern "C" {

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
    set_int(dinfo, 0, st);
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

}  // extern "C"
