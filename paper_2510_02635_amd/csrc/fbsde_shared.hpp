// Shared-increment form of one backward level (the common-randomness remark after Lemma 3.7):
// all P evaluation points use the same particle cloud W [M][ld], so the kernel weights, the weighted
// mean and the ridge system are shared and only the responses Y [P][M] differ.  Per level
//   w_j            from |W_j|^2 (eq. Dj, Gaussian kernel)
//   Dt_j           = sqrt(w_j) (W_j - Wbar)                       [M][ld]
//   K              = lam I + s^2 Dt Dt^T                          [M][M] (Gram, MFMA)   -> Cholesky
//   R[p][j]        = sqrt(w_j) (Y_pj - Ybar_p)                    [P][M]
//   F              = R K^{-1}                                     (K^{-1} from the factor, one GEMM)
//   alpha_x[p]     = s F[p] Dt   (the dual form of the ridge normal equations: A^{-1} D'^T W (Y - Ybar))
//   alpha_p        = Ybar_p - s alpha_x[p] . Wbar
//   C[p][m]        = alpha_p + s alpha_x[p] . W^m_k  -> Newton in the GEMM epilogue
// The two [P x M] x [M x d] / [P x d] x [d x M] contractions and the Gram are the MFMA GEMMs of
// fbsde_mfma.hpp.
#pragma once
#include "fbsde_mfma.hpp"

namespace fbsde {

// Dual Gram matrix with the known small eigenvalue lifted: K' = lam I + s^2 Dt Dt^T + c sqrt(w) sqrt(w)^T.
// The weighted centring makes sqrt(w) an exact null vector of Dt^T, so K itself has the eigenvalue lam
// there (condition near 10^3 d / M); every right-hand side K^{-1} is applied to -- sqrt(w_j)(Y_j - Ybar)
// and alpha_xbar Dt^T -- is orthogonal to sqrt(w), so K'^{-1} gives the same products while its
// explicit inverse keeps the condition of the rest of the spectrum (c of the order of its mean).
template <typename T>
struct EpiGram {
    T* K;
    int64_t ldk;
    double s2, lam, c;
    const double* sqw;
    __device__ __forceinline__ void operator()(int m, int n, double v) const {
        double r = s2 * v + c * sqw[m] * sqw[n];
        if (m == n) r += lam;
        K[(int64_t)m * ldk + n] = (T)r;
    }
};

// Terminal values from the contraction v = xc_p . W_j (radial g): |X|^2 = |xc_p|^2 + 2 s v + s^2 |W_j|^2.
struct EpiTerminal {
    double* Y;
    const double* xc2;
    const double* rn2;
    double s, ga, gb;
    int g_kind, M, d;
    uint32_t* status;
    double* q_tape;   // [P][M] |X|^2 for the adjoint, or null
    __device__ __forceinline__ void operator()(int p, int j, double v) const {
        const double q = xc2[p] + 2.0 * s * v + s * s * rn2[j];
        const double y = g_of(g_kind, ga, gb, q, d);
        Y[(int64_t)p * M + j] = y;
        if (q_tape) q_tape[(int64_t)p * M + j] = q;
        if (!isfinite(y)) atomicOr(&status[p], (uint32_t)ST_NONFINITE);
    }
};

// Newton for Y^m_k of point p from the contraction v = alpha_x[p] . W^m_k.
struct EpiNewton {
    double* Y;
    const double* scal;
    int ns, M, newton_iters;
    FSpec f;
    double s, dt;
    uint32_t* status;
    __device__ __forceinline__ void operator()(int p, int j, double v) const {
        uint32_t st = 0;
        double Fp;
        const double y = newton_y(f, scal[(int64_t)p * ns + 5] + s * v, scal[(int64_t)p * ns + 6],
                                  scal[(int64_t)p * ns + 8], dt, newton_iters, Fp, st);
        Y[(int64_t)p * M + j] = y;
        if (st) atomicOr(&status[p], st);
    }
};

// x0 + mu T (element type T, pad zero) and its squared norm.
template <typename T>
__global__ void __launch_bounds__(256)
k_sh_xc(const double* __restrict__ x0, const double* __restrict__ mu, int d, int ld, double Tend, T* __restrict__ xc,
        double* __restrict__ xc2) {
    __shared__ double lds[16];
    const int p = blockIdx.x;
    double s = 0.0;
    for (int i = threadIdx.x; i < ld; i += blockDim.x) {
        const double v = (i < d) ? x0[(int64_t)p * d + i] + (mu ? mu[i] * Tend : 0.0) : 0.0;
        xc[(int64_t)p * ld + i] = (T)v;
        s += v * v;
    }
    s = block_sum(s, lds);
    if (threadIdx.x == 0) xc2[p] = s;
}

// Terminal g of q = gvec . (xc_p + s W_j) (affine: q + b; logistic: 1 / (1 + e^-(q + b))): per-particle
// gvec . W_j then per (p, j); q_tape (or null) keeps q for the adjoint.
template <typename T>
__global__ void __launch_bounds__(256)
k_sh_affine_terminal(const T* __restrict__ W, int ld, int M, int d, const double* __restrict__ gvec,
                     const double* __restrict__ x0, const double* __restrict__ mu, double Tend, double s, double b,
                     int P, int g_kind, double* __restrict__ Y, double* __restrict__ q_tape, uint32_t* __restrict__ status) {
    __shared__ double lds[16];
    const int p = blockIdx.x;
    double gx = 0.0;
    for (int i = threadIdx.x; i < d; i += blockDim.x) gx += gvec[i] * (x0[(int64_t)p * d + i] + (mu ? mu[i] * Tend : 0.0));
    gx = block_sum(gx, lds);
    for (int j = 0; j < M; ++j) {
        double gw = 0.0;
        for (int i = threadIdx.x; i < d; i += blockDim.x) gw += gvec[i] * (double)W[(int64_t)j * ld + i];
        gw = block_sum(gw, lds);
        if (threadIdx.x == 0) {
            const double q = gx + s * gw;
            const double y = g_of(g_kind, b, 0.0, q, d);
            Y[(int64_t)p * M + j] = y;
            if (q_tape) q_tape[(int64_t)p * M + j] = q;
            if (!isfinite(y)) atomicOr(&status[p], (uint32_t)ST_NONFINITE);
        }
    }
}

// Shared kernel weights (one block): w_j, sqrt(w_j).
__global__ void __launch_bounds__(256)
k_sh_weights(const double* __restrict__ rn2, int M, double s2, double eps2, double* __restrict__ w,
             double* __restrict__ sqw) {
    __shared__ double lds[16];
    double mn = INFINITY;
    for (int j = threadIdx.x; j < M; j += blockDim.x) mn = fmin(mn, rn2[j]);
    mn = block_min(mn, lds);
    double se = 0.0;
    for (int j = threadIdx.x; j < M; j += blockDim.x) {
        const double e = (eps2 > 0.0) ? exp(-(s2 * rn2[j] - s2 * mn) / eps2) : 1.0;
        w[j] = e;
        se += e;
    }
    se = block_sum(se, lds);
    for (int j = threadIdx.x; j < M; j += blockDim.x) {
        const double wj = w[j] / se;
        w[j] = wj;
        sqw[j] = sqrt(wj);
    }
}

// Per point: Ybar_p = sum_j w_j Y_pj and R[p][j] = sqrt(w_j) (Y_pj - Ybar_p).
template <typename T>
__global__ void __launch_bounds__(256)
k_sh_rhs(const double* __restrict__ Y, const double* __restrict__ w, const double* __restrict__ sqw, int M,
         T* __restrict__ R, double* __restrict__ scal, int ns) {
    __shared__ double lds[16];
    const int p = blockIdx.x;
    const double* y = Y + (int64_t)p * M;
    double yb = 0.0;
    for (int j = threadIdx.x; j < M; j += blockDim.x) yb += w[j] * y[j];
    yb = block_sum(yb, lds);
    for (int j = threadIdx.x; j < M; j += blockDim.x) R[(int64_t)p * M + j] = (T)(sqw[j] * (y[j] - yb));
    if (threadIdx.x == 0) scal[(int64_t)p * ns + 4] = yb;
}

// Weighted mean of the cloud, two stages: part[c][i] = sum over the rows of chunk c of w_j W_j[i].
template <typename T>
__global__ void __launch_bounds__(256)
k_sh_colsum(const T* __restrict__ W, int ld, int M, int rows_per_chunk, const double* __restrict__ w,
            double* __restrict__ part) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= ld) return;
    const int r0 = c * rows_per_chunk, r1 = min(M, r0 + rows_per_chunk);
    double s = 0.0;
    for (int j = r0; j < r1; ++j) s += w[j] * (double)W[(int64_t)j * ld + i];
    part[(int64_t)c * ld + i] = s;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_sh_dtilde(const T* __restrict__ W, int ld, int M, const double* __restrict__ part, int nchunk,
            const double* __restrict__ sqw, double* __restrict__ Wbar, T* __restrict__ Dt) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= ld) return;
    double wb = 0.0;
    for (int c = 0; c < nchunk; ++c) wb += part[(int64_t)c * ld + i];
    if (blockIdx.y == 0) Wbar[i] = wb;
    const int rows = (M + gridDim.y - 1) / gridDim.y;
    const int r0 = blockIdx.y * rows, r1 = min(M, r0 + rows);
    for (int j = r0; j < r1; ++j) Dt[(int64_t)j * ld + i] = (T)(sqw[j] * ((double)W[(int64_t)j * ld + i] - wb));
}

// out[c][r] = in[r][c] for r < rows, c < cols (32 x 32 tiles through LDS).
template <typename T>
__global__ void __launch_bounds__(256)
k_transpose(const T* __restrict__ in, int64_t ldi, int rows, int cols, T* __restrict__ out, int64_t ldo) {
    __shared__ T tile[32][33];
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int i = ty; i < 32; i += 8) {
        const int r = r0 + i, c = c0 + tx;
        tile[i][tx] = (r < rows && c < cols) ? in[(int64_t)r * ldi + c] : (T)0;
    }
    __syncthreads();
    for (int i = ty; i < 32; i += 8) {
        const int c = c0 + i, r = r0 + tx;
        if (c < cols && r < rows) out[(int64_t)c * ldo + r] = tile[tx][i];
    }
}

// Per point: alpha_p = Ybar_p - s alpha_x[p] . Wbar,  zz_p = s^2 |alpha_x[p]|^2,  zs_p = s sum_i alpha_x[p]_i.
template <typename T>
__global__ void __launch_bounds__(256)
k_sh_point_finish(const T* __restrict__ ax, int ld, const double* __restrict__ Wbar, double s,
                  double* __restrict__ scal, int ns) {
    __shared__ double lds[16];
    const int p = blockIdx.x;
    double xw = 0.0, xx = 0.0, xs = 0.0;
    for (int i = threadIdx.x; i < ld; i += blockDim.x) {
        const double a = (double)ax[(int64_t)p * ld + i];
        xw += a * Wbar[i];
        xx += a * a;
        xs += a;
    }
    xw = block_sum(xw, lds);
    xx = block_sum(xx, lds);
    xs = block_sum(xs, lds);
    if (threadIdx.x == 0) {
        scal[(int64_t)p * ns + 5] = scal[(int64_t)p * ns + 4] - s * xw;
        scal[(int64_t)p * ns + 6] = s * s * xx;
        scal[(int64_t)p * ns + 8] = s * xs;
    }
}

// Level-0 outputs in the shared form: u_p = Newton(alpha_p), grad = alpha_x[p] / F'(u).
template <typename T>
__global__ void __launch_bounds__(256)
k_sh_outputs(const T* __restrict__ ax, int ld, int d, const double* __restrict__ scal, int ns, FSpec f, double dt,
             int newton_iters, double* __restrict__ u, double* __restrict__ grad, uint32_t* __restrict__ status) {
    const int p = blockIdx.x;
    uint32_t st = 0;
    double Fp;
    const double y = newton_y(f, scal[(int64_t)p * ns + 5], scal[(int64_t)p * ns + 6], scal[(int64_t)p * ns + 8], dt,
                              newton_iters, Fp, st);
    if (threadIdx.x == 0) u[p] = y;
    if (grad)
        for (int i = threadIdx.x; i < d; i += blockDim.x) grad[(int64_t)p * d + i] = (double)ax[(int64_t)p * ld + i] / Fp;
    if (st && threadIdx.x == 0) atomicOr(&status[p], st);
}

// ------------------------------------------------------------------ reverse mode of the shared form
// Per level k (walked from k = 0 upwards, the shared cloud regenerated forward in time), with G the
// adjoint of Y_k and cbar = G / F' from the Newton adjoint:
//   alpha_xbar[p] = s sum_m cbar[p][m] W^m_k + s^2 zc_p alpha_x[p] - alphabar_p s Wbar      (GEMM, epilogue)
//   the ridge solve alpha_x = A^{-1} b, A = lam I + s^2 Dt^T Dt symmetric and independent of Y, enters
//   only through sqrt(w_j) D'_j . bbar = s [A^{-1}-free form]:
//     dual   (M <= d): V = (alpha_xbar Dt^T) K^{-1},  K = lam I + s^2 Dt Dt^T   (push-through identity)
//     primal (M >  d): V = (alpha_xbar A^{-1}) Dt^T
//   G_{k+1}[p][j] = s sqrt(w_j) V[p][j] + w_j (alphabar_p - s sum_i sqrt(w_i) V[p][i])
// The dual form never forms bbar itself, whose component in the ridge-only null space of the design
// is scaled by 1/lam.

// alpha_xbar from the GEMM value v = sum_m cbar[p][m] W^m_k (element type T); Zbar = zc Z + z1 (1, ..., 1)
// over the d coordinates.
template <typename T>
struct EpiAxbar {
    T* out;
    const T* ax;
    const double* Wbar;
    const double* adj;
    int ld, d;
    double s;
    __device__ __forceinline__ void operator()(int p, int i, double v) const {
        const double* a = adj + (int64_t)p * A_NS;
        const double r = s * v + s * s * a[A_ZC] * (double)ax[(int64_t)p * ld + i] + ((i < d) ? s * a[A_Z1] : 0.0) -
                         a[A_ABAR] * s * Wbar[i];
        out[(int64_t)p * ld + i] = (T)r;
    }
};

// The same at k = 0, where the cloud is W_0 = 0 and the GEMM term vanishes.
template <typename T>
__global__ void __launch_bounds__(256)
k_sha_axbar0(T* __restrict__ out, const T* __restrict__ ax, const double* __restrict__ Wbar,
             const double* __restrict__ adj, int ld, int d, double s) {
    const int p = blockIdx.x;
    const double* a = adj + (int64_t)p * A_NS;
    for (int i = threadIdx.x; i < ld; i += blockDim.x)
        out[(int64_t)p * ld + i] = (T)(s * s * a[A_ZC] * (double)ax[(int64_t)p * ld + i] +
                                       ((i < d) ? s * a[A_Z1] : 0.0) - a[A_ABAR] * s * Wbar[i]);
}

// FP64 [P][M] -> element type.
template <typename T>
__global__ void __launch_bounds__(256)
k_sha_to_elem(const double* __restrict__ a, int64_t n, T* __restrict__ b) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (T)a[i];
}

// Dt_j = sqrt(w_j) (W_j - Wbar) from the taped weights and mean (all ld columns; the pad stays 0).
template <typename T>
__global__ void __launch_bounds__(256)
k_sha_dtilde(const T* __restrict__ W, int ld, int M, const double* __restrict__ Wbar,
             const double* __restrict__ sqw, T* __restrict__ Dt) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= ld) return;
    const double wb = Wbar[i];
    const int rows = (M + gridDim.y - 1) / gridDim.y;
    const int r0 = blockIdx.y * rows, r1 = min(M, r0 + rows);
    for (int j = r0; j < r1; ++j) Dt[(int64_t)j * ld + i] = (T)(sqw[j] * ((double)W[(int64_t)j * ld + i] - wb));
}

// G[p][j] = s sqrt(w_j) V[p][j] (the part before the mean-response term) and tau_p = sum_j of it,
// stored as the per-point row-pass sum that the next Newton adjoint completes G with.
template <typename T>
__global__ void __launch_bounds__(256)
k_sha_G(const T* __restrict__ V, int M, const double* __restrict__ sqw, double s, double* __restrict__ G,
        double* __restrict__ psc) {
    __shared__ double lds[16];
    const int p = blockIdx.x;
    double tau = 0.0;
    for (int j = threadIdx.x; j < M; j += blockDim.x) {
        const double g = s * sqw[j] * (double)V[(int64_t)p * M + j];
        G[(int64_t)p * M + j] = g;
        tau += g;
    }
    tau = block_sum(tau, lds);
    if (threadIdx.x == 0) psc[(int64_t)p * 4] = tau;
}

// Terminal adjoint, per point: phi_j = 2 h'(|X_j|^2) G_j (element type, for the x0bar GEMM) and the
// sums sum_j phi_j, sum_j G_j dg/dgp0, sum_j G_j dg/dgp1, sum_j G_j (affine g: only the last two).
template <typename T>
__global__ void __launch_bounds__(256)
k_sha_terminal(const double* __restrict__ G, const double* __restrict__ qt, int M, int d, int g_kind, double ga,
               T* __restrict__ phi, double* __restrict__ adj) {
    __shared__ double lds[16];
    const int p = blockIdx.x;
    double s1 = 0.0, g0 = 0.0, g1 = 0.0, sg = 0.0;
    for (int j = threadIdx.x; j < M; j += blockDim.x) {
        const double gj = G[(int64_t)p * M + j];
        double hp = 0.0, d0 = 0.0, d1 = 0.0;
        if (g_kind == G_AFFINE) {
            d0 = 1.0;
        } else if (g_kind == G_LOGISTIC) {
            const double gv = 1.0 / (1.0 + exp(-(qt[(int64_t)p * M + j] + ga)));
            d0 = gv * (1.0 - gv);
        } else {
            const double q = qt[(int64_t)p * M + j];
            if (g_kind == G_QUAD) { hp = ga / (double)d; d0 = q / (double)d; d1 = 1.0; }
            else if (g_kind == G_AC) { const double den = 2.0 + ga * q; hp = -ga / (den * den); d0 = -q / (den * den); }
            else if (g_kind == G_HJ_GAUSS) {   // g = (1 + 4a)^(-d/2) e^(-q / (1 + 4a))
                const double a4 = 1.0 + 4.0 * ga, gv = g_of(G_HJ_GAUSS, ga, 0.0, q, d);
                hp = -gv / a4;
                d0 = gv * (-2.0 * (double)d / a4 + 4.0 * q / (a4 * a4));
            }
            else { const double den = 1.0 + ga * q; hp = ga / den; d0 = q / den; }
        }
        const double ph = 2.0 * hp * gj;
        if (phi) phi[(int64_t)p * M + j] = (T)ph;
        s1 += ph; g0 += gj * d0; g1 += gj * d1; sg += gj;
    }
    s1 = block_sum(s1, lds);
    g0 = block_sum(g0, lds);
    g1 = block_sum(g1, lds);
    sg = block_sum(sg, lds);
    if (threadIdx.x == 0) {
        double* a = adj + (int64_t)p * A_NS;
        a[A_S1] = s1;
        a[A_GP + 0] = g0;
        a[A_GP + 1] = g1;
        a[A_SG] = sg;
    }
}

// x0bar[p][i] = S1_p xc_p[i] + s v  (v = sum_j phi_pj W^j_N), xc = x0 + mu T; columns i < d.
struct EpiX0bar {
    double* x0bar;
    const double* x0;
    const double* mu;
    const double* adj;
    int d;
    double s, T;
    __device__ __forceinline__ void operator()(int p, int i, double v) const {
        if (i >= d) return;
        const double xc = x0[(int64_t)p * d + i] + (mu ? mu[i] * T : 0.0);
        x0bar[(int64_t)p * d + i] = adj[(int64_t)p * A_NS + A_S1] * xc + s * v;
    }
};

// g of gvec . X: x0bar[p] = c_p gvec with c_p the adjoint slot `slot` (affine: sum_j G_j; logistic:
// sum_j G_j g'_j, the gp0 sum).
__global__ void __launch_bounds__(256)
k_sha_x0bar_affine(const double* __restrict__ gvec, int d, const double* __restrict__ adj, int slot,
                   double* __restrict__ x0bar) {
    const int p = blockIdx.x;
    const double sg = adj[(int64_t)p * A_NS + slot];
    for (int i = threadIdx.x; i < d; i += blockDim.x) x0bar[(int64_t)p * d + i] = sg * gvec[i];
}

}  // namespace fbsde
