// Direct dual solve of a level's ridge regression for small, rank-deficient clouds (M <= d + 1,
// M <= FBSDE_DUAL_MAXM).  The normal equations of Sec. 2.4, (D'^T W D' + lambda I) alpha_x = D'^T W (Y - Ybar)
// with D'_j = s (W_j - Wbar), are solved through the push-through identity
//   alpha_x = B^T (B B^T + lambda I)^{-1} W^1/2 (Y - Ybar),   B = W^1/2 D'  (M x d),
// i.e. one M x M Cholesky factorisation per point instead of the matrix-free CG, whose iteration count on
// such clouds (all but one eigenvalue of the d x d system spread over the cloud's M - 1 directions, the
// rest at lambda) runs to dozens or, at M = d + 1, past M.  Two kernels, one block per point:
//   k_dual_gram:  K = s^2 W^1/2 G W^1/2 + lambda I with G_ij = (W_i - Wbar) . (W_j - Wbar), FP64 sums
//                 over d in chunks of 32 coordinates staged through LDS, 4 x 4 register blocks of (i, j);
//                 and the right-hand side W^1/2 (Y - Ybar), times the scale k_moments_finish chose;
//   k_dual_solve: K factored in LDS (column by column, the trailing triangle updated by all threads),
//                 forward and back substitution, then alpha_x = s sum_j w_j^1/2 c_j (W_j - Wbar) over
//                 the cloud.  The result goes where the CG iterate goes (scaled like it), so the level's
//                 finish is the same.
#pragma once
#include "fbsde.h"
#include "fbsde_rowteam.hpp"

namespace fbsde {

constexpr int DUAL_MAXM = FBSDE_DUAL_MAXM;

template <typename S>
__global__ void __launch_bounds__(256)
k_dual_gram(const S* __restrict__ W, int64_t ldw, int M, int d, int ld, double s, const double* __restrict__ Wbar,
            const double* __restrict__ w, const double* __restrict__ Y, const double* __restrict__ scal, int ns,
            double* __restrict__ K, double* __restrict__ rhs) {
    __shared__ double rows[DUAL_MAXM][33];
    const int p = blockIdx.x, t = threadIdx.x;
    const int nbk = (M + 3) / 4;                 // blocks of four rows
    const int nblk = nbk * (nbk + 1) / 2;        // block pairs (bi >= bj), at most 528
    int bi[3], bj[3];
    bool own[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int idx = t + 256 * q;
        own[q] = idx < nblk;
        int b = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
        while (b > 0 && b * (b + 1) / 2 > idx) --b;
        while ((b + 1) * (b + 2) / 2 <= idx) ++b;
        bi[q] = b;
        bj[q] = idx - b * (b + 1) / 2;
    }
    double acc[3][16];
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[q][e] = 0.0;
    const S* Wp = W + (int64_t)p * M * ldw;
    const double* wb = Wbar + (int64_t)p * ld;
    for (int c0 = 0; c0 < d; c0 += 32) {
        __syncthreads();
        for (int e = t; e < 4 * nbk * 32; e += 256) {
            const int r = e >> 5, c = e & 31;
            rows[r][c] = (r < M && c0 + c < d) ? (double)Wp[(int64_t)r * ldw + c0 + c] - wb[c0 + c] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            if (!own[q]) continue;
            for (int c = 0; c < 32; ++c) {
                double a[4], b[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    a[u] = rows[4 * bi[q] + u][c];
                    b[u] = rows[4 * bj[q] + u][c];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[q][4 * u + v] += a[u] * b[v];
            }
        }
    }
    const double lam = scal[(int64_t)p * ns + 3];
    const double* wp = w + (int64_t)p * M;
    double* Kp = K + (int64_t)p * M * M;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        if (!own[q]) continue;
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 4 * bi[q] + u, j = 4 * bj[q] + v;
                if (i < M && j <= i)
                    Kp[(int64_t)i * M + j] = s * s * sqrt(wp[i] * wp[j]) * acc[q][4 * u + v] + ((i == j) ? lam : 0.0);
            }
    }
    // W^1/2 (Y - Ybar) at the scale of the level's CG right-hand side (k_moments_finish keeps 1 / scale)
    const double yb = scal[(int64_t)p * ns + 4], isc = scal[(int64_t)p * ns + 9];
    for (int i = t; i < M; i += 256) rhs[(int64_t)p * M + i] = sqrt(wp[i]) * (Y[(int64_t)p * M + i] - yb) / isc;
}

template <typename S>
__global__ void __launch_bounds__(256)
k_dual_solve(const double* __restrict__ K, const double* __restrict__ rhs, int M, const S* __restrict__ W,
             int64_t ldw, int d, int ld, double s, const double* __restrict__ Wbar, const double* __restrict__ w,
             double* __restrict__ x, int* __restrict__ iscal, uint32_t* __restrict__ status) {
    __shared__ double A[DUAL_MAXM][DUAL_MAXM + 1];
    __shared__ double y[DUAL_MAXM];
    __shared__ double red[16];
    __shared__ int bad;
    const int p = blockIdx.x, t = threadIdx.x;
    const double* Kp = K + (int64_t)p * M * M;
    for (int e = t; e < M * M; e += 256) {
        const int i = e / M, j = e - (e / M) * M;
        A[i][j] = (j <= i) ? Kp[(int64_t)i * M + j] : 0.0;
    }
    for (int i = t; i < M; i += 256) y[i] = rhs[(int64_t)p * M + i];
    if (t == 0) bad = 0;
    __syncthreads();
    // Cholesky K = L L^T in place (lower)
    for (int j = 0; j < M; ++j) {
        double dj = A[j][j];
        if (!(dj > 0.0)) {
            if (t == 0) bad = 1;
            dj = 1.0;
        }
        const double piv = sqrt(dj);
        __syncthreads();   // every thread has read the pivot
        if (t == j) A[j][j] = piv;
        for (int r = j + 1 + t; r < M; r += 256) A[r][j] /= piv;
        __syncthreads();
        for (int r = j + 1 + (t >> 2); r < M; r += 64) {
            const double lrj = A[r][j];
            for (int c = j + 1 + (t & 3); c <= r; c += 4) A[r][c] -= lrj * A[c][j];
        }
        __syncthreads();
    }
    // L z = rhs, then L^T c = z (column-oriented, in y)
    for (int j = 0; j < M; ++j) {
        if (t == 0) y[j] /= A[j][j];
        __syncthreads();
        for (int r = j + 1 + t; r < M; r += 256) y[r] -= A[r][j] * y[j];
        __syncthreads();
    }
    for (int j = M - 1; j >= 0; --j) {
        if (t == 0) y[j] /= A[j][j];
        __syncthreads();
        for (int r = t; r < j; r += 256) y[r] -= A[j][r] * y[j];
        __syncthreads();
    }
    // alpha_x = s sum_j w_j^1/2 c_j (W_j - Wbar): the coefficients in y, their sum for the Wbar term
    double cs = 0.0;
    for (int i = t; i < M; i += 256) {
        const double cj = s * sqrt(w[(int64_t)p * M + i]) * y[i];
        y[i] = cj;
        cs += cj;
    }
    cs = block_sum(cs, red);   // its barriers also publish the coefficients
    const S* Wp = W + (int64_t)p * M * ldw;
    for (int i = t; i < ld; i += 256) {
        double a = 0.0;
        if (i < d) {
            for (int j = 0; j < M; ++j) a += y[j] * (double)Wp[(int64_t)j * ldw + i];
            a -= cs * Wbar[(int64_t)p * ld + i];
        }
        x[(int64_t)p * ld + i] = a;
    }
    if (t == 0) {
        iscal[p * 4 + 0] = 0;   // no CG iterations
        iscal[p * 4 + 1] = 1;
        if (bad) atomicOr(&status[p], (uint32_t)ST_NONFINITE);
    }
}

}  // namespace fbsde
