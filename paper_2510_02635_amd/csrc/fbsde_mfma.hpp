// Dense contractions on the gfx950 matrix cores for the shared-increment form of the scheme.
//
// When every evaluation point uses the same increments (the common-randomness remark after
// Lemma 3.7), the cloud, its kernel weights and the regression matrix are shared and only the
// responses differ per point, so the local linear regression of all P points is a set of dense
// products: [P x M] x [M x d] and [P x d] x [d x M] contractions and one M x M Gram / Cholesky per
// level.  This header holds the MFMA GEMM used for all of them (with fused epilogues), and the
// blocked Cholesky factorisation and triangular solves built on it.
//
// GEMM: C[m][n] (+)= sum_k A[m][k] * B(k, n), A row-major with k contiguous; B either [n][k]
// (NT, k contiguous) or [k][n] (NN, n contiguous).  256 threads = 4 waves in a 2 x 2 layout; block
// tile BM x BN, K step BK, staged through LDS k-major (padded against bank conflicts), next K tile
// prefetched into registers while the current one feeds the MFMAs.
//   float : v_mfma_f32_16x16x4f32, block 128 x 128 x 32, each wave 64 x 64 (4 x 4 MFMA tiles)
//   double: v_mfma_f64_16x16x4f64, block  64 x  64 x 16, each wave 32 x 32 (2 x 2 MFMA tiles)
// MFMA 16x16x4 operand layout (lane l of the wave): A[i][k] with i = l % 16, k = l / 16;
// B[k][j] with j = l % 16, k = l / 16; result register r holds D[4 (l / 16) + r][l % 16] for the FP32
// instruction and D[4 r + l / 16][l % 16] for the FP64 one (both checked on gfx950).
#pragma once
#include "fbsde_device.hpp"

namespace fbsde {

template <typename T> struct GemmCfg;
template <> struct GemmCfg<float> {
    static constexpr int BM = 128, BN = 128, BK = 32, PAD = 16;
    using vec4 = __attribute__((__vector_size__(4 * sizeof(float)))) float;
    __device__ static __forceinline__ vec4 mfma(float a, float b, vec4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // result register r of lane group g = lane / 16 holds row 4 g + r
    __device__ static __forceinline__ int row_of(int g, int r) { return 4 * g + r; }
};
template <> struct GemmCfg<double> {
    static constexpr int BM = 64, BN = 64, BK = 16, PAD = 4;
    using vec4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;
    __device__ static __forceinline__ vec4 mfma(double a, double b, vec4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // result register r of lane group g = lane / 16 holds row 4 r + g (interleaved, unlike FP32)
    __device__ static __forceinline__ int row_of(int g, int r) { return 4 * r + g; }
};

// C = alpha * acc + beta * C, plus diag on m == n < dlim and dpad on m == n >= dlim (dense store,
// row-major, ldc).  dlim / dpad let a padded Gram matrix keep unit pivots in its pad.
template <typename T>
struct EpiStore {
    T* C;
    int64_t ldc;
    double alpha, beta, diag;
    int dlim = 0x7FFFFFFF;
    double dpad = 0.0;
    __device__ __forceinline__ void operator()(int m, int n, double v) const {
        double r = alpha * v;
        if (beta != 0.0) r += beta * (double)C[(int64_t)m * ldc + n];
        if (m == n) r += (m < dlim) ? diag : dpad;
        C[(int64_t)m * ldc + n] = (T)r;
    }
};

template <typename T, bool NT, typename Epi>
__global__ void __launch_bounds__(256)
k_gemm(int Md, int Nd, int Kd, const T* __restrict__ A, int64_t lda, const T* __restrict__ B, int64_t ldb,
       Epi epi, int lower_only) {
    using Cfg = GemmCfg<T>;
    using vec4 = typename Cfg::vec4;
    constexpr int BM = Cfg::BM, BN = Cfg::BN, BK = Cfg::BK, PAD = Cfg::PAD;
    constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 16, TN = WN / 16;
    constexpr int AV = BM * BK / 4 / 256;   // 4-vectors of A per thread per K tile
    constexpr int BV = BN * BK / 4 / 256;
    __shared__ T As[BK][BM + PAD];
    __shared__ T Bs[BK][BN + PAD];
    const int bm = blockIdx.y, bn = blockIdx.x;
    if (lower_only && bn * BN > bm * BM + BM - 1) return;   // tile entirely above the diagonal
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = bm * BM, n0 = bn * BN;

    T ra[AV][4], rb[BV][4];
    auto load_tile = [&](int k0) {
#pragma unroll
        for (int v = 0; v < AV; ++v) {
            const int idx = tid + 256 * v;
            const int row = idx / (BK / 4), kq = idx % (BK / 4);
            const int gm = m0 + row, gk = k0 + 4 * kq;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                ra[v][e] = (gm < Md && gk + e < Kd) ? A[(int64_t)gm * lda + gk + e] : (T)0;
        }
#pragma unroll
        for (int v = 0; v < BV; ++v) {
            const int idx = tid + 256 * v;
            if constexpr (NT) {
                const int row = idx / (BK / 4), kq = idx % (BK / 4);
                const int gn = n0 + row, gk = k0 + 4 * kq;
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    rb[v][e] = (gn < Nd && gk + e < Kd) ? B[(int64_t)gn * ldb + gk + e] : (T)0;
            } else {
                const int krow = idx / (BN / 4), nq = idx % (BN / 4);
                const int gk = k0 + krow, gn = n0 + 4 * nq;
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    rb[v][e] = (gk < Kd && gn + e < Nd) ? B[(int64_t)gk * ldb + gn + e] : (T)0;
            }
        }
    };
    auto store_tile = [&]() {
#pragma unroll
        for (int v = 0; v < AV; ++v) {
            const int idx = tid + 256 * v;
            const int row = idx / (BK / 4), kq = idx % (BK / 4);
#pragma unroll
            for (int e = 0; e < 4; ++e) As[4 * kq + e][row] = ra[v][e];
        }
#pragma unroll
        for (int v = 0; v < BV; ++v) {
            const int idx = tid + 256 * v;
            if constexpr (NT) {
                const int row = idx / (BK / 4), kq = idx % (BK / 4);
#pragma unroll
                for (int e = 0; e < 4; ++e) Bs[4 * kq + e][row] = rb[v][e];
            } else {
                const int krow = idx / (BN / 4), nq = idx % (BN / 4);
#pragma unroll
                for (int e = 0; e < 4; ++e) Bs[krow][4 * nq + e] = rb[v][e];
            }
        }
    };

    vec4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[i][j][r] = (T)0;

    const int nk = (Kd + BK - 1) / BK;
    load_tile(0);
    store_tile();
    __syncthreads();
    const int li = lane & 15, lk = lane >> 4;
    for (int kt = 0; kt < nk; ++kt) {
        if (kt + 1 < nk) load_tile((kt + 1) * BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            T af[TM], bf[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) af[i] = As[kk + lk][wm * WM + 16 * i + li];
#pragma unroll
            for (int j = 0; j < TN; ++j) bf[j] = Bs[kk + lk][wn * WN + 16 * j + li];
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) acc[i][j] = Cfg::mfma(af[i], bf[j], acc[i][j]);
        }
        __syncthreads();
        if (kt + 1 < nk) {
            store_tile();
            __syncthreads();
        }
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm * WM + 16 * i + Cfg::row_of(lk, r);
                const int n = n0 + wn * WN + 16 * j + li;
                if (m < Md && n < Nd) epi(m, n, (double)acc[i][j][r]);
            }
}

template <typename T, bool NT, typename Epi>
inline void gemm(int Md, int Nd, int Kd, const T* A, int64_t lda, const T* B, int64_t ldb, const Epi& epi,
                 hipStream_t st, int lower_only = 0) {
    using Cfg = GemmCfg<T>;
    if (Md <= 0 || Nd <= 0) return;
    const dim3 grid((Nd + Cfg::BN - 1) / Cfg::BN, (Md + Cfg::BM - 1) / Cfg::BM);
    hipLaunchKernelGGL((k_gemm<T, NT, Epi>), grid, dim3(256), 0, st, Md, Nd, Kd, A, lda, B, ldb, epi, lower_only);
}

// ------------------------------------------------------------------ blocked Cholesky
// K = L L^T in place (lower triangle), block size CB.  Per diagonal block: k_potrf_diag factors it
// and writes the inverse of its triangle; the panel below becomes A_panel L_kk^{-T} (a GEMM with the
// inverse), and the trailing lower triangle takes the rank-CB update (GEMM, lower tiles only).
constexpr int CB = 64;

// Factor the CB x CB diagonal block at (kb, kb) of K (row-major, ldk) and write L_kk^{-1} into Linv
// (CB x CB row-major, upper part zero).  One block of 256 threads; the block sits in LDS (in FP64).
template <typename T>
__global__ void __launch_bounds__(256)
k_potrf_diag(T* __restrict__ K, int64_t ldk, int n, int kb, T* __restrict__ Linv, int* __restrict__ info) {
    __shared__ double a[CB][CB + 1];
    __shared__ double li[CB][CB + 1];
    const int o = kb * CB;
    const int nb = min(CB, n - o);
    const int tid = threadIdx.x;
    for (int t = tid; t < CB * CB; t += 256) {
        const int i = t / CB, j = t % CB;
        a[i][j] = (i < nb && j < nb && j <= i) ? (double)K[(int64_t)(o + i) * ldk + o + j] : (i == j ? 1.0 : 0.0);
        li[i][j] = 0.0;
    }
    __syncthreads();
    // right-looking unblocked Cholesky of the block
    for (int j = 0; j < CB; ++j) {
        if (tid == 0) {
            const double djj = a[j][j];
            if (!(djj > 0.0)) { if (j < nb) atomicOr(info, 1); a[j][j] = 1.0; }
            else a[j][j] = sqrt(djj);
        }
        __syncthreads();
        const double djj = a[j][j];
        for (int i = j + 1 + tid; i < CB; i += 256) a[i][j] /= djj;
        __syncthreads();
        const int rem = CB - j - 1;
        for (int t = tid; t < rem * rem; t += 256) {
            const int i = j + 1 + t / rem, c = j + 1 + t % rem;
            if (c <= i) a[i][c] -= a[i][j] * a[c][j];
        }
        __syncthreads();
    }
    // inverse of the lower triangle, column by column: L X = I
    for (int c = tid; c < CB; c += 256) {
        for (int i = 0; i < CB; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int k = c; k < i; ++k) s -= a[i][k] * li[k][c];
            li[i][c] = (i >= c) ? s / a[i][i] : 0.0;
        }
    }
    __syncthreads();
    for (int t = tid; t < CB * CB; t += 256) {
        const int i = t / CB, j = t % CB;
        if (i < nb && j < nb) K[(int64_t)(o + i) * ldk + o + j] = (T)((j <= i) ? a[i][j] : 0.0);
        Linv[t] = (T)li[i][j];
    }
}

// Copy rows r0.. (rows of them) x columns c0..c0+cols-1 of K into scratch [rows][CB], zero beyond cols
// (the panel GEMMs may not read and write the same memory across blocks).
template <typename T>
__global__ void k_copy_panel(const T* __restrict__ K, int64_t ldk, int r0, int rows, int c0, int cols,
                             T* __restrict__ out) {
    const int64_t n = (int64_t)rows * CB;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t / CB), j = (int)(t % CB);
        out[t] = (j < cols) ? K[(int64_t)(r0 + i) * ldk + c0 + j] : (T)0;
    }
}

// Blocked Cholesky of the n x n SPD matrix K (lower triangle used and overwritten with L).
// Linv: nblocks x CB x CB inverses of the diagonal blocks; scratch: n x CB.
template <typename T>
inline void cholesky(T* K, int64_t ldk, int n, T* Linv, T* scratch, int* info, hipStream_t st) {
    const int nb = (n + CB - 1) / CB;
    for (int kb = 0; kb < nb; ++kb) {
        const int o = kb * CB;
        hipLaunchKernelGGL((k_potrf_diag<T>), dim3(1), dim3(256), 0, st, K, ldk, n, kb, Linv + (size_t)kb * CB * CB,
                           info);
        const int rows = n - o - CB;
        if (rows <= 0) break;
        // panel: L[i][kb] = A[i][kb] L_kk^{-T}, i.e. C[i][c] = sum_k P[i][k] Linv[c][k]
        hipLaunchKernelGGL((k_copy_panel<T>), dim3((unsigned)std::min<int64_t>(((int64_t)rows * CB + 255) / 256, 4096)),
                           dim3(256), 0, st, K, ldk, o + CB, rows, o, CB, scratch);
        gemm<T, true>(rows, CB, CB, scratch, CB, Linv + (size_t)kb * CB * CB, CB,
                      EpiStore<T>{K + (int64_t)(o + CB) * ldk + o, ldk, 1.0, 0.0, 0.0}, st);
        // trailing update of the lower triangle: K[i][j] -= sum_c L[i][c] L[j][c]
        gemm<T, true>(rows, rows, CB, K + (int64_t)(o + CB) * ldk + o, ldk, K + (int64_t)(o + CB) * ldk + o, ldk,
                      EpiStore<T>{K + (int64_t)(o + CB) * ldk + o + CB, ldk, -1.0, 1.0, 0.0}, st, 1);
    }
}

// Solve (L L^T) X^T = R^T for the P right-hand sides stored as rows of R [P][n] (in place), with the
// factor from cholesky().  Blocked forward then backward substitution on row blocks of CB columns;
// diagonal blocks apply the stored inverses, off-diagonal parts are GEMM updates.  scratch: P x CB.
template <typename T>
inline void cholesky_solve_rows(const T* L, int64_t ldl, int n, const T* Linv, T* R, int64_t ldr, int P, T* scratch,
                                hipStream_t st) {
    const int nb = (n + CB - 1) / CB;
    // forward: L Y^T = R^T  <=>  Y[p][blk kb] = (R[p][kb] - sum_{j<kb} Y[p][j] L[kb][j]) L_kk^{-T}
    for (int kb = 0; kb < nb; ++kb) {
        const int o = kb * CB, w = std::min(CB, n - o);
        if (kb > 0)   // R[p][o..o+w) -= sum_{j < o} Y[p][j] L[o + c][j]
            gemm<T, true>(P, w, o, R, ldr, L + (int64_t)o * ldl, ldl, EpiStore<T>{R + o, ldr, -1.0, 1.0, 0.0}, st);
        // Y[p][o + c] = sum_k R[p][o + k] Linv[c][k]
        hipLaunchKernelGGL((k_copy_panel<T>), dim3((unsigned)std::min<int64_t>(((int64_t)P * CB + 255) / 256, 4096)),
                           dim3(256), 0, st, R, ldr, 0, P, o, w, scratch);
        gemm<T, true>(P, w, w, scratch, CB, Linv + (size_t)kb * CB * CB, CB, EpiStore<T>{R + o, ldr, 1.0, 0.0, 0.0}, st);
    }
    // backward: L^T X^T = Y^T  <=>  X[p][kb] = (Y[p][kb] - sum_{j>kb} X[p][j] L[j][kb]) L_kk^{-1}
    for (int kb = nb - 1; kb >= 0; --kb) {
        const int o = kb * CB, w = std::min(CB, n - o);
        const int after = n - (o + w);
        if (after > 0)   // Y[p][o + c] -= sum_{j >= o + w} X[p][j] L[j][o + c]   (NN: B[k = j][n = c])
            gemm<T, false>(P, w, after, R + o + w, ldr, L + (int64_t)(o + w) * ldl + o, ldl,
                           EpiStore<T>{R + o, ldr, -1.0, 1.0, 0.0}, st);
        // X[p][o + r] = sum_c Y[p][o + c] Linv[c][r]   (L_kk^T x = y  =>  x = L_kk^{-T} y)
        hipLaunchKernelGGL((k_copy_panel<T>), dim3((unsigned)std::min<int64_t>(((int64_t)P * CB + 255) / 256, 4096)),
                           dim3(256), 0, st, R, ldr, 0, P, o, w, scratch);
        gemm<T, false>(P, w, w, scratch, CB, Linv + (size_t)kb * CB * CB, CB, EpiStore<T>{R + o, ldr, 1.0, 0.0, 0.0},
                       st);
    }
}

}  // namespace fbsde
