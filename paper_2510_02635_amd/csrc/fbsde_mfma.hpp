// Dense contractions on the gfx950 matrix cores for the shared-increment form of the scheme.
//
// When every evaluation point uses the same increments (the common-randomness remark after
// Lemma 3.7), the cloud, its kernel weights and the regression matrix are shared and only the
// responses differ per point, so the local linear regression of all P points is a set of dense
// products: [P x M] x [M x d] and [P x d] x [d x M] contractions and one M x M Gram / Cholesky per
// level.  This header holds the MFMA GEMM used for all of them (with fused epilogues), and the
// blocked Cholesky factorisation and triangular solves built on it (row-parallel substitutions for
// the diagonal blocks, matrix-core GEMMs for every update).
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
// K = L L^T in place (lower triangle), block size CB, right-looking: per diagonal block, factor it
// (one wavefront, LDS), solve the panel below it row by row (k_trsm_rows: every row is independent),
// and give the trailing lower triangle the rank-CB update on the matrix cores (GEMM, lower tiles only).
constexpr int CB = 64;

// Broadcast lane src's value to the whole wavefront (src uniform).
__device__ __forceinline__ double lane_bcast(double v, int src) {
    const uint64_t b = __double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)b, src);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(b >> 32), src);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Factor the CB x CB diagonal block at (kb, kb) in place (lower; upper part of the block zeroed).
// One wavefront: lane i owns row i in registers; the column being eliminated is read from its owner
// lanes with readlane (no LDS, no barriers).
template <typename T>
__global__ void __launch_bounds__(64)
k_potrf_diag(T* __restrict__ K, int64_t ldk, int n, int kb, int* __restrict__ info) {
    const int o = kb * CB;
    const int nb = min(CB, n - o);
    const int i = threadIdx.x;
    double a[CB];
#pragma unroll
    for (int j = 0; j < CB; ++j)
        a[j] = (i < nb && j < nb && j <= i) ? (double)K[(int64_t)(o + i) * ldk + o + j] : ((i == j) ? 1.0 : 0.0);
    int bad = 0;
#pragma unroll
    for (int j = 0; j < CB; ++j) {
        double d = lane_bcast(a[j], j);
        if (!(d > 0.0)) { bad |= (j < nb); d = 1.0; }
        const double piv = sqrt(d);
        if (i == j) a[j] = piv;
        else if (i > j) a[j] /= piv;
#pragma unroll
        for (int c = j + 1; c < CB; ++c) {
            const double lcj = lane_bcast(a[j], c);   // L[c][j]
            if (i >= c) a[c] -= a[j] * lcj;
        }
    }
    if (bad && i == 0) atomicOr(info, 1);
    if (i < nb)
#pragma unroll
        for (int j = 0; j < CB; ++j)
            if (j < nb) K[(int64_t)(o + i) * ldk + o + j] = (T)((j <= i) ? a[j] : 0.0);
}

// Row-wise triangular solves with the CB x CB lower factor Lkk (row-major, ldl) for rows r of X
// (row stride ldx, columns c0 .. c0 + w - 1, in place), one wavefront per row, lane c owning column c
// (column-oriented substitution):
//   upper = 0: x Lkk^T = a   (x_c = (a_c - sum_{k<c} x_k L[c][k]) / L[c][c], c ascending)
//   upper = 1: x Lkk   = a   (x_c = (a_c - sum_{k>c} x_k L[k][c]) / L[c][c], c descending)
template <typename T>
__global__ void __launch_bounds__(256)
k_trsm_rows(const T* __restrict__ Lkk, int64_t ldl, int w, T* __restrict__ X, int64_t ldx, int rows, int c0, int upper) {
    __shared__ double L[CB][CB + 1];
    for (int t = threadIdx.x; t < CB * CB; t += 256) {
        const int i = t / CB, j = t % CB;
        L[i][j] = (i < w && j < w) ? (double)Lkk[(int64_t)i * ldl + j] : ((i == j) ? 1.0 : 0.0);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int r = blockIdx.x * 4 + wave; r < rows; r += gridDim.x * 4) {
        T* row = X + (int64_t)r * ldx + c0;
        double a = (lane < w) ? (double)row[lane] : 0.0;
        if (!upper) {
            for (int c = 0; c < CB; ++c) {
                const double xc = lane_bcast(a, c) / L[c][c];
                if (lane == c) a = xc;
                else if (lane > c) a -= xc * L[lane][c];
            }
        } else {
            for (int c = CB - 1; c >= 0; --c) {
                const double xc = lane_bcast(a, c) / L[c][c];
                if (lane == c) a = xc;
                else if (lane < c) a -= xc * L[c][lane];
            }
        }
        if (lane < w) row[lane] = (T)a;
    }
}

// Blocked Cholesky of the n x n SPD matrix K (lower triangle used and overwritten with L).
template <typename T>
inline void cholesky(T* K, int64_t ldk, int n, int* info, hipStream_t st) {
    const int nb = (n + CB - 1) / CB;
    for (int kb = 0; kb < nb; ++kb) {
        const int o = kb * CB;
        hipLaunchKernelGGL((k_potrf_diag<T>), dim3(1), dim3(64), 0, st, K, ldk, n, kb, info);
        const int rows = n - o - CB;
        if (rows <= 0) break;
        // panel: L[i][kb] solves L[i][kb] L_kk^T = A[i][kb]
        hipLaunchKernelGGL((k_trsm_rows<T>), dim3((unsigned)std::min((rows + 3) / 4, 4096)), dim3(256), 0, st,
                           K + (int64_t)o * ldk + o, ldk, CB, K + (int64_t)(o + CB) * ldk, ldk, rows, o, 0);
        // trailing update of the lower triangle: K[i][j] -= sum_c L[i][c] L[j][c]
        gemm<T, true>(rows, rows, CB, K + (int64_t)(o + CB) * ldk + o, ldk, K + (int64_t)(o + CB) * ldk + o, ldk,
                      EpiStore<T>{K + (int64_t)(o + CB) * ldk + o + CB, ldk, -1.0, 1.0, 0.0}, st, 1);
    }
}

// Solve X (L L^T) = R for the P right-hand sides stored as rows of R [P][n] (in place), with the factor
// from cholesky().  Right-looking blocked substitutions: per column block, the row-wise triangular solve,
// then one wide GEMM update of all remaining columns.
template <typename T>
inline void cholesky_solve_rows(const T* L, int64_t ldl, int n, T* R, int64_t ldr, int P, hipStream_t st) {
    const int nb = (n + CB - 1) / CB;
    const unsigned rblocks = (unsigned)std::min((P + 3) / 4, 4096);
    // forward: Y L^T = R
    for (int kb = 0; kb < nb; ++kb) {
        const int o = kb * CB, w = std::min(CB, n - o);
        hipLaunchKernelGGL((k_trsm_rows<T>), dim3(rblocks), dim3(256), 0, st, L + (int64_t)o * ldl + o, ldl, w, R, ldr,
                           P, o, 0);
        const int rest = n - o - w;
        if (rest > 0)   // R[p][o + w + c] -= sum_k Y[p][o + k] L[o + w + c][o + k]
            gemm<T, true>(P, rest, w, R + o, ldr, L + (int64_t)(o + w) * ldl + o, ldl,
                          EpiStore<T>{R + o + w, ldr, -1.0, 1.0, 0.0}, st);
    }
    // backward: X L = Y
    for (int kb = nb - 1; kb >= 0; --kb) {
        const int o = kb * CB, w = std::min(CB, n - o);
        hipLaunchKernelGGL((k_trsm_rows<T>), dim3(rblocks), dim3(256), 0, st, L + (int64_t)o * ldl + o, ldl, w, R, ldr,
                           P, o, 1);
        if (o > 0)   // Y[p][c] -= sum_r X[p][o + r] L[o + r][c]   for c < o   (NN: B[k = r][n = c])
            gemm<T, false>(P, o, w, R + o, ldr, L + (int64_t)o * ldl, ldl, EpiStore<T>{R, ldr, -1.0, 1.0, 0.0}, st);
    }
}

// out[c][r] = in[r][c] for an n x n block (32 x 32 tiles through LDS).
template <typename T>
__global__ void __launch_bounds__(256)
k_transpose_sq(const T* __restrict__ in, int64_t ldi, int n, T* __restrict__ out, int64_t ldo) {
    __shared__ T tile[32][33];
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int i = ty; i < 32; i += 8) {
        const int r = r0 + i, c = c0 + tx;
        tile[i][tx] = (r < n && c < n) ? in[(int64_t)r * ldi + c] : (T)0;
    }
    __syncthreads();
    for (int i = ty; i < 32; i += 8) {
        const int c = c0 + i, r = r0 + tx;
        if (c < n && r < n) out[(int64_t)c * ldo + r] = tile[tx][i];
    }
}

// Zero an n x n block (row pitch ld).
template <typename T>
__global__ void __launch_bounds__(256) k_zero_square(T* __restrict__ A, int64_t ld, int n) {
    const int64_t total = (int64_t)n * n;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x)
        A[(t / n) * ld + (t % n)] = (T)0;
}

// ------------------------------------------------------------------ recursive Cholesky with the inverse
// For the shared form only K^{-1} is needed.  With K = [[A, B^T], [B, C]] and L its factor:
//   L11 = chol(A);  L21 = B L11^{-T};  L22 = chol(C - L21 L21^T);
//   L^{-1} = [[L11^{-1}, 0], [-L22^{-1} L21 L11^{-1}, L22^{-1}]]
// so the factor's inverse follows by recursion on halves, every off-diagonal step a GEMM on the matrix
// cores; only the CB x CB leaves (factor and inverse together in LDS) run one after another.

// Leaf: the w x w SPD block at K (lower triangle read), w <= CB: its factor's inverse into Li (lower,
// zeros above).  256 threads, FP64 in LDS: right-looking factorisation (column scale, then the trailing
// update split over the threads), then lane c of the first wave forms column c of the inverse.
template <typename T>
__global__ void __launch_bounds__(256)
k_chol_inv_leaf(const T* __restrict__ K, int64_t ldk, int w, T* __restrict__ Li, int64_t ldi, int* __restrict__ info) {
    __shared__ double Ls[CB][CB + 1];
    __shared__ double xs[CB][CB + 1];
    const int t = threadIdx.x;
    for (int e = t; e < CB * CB; e += 256) {
        const int i = e / CB, j = e % CB;
        Ls[i][j] = (i < w && j <= i) ? (double)K[(int64_t)i * ldk + j] : ((i == j) ? 1.0 : 0.0);
    }
    __syncthreads();
    int bad = 0;
    const int r = t >> 2, cq = t & 3;   // thread t updates row r, columns c = cq (mod 4)
    for (int j = 0; j < w; ++j) {
        double dj = Ls[j][j];
        if (!(dj > 0.0)) { bad = 1; dj = 1.0; }
        const double piv = sqrt(dj);
        __syncthreads();   // every thread has read the pivot before it changes
        if (cq == 0 && r < w) {
            if (r == j) Ls[j][j] = piv;
            else if (r > j) Ls[r][j] /= piv;
        }
        __syncthreads();
        if (r > j && r < w) {
            const double lrj = Ls[r][j];
            for (int c = j + 1 + ((cq - (j + 1)) & 3); c <= r; c += 4) Ls[r][c] -= lrj * Ls[c][j];
        }
        __syncthreads();
    }
    if (t < CB) {
        const int c = t;
        for (int rr = 0; rr < CB; ++rr) {
            double acc = (rr == c) ? 1.0 : 0.0;
            for (int k = c; k < rr; ++k) acc -= Ls[rr][k] * xs[k][c];
            xs[rr][c] = (rr >= c) ? acc / Ls[rr][rr] : 0.0;
        }
        if (c < w)
            for (int rr = 0; rr < w; ++rr) Li[(int64_t)rr * ldi + c] = (T)xs[rr][c];
    }
    if (bad && t == 0) atomicOr(info, 1);
}

// Li = (chol K)^{-1} for the n x n SPD K (lower triangle read; its strictly lower blocks are left as
// they are, the lower triangle of each diagonal block is read only).  Li needs zeros above the
// diagonal: the caller clears it once.  S: scratch of at least (n/2 + CB)^2 elements.
template <typename T>
inline void chol_inverse_rec(T* K, int64_t ldk, int n, T* Li, int64_t ldi, T* S, int* info, hipStream_t st) {
    if (n <= CB) {
        hipLaunchKernelGGL((k_chol_inv_leaf<T>), dim3(1), dim3(256), 0, st, K, ldk, n, Li, ldi, info);
        return;
    }
    const int n1 = ((n / CB + 1) / 2) * CB, n2 = n - n1;
    T* C = K + (int64_t)n1 * ldk + n1;
    const T* B = K + (int64_t)n1 * ldk;
    T* Li11 = Li;
    T* Li21 = Li + (int64_t)n1 * ldi;
    T* Li22 = Li + (int64_t)n1 * ldi + n1;
    chol_inverse_rec<T>(K, ldk, n1, Li11, ldi, S, info, st);
    // L21 = B L11^{-T}, kept for now in the lower-left block of Li
    gemm<T, true>(n2, n1, n1, B, ldk, Li11, ldi, EpiStore<T>{Li21, ldi, 1.0, 0.0, 0.0}, st);
    // C <- C - L21 L21^T (lower tiles)
    gemm<T, true>(n2, n2, n1, Li21, ldi, Li21, ldi, EpiStore<T>{C, ldk, -1.0, 1.0, 0.0}, st, 1);
    chol_inverse_rec<T>(C, ldk, n2, Li22, ldi, S, info, st);
    // Li21 = -L22^{-1} (L21 L11^{-1})
    gemm<T, false>(n2, n1, n1, Li21, ldi, Li11, ldi, EpiStore<T>{S, (int64_t)n1, 1.0, 0.0, 0.0}, st);
    gemm<T, false>(n2, n1, n2, Li22, ldi, S, n1, EpiStore<T>{Li21, ldi, -1.0, 0.0, 0.0}, st);
}

// K^{-1} of the SPD K (lower triangle read and overwritten) into Kinv (may be K): Li [n][n] and S [n][n]
// scratch; *info (device) gets 1 for a non-positive pivot.
template <typename T>
inline void spd_inverse(T* K, int64_t ldk, int n, T* Kinv, int64_t ldkinv, T* Li, T* S, int* info, hipStream_t st) {
    hipLaunchKernelGGL((k_zero_square<T>), dim3((unsigned)std::min<int64_t>(((int64_t)n * n + 255) / 256, 4096)),
                       dim3(256), 0, st, Li, (int64_t)n, n);
    chol_inverse_rec<T>(K, ldk, n, Li, n, S, info, st);
    const unsigned tb = (unsigned)((n + 31) / 32);
    hipLaunchKernelGGL((k_transpose_sq<T>), dim3(tb, tb), dim3(256), 0, st, Li, (int64_t)n, n, S, (int64_t)n);
    gemm<T, false>(n, n, n, S, n, Li, n, EpiStore<T>{Kinv, ldkinv, 1.0, 0.0, 0.0}, st);
}

}  // namespace fbsde
