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

#include <type_traits>

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

// Four consecutive elements from a 16-byte aligned address.
__device__ __forceinline__ void gload4(const float* __restrict__ p, float v[4]) {
    const float4 a = *reinterpret_cast<const float4*>(p);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}
__device__ __forceinline__ void gload4(const double* __restrict__ p, double v[4]) {
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 2);
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}

template <typename T, bool NT, typename Epi, bool FOLD_LONG = false>
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
    // groups of four consecutive elements: one 16-byte (FP32) or two (FP64) loads when the group is in
    // bounds and the operand's rows are 16-byte aligned, element loads at the edges
    const bool avec = (lda % 4 == 0) && (((uintptr_t)A & 15) == 0);
    const bool bvec = (ldb % 4 == 0) && (((uintptr_t)B & 15) == 0);
    auto load_tile = [&](int k0) {
#pragma unroll
        for (int v = 0; v < AV; ++v) {
            const int idx = tid + 256 * v;
            const int row = idx / (BK / 4), kq = idx % (BK / 4);
            const int gm = m0 + row, gk = k0 + 4 * kq;
            if (avec && gm < Md && gk + 3 < Kd) {
                gload4(A + (int64_t)gm * lda + gk, ra[v]);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    ra[v][e] = (gm < Md && gk + e < Kd) ? A[(int64_t)gm * lda + gk + e] : (T)0;
            }
        }
#pragma unroll
        for (int v = 0; v < BV; ++v) {
            const int idx = tid + 256 * v;
            if constexpr (NT) {
                const int row = idx / (BK / 4), kq = idx % (BK / 4);
                const int gn = n0 + row, gk = k0 + 4 * kq;
                if (bvec && gn < Nd && gk + 3 < Kd) {
                    gload4(B + (int64_t)gn * ldb + gk, rb[v]);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        rb[v][e] = (gn < Nd && gk + e < Kd) ? B[(int64_t)gn * ldb + gk + e] : (T)0;
                }
            } else {
                const int krow = idx / (BN / 4), nq = idx % (BN / 4);
                const int gk = k0 + krow, gn = n0 + 4 * nq;
                if (bvec && gk < Kd && gn + 3 < Nd) {
                    gload4(B + (int64_t)gk * ldb + gn, rb[v]);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        rb[v][e] = (gk < Kd && gn + e < Nd) ? B[(int64_t)gk * ldb + gn + e] : (T)0;
                }
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
    // Long FP32 contractions (FOLD_LONG, chosen by the launcher for K > 1024): the matrix cores
    // accumulate eight K tiles (256 terms) in FP32, then those sums are added into FP64 running sums, so
    // the rounding grows with 256 terms, not with K (measured at d = 10^4, P = 4096, M = 2048: gradient
    // error 1.8e-5 with plain FP32 accumulation, 3.3e-6 folded, 8.4e-6 folding only K > 4096).  The
    // folding costs about a sixth of the kernel's speed, so short contractions (the K = 64 updates of the
    // factorisation and of the inverse) keep plain FP32 accumulation.
    constexpr bool FOLD = FOLD_LONG && std::is_same<T, float>::value;
    double fsum[FOLD ? TM : 1][FOLD ? TN : 1][4];
    constexpr int FOLD_TILES = (256 / BK > 0) ? 256 / BK : 1;   // K tiles per 256-term FP32 partial sum
    if constexpr (FOLD) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) fsum[i][j][r] = 0.0;
    }

    const int nk = (Kd + BK - 1) / BK;
    load_tile(0);
    store_tile();
    __syncthreads();
    const int li = lane & 15, lk = lane >> 4;
    // operand fragments of one 4-deep K step, double-buffered in registers; the scheduling groups
    // below order the LDS reads of step kk + 4 ahead of the MFMAs of step kk, so their latency hides
    // behind the matrix cores instead of stalling them once per step
    T af[2][TM], bf[2][TN];
    auto frag = [&](int kk, int b) {
#pragma unroll
        for (int i = 0; i < TM; ++i) af[b][i] = As[kk + lk][wm * WM + 16 * i + li];
#pragma unroll
        for (int j = 0; j < TN; ++j) bf[b][j] = Bs[kk + lk][wn * WN + 16 * j + li];
    };
    for (int kt = 0; kt < nk; ++kt) {
        if (kt + 1 < nk) load_tile((kt + 1) * BK);
        frag(0, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, (TM + TN) / 2, 0);   // the first step's reads
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            const int b = (kk / 4) & 1;
            if (kk + 4 < BK) frag(kk + 4, b ^ 1);
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) acc[i][j] = Cfg::mfma(af[b][i], bf[b][j], acc[i][j]);
            if (kk + 4 < BK) __builtin_amdgcn_sched_group_barrier(0x100, (TM + TN) / 2, 0);   // LDS reads
            __builtin_amdgcn_sched_group_barrier(0x008, TM * TN, 0);                           // MFMAs
        }
        if constexpr (FOLD) {
            if (kt % FOLD_TILES == FOLD_TILES - 1 || kt + 1 == nk) {
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            fsum[i][j][r] += (double)acc[i][j][r];
                            acc[i][j][r] = (T)0;
                        }
            }
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
                double val;
                if constexpr (FOLD) val = fsum[i][j][r];
                else val = (double)acc[i][j][r];
                if (m < Md && n < Nd) epi(m, n, val);
            }
}

// FP32 GEMM, pipelined form (the one the launcher picks for FP32): the same block and wave tiles as
// k_gemm<float>, with
//   * two LDS buffers and a prefetch distance of two tiles: tile kt + 2 is loaded into registers while
//     the MFMAs consume tile kt, and written at the start of tile kt + 1 into the buffer tile kt read, so
//     a K tile costs one barrier and the loads have a whole tile to arrive;
//   * operands k-contiguous in LDS (A rows and, for NT, B rows of BK + 4 floats: 16-byte aligned rows
//     whose 8-lane groups of 128-bit accesses cover all 32 banks once), written with 128-bit stores;
//   * a permuted contraction order: at step s of the tile the four k of the 4-deep MFMA are 8 g + s
//     (g = lane / 16, the operand's k slot), the same permutation for both operands, so a lane's A
//     (and NT B) fragments for the whole tile are 8 consecutive k of one row: two 128-bit LDS reads
//     per 16-row tile instead of eight 32-bit ones.  NN B stays n-contiguous ([BK][BN + 4]) and is read
//     32 bits at a time.
// FOLD as in k_gemm: FP32 partial sums of 256 terms added into FP64 running sums.
template <bool NT, typename Epi, bool FOLD, int NW>
__global__ void __launch_bounds__(64 * NW)
k_gemm_f32p(int Md, int Nd, int Kd, const float* __restrict__ A, int64_t lda, const float* __restrict__ B,
            int64_t ldb, Epi epi, int lower_only) {
    constexpr int BM = 128, BN = 128, BK = 32, SA = BK + 4, SBN = BN + 4;
    constexpr int BSZ = NT ? BN * SA : BK * SBN;
    // NW waves: 2 along m (64 rows each) x NW / 2 along n (WNT columns each, TN 16-column MFMA tiles)
    constexpr int WGN = NW / 2, WNT = BN / WGN, TN = WNT / 16;
    constexpr int LV = 16 / NW;   // 128-bit loads per thread and operand per K tile
    using vec4 = GemmCfg<float>::vec4;
    __shared__ __attribute__((aligned(16))) float As[2][BM * SA];
    __shared__ __attribute__((aligned(16))) float Bs[2][BSZ];
    const int bm = blockIdx.y, bn = blockIdx.x;
    if (lower_only && bn * BN > bm * BM + BM - 1) return;   // tile entirely above the diagonal
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WGN, wn = wave % WGN;
    const int m0 = bm * BM, n0 = bn * BN;
    const int li = lane & 15, lk = lane >> 4;
    const bool avec = (lda % 4 == 0) && (((uintptr_t)A & 15) == 0);
    const bool bvec = (ldb % 4 == 0) && (((uintptr_t)B & 15) == 0);
    float ra[LV][4], rb[LV][4];
    // a K tile into registers: A (and NT B) as 32 rows x 8 groups of four k per pass, NN B as 8 k rows x
    // 32 groups of four n per pass; 128-bit loads where the group is in bounds and aligned
    auto load_tile = [&](int k0) {
#pragma unroll
        for (int v = 0; v < LV; ++v) {
            const int row = (tid >> 3) + 8 * NW * v, kq = tid & 7;
            const int gm = m0 + row, gk = k0 + 4 * kq;
            if (avec && gm < Md && gk + 3 < Kd) {
                gload4(A + (int64_t)gm * lda + gk, ra[v]);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) ra[v][e] = (gm < Md && gk + e < Kd) ? A[(int64_t)gm * lda + gk + e] : 0.0f;
            }
        }
#pragma unroll
        for (int v = 0; v < LV; ++v) {
            if constexpr (NT) {
                const int row = (tid >> 3) + 8 * NW * v, kq = tid & 7;
                const int gn = n0 + row, gk = k0 + 4 * kq;
                if (bvec && gn < Nd && gk + 3 < Kd) {
                    gload4(B + (int64_t)gn * ldb + gk, rb[v]);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        rb[v][e] = (gn < Nd && gk + e < Kd) ? B[(int64_t)gn * ldb + gk + e] : 0.0f;
                }
            } else {
                const int krow = (tid >> 5) + 2 * NW * v, nq = tid & 31;
                const int gk = k0 + krow, gn = n0 + 4 * nq;
                if (bvec && gk < Kd && gn + 3 < Nd) {
                    gload4(B + (int64_t)gk * ldb + gn, rb[v]);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        rb[v][e] = (gk < Kd && gn + e < Nd) ? B[(int64_t)gk * ldb + gn + e] : 0.0f;
                }
            }
        }
    };
    auto store_tile = [&](int buf) {
#pragma unroll
        for (int v = 0; v < LV; ++v) {
            const int row = (tid >> 3) + 8 * NW * v, kq = tid & 7;
            *reinterpret_cast<float4*>(&As[buf][row * SA + 4 * kq]) = make_float4(ra[v][0], ra[v][1], ra[v][2], ra[v][3]);
        }
#pragma unroll
        for (int v = 0; v < LV; ++v) {
            if constexpr (NT) {
                const int row = (tid >> 3) + 8 * NW * v, kq = tid & 7;
                *reinterpret_cast<float4*>(&Bs[buf][row * SA + 4 * kq]) =
                    make_float4(rb[v][0], rb[v][1], rb[v][2], rb[v][3]);
            } else {
                const int krow = (tid >> 5) + 2 * NW * v, nq = tid & 31;
                *reinterpret_cast<float4*>(&Bs[buf][krow * SBN + 4 * nq]) =
                    make_float4(rb[v][0], rb[v][1], rb[v][2], rb[v][3]);
            }
        }
    };

    vec4 acc[4][TN];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.0f;
    double fsum[FOLD ? 4 : 1][FOLD ? TN : 1][4];
    if constexpr (FOLD) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) fsum[i][j][r] = 0.0;
    }
    // Tile kt + 1 is loaded into registers during tile kt - 1 and written to LDS at the start of tile kt,
    // into the buffer tile kt - 1 read (free since the barrier that ended it): the loads have a whole
    // tile's MFMAs to arrive in.
    const int nk = (Kd + BK - 1) / BK;
    load_tile(0);
    store_tile(0);
    if (nk > 1) load_tile(BK);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) store_tile(buf ^ 1);
        if (kt + 2 < nk) load_tile((kt + 2) * BK);
        // the tile's fragments: a[i][s] = A(row of tile i, k = 8 lk + s), b[j][s] likewise
        // in two halves (s = 0..3, then 4..7): the first half's reads are all issued before the second
        // half's, so the first MFMAs wait only for them
        float a[4][8], b[TN][8];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float4 x = *reinterpret_cast<const float4*>(&As[buf][(wm * 64 + 16 * i + li) * SA + 8 * lk + 4 * h]);
                a[i][4 * h + 0] = x.x; a[i][4 * h + 1] = x.y; a[i][4 * h + 2] = x.z; a[i][4 * h + 3] = x.w;
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                if constexpr (NT) {
                    const float4 y = *reinterpret_cast<const float4*>(&Bs[buf][(wn * WNT + 16 * j + li) * SA + 8 * lk + 4 * h]);
                    b[j][4 * h + 0] = y.x; b[j][4 * h + 1] = y.y; b[j][4 * h + 2] = y.z; b[j][4 * h + 3] = y.w;
                } else {
#pragma unroll
                    for (int s = 4 * h; s < 4 * h + 4; ++s) b[j][s] = Bs[buf][(8 * lk + s) * SBN + wn * WNT + 16 * j + li];
                }
            }
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][s], b[j][s], acc[i][j], 0, 0, 0);
#pragma unroll
        for (int s = 4; s < 8; ++s)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][s], b[j][s], acc[i][j], 0, 0, 0);
        if constexpr (FOLD) {
            if ((kt & 7) == 7 || kt + 1 == nk) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            fsum[i][j][r] += (double)acc[i][j][r];
                            acc[i][j][r] = 0.0f;
                        }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm * 64 + 16 * i + 4 * lk + r;
                const int n = n0 + wn * WNT + 16 * j + li;
                double val;
                if constexpr (FOLD) val = fsum[i][j][r];
                else val = (double)acc[i][j][r];
                if (m < Md && n < Nd) epi(m, n, val);
            }
}

template <typename T, bool NT, typename Epi>
inline void gemm(int Md, int Nd, int Kd, const T* A, int64_t lda, const T* B, int64_t ldb, const Epi& epi,
                 hipStream_t st, int lower_only = 0) {
    using Cfg = GemmCfg<T>;
    if (Md <= 0 || Nd <= 0) return;
    const dim3 grid((Nd + Cfg::BN - 1) / Cfg::BN, (Md + Cfg::BM - 1) / Cfg::BM);
    if constexpr (std::is_same<T, float>::value) {
        // the FP64-folded form keeps 64 x 32 wave tiles (8 waves): half the FP64 running sums per lane, so
        // two waves share each SIMD
        if (Kd > 1024)
            hipLaunchKernelGGL((k_gemm_f32p<NT, Epi, true, 8>), grid, dim3(512), 0, st, Md, Nd, Kd, A, lda, B, ldb, epi,
                               lower_only);
        else
            hipLaunchKernelGGL((k_gemm_f32p<NT, Epi, false, 4>), grid, dim3(256), 0, st, Md, Nd, Kd, A, lda, B, ldb,
                               epi, lower_only);
    } else {
        hipLaunchKernelGGL((k_gemm<T, NT, Epi, false>), grid, dim3(256), 0, st, Md, Nd, Kd, A, lda, B, ldb, epi,
                           lower_only);
    }
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
// 256 threads: thread t holds 16 entries of row t / 4 (columns 16 (t % 4) ..) in registers.  Per column j
// the owners of column j publish it unscaled, A[.][j], in LDS (two buffers, alternating), one barrier,
// and then every thread updates its entries right of the column with x -= A[r][j] A[c][j] / A[j][j]
// (= L[r][j] L[c][j]) from same-address (broadcast) reads, while the owners scale their entry of the
// column to L[r][j].  One barrier per column; the update is branch-free so that its reads are issued
// together.  (One wavefront holding a whole row per lane and broadcasting the column with readlane
// needed a scalar register per broadcast value; the compiler spilled about 3100 of them and a block
// took 67 us.  With the pivot and the scaled column each behind a barrier and a branch per entry, 70 us;
// this form, 40 us at n = 2048.)
template <typename T>
__global__ void __launch_bounds__(256)
k_potrf_diag(T* __restrict__ K, int64_t ldk, int n, int kb, int* __restrict__ info) {
    static_assert(CB == 64, "four 16-column groups per row");
    __shared__ double col[2][CB];
    const int o = kb * CB;
    const int nb = min(CB, n - o);
    const int t = threadIdx.x, r = t >> 2, g = t & 3;
    double x[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int c = 16 * g + e;
        x[e] = (r < nb && c < nb && c <= r) ? (double)K[(int64_t)(o + r) * ldk + o + c] : ((r == c) ? 1.0 : 0.0);
    }
    int bad = 0;
    // the group loop is not unrolled (straight-line code for all 64 columns runs once and is fetched
    // once); the 16 columns of a group are, so that x[ej] is a register
#pragma unroll 1
    for (int gj = 0; gj < 4; ++gj)
#pragma unroll
    for (int ej = 0; ej < 16; ++ej) {
        const int j = 16 * gj + ej;
        double* cj = col[ej & 1];
        if (g == gj) cj[r] = x[ej];   // A[r][j] (updated by the columns before j)
        __syncthreads();
        double d = cj[j];
        if (!(d > 0.0)) { bad |= (j < nb); d = 1.0; }
        const double inv = 1.0 / d;
        const double arj = cj[r];
        double cv[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) cv[e] = cj[16 * g + e];
        const double s = arj * inv;   // L[r][j] / L[j][j]
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int c = 16 * g + e;
            const double upd = x[e] - s * cv[e];
            x[e] = (c > j && c <= r) ? upd : x[e];
        }
        if (g == gj) {
            const double piv = sqrt(d);
            x[ej] = (r == j) ? piv : ((r > j) ? arj / piv : x[ej]);
        }
    }
    if (bad && t == 0) atomicOr(info, 1);
    if (r < nb)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int c = 16 * g + e;
            if (c < nb) K[(int64_t)(o + r) * ldk + o + c] = (T)((c <= r) ? x[e] : 0.0);
        }
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
    __shared__ double inv[CB];   // 1 / L[c][c], so that the substitution chain multiplies
    for (int t = threadIdx.x; t < CB * CB; t += 256) {
        const int i = t / CB, j = t % CB;
        L[i][j] = (i < w && j < w) ? (double)Lkk[(int64_t)i * ldl + j] : ((i == j) ? 1.0 : 0.0);
    }
    __syncthreads();
    if (threadIdx.x < CB) inv[threadIdx.x] = 1.0 / L[threadIdx.x][threadIdx.x];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int r = blockIdx.x * 4 + wave; r < rows; r += gridDim.x * 4) {
        T* row = X + (int64_t)r * ldx + c0;
        double a = (lane < w) ? (double)row[lane] : 0.0;
        if (!upper) {
            for (int c = 0; c < CB; ++c) {
                const double xc = lane_bcast(a, c) * inv[c];
                if (lane == c) a = xc;
                else if (lane > c) a -= xc * L[lane][c];
            }
        } else {
            for (int c = CB - 1; c >= 0; --c) {
                const double xc = lane_bcast(a, c) * inv[c];
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
        hipLaunchKernelGGL((k_potrf_diag<T>), dim3(1), dim3(256), 0, st, K, ldk, n, kb, info);
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

// ------------------------------------------------------------------ inverse from the factor
// For the shared form only K^{-1} is needed: K = L L^T by the blocked Cholesky above, then L^{-1}
// blockwise -- every CB x CB diagonal block inverted in one launch (one wavefront each, forward
// substitution of the unit columns, FP64 sums), then recursive doubling joins neighbouring
// lower-triangular blocks [[A, 0], [B, C]] into one, whose lower-left block of the inverse is
// -C^{-1} B A^{-1} (two GEMMs on the matrix cores) -- and K^{-1} = (L^{-1})^T L^{-1} (one GEMM).

template <typename T>
__global__ void __launch_bounds__(64)
k_trtri_diag(const T* __restrict__ L, int64_t ldl, int n, T* __restrict__ Li, int64_t ldi) {
    __shared__ double Ls[CB][CB];
    __shared__ double xs[CB][CB];
    const int o = blockIdx.x * CB, w = min(CB, n - o);
    const int c = threadIdx.x;
    for (int r = 0; r < w; ++r) Ls[r][c] = (c <= r) ? (double)L[(int64_t)(o + r) * ldl + o + c] : 0.0;
    __syncthreads();
    if (c < w) {
        for (int r = 0; r < w; ++r) {
            double acc = (r == c) ? 1.0 : 0.0;
            for (int k = c; k < r; ++k) acc -= Ls[r][k] * xs[k][c];
            xs[r][c] = (r >= c) ? acc / Ls[r][r] : 0.0;
        }
        for (int r = 0; r < w; ++r) Li[(int64_t)(o + r) * ldi + o + c] = (T)xs[r][c];
    }
}

// Li = L^{-1} (lower triangle, zeros above) of the factor in L; S: scratch of at least n^2 / 4 elements.
template <typename T>
inline void triangular_inverse(const T* L, int64_t ldl, int n, T* Li, int64_t ldi, T* S, hipStream_t st) {
    const int nb = (n + CB - 1) / CB;
    hipLaunchKernelGGL((k_zero_square<T>), dim3((unsigned)std::min<int64_t>(((int64_t)n * n + 255) / 256, 4096)),
                       dim3(256), 0, st, Li, ldi, n);
    hipLaunchKernelGGL((k_trtri_diag<T>), dim3((unsigned)nb), dim3(64), 0, st, L, ldl, n, Li, ldi);
    for (int sb = 1; sb < nb; sb *= 2)
        for (int a0 = 0; a0 + sb < nb; a0 += 2 * sb) {
            const int oa = a0 * CB, sa = sb * CB;              // A: rows / cols [oa, oa + sa)
            const int oc = oa + sa, sc = std::min(sa, n - oc);  // C: rows / cols [oc, oc + sc)
            // S = B A^{-1}  (B = L[oc.., oa..], sc x sa)
            gemm<T, false>(sc, sa, sa, L + (int64_t)oc * ldl + oa, ldl, Li + (int64_t)oa * ldi + oa, ldi,
                           EpiStore<T>{S, (int64_t)sa, 1.0, 0.0, 0.0}, st);
            // Li[oc.., oa..] = -C^{-1} S
            gemm<T, false>(sc, sa, sc, Li + (int64_t)oc * ldi + oc, ldi, S, sa,
                           EpiStore<T>{Li + (int64_t)oc * ldi + oa, ldi, -1.0, 0.0, 0.0}, st);
        }
}

// K^{-1} of the SPD K (lower triangle read and overwritten by the factor) into Kinv (may be K): Li [n][n]
// and S [n][n] scratch; *info (device) gets 1 for a non-positive pivot.
template <typename T>
inline void spd_inverse(T* K, int64_t ldk, int n, T* Kinv, int64_t ldkinv, T* Li, T* S, int* info, hipStream_t st) {
    cholesky<T>(K, ldk, n, info, st);
    triangular_inverse<T>(K, ldk, n, Li, n, S, st);
    const unsigned tb = (unsigned)((n + 31) / 32);
    hipLaunchKernelGGL((k_transpose_sq<T>), dim3(tb, tb), dim3(256), 0, st, Li, (int64_t)n, n, S, (int64_t)n);
    gemm<T, false>(n, n, n, S, n, Li, n, EpiStore<T>{Kinv, ldkinv, 1.0, 0.0, 0.0}, st);
}

}  // namespace fbsde
