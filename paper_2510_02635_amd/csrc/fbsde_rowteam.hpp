// Row-team building blocks shared by the per-point kernels and the persistent batched kernel: the
// geometry of a team of wavefronts owning one particle row, compensated sums, 16/32-byte loads and
// stores of four coordinates, team and block reductions of columns.
#pragma once
#include "fbsde_device.hpp"

namespace fbsde {

template <int Q, int TEAM>
struct Geo {
    static constexpr int TL = 64 * TEAM;                 // lanes per team
    static constexpr int BS = 64 * (TEAM > 4 ? TEAM : 4);  // threads per block
    static constexpr int TPW = BS / TL;                   // teams per block
};

// compensated running sum
template <typename R> struct CSum;
template <> struct CSum<double> {
    double s = 0.0;
    __device__ __forceinline__ void add(double v) { s += v; }
    __device__ __forceinline__ double get() const { return s; }
};
template <> struct CSum<float> {
    float s = 0.0f, c = 0.0f;
    __device__ __forceinline__ void add(float v) {
        const float y = v - c;
        const float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ __forceinline__ double get() const { return (double)s - (double)c; }
};

// Loads of state rows: each pass streams the [P][M][ld] state once and never re-reads a row, so the
// loads carry the non-temporal hint (measured: the FP32 CG product 2.87 -> 2.53 ms at d = 1000,
// P = 1024, M = 4096; no change in FP64).
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef double nt_d2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void load4(const double* __restrict__ p, double v[4]) {
    const nt_d2 a = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p));
    const nt_d2 b = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p + 2));
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
__device__ __forceinline__ void load4(const float* __restrict__ p, float v[4]) {
    const nt_f4 a = __builtin_nontemporal_load(reinterpret_cast<const nt_f4*>(p));
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}
// One row of the state into a lane's registers: groups of four at 4 (L + q TL), zero beyond ld.
template <typename S, int Q, int TL>
__device__ __forceinline__ void load_row(const S* __restrict__ row, int ld, int L, S x[Q][4]) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int e0 = 4 * (L + q * TL);
        if (e0 < ld) load4(row + e0, x[q]);
        else {
#pragma unroll
            for (int e = 0; e < 4; ++e) x[q][e] = (S)0;
        }
    }
}

__device__ __forceinline__ void store4(double* __restrict__ p, const double v[4]) {
    *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
    *reinterpret_cast<double2*>(p + 2) = make_double2(v[2], v[3]);
}
__device__ __forceinline__ void store4(float* __restrict__ p, const float v[4]) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
}

// Reduce two values over the team owning a row; every lane of the team gets the totals.
// For TEAM > 1 all waves of the block must call it the same number of times.
template <int TEAM>
__device__ __forceinline__ void team_sum2(double& a, double& b, double* red, int team) {
    a = wave_sum(a);
    b = wave_sum(b);
    if constexpr (TEAM > 1) {
        const int wv = (threadIdx.x >> 6) % TEAM, ln = threadIdx.x & 63;
        if (ln == 0) { red[2 * (team * TEAM + wv)] = a; red[2 * (team * TEAM + wv) + 1] = b; }
        __syncthreads();
        a = 0.0; b = 0.0;
#pragma unroll
        for (int i = 0; i < TEAM; ++i) { a += red[2 * (team * TEAM + i)]; b += red[2 * (team * TEAM + i) + 1]; }
        __syncthreads();
    }
}

// Combine the coordinate-product pairs (P, Q) of pq_add / pq_combine over the team owning a row; every
// lane of the team gets the totals (a butterfly: both partners combine the same two pairs).  For TEAM > 1
// all waves of the block must call it the same number of times.
template <int TEAM>
__device__ __forceinline__ void team_pq(double& P, double& Q, double* red, int team) {
    for (int off = 32; off > 0; off >>= 1) {
        const double Pb = __shfl_xor(P, off, 64), Qb = __shfl_xor(Q, off, 64);
        pq_combine(P, Q, Pb, Qb);
    }
    if constexpr (TEAM > 1) {
        const int wv = (threadIdx.x >> 6) % TEAM, ln = threadIdx.x & 63;
        if (ln == 0) { red[2 * (team * TEAM + wv)] = P; red[2 * (team * TEAM + wv) + 1] = Q; }
        __syncthreads();
        P = 1.0; Q = 0.0;
#pragma unroll
        for (int i = 0; i < TEAM; ++i) pq_combine(P, Q, red[2 * (team * TEAM + i)], red[2 * (team * TEAM + i) + 1]);
        __syncthreads();
    }
}

// Per-block combination of per-lane column accumulators into out[0..ld) (double), in team order.
template <int Q, int TEAM, typename R>
__device__ __forceinline__ void block_columns_out(CSum<R> (&acc)[Q][4], double* lds, double* __restrict__ out,
                                                  int ld, int team, int L) {
    using G = Geo<Q, TEAM>;
    if constexpr (G::TPW == 1) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int e0 = 4 * (L + q * G::TL);
            if (e0 < ld) {
                double v[4] = {acc[q][0].get(), acc[q][1].get(), acc[q][2].get(), acc[q][3].get()};
                store4(out + e0, v);
            }
        }
    } else {
        // lds holds TPW * 256 Q TEAM doubles
        constexpr int SPAN = 4 * Q * G::TL;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int e0 = 4 * (L + q * G::TL);
#pragma unroll
            for (int e = 0; e < 4; ++e) lds[team * SPAN + e0 + e] = acc[q][e].get();
        }
        __syncthreads();
        for (int i = threadIdx.x; i < ld; i += G::BS) {
            double s = 0.0;
#pragma unroll
            for (int t = 0; t < G::TPW; ++t) s += lds[t * SPAN + i];
            out[i] = s;
        }
        __syncthreads();
    }
}

}  // namespace fbsde
