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

__device__ __forceinline__ void load4(const double* __restrict__ p, double v[4]) {
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 2);
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
__device__ __forceinline__ void load4(const float* __restrict__ p, float v[4]) {
    const float4 a = *reinterpret_cast<const float4*>(p);
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
