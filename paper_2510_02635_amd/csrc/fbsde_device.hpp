// Device-side building blocks of the FBSDE-LLR kernels for gfx950 (wave64).
//
//  * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) in registers and the Box-Muller map
//    that turns one call (four 32-bit words) into four N(0, 1) coordinates of a particle
//    increment (paper Sec. 2.3, eq. Xk: dW ~ N(0, dt I)).
//  * The built-in f and g families of the problem (Sec. 2.1) and the scalar Newton iteration
//    for Y (Sec. 2.5, eqs. nonlinearf / NRiter).
//  * Wave and team reductions (DPP-free shuffles; a "team" is TEAM wavefronts that share one
//    particle row, used when a row of d coordinates does not fit one wavefront's registers).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fbsde {

struct Words4 { uint32_t x, y, z, w; };

__device__ __forceinline__ Words4 philox4x32_10(Words4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        const Words4 n = {(uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1,
                          (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0};
        c = n;
    }
    return c;
}

// Four normals from one Philox call: Box-Muller on the word pairs (x, y) and (z, w) with
// u = (w + 1/2) 2^-32 in (0, 1); radius sqrt(-2 ln u_even), angle 2 pi u_odd.
__device__ __forceinline__ void box_muller4(const Words4& w, double z[4]) {
    const double two_m32 = 2.3283064365386963e-10;   // 2^-32
    const double two_pi = 6.283185307179586;
    const double u0 = ((double)w.x + 0.5) * two_m32;
    const double u1 = ((double)w.y + 0.5) * two_m32;
    const double u2 = ((double)w.z + 0.5) * two_m32;
    const double u3 = ((double)w.w + 0.5) * two_m32;
    const double r0 = sqrt(-2.0 * log(u0));
    const double r2 = sqrt(-2.0 * log(u2));
    double s1, c1, s3, c3;
    sincos(two_pi * u1, &s1, &c1);
    sincos(two_pi * u3, &s3, &c3);
    z[0] = r0 * c1; z[1] = r0 * s1; z[2] = r2 * c3; z[3] = r2 * s3;
}

// Normals of coordinates 4g..4g+3 of particle j, level k, stream q (point or shared).
__device__ __forceinline__ void increment4(uint32_t g, uint32_t j, uint32_t k, uint32_t q,
                                           uint32_t k0, uint32_t k1, double z[4]) {
    const Words4 c = {g, j, k, q};
    box_muller4(philox4x32_10(c, k0, k1), z);
}

// ------------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}

// Sum of v over all threads of the block (blockDim.x multiple of 64, <= 1024).
__device__ __forceinline__ double block_sum(double v, double* lds /* >= 16 */) {
    v = wave_sum(v);
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63, nw = blockDim.x >> 6;
    __syncthreads();
    if (ln == 0) lds[wv] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += lds[i];
    __syncthreads();
    return s;
}
__device__ __forceinline__ double block_min(double v, double* lds) {
    v = wave_min(v);
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63, nw = blockDim.x >> 6;
    __syncthreads();
    if (ln == 0) lds[wv] = v;
    __syncthreads();
    double s = lds[0];
    for (int i = 1; i < nw; ++i) s = fmin(s, lds[i]);
    __syncthreads();
    return s;
}

// ------------------------------------------------------------------ f, g, Newton
enum { F_ZERO = 0, F_ALLEN_CAHN = 1, F_HJB = 2 };
enum { G_QUAD = 0, G_AC = 1, G_HJB_LOG = 2, G_AFFINE = 3 };
enum { ST_CG_MAXIT = 1, ST_NEWTON_FLAT = 2, ST_NONFINITE = 4 };

struct FSpec { int kind; double p0, p1; };

// f(t, x, y, z) and d f / d y of the built-in families; zz = |z|^2 (z shared by the cloud).
__device__ __forceinline__ void f_and_fy(const FSpec& f, double y, double zz, double& fv, double& fy) {
    if (f.kind == F_ALLEN_CAHN) { fv = f.p0 * y - f.p1 * y * y * y; fy = f.p0 - 3.0 * f.p1 * y * y; }
    else if (f.kind == F_HJB) { fv = -f.p0 * zz; fy = 0.0; }
    else { fv = 0.0; fy = 0.0; }
}

// Fixed-count Newton for F(y) = y - C - dt f(y) from y = C; returns y and F'(y).
__device__ __forceinline__ double newton_y(const FSpec& f, double C, double zz, double dt, int iters,
                                           double& Fp, uint32_t& st) {
    double y = C, fv, fy;
    for (int n = 0; n < iters; ++n) {
        f_and_fy(f, y, zz, fv, fy);
        const double F = y - C - dt * fv;
        const double dF = 1.0 - dt * fy;
        if (fabs(dF) < 1e-12) st |= ST_NEWTON_FLAT;
        y = y - F / dF;
    }
    f_and_fy(f, y, zz, fv, fy);
    Fp = 1.0 - dt * fy;
    if (!isfinite(y)) st |= ST_NONFINITE;
    return y;
}

// Terminal g from q = |X|^2 (radial families) or q = gvec . X (affine).
__device__ __forceinline__ double g_of(int kind, double a, double b, double q, int64_t d) {
    if (kind == G_QUAD) return a * q / (double)d + b;
    if (kind == G_AC) return 1.0 / (2.0 + a * q);
    if (kind == G_HJB_LOG) return log((1.0 + a * q) * 0.5);
    return q + a;   // G_AFFINE: q = gvec . X, a = offset
}

}  // namespace fbsde
