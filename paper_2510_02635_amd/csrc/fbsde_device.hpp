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

// sin and cos of the angle 2 pi (w + 1/2) 2^-32 of one Philox word w.  The octant comes exactly from
// the top three bits; the angle left over, |psi| <= pi/4, is taken from the low 29 bits in integer
// arithmetic (for odd octants as the distance to the next octant boundary, also exact), so no
// floating-point range reduction is needed; sin and cos of psi are their Taylor series, truncated where
// the next term is below half an ulp of the type (psi^19/19! for double, psi^11/11! for float).
template <typename R>
__device__ __forceinline__ void sincos_turn(uint32_t w, R& sn, R& cs);

template <>
__device__ __forceinline__ void sincos_turn<double>(uint32_t w, double& sn, double& cs) {
    const uint32_t o = w >> 29;                       // octant 0..7
    const uint32_t f = w & 0x1FFFFFFFu;
    const double two_pi_2m32 = 1.4629180792671596e-09;  // 2 pi 2^-32
    // even octant: psi = theta in [0, pi/4); odd: psi = theta - pi/4 in [-pi/4, 0)
    const double t = (o & 1u) ? -((double)(0x1FFFFFFFu - f) + 0.5) : ((double)f + 0.5);
    const double psi = t * two_pi_2m32;
    const double z = psi * psi;
    double ps = 1.0 / 121645100408832000.0;            // 1/19!
    ps = ps * z - 1.0 / 355687428096000.0;             // 1/17!
    ps = ps * z + 1.0 / 1307674368000.0;               // 1/15!
    ps = ps * z - 1.0 / 6227020800.0;                  // 1/13!
    ps = ps * z + 1.0 / 39916800.0;                    // 1/11!
    ps = ps * z - 1.0 / 362880.0;                      // 1/9!
    ps = ps * z + 1.0 / 5040.0;                        // 1/7!
    ps = ps * z - 1.0 / 120.0;                         // 1/5!
    ps = ps * z + 1.0 / 6.0;                           // 1/3!
    const double s_ = psi - psi * z * ps;
    double pc = 1.0 / 6402373705728000.0;              // 1/18!
    pc = pc * z - 1.0 / 20922789888000.0;              // 1/16!
    pc = pc * z + 1.0 / 87178291200.0;                 // 1/14!
    pc = pc * z - 1.0 / 479001600.0;                   // 1/12!
    pc = pc * z + 1.0 / 3628800.0;                     // 1/10!
    pc = pc * z - 1.0 / 40320.0;                       // 1/8!
    pc = pc * z + 1.0 / 720.0;                         // 1/6!
    pc = pc * z - 1.0 / 24.0;                          // 1/4!
    pc = pc * z + 0.5;                                 // 1/2!
    const double c_ = 1.0 - z * pc;
    const uint32_t q = ((o + 1u) >> 1) & 3u;          // angle = psi + q pi/2
    sn = (q == 0) ? s_ : (q == 1) ? c_ : (q == 2) ? -s_ : -c_;
    cs = (q == 0) ? c_ : (q == 1) ? -s_ : (q == 2) ? -c_ : s_;
}

template <>
__device__ __forceinline__ void sincos_turn<float>(uint32_t w, float& sn, float& cs) {
    const uint32_t o = w >> 29;
    const uint32_t f = w & 0x1FFFFFFFu;
    const float two_pi_2m32 = 1.46291808e-09f;
    const float t = (o & 1u) ? -((float)(0x1FFFFFFFu - f) + 0.5f) : ((float)f + 0.5f);
    const float psi = t * two_pi_2m32;
    const float z = psi * psi;
    float ps = 1.0f / 362880.0f;                       // 1/9!
    ps = ps * z - 1.0f / 5040.0f;
    ps = ps * z + 1.0f / 120.0f;
    ps = ps * z - 1.0f / 6.0f;
    const float s_ = psi + psi * z * ps;
    float pc = 1.0f / 3628800.0f;                      // 1/10!
    pc = pc * z - 1.0f / 40320.0f;
    pc = pc * z + 1.0f / 720.0f;
    pc = pc * z - 1.0f / 24.0f;
    pc = pc * z + 0.5f;
    const float c_ = 1.0f - z * pc;
    // angle = psi + q pi/2: odd q swaps sin and cos, and the signs are flipped in the sign bit
    // (sin: q = 2, 3; cos: q = 1, 2)
    const uint32_t q = ((o + 1u) >> 1) & 3u;
    const bool sw = (q & 1u) != 0u;
    const float a = sw ? c_ : s_, b = sw ? s_ : c_;
    sn = __uint_as_float(__float_as_uint(a) ^ ((q >> 1) << 31));
    cs = __uint_as_float(__float_as_uint(b) ^ (((q ^ (q >> 1)) & 1u) << 31));
}

// ln u for u = (w + 1/2) 2^-32 in FP64.  x = w + 1/2 is exact; frexp gives x = m 2^e exactly with
// m in [sqrt(1/2), sqrt(2)); ln m = 2 atanh(z) = 2 (z + z^3/3 + z^5/5 + ...) with z = (m - 1)/(m + 1),
// |z| <= 0.1716, so twelve odd terms reach the double rounding level (m - 1 is exact, so the result
// keeps full relative accuracy as u -> 1); (e - 32) ln 2 uses ln 2 split into a 32-bit head and a tail.
__device__ __forceinline__ double log_unit(uint32_t w) {
    const double x = (double)w + 0.5;
    int e;
    double m = frexp(x, &e);                 // x = m 2^e, m in [1/2, 1)
    if (m < 0.7071067811865476) { m += m; --e; }
    const double z = (m - 1.0) / (m + 1.0);
    const double z2 = z * z;
    double sr = 1.0 / 23.0;
    sr = sr * z2 + 1.0 / 21.0;
    sr = sr * z2 + 1.0 / 19.0;
    sr = sr * z2 + 1.0 / 17.0;
    sr = sr * z2 + 1.0 / 15.0;
    sr = sr * z2 + 1.0 / 13.0;
    sr = sr * z2 + 1.0 / 11.0;
    sr = sr * z2 + 1.0 / 9.0;
    sr = sr * z2 + 1.0 / 7.0;
    sr = sr * z2 + 1.0 / 5.0;
    sr = sr * z2 + 1.0 / 3.0;
    const double lnm = 2.0 * z + 2.0 * z * z2 * sr;
    const double k = (double)(e - 32);
    const double ln2_hi = 0.6931471803691238, ln2_lo = 1.9082149292705877e-10;
    return k * ln2_hi + (k * ln2_lo + lnm);
}

// ln u for u = (w + 1/2) 2^-32 in FP32 (the FP32C mode, whose state is FP32).  The reduction is done in
// integers so that m - 1 keeps full relative accuracy as u -> 1: with x = w + 1/2 = 2^e (1 + f),
// e = floor(log2 w), the numerator of m - 1 over 2^(e+1) is the exact integer 2 (w - 2^e) + 1; once
// w / 2^e reaches sqrt(2) the mantissa is halved, m/2 - 1 = -(2^(e+2) - 2w - 1) / 2^(e+2) (both
// numerators fit 32 bits; 2^(e+2) wraps to 0 for e >= 30, which leaves the difference exact).  Both
// candidates are formed and one is selected, with no branch.  Then ln m = 2 atanh(z),
// z = (m - 1)/(m + 1), |z| <= 0.1716, with the hardware reciprocal (about 1 ulp) for the division and
// five odd terms (truncation below 2e-9 relative); (e - 32) ln 2 with ln 2 split into a 16-bit head
// (exact products) and a tail.  Over all 2^32 words, sqrt(-2 ln u) from this logarithm and the hardware
// square root stays within 2.5 FP32 ulps of the FP64 form.
__device__ __forceinline__ float log_unit_f32(uint32_t w) {
    const int e = 31 - __clz((int)(w | 1u));                 // 2^e <= w < 2^(e+1); w = 0 selected below
    const bool upper = (w << (31 - e)) >= 0xB504F334u;       // w / 2^e >= sqrt(2)
    const uint32_t t_lo = 2u * (w - (1u << e)) + 1u;
    const uint32_t t_hi = ((e >= 30) ? 0u : (1u << (e + 2))) - 2u * w - 1u;
    const float mag = ldexpf((float)(upper ? t_hi : t_lo), upper ? -(e + 2) : -(e + 1));   // one rounding
    const float mm1 = upper ? -mag : mag;                    // m - 1 (or m/2 - 1)
    const int k = upper ? (e - 31) : (e - 32);
    const float z = mm1 * __builtin_amdgcn_rcpf(2.0f + mm1);
    const float z2 = z * z;
    float sr = 1.0f / 9.0f;
    sr = sr * z2 + 1.0f / 7.0f;
    sr = sr * z2 + 1.0f / 5.0f;
    sr = sr * z2 + 1.0f / 3.0f;
    const float lnm = 2.0f * z + 2.0f * z * z2 * sr;
    const float kf = (float)k;
    const float r = kf * 0.693145751953125f + (kf * 1.4286068e-06f + lnm);
    return (w == 0u) ? (-33.0f * 0.693145751953125f - 33.0f * 1.4286068e-06f) : r;   // u = 2^-33
}


// Four normals from one Philox call: Box-Muller on the word pairs (x, y) and (z, w) with
// u = (w + 1/2) 2^-32 in (0, 1); radius sqrt(-2 ln u_even) and angle 2 pi u_odd, both in the element
// type (FP64 logarithm for the FP64 mode, the FP32 one above for FP32C).
template <typename R> __device__ __forceinline__ R radius_of(uint32_t w);
template <> __device__ __forceinline__ double radius_of<double>(uint32_t w) { return sqrt(-2.0 * log_unit(w)); }
// -2 ln u lies in [2.3e-10, 46]: no zero, denormal or overflow, so the hardware square root (not the
// correctly rounded sequence) is enough
template <> __device__ __forceinline__ float radius_of<float>(uint32_t w) {
    return __builtin_amdgcn_sqrtf(-2.0f * log_unit_f32(w));
}

template <typename R>
__device__ __forceinline__ void box_muller4(const Words4& w, R z[4]) {
    const R r0 = radius_of<R>(w.x);
    const R r2 = radius_of<R>(w.z);
    R s1, c1, s3, c3;
    sincos_turn<R>(w.y, s1, c1);
    sincos_turn<R>(w.w, s3, c3);
    z[0] = r0 * c1; z[1] = r0 * s1; z[2] = r2 * c3; z[3] = r2 * s3;
}

// Normals of coordinates 4g..4g+3 of particle j, level k, stream q (point or shared).
template <typename R>
__device__ __forceinline__ void increment4(uint32_t g, uint32_t j, uint32_t k, uint32_t q,
                                           uint32_t k0, uint32_t k1, R z[4]) {
    const Words4 c = {g, j, k, q};
    box_muller4<R>(philox4x32_10(c, k0, k1), z);
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
enum { F_ZERO = 0, F_ALLEN_CAHN = 1, F_HJB = 2, F_BURGERS = 3, F_HJ_SINK = 4, F_LOG_POT = 5 };
enum { G_QUAD = 0, G_AC = 1, G_HJB_LOG = 2, G_AFFINE = 3, G_LOGISTIC = 4, G_HJ_GAUSS = 5, G_CASE2 = 6 };

// g families whose argument is q = gvec . X (the others take q = |X|^2)
__device__ __forceinline__ bool g_dot_arg(int kind) { return kind == G_AFFINE || kind == G_LOGISTIC; }

// Per-point FP64 slots of the reverse mode: alphabar, row-pass sum, Zbar coefficient along z, Wbar.bbar,
// f-parameter sums [4], g-parameter sums [4], terminal sum of 2h'G, terminal sum of G, Zbar coefficient
// along the all-ones vector (the Burgers family, whose d f / d z_i is the same for every i).
enum { A_ABAR = 0, A_TAU = 1, A_ZC = 2, A_WB = 3, A_FP = 4, A_GP = 8, A_S1 = 12, A_SG = 13, A_Z1 = 14, A_NS = 16 };
enum { ST_CG_MAXIT = 1, ST_NEWTON_FLAT = 2, ST_NONFINITE = 4 };

struct FSpec { int kind; double p0, p1, p2 = 0.0; };

// x-dependent coefficients mu(x) = mu0 x + mu1, sigma(x) = diag(sigma0 x + sigma1) in the per-point form:
// the state holds D = X - m, m the Euler-Maruyama mean path, with m_k = x0 A_k + B_k (A_k = (1 + mu0 dt)^k,
// B_k its drift part); a, b: the levels a kernel touches (the reversal reads k + 1 and writes k).
struct CoefArgs { double mu0, s0, mu1, s1, dt, Aa, Ba, Ab, Bb; };

// f(t, x, y, z) and d f / d y of the built-in families; zz = |z|^2 and zs = sum_i z_i (z shared by the
// cloud).  BURGERS: fp0 (y - fp1) sum_i z_i, the Burgers-type nonlinearity of the Sec. 4 experiments in
// a form whose logistic solution is exact (fp0 = s/d, fp1 = d/s^2 + 1/2).
// HJ_SINK: the sink -fp0 y |z|^2 / s^2 with p1 = 1 / s^2; its x-dependent source S(t, x) does not depend
// on y and enters Newton through C (hj_source).
__device__ __forceinline__ void f_and_fy(const FSpec& f, double y, double zz, double zs, double& fv, double& fy) {
    if (f.kind == F_ALLEN_CAHN) { fv = f.p0 * y - f.p1 * y * y * y; fy = f.p0 - 3.0 * f.p1 * y * y; }
    else if (f.kind == F_HJB) { fv = -f.p0 * zz; fy = 0.0; }
    else if (f.kind == F_BURGERS) { fv = f.p0 * (y - f.p1) * zs; fy = f.p0 * zs; }
    else if (f.kind == F_HJ_SINK) { fv = -f.p0 * f.p1 * y * zz; fy = -f.p0 * f.p1 * zz; }
    else if (f.kind == F_LOG_POT) {
        fv = 0.5 * f.p0 * log((1.0 + y) / (1.0 - y)) - f.p1 * y;
        fy = f.p0 / (1.0 - y * y) - f.p1;
    }
    else { fv = 0.0; fy = 0.0; }
}

// Products over the coordinates of a point, for Allen-Cahn Case 2: the pair (P, Q) = (prod_j x_j,
// sum_i prod_{j != i} x_j^2) of a set of coordinates; one coordinate is (x, 1), and two disjoint sets
// combine as (Pa Pb, Qa Pb^2 + Qb Pa^2) (associative and commutative, identity (1, 0)).
__device__ __forceinline__ void pq_add(double& P, double& Q, double x) {
    Q = Q * x * x + P * P;
    P *= x;
}
__device__ __forceinline__ void pq_combine(double& P, double& Q, double Pb, double Qb) {
    Q = Q * Pb * Pb + Qb * P * P;
    P *= Pb;
}

// Source of Allen-Cahn Case 2 at time t for r2 = |x|^2 and (P, Q2) of x: with v = amp cos(P) w,
// w = e^(cos t - r2), S2 = v_t + (s^2/2) Lap v + F(v), v_t = -sin(t) v,
// Lap v = amp w (-cos(P) Q2 + 4 d P sin(P) + cos(P) (4 r2 - 2 d)), F the log potential (theta, theta_c).
__device__ __forceinline__ double case2_source(double t, double r2, double P, double Q2, double d, double s,
                                               double theta, double theta_c, double amp) {
    const double w = exp(cos(t) - r2), cP = cos(P), sP = sin(P);
    const double v = amp * cP * w;
    const double lap = amp * w * (-cP * Q2 + 4.0 * d * P * sP + cP * (4.0 * r2 - 2.0 * d));
    return -sin(t) * v + 0.5 * s * s * lap + 0.5 * theta * log((1.0 + v) / (1.0 - v)) - theta_c * v;
}

// d S2 / d x_k for the same point: Pk, Q2k are P and Q2 of the coordinates other than k, so that
// d_k P = Pk and d_k Q2 = 2 x_k Q2k; the derivatives of w, v, the Laplacian's bracket and F written out.
__device__ __forceinline__ double case2_source_dk(double t, double r2, double P, double Q2, double xk, double Pk,
                                                  double Q2k, double d, double s, double theta, double theta_c,
                                                  double amp) {
    const double w = exp(cos(t) - r2), cP = cos(P), sP = sin(P);
    const double v = amp * cP * w;
    const double D = -cP * Q2 + 4.0 * d * P * sP + cP * (4.0 * r2 - 2.0 * d);
    const double dv = amp * w * (-sP * Pk - 2.0 * xk * cP);
    const double dD = sP * Pk * Q2 - cP * 2.0 * xk * Q2k + 4.0 * d * (Pk * sP + P * cP * Pk) -
                      sP * Pk * (4.0 * r2 - 2.0 * d) + cP * 8.0 * xk;
    const double dlap = amp * (-2.0 * xk * w * D + w * dD);
    return -sin(t) * dv + 0.5 * s * s * dlap + (theta / (1.0 - v * v) - theta_c) * dv;
}

// Source of the Hamilton-Jacobi-type family at time t and r2 = |x|^2, and its derivative in r2: with
// v = a^(-d/2) exp(-r2/a), a = 1 + 4t (a heat kernel: Lap v = v_t), the source that makes v exact for
// v_t + (s^2/2) Lap v + S - kappa v |grad v|^2 = 0 is S = -(1 + s^2/2) v_t + kappa v |grad v|^2, where
// v_t = v (-2d/a + 4 r2/a^2) and |grad v|^2 = 4 r2 v^2 / a^2.
__device__ __forceinline__ double hj_source(double t, double r2, double d, double s, double kappa, double* dS) {
    const double a = 1.0 + 4.0 * t, ia = 1.0 / a;
    const double c = 1.0 + 0.5 * s * s;
    const double v = exp(-0.5 * d * log(a) - r2 * ia);
    const double B = -2.0 * d * ia + 4.0 * r2 * ia * ia;
    const double E = 4.0 * r2 * ia * ia;
    if (dS) {
        const double dv = -v * ia;
        *dS = -c * (dv * B + v * 4.0 * ia * ia) + kappa * (3.0 * v * v * dv * E + v * v * v * 4.0 * ia * ia);
    }
    return -c * v * B + kappa * v * v * v * E;
}

// Fixed-count Newton for F(y) = y - C - dt f(y) from y = C; returns y and F'(y).
__device__ __forceinline__ double newton_y(const FSpec& f, double C, double zz, double zs, double dt, int iters,
                                           double& Fp, uint32_t& st) {
    double y = C, fv, fy;
    for (int n = 0; n < iters; ++n) {
        f_and_fy(f, y, zz, zs, fv, fy);
        const double F = y - C - dt * fv;
        const double dF = 1.0 - dt * fy;
        if (fabs(dF) < 1e-12) st |= ST_NEWTON_FLAT;
        y = y - F / dF;
    }
    f_and_fy(f, y, zz, zs, fv, fy);
    Fp = 1.0 - dt * fy;
    if (!isfinite(y)) st |= ST_NONFINITE;
    return y;
}

// Terminal g from q = |X|^2 (radial families) or q = gvec . X (affine, logistic).
__device__ __forceinline__ double g_of(int kind, double a, double b, double q, int64_t d) {
    if (kind == G_QUAD) return a * q / (double)d + b;
    if (kind == G_AC) return 1.0 / (2.0 + a * q);
    if (kind == G_HJB_LOG) return log((1.0 + a * q) * 0.5);
    if (kind == G_LOGISTIC) return 1.0 / (1.0 + exp(-(q + a)));   // a = offset
    if (kind == G_HJ_GAUSS) return exp(-0.5 * (double)d * log1p(4.0 * a) - q / (1.0 + 4.0 * a));
    return q + a;   // G_AFFINE: q = gvec . X, a = offset
}

}  // namespace fbsde
