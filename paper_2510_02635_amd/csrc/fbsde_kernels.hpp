// HIP kernels of one level of the localized FBSDE-LLR scheme on gfx950.
//
// Data layout in HBM (per evaluation point p):
//   W   [P][M][ld]  Brownian displacement of every particle (X = x0 + t mu + s W); the state
//                   that the sweeps stream.  ld = d rounded up to 128 bytes, pad kept at zero.
//   per-particle scalars [P][M]: |W|^2, Y, kernel weights w, w (Y - Ybar).
//   per-point vectors   [P][ld]: CG iterate, residual, direction, A p, weighted mean of W.
//   two-stage partial sums [P][nchunk][ld] (fixed reduction order: results are deterministic).
//
// Row geometry: a "team" of TEAM wavefronts owns one particle row; lane L of a team holds
// coordinate groups g = L + q * 64 TEAM (q < Q), each four consecutive coordinates (one Philox
// call, one 16/32-byte load), so a team covers 256 Q TEAM coordinates and consecutive lanes read
// consecutive 16/32-byte pieces of the row (fully coalesced).  A block has max(4, TEAM) waves:
// 4 / TEAM teams for small d, one team for large d.  Row dot products reduce in registers and
// across the wave with shuffles, across a team's waves through LDS; column sums over particles
// accumulate in registers and are combined per block through LDS, then across blocks in a
// second, fixed-order stage.
//
// Element types: S = double (FP64 mode) or float (FP32C mode: FP32 state and FP32 arithmetic with
// Kahan-compensated per-lane sums; row dots are finished and all CG / Newton scalars kept in FP64).
#pragma once
#include "fbsde_rowteam.hpp"

namespace fbsde {

// ------------------------------------------------------------------------------------------
// Forward sweep and terminal condition (Algorithm 1, first two loops; eq. Xk):
//   W^j_N = sum_k sqrt(dt) xi^j_k in registers, one store; Y^j_N = g(x0 + mu T + s W^j_N).
// COEF: x-dependent coefficients (CoefArgs): every coordinate follows the Euler-Maruyama step
// X_{k+1} = X_k + (mu0 X_k + mu1) dt + (sigma0 X_k + sigma1) sqrt(dt) xi_k from x0, and the state holds
// D_N = X_N - m_N (cf.Aa, cf.Ba: A_N, B_N).
template <typename S, int Q, int TEAM, bool COEF = false>
__global__ void __launch_bounds__((Geo<Q, TEAM>::BS))
k_forward(S* __restrict__ W, int64_t ldw, int M, int rows_per_chunk, const double* __restrict__ x0,
          const double* __restrict__ mu, const double* __restrict__ gvec, int d, int ld, int N,
          double sqdt, double s, double T, int g_kind, double ga, double gb, uint32_t k0, uint32_t k1,
          uint32_t point_base, int shared, double* __restrict__ Y, double* __restrict__ rn2,
          uint32_t* __restrict__ status, CoefArgs cf = CoefArgs{}) {
    using G = Geo<Q, TEAM>;
    __shared__ double red[2 * G::BS / 64];
    const int p = blockIdx.y;
    const int team = threadIdx.x / G::TL, L = threadIdx.x % G::TL;
    const int r0 = blockIdx.x * rows_per_chunk;
    const int r1 = min(M, r0 + rows_per_chunk);
    const uint32_t qs = shared ? 0xFFFFFFFFu : point_base + (uint32_t)p;
    double xc[Q][4];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int i = 4 * (L + q * G::TL) + e;
            xc[q][e] = (i < d) ? (x0 ? x0[(int64_t)p * d + i] : 0.0) + ((mu && !COEF) ? mu[i] * T : 0.0) : 0.0;
        }
    uint32_t st = 0;
    for (int jb = r0; jb < r1; jb += G::TPW) {
        const int j = jb + team;
        const bool valid = j < r1;
        double w[Q][4];   // COEF: the position X; otherwise the Brownian displacement W
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) w[q][e] = COEF ? xc[q][e] : 0.0;
        if (valid) {
            for (int k = 0; k < N; ++k) {
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int g = L + q * G::TL;
                    if (4 * g < d) {
                        S z[4];
                        increment4<S>((uint32_t)g, (uint32_t)j, (uint32_t)k, qs, k0, k1, z);
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (4 * g + e < d) {
                                if constexpr (COEF) {
                                    const double xv = w[q][e];
                                    w[q][e] = xv + (cf.mu0 * xv + cf.mu1) * cf.dt + (cf.s0 * xv + cf.s1) * (sqdt * (double)z[e]);
                                } else {
                                    w[q][e] += sqdt * (double)z[e];
                                }
                            }
                    }
                }
            }
        }
        double n2 = 0.0, gq = 0.0, Pp = 1.0, Pq = 0.0;   // Pp: product of the coordinates (G_CASE2)
        if (valid) {
            S* row = W + ((int64_t)(shared ? 0 : p) * M + j) * ldw;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int e0 = 4 * (L + q * G::TL);
                if (e0 < ld) {
                    S v[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        v[e] = COEF ? ((e0 + e < d) ? (S)(w[q][e] - (xc[q][e] * cf.Aa + cf.Ba)) : (S)0) : (S)w[q][e];
                    if (!shared || p == 0) store4(row + e0, v);
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const double ws = (double)v[e];
                        n2 += ws * ws;
                        const double X = COEF ? w[q][e] : xc[q][e] + s * ws;
                        if (g_dot_arg(g_kind)) gq += ((e0 + e < d) ? gvec[e0 + e] : 0.0) * X;
                        else gq += X * X;
                        if (g_kind == G_CASE2 && e0 + e < d) Pp *= X;
                    }
                }
            }
        }
        team_sum2<TEAM>(n2, gq, red, team);
        if (g_kind == G_CASE2) team_pq<TEAM>(Pp, Pq, red, team);
        if (valid && (L == 0)) {
            // G_CASE2: gb cos(prod x) e^(cos ga - |x|^2)
            const double y = (g_kind == G_CASE2) ? gb * cos(Pp) * exp(cos(ga) - gq) : g_of(g_kind, ga, gb, gq, d);
            Y[(int64_t)p * M + j] = y;
            if (rn2) rn2[(int64_t)p * M + j] = n2;
            if (!isfinite(y)) st |= ST_NONFINITE;
        }
    }
    if (st) atomicOr(&status[p], st);
}

// Kernel weights of the cloud (eq. Dj with the Gaussian kernel), weighted mean of Y and the
// centred response coefficients w_j (Y_j - Ybar).  One block per point.  warm: c2 holds
// dY_j/dC_j = 1/F'(Y_j) from the previous level's Newton solve, and rho = sum_j w_j dY_j/dC_j is
// stored in scal[7] (the scale of the CG warm start).
__global__ void __launch_bounds__(256)
k_weights(const double* __restrict__ rn2, const double* __restrict__ Y, int M, double s2, double eps2_all,
          double* __restrict__ w, double* __restrict__ c2, double* __restrict__ scal, int ns, int* active, int P,
          int warm, const double* __restrict__ vt = nullptr, int vstride = 0, double vfac = 0.0) {
    __shared__ double lds[16];
    const int p = blockIdx.x;
    // x-dependent coefficients: the bandwidth of the point's own cloud, vfac V (vt[p vstride] = V of its
    // Euler-Maruyama particles at this level)
    const double eps2 = vt ? vfac * vt[(int64_t)p * vstride] : eps2_all;
    const double* n = rn2 + (int64_t)p * M;
    const double* y = Y + (int64_t)p * M;
    double* wp = w + (int64_t)p * M;
    double* cp = c2 + (int64_t)p * M;
    double mn = INFINITY;
    for (int j = threadIdx.x; j < M; j += blockDim.x) mn = fmin(mn, n[j]);
    mn = block_min(mn, lds);
    double se = 0.0;
    for (int j = threadIdx.x; j < M; j += blockDim.x) {
        const double e = (eps2 > 0.0) ? exp(-(s2 * n[j] - s2 * mn) / eps2) : 1.0;
        wp[j] = e;
        se += e;
    }
    se = block_sum(se, lds);
    double yb = 0.0, rho = 0.0;
    for (int j = threadIdx.x; j < M; j += blockDim.x) {
        const double wj = wp[j] / se;
        wp[j] = wj;
        yb += wj * y[j];
        if (warm) rho += wj * cp[j];
    }
    yb = block_sum(yb, lds);
    rho = block_sum(rho, lds);
    for (int j = threadIdx.x; j < M; j += blockDim.x) cp[j] = wp[j] * (y[j] - yb);
    if (threadIdx.x == 0) {
        scal[(int64_t)p * ns + 4] = yb;
        scal[(int64_t)p * ns + 7] = warm ? rho : 0.0;
        if (p == 0) *active = P;
    }
}

// Weighted first moments of the cloud: sum_j w_j W_j and sum_j w_j (Y_j - Ybar) W_j (column sums
// over particles; the normal-equation right-hand side, eq. normal-eq), per block.  warm: also the
// pieces of A x0 for the CG warm start x0 = rho * xw (xw = previous level's slope):
// t_j = W_j . x0, sum_j w_j t_j W_j and sum_j w_j t_j, with the row still in registers.  R is the
// arithmetic type (FP64 on the FP32 state for a rank-deficient design, as in the CG product).
template <typename S, typename R, int Q, int TEAM>
__global__ void __launch_bounds__((Geo<Q, TEAM>::BS))
k_moments(const S* __restrict__ W, int64_t ldw, int M, int rows_per_chunk, int nchunk, int ld,
          const double* __restrict__ w, const double* __restrict__ c2, const double* __restrict__ xw,
          const double* __restrict__ scal, int ns, int warm, double* __restrict__ part1, double* __restrict__ part2,
          double* __restrict__ part3, double* __restrict__ psc) {
    using G = Geo<Q, TEAM>;
    __shared__ double lds[(G::TPW > 1) ? G::TPW * 4 * Q * G::TL : 1];
    __shared__ double red[2 * G::BS / 64];
    const int p = blockIdx.y, c = blockIdx.x;
    const int team = threadIdx.x / G::TL, L = threadIdx.x % G::TL;
    const int r0 = c * rows_per_chunk;
    const int r1 = min(M, r0 + rows_per_chunk);
    R v[Q][4];
    const double rho = warm ? scal[(int64_t)p * ns + 7] : 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int e0 = 4 * (L + q * G::TL);
#pragma unroll
        for (int e = 0; e < 4; ++e) v[q][e] = (warm && e0 < ld) ? (R)(rho * xw[(int64_t)p * ld + e0 + e]) : (R)0;
    }
    CSum<R> a1[Q][4], a2[Q][4], a3[Q][4];
    double sig = 0.0, tau = 0.0;
    for (int jb = r0; jb < r1; jb += G::TPW) {
        const int j = jb + team;
        const bool valid = j < r1;
        S x[Q][4];
        CSum<R> dl;
        double wjd = 0.0;
        if (valid) {
            const S* row = W + ((int64_t)p * M + j) * ldw;
            wjd = w[(int64_t)p * M + j];
            const R wj = (R)wjd;
            const double cjd = c2[(int64_t)p * M + j];
            const R cj = (R)cjd;
            sig += cjd;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int e0 = 4 * (L + q * G::TL);
                if (e0 < ld) load4(row + e0, x[q]);
                else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) x[q][e] = (S)0;
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const R xr = (R)x[q][e];
                    a1[q][e].add(wj * xr);
                    a2[q][e].add(cj * xr);
                    if (warm) dl.add(xr * v[q][e]);
                }
            }
        }
        if (warm) {
            double t = dl.get(), unused = 0.0;
            team_sum2<TEAM>(t, unused, red, team);
            if (valid) {
                const double ct = wjd * t;
                tau += ct;
                const R cr = (R)ct;
#pragma unroll
                for (int q = 0; q < Q; ++q)
#pragma unroll
                    for (int e = 0; e < 4; ++e) a3[q][e].add(cr * (R)x[q][e]);
            }
        }
    }
    const int64_t off = ((int64_t)p * nchunk + c) * ld;
    block_columns_out<Q, TEAM, R>(a1, lds, part1 + off, ld, team, L);
    block_columns_out<Q, TEAM, R>(a2, lds, part2 + off, ld, team, L);
    if (warm) block_columns_out<Q, TEAM, R>(a3, lds, part3 + off, ld, team, L);
    // sig and tau are identical on every lane of a team: one lane per team contributes
    const double ts = block_sum((L == 0) ? sig : 0.0, red);
    const double tt = block_sum((L == 0) ? tau : 0.0, red);
    if (threadIdx.x == 0) {
        psc[((int64_t)p * nchunk + c) * 2] = ts;
        psc[((int64_t)p * nchunk + c) * 2 + 1] = tt;
    }
}

// Finish the moments and start CG on (sum_j w_j D'_j D'_j^T + lam I) a_x = b.
// Cold start x0 = 0; warm start x0 = rho * (previous level's slope, in x) with
// A x0 = s^2 (sum_j w_j t_j W_j - (sum_j w_j t_j) Wbar) + lam x0, t_j = W_j . x0.
// Per-point sum of the per-chunk partial vectors into chunk 0 of each buffer, spread over the
// chip: block (x, p) owns 64 elements of point p; its four waves sum four contiguous chunk ranges
// and wave 0 adds the four range sums in order.  Deterministic for a fixed chunk count.  Used when
// a point is split over many chunks, where a one-block-per-point finish would read them serially.
__global__ void __launch_bounds__(256)
k_fold_chunks(double* __restrict__ a, double* __restrict__ b, double* __restrict__ c3, int nchunk, int ld) {
    __shared__ double red[3][4][64];
    const int p = blockIdx.y;
    const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lane;
    const int per = (nchunk + 3) / 4;
    const int c0 = min(nchunk, g * per), c1 = min(nchunk, c0 + per);
    double* bufs[3] = {a, b, c3};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double acc = 0.0;
        if (bufs[k] && i < ld)
            for (int c = c0; c < c1; ++c) acc += bufs[k][((int64_t)p * nchunk + c) * ld + i];
        red[k][g][lane] = acc;
    }
    __syncthreads();
    if (g == 0 && i < ld) {
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (bufs[k])
                bufs[k][(int64_t)p * nchunk * ld + i] = ((red[k][0][lane] + red[k][1][lane]) + red[k][2][lane]) + red[k][3][lane];
    }
}

// scal layout per point: 0 rr, 1 |b|^2, 2 wv = Wbar.p, 3 lam, 4 Ybar, 5 alpha, 6 zz = |Z|^2, 7 rho,
// 8 zs = sum_i Z_i.
// iscal: 0 iterations, 1 done.
__global__ void __launch_bounds__(256)
k_moments_finish(const double* __restrict__ part1, const double* __restrict__ part2,
                 const double* __restrict__ part3, const double* __restrict__ psc, int nchunk, int vchunks, int ld,
                 double s, double lam_all, int warm, double* __restrict__ Wbar, double* __restrict__ x, double* __restrict__ r,
                 double* __restrict__ pv, double* __restrict__ scal, int ns, int* __restrict__ iscal, int* active,
                 const double* __restrict__ vt = nullptr, int vstride = 0, double vfac = 0.0) {
    __shared__ double lds[16];
    const int p = blockIdx.x;
    const double lam = vt ? vfac * vt[(int64_t)p * vstride] : lam_all;   // per point (x-dependent coefficients)
    double sig = 0.0, tau = 0.0;
    for (int c = 0; c < nchunk; ++c) {
        sig += psc[((int64_t)p * nchunk + c) * 2];
        tau += psc[((int64_t)p * nchunk + c) * 2 + 1];
    }
    const double rho = warm ? scal[(int64_t)p * ns + 7] : 0.0;
    // Pass 1: b, the warm start x0 and the residual b - A x0 (b in r, the residual in pv), and the
    // largest magnitude among them.
    double big = 0.0;
    for (int i = threadIdx.x; i < ld; i += blockDim.x) {
        double wb = 0.0, bb = 0.0, ab = 0.0;
        for (int c = 0; c < vchunks; ++c) {
            wb += part1[((int64_t)p * nchunk + c) * ld + i];
            bb += part2[((int64_t)p * nchunk + c) * ld + i];
            if (warm) ab += part3[((int64_t)p * nchunk + c) * ld + i];
        }
        const double b = s * (bb - sig * wb);
        double x0 = 0.0, res = b;
        if (warm) {
            x0 = rho * x[(int64_t)p * ld + i];
            res = b - (s * s * (ab - tau * wb) + lam * x0);
        }
        Wbar[(int64_t)p * ld + i] = wb;
        x[(int64_t)p * ld + i] = x0;
        r[(int64_t)p * ld + i] = b;
        pv[(int64_t)p * ld + i] = res;
        big = fmax(big, fmax(fabs(b), fabs(res)));
    }
    // The system is solved for sc b with sc a power of two that brings the right-hand side to order one:
    // A does not depend on Y, so the CG iterates scale exactly, while squared norms of a right-hand side
    // far from one (|Y - Ybar| ~ 1e-150 where the terminal value is a d = 500 Gaussian) would leave the
    // normal range.  k_level_finish takes the scale back out of the slope.
    big = -block_min(-big, lds);
    const double sc = (big > 0.0 && isfinite(big)) ? ldexp(1.0, -max(-1000, min(1000, ilogb(big)))) : 1.0;
    double rr = 0.0, bb2 = 0.0, wv = 0.0;
    for (int i = threadIdx.x; i < ld; i += blockDim.x) {
        const double b = sc * r[(int64_t)p * ld + i], res = sc * pv[(int64_t)p * ld + i];
        x[(int64_t)p * ld + i] *= sc;
        r[(int64_t)p * ld + i] = res;
        pv[(int64_t)p * ld + i] = res;
        rr += res * res;
        bb2 += b * b;
        wv += Wbar[(int64_t)p * ld + i] * res;
    }
    rr = block_sum(rr, lds);
    bb2 = block_sum(bb2, lds);
    wv = block_sum(wv, lds);
    if (threadIdx.x == 0) {
        scal[(int64_t)p * ns + 0] = rr;
        scal[(int64_t)p * ns + 1] = bb2;
        scal[(int64_t)p * ns + 2] = wv;
        scal[(int64_t)p * ns + 3] = lam;
        scal[(int64_t)p * ns + 9] = 1.0 / sc;
        iscal[p * 4 + 0] = 0;
        const int done = (rr == 0.0) ? 1 : 0;
        iscal[p * 4 + 1] = done;
        if (done) atomicSub(active, 1);
    }
}

// One pass of the fused matrix-free product of the centred weighted normal matrix with the CG
// direction p (the two steps of the paper's matrix-free scheme done per particle row while the
// row sits in registers): t_j = D'_j . p = s (W_j . p - Wbar . p), then sum_j w_j t_j W_j and
// sum_j w_j t_j, per block.  One read of the state per CG iteration.  R is the arithmetic type: the
// element type with compensated FP32 sums for the forward solve, or FP64 on the FP32 state for the
// adjoint solve, whose right-hand side reaches the ridge-only null space of the centred design (there
// the iterate grows like 1/lam and FP32 row dots would leak eps32 |W| |x| back into the range).
template <typename S, typename R, int Q, int TEAM>
__global__ void __launch_bounds__((Geo<Q, TEAM>::BS))
k_matvec(const S* __restrict__ W, int64_t ldw, int M, int rows_per_chunk, int nchunk, int ld, double s,
         const double* __restrict__ w, const double* __restrict__ pv, const double* __restrict__ scal,
         int ns, const int* __restrict__ iscal, double* __restrict__ part, double* __restrict__ psc) {
    using G = Geo<Q, TEAM>;
    __shared__ double lds[(G::TPW > 1) ? G::TPW * 4 * Q * G::TL : 1];
    __shared__ double red[2 * G::BS / 64];
    const int p = blockIdx.y, c = blockIdx.x;
    if (iscal[p * 4 + 1]) return;
    const int team = threadIdx.x / G::TL, L = threadIdx.x % G::TL;
    const int r0 = c * rows_per_chunk;
    const int r1 = min(M, r0 + rows_per_chunk);
    R v[Q][4];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int e0 = 4 * (L + q * G::TL);
#pragma unroll
        for (int e = 0; e < 4; ++e) v[q][e] = (e0 < ld) ? (R)pv[(int64_t)p * ld + e0 + e] : (R)0;
    }
    const double wvp = scal[(int64_t)p * ns + 2];
    CSum<R> acc[Q][4];
    double tau = 0.0;
    // rows are double-buffered: the loads of the team's next row are issued before the reduction of
    // the current one, so a wave keeps two rows in flight across the team barrier (not in 1024-lane
    // blocks, whose 128-register cap the second buffer would overflow, nor with FP64 arithmetic on
    // eight groups per lane, which already fills the register file)
    constexpr bool PF = G::BS < 1024 && !(sizeof(R) > sizeof(S) && Q == 8);
    const S* base = W + (int64_t)p * M * ldw;
    S x[Q][4];
    if (PF && r0 + team < r1) load_row<S, Q, G::TL>(base + (int64_t)(r0 + team) * ldw, ld, L, x);
    for (int jb = r0; jb < r1; jb += G::TPW) {
        const int j = jb + team;
        const bool valid = j < r1;
        S xn[Q][4];
        if (PF) {
            if (j + G::TPW < r1) load_row<S, Q, G::TL>(base + (int64_t)(j + G::TPW) * ldw, ld, L, xn);
        } else if (valid) {
            load_row<S, Q, G::TL>(base + (int64_t)j * ldw, ld, L, x);
        }
        CSum<R> dl;
        if (valid) {
#pragma unroll
            for (int q = 0; q < Q; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) dl.add((R)x[q][e] * v[q][e]);
        }
        double t = dl.get(), unused = 0.0;
        team_sum2<TEAM>(t, unused, red, team);
        if (valid) {
            const double cj = w[(int64_t)p * M + j] * s * (t - wvp);
            tau += cj;
            const R cr = (R)cj;
#pragma unroll
            for (int q = 0; q < Q; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[q][e].add(cr * (R)x[q][e]);
        }
        if (PF) {
#pragma unroll
            for (int q = 0; q < Q; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) x[q][e] = xn[q][e];
        }
    }
    block_columns_out<Q, TEAM, R>(acc, lds, part + ((int64_t)p * nchunk + c) * ld, ld, team, L);
    const double contrib = (L == 0) ? tau : 0.0;
    const double tot = block_sum(contrib, red);
    if (threadIdx.x == 0) psc[(int64_t)p * nchunk + c] = tot;
}

// CG step on the per-point vectors (one block per point): q = s (sum_c part_c - tau Wbar) + lam p,
// then the usual conjugate-gradient updates; convergence |r| <= rtol |b| or the iteration cap.
__global__ void __launch_bounds__(256)
k_cg_update(const double* __restrict__ part, const double* __restrict__ psc, int nchunk, int vchunks, int ld,
            double s,
            const double* __restrict__ Wbar, double* __restrict__ x, double* __restrict__ r,
            double* __restrict__ pv, double* __restrict__ qv, double* __restrict__ scal, int ns,
            int* __restrict__ iscal, double rtol2, int maxit, int* active, uint32_t* __restrict__ status) {
    __shared__ double lds[16];
    const int p = blockIdx.x;
    if (iscal[p * 4 + 1]) return;
    double* sc = scal + (int64_t)p * ns;
    const double lam = sc[3];
    double tau = 0.0;
    for (int c = 0; c < nchunk; ++c) tau += psc[(int64_t)p * nchunk + c];
    const int64_t o = (int64_t)p * ld;
    double pq = 0.0;
    for (int i = threadIdx.x; i < ld; i += blockDim.x) {
        double a = 0.0;
        for (int c = 0; c < vchunks; ++c) a += part[((int64_t)p * nchunk + c) * ld + i];
        const double q = s * (a - tau * Wbar[o + i]) + lam * pv[o + i];
        qv[o + i] = q;
        pq += pv[o + i] * q;
    }
    pq = block_sum(pq, lds);
    const double rr = sc[0];
    const double alpha = (pq > 0.0) ? rr / pq : 0.0;
    double rr2 = 0.0;
    for (int i = threadIdx.x; i < ld; i += blockDim.x) {
        x[o + i] += alpha * pv[o + i];
        const double ri = r[o + i] - alpha * qv[o + i];
        r[o + i] = ri;
        rr2 += ri * ri;
    }
    rr2 = block_sum(rr2, lds);
    const int it = iscal[p * 4 + 0] + 1;
    int done = 0;
    uint32_t st = 0;
    if (!(pq > 0.0) || rr2 <= rtol2 * sc[1]) done = 1;
    else if (it >= maxit) { done = 1; st = ST_CG_MAXIT; }
    double wv = 0.0;
    if (!done) {
        const double beta = rr2 / rr;
        for (int i = threadIdx.x; i < ld; i += blockDim.x) {
            const double pi = r[o + i] + beta * pv[o + i];
            pv[o + i] = pi;
            wv += Wbar[o + i] * pi;
        }
        wv = block_sum(wv, lds);
    }
    if (threadIdx.x == 0) {
        sc[0] = rr2;
        sc[2] = wv;
        iscal[p * 4 + 0] = it;
        iscal[p * 4 + 1] = done;
        if (done) atomicSub(active, 1);
        if (st) atomicOr(&status[p], st);
    }
}

// Intercept alpha = Ybar - s alpha_x . Wbar (eq. taylorexp / Schur form), |Z|^2 = s^2 |alpha_x|^2 and
// sum_i Z_i = s sum_i alpha_x,i; optional dense copies of alpha, alpha_x for the caller.
__global__ void __launch_bounds__(256)
k_level_finish(double* __restrict__ x, const double* __restrict__ Wbar, int ld, int d, double s,
               double* __restrict__ scal, int ns, double* __restrict__ alpha_out,
               double* __restrict__ alpha_x_out) {
    __shared__ double lds[16];
    const int p = blockIdx.x;
    const int64_t o = (int64_t)p * ld;
    // the CG solved for the scaled right-hand side (k_moments_finish): the slope is the iterate over sc
    const double isc = scal[(int64_t)p * ns + 9];
    double xw = 0.0, xx = 0.0, xs = 0.0;
    for (int i = threadIdx.x; i < ld; i += blockDim.x) {
        if (isc != 1.0) x[o + i] *= isc;
        xw += x[o + i] * Wbar[o + i];
        xx += x[o + i] * x[o + i];
        xs += x[o + i];
        if (alpha_x_out && i < d) alpha_x_out[(int64_t)p * d + i] = x[o + i];
    }
    xw = block_sum(xw, lds);
    xx = block_sum(xx, lds);
    xs = block_sum(xs, lds);
    if (threadIdx.x == 0) {
        double* sc = scal + (int64_t)p * ns;
        const double alpha = sc[4] - s * xw;
        sc[5] = alpha;
        sc[6] = s * s * xx;
        sc[8] = s * xs;
        if (alpha_out) alpha_out[p] = alpha;
    }
}

// Particle reversal W_k = W_{k+1} - sqrt(dt) xi_k (Philox regenerated, in place) fused with the
// per-particle dots |W_k|^2 and alpha_x . W_k, the local linear model C = alpha + s alpha_x . W_k
// and the Newton solve for Y_k (eqs. nonlinearf / NRiter).  zero_state: level 0, W_0 = 0.
// XK != 0: f has an x-dependent source, evaluated at the particle's position X = b + s W_k with
// b = x0 + t_k mu (a third row dot b . W_k gives |X|^2) and moved into C (Newton's F(y) = y - C - dt f
// with f = f(y) + source): XK = 1 the Hamilton-Jacobi-type source (a function of |X|^2), XK = 2 the
// Allen-Cahn Case 2 source, which also needs the coordinate products (P, Q2) of X (pq_add per lane,
// team_pq across the team).  XK = 3: x-dependent coefficients (CoefArgs; b = x0): the state holds
// D = X - m, the reversal inverts the Euler-Maruyama step, X_k = (X_{k+1} - mu1 dt - sigma1 dW) /
// (1 + mu0 dt + sigma0 dW), the model is taken at the drift-transported particle, C = alpha +
// (1 + mu0 dt) alpha_x . D_k, and Z = (sigma0 X_k + sigma1) * alpha_x is the particle's own (|Z|^2 and
// sum_i Z_i per row).
template <typename S, int Q, int TEAM, int XK = 0>
__global__ void __launch_bounds__((Geo<Q, TEAM>::BS))
k_reverse(S* __restrict__ W, int64_t ldw, int M, int rows_per_chunk, int d, int ld, int k, int zero_state,
          double sqdt, double s, double dt, const double* __restrict__ ax, const double* __restrict__ scal,
          int ns, FSpec f, int newton_iters, uint32_t k0, uint32_t k1, uint32_t point_base,
          double* __restrict__ Y, double* __restrict__ rn2, double* __restrict__ dydc, uint32_t* __restrict__ status,
          int shared, const double* __restrict__ x0 = nullptr, const double* __restrict__ mu = nullptr,
          double tk = 0.0, CoefArgs cf = CoefArgs{}, double* __restrict__ zz_out = nullptr,
          double* __restrict__ zs_out = nullptr) {
    using G = Geo<Q, TEAM>;
    using R = S;
    __shared__ double red[2 * G::BS / 64];
    const int p = blockIdx.y;
    const int team = threadIdx.x / G::TL, L = threadIdx.x % G::TL;
    const int r0 = blockIdx.x * rows_per_chunk;
    const int r1 = min(M, r0 + rows_per_chunk);
    const uint32_t qs = shared ? 0xFFFFFFFFu : point_base + (uint32_t)p;
    R a[Q][4];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int e0 = 4 * (L + q * G::TL);
#pragma unroll
        for (int e = 0; e < 4; ++e) a[q][e] = (e0 < ld) ? (R)ax[(int64_t)p * ld + e0 + e] : (R)0;
    }
    const double alpha = scal[(int64_t)p * ns + 5];
    const double zz = scal[(int64_t)p * ns + 6], zs = scal[(int64_t)p * ns + 8];
    uint32_t st = 0;
    R b[Q][4];        // XK: the lane's coordinates of b = x0 + t_k mu
    double bb = 0.0;  // XK: |b|^2
    if constexpr (XK != 0) {
        double lb = 0.0, unused = 0.0;
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = 4 * (L + q * G::TL) + e;
                const double v = (i < d) ? (x0 ? x0[(int64_t)p * d + i] : 0.0) + (mu ? mu[i] * tk : 0.0) : 0.0;
                b[q][e] = (R)v;
                lb += v * v;
            }
        team_sum2<TEAM>(lb, unused, red, team);
        bb = lb;
    }
    // Newton runs 64 rows at a time: lane (row count mod 64) of the team's first wave keeps the row's
    // C and |W|^2, and every 64 rows those lanes solve together instead of one lane per row
    int j_keep = -1;
    double c_keep = 0.0, n2_keep = 0.0, zz_keep = zz, zs_keep = zs;   // XK == 3: the particle's own Z
    auto flush = [&]() {
        if (j_keep >= 0) {
            double Fp;
            const double y = newton_y(f, c_keep, zz_keep, zs_keep, dt, newton_iters, Fp, st);
            Y[(int64_t)p * M + j_keep] = y;
            rn2[(int64_t)p * M + j_keep] = n2_keep;
            if (dydc) dydc[(int64_t)p * M + j_keep] = 1.0 / Fp;
            if (zz_out) {   // XK == 3 with a tape: the particle's |Z|^2 and sum_i Z_i for the reverse mode
                zz_out[(int64_t)p * M + j_keep] = zz_keep;
                zs_out[(int64_t)p * M + j_keep] = zs_keep;
            }
        }
        j_keep = -1;
    };
    int cnt = 0;
    for (int jb = r0; jb < r1; jb += G::TPW) {
        const int j = jb + team;
        const bool valid = j < r1;
        CSum<R> n2s, dots, xbs, zsum;   // XK == 3: xbs sums |Z|^2, zsum sum_i Z_i
        double Pp = 1.0, Pq = 0.0;   // XK == 2: (P, Q2) of the lane's coordinates of X
        if (valid) {
            S* row = W + ((int64_t)p * M + j) * ldw;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int g = L + q * G::TL;
                const int e0 = 4 * g;
                if (e0 < ld) {
                    S v[4];
                    if (zero_state) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) v[e] = (S)0;
                    } else {
                        load4(row + e0, v);
                        if (e0 < d) {
                            S z[4];
                            increment4<S>((uint32_t)g, (uint32_t)j, (uint32_t)k, qs, k0, k1, z);
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                if (e0 + e < d) {
                                    if constexpr (XK == 3) {
                                        const double xb0 = (double)b[q][e];
                                        const double dW = sqdt * (double)z[e];
                                        const double X1 = xb0 * cf.Ab + cf.Bb + (double)v[e];
                                        const double X0 = (X1 - cf.mu1 * cf.dt - cf.s1 * dW) / (1.0 + cf.mu0 * cf.dt + cf.s0 * dW);
                                        v[e] = (S)(X0 - (xb0 * cf.Aa + cf.Ba));
                                        const double zi = (cf.s0 * X0 + cf.s1) * (double)a[q][e];
                                        xbs.add((R)(zi * zi));
                                        zsum.add((R)zi);
                                    } else {
                                        v[e] = (S)((double)v[e] - sqdt * (double)z[e]);
                                    }
                                }
                        }
                    }
                    store4(row + e0, v);
#pragma unroll
                    for (int e = 0; e < 4; ++e) { n2s.add(v[e] * v[e]); dots.add(a[q][e] * v[e]); }
                    if constexpr (XK == 1 || XK == 2) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) xbs.add(b[q][e] * v[e]);
                    }
                    if constexpr (XK == 2) {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (e0 + e < d) pq_add(Pp, Pq, (double)b[q][e] + s * (double)v[e]);
                    }
                }
            }
        }
        double n2 = n2s.get(), dt_ = dots.get();
        team_sum2<TEAM>(n2, dt_, red, team);
        double src = 0.0, zz_row = zz, zs_row = zs;
        if constexpr (XK == 3) {
            zz_row = xbs.get();
            zs_row = zsum.get();
            team_sum2<TEAM>(zz_row, zs_row, red, team);
            dt_ *= 1.0 + cf.mu0 * cf.dt;   // the drift-transported particle
        }
        if constexpr (XK == 1 || XK == 2) {
            double xb = xbs.get(), unused = 0.0;
            team_sum2<TEAM>(xb, unused, red, team);
            const double r2 = bb + 2.0 * s * xb + s * s * n2;
            if constexpr (XK == 1) src = dt * hj_source(tk, r2, (double)d, s, f.p0, nullptr);
            if constexpr (XK == 2) {
                team_pq<TEAM>(Pp, Pq, red, team);
                src = -dt * case2_source(tk, r2, Pp, Pq, (double)d, s, f.p0, f.p1, f.p2);
            }
        }
        if (valid && L == (cnt & 63)) {
            j_keep = j;
            c_keep = alpha + s * dt_ + src;
            n2_keep = n2;
            zz_keep = zz_row;
            zs_keep = zs_row;
        }
        if ((++cnt & 63) == 0) flush();
    }
    flush();
    if (st) atomicOr(&status[p], st);
}

// x-dependent coefficients: V[p][k] = E|X_k - m_k|^2 of point p's Euler-Maruyama particles, k = 0..N, from
// the moment recursion per coordinate, m_{k+1} = m_k + (mu0 m_k + mu1) dt (m_0 = x0) and
// v_{k+1} = v_k (1 + mu0 dt)^2 + dt (sigma0^2 (v_k + m_k^2) + 2 sigma0 sigma1 m_k + sigma1^2) (v_0 = 0).
// One block per point; m and v of the coordinates live in mbuf, vbuf [P][ld] between levels.
__global__ void __launch_bounds__(256)
k_coef_moments(const double* __restrict__ x0, int d, int ld, int N, CoefArgs cf, double* __restrict__ mbuf,
               double* __restrict__ vbuf, double* __restrict__ V) {
    __shared__ double lds[16];
    const int p = blockIdx.x;
    double* m = mbuf + (int64_t)p * ld;
    double* v = vbuf + (int64_t)p * ld;
    for (int i = threadIdx.x; i < d; i += blockDim.x) {
        m[i] = x0[(int64_t)p * d + i];
        v[i] = 0.0;
    }
    if (threadIdx.x == 0) V[(int64_t)p * (N + 1)] = 0.0;
    const double a = 1.0 + cf.mu0 * cf.dt;
    for (int k = 0; k < N; ++k) {
        double sv = 0.0;
        for (int i = threadIdx.x; i < d; i += blockDim.x) {
            const double mi = m[i], vi = v[i];
            const double vn = vi * a * a + cf.dt * (cf.s0 * cf.s0 * (vi + mi * mi) + 2.0 * cf.s0 * cf.s1 * mi + cf.s1 * cf.s1);
            v[i] = vn;
            m[i] = mi + (cf.mu0 * mi + cf.mu1) * cf.dt;
            sv += vn;
        }
        sv = block_sum(sv, lds);
        if (threadIdx.x == 0) V[(int64_t)p * (N + 1) + k + 1] = sv;
    }
}

// Level-0 outputs: u = Y^m_0 (every particle sits at x0, so C = alpha) and
// grad u = (alpha_x + dt grad_x f) / F'(u) (the x-derivative of the level-0 Newton equation).  x0: the
// points [P][d], read only when f depends on x: the source at t = 0 and x0 moves into C, and its
// x-gradient enters grad u.  HJ type: a function of |x0|^2 (gradient 2 x0 dS/d|x|^2).  Allen-Cahn Case 2:
// also of the coordinate products of x0; d_k of them needs the products of the coordinates other than k,
// formed per thread over a contiguous segment of coordinates with the other segments' products combined
// on either side (no division, so zero coordinates are exact).
__global__ void __launch_bounds__(256)
k_outputs(const double* __restrict__ x, int ld, int d, const double* __restrict__ scal, int ns, FSpec f,
          double dt, int newton_iters, double* __restrict__ u, double* __restrict__ grad,
          uint32_t* __restrict__ status, const double* __restrict__ x0 = nullptr, double s = 0.0,
          int coef_on = 0, CoefArgs cfo = CoefArgs{}) {
    const CoefArgs* coef = coef_on ? &cfo : nullptr;   // x-dependent coefficients
    __shared__ double lds[16];
    __shared__ double segP[256], segQ[256];
    const int p = blockIdx.x;
    const double* xp = x0 ? x0 + (int64_t)p * d : nullptr;
    uint32_t st = 0;
    double csrc = 0.0, dsrc = 0.0, r2 = 0.0, Pall = 1.0, Qall = 0.0;
    const int nt = blockDim.x, seg = (d + nt - 1) / nt;
    const int lo = min(d, (int)threadIdx.x * seg), hi = min(d, lo + seg);
    if (f.kind == F_HJ_SINK) {
        if (xp)
            for (int i = threadIdx.x; i < d; i += blockDim.x) r2 += xp[i] * xp[i];
        r2 = block_sum(r2, lds);
        csrc = hj_source(0.0, r2, (double)d, s, f.p0, &dsrc);
    } else if (f.kind == F_LOG_POT) {
        double P = 1.0, Q = 0.0;
        for (int i = lo; i < hi; ++i) {
            const double xi = xp ? xp[i] : 0.0;
            r2 += xi * xi;
            pq_add(P, Q, xi);
        }
        segP[threadIdx.x] = P;
        segQ[threadIdx.x] = Q;
        r2 = block_sum(r2, lds);   // its barrier also publishes the segments
        for (int t = 0; t < nt; ++t) pq_combine(Pall, Qall, segP[t], segQ[t]);
        csrc = -case2_source(0.0, r2, Pall, Qall, (double)d, s, f.p0, f.p1, f.p2);   // f = F(y) - S2
    }
    // x-dependent coefficients: Z_0 = (sigma0 x0 + sigma1) * alpha_x at x0, where every particle sits
    double zz0 = scal[(int64_t)p * ns + 6], zs0 = scal[(int64_t)p * ns + 8];
    if (coef) {
        double a = 0.0, b = 0.0;
        for (int i = threadIdx.x; i < d; i += blockDim.x) {
            const double zi = (coef->s0 * (xp ? xp[i] : 0.0) + coef->s1) * x[(int64_t)p * ld + i];
            a += zi * zi;
            b += zi;
        }
        zz0 = block_sum(a, lds);
        zs0 = block_sum(b, lds);
    }
    double Fp;
    const double y = newton_y(f, scal[(int64_t)p * ns + 5] + dt * csrc, zz0, zs0, dt, newton_iters, Fp, st);
    if (threadIdx.x == 0) u[p] = y;
    if (grad && coef) {
        // the x-derivative of y = alpha + (1 + mu0 dt) alpha_x . (x - x0) + dt f(0, x, y, Z(x)),
        // Z(x) = (sigma0 x + sigma1) * alpha_x: ((1 + mu0 dt) alpha_x + dt sigma0 alpha_x * d f / d z) / F'
        for (int i = threadIdx.x; i < d; i += blockDim.x) {
            const double ai = x[(int64_t)p * ld + i];
            const double zi = (coef->s0 * (xp ? xp[i] : 0.0) + coef->s1) * ai;
            const double fz = (f.kind == F_HJB) ? -2.0 * f.p0 * zi : (f.kind == F_BURGERS) ? f.p0 * (y - f.p1) : 0.0;
            const double gi = ((1.0 + coef->mu0 * coef->dt) * ai + dt * coef->s0 * ai * fz) / Fp;
            grad[(int64_t)p * d + i] = gi;
            if (!isfinite(gi)) st |= ST_NONFINITE;
        }
    } else if (grad) {
        if (f.kind == F_LOG_POT) {
            double EP = 1.0, EQ = 0.0, FP = 1.0, FQ = 0.0;   // segments before / after this thread's
            for (int t = 0; t < nt; ++t) {
                if (t < (int)threadIdx.x) pq_combine(EP, EQ, segP[t], segQ[t]);
                else if (t > (int)threadIdx.x) pq_combine(FP, FQ, segP[t], segQ[t]);
            }
            double preP = 1.0, preQ = 0.0;
            for (int k = lo; k < hi; ++k) {
                double sP = 1.0, sQ = 0.0;
                for (int j = k + 1; j < hi; ++j) pq_add(sP, sQ, xp ? xp[j] : 0.0);
                double lP = EP, lQ = EQ;
                pq_combine(lP, lQ, preP, preQ);
                pq_combine(lP, lQ, sP, sQ);
                pq_combine(lP, lQ, FP, FQ);
                const double xk = xp ? xp[k] : 0.0;
                const double gx = -case2_source_dk(0.0, r2, Pall, Qall, xk, lP, lQ, (double)d, s, f.p0, f.p1, f.p2);
                const double gi = (x[(int64_t)p * ld + k] + dt * gx) / Fp;
                grad[(int64_t)p * d + k] = gi;
                if (!isfinite(gi)) st |= ST_NONFINITE;
                pq_add(preP, preQ, xk);
            }
        } else {
            for (int i = threadIdx.x; i < d; i += blockDim.x) {
                const double gx = (f.kind == F_HJ_SINK && xp) ? 2.0 * dsrc * xp[i] : 0.0;
                const double gi = (x[(int64_t)p * ld + i] + dt * gx) / Fp;
                grad[(int64_t)p * d + i] = gi;
                if (!isfinite(gi)) st |= ST_NONFINITE;
            }
        }
    }
    if (st) atomicOr(&status[p], st);
}

__global__ void k_fill_u32(uint32_t* __restrict__ a, int64_t n, uint32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) a[i] = v;
}

// Row norms |W_j|^2 of a caller-provided state (used by the single-level entry point).
template <typename S, int Q, int TEAM>
__global__ void __launch_bounds__((Geo<Q, TEAM>::BS))
k_rownorm(const S* __restrict__ W, int64_t ldw, int M, int rows_per_chunk, int ld, double* __restrict__ rn2) {
    using G = Geo<Q, TEAM>;
    __shared__ double red[2 * G::BS / 64];
    const int p = blockIdx.y;
    const int team = threadIdx.x / G::TL, L = threadIdx.x % G::TL;
    const int r0 = blockIdx.x * rows_per_chunk;
    const int r1 = min(M, r0 + rows_per_chunk);
    for (int jb = r0; jb < r1; jb += G::TPW) {
        const int j = jb + team;
        const bool valid = j < r1;
        CSum<S> n2s;
        if (valid) {
            const S* row = W + ((int64_t)p * M + j) * ldw;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int e0 = 4 * (L + q * G::TL);
                if (e0 < ld) {
                    S v[4];
                    load4(row + e0, v);
#pragma unroll
                    for (int e = 0; e < 4; ++e) n2s.add(v[e] * v[e]);
                }
            }
        }
        double n2 = n2s.get(), z = 0.0;
        team_sum2<TEAM>(n2, z, red, team);
        if (valid && L == 0) rn2[(int64_t)p * M + j] = n2;
    }
}

// Diagnostic: normals (in the element type R of the precision mode, written as FP64) and raw Philox
// words of rows j0.. of one level.
template <typename R>
__global__ void k_normals(int d, int64_t j0, int64_t rows, int k, uint32_t q, uint32_t k0, uint32_t k1,
                          double* __restrict__ out, uint32_t* __restrict__ words) {
    const int ng = (d + 3) / 4;
    const int64_t n = rows * ng;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = t / ng;
        const int g = (int)(t % ng);
        const Words4 c = {(uint32_t)g, (uint32_t)(j0 + r), (uint32_t)k, q};
        const Words4 wd = philox4x32_10(c, k0, k1);
        R z[4];
        box_muller4<R>(wd, z);
        for (int e = 0; e < 4; ++e)
            if (4 * g + e < d) out[r * d + 4 * g + e] = (double)z[e];
        if (words) {
            uint32_t* wp = words + (r * ng + g) * 4;
            wp[0] = wd.x; wp[1] = wd.y; wp[2] = wd.z; wp[3] = wd.w;
        }
    }
}

}  // namespace fbsde
