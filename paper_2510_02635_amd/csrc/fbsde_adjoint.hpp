// Adjoint (reverse mode) of the backward level chain for L = sum_p ubar_p u(0, x0_p).
//
// The forward pass keeps, per level k, the kernel weights w^(k) and weighted mean Wbar^(k) of the
// cloud at t_{k+1}, the slope alpha_x^(k), the level scalars and Y_k.  The adjoint then walks
// k = 0 .. N-1 forward in time, regenerating the particles from their Philox counters
// (W_{k+1} = W_k + sqrt(dt) xi_k, W_0 = 0), and per level applies the transposes of
//   Newton (implicit-function rule: cbar = G / F'(Y_k)),
//   C^m = alpha + s alpha_x . W^m_k,   Z = s alpha_x,   alpha = Ybar - s alpha_x . Wbar,
//   alpha_x = A^{-1} b with A = sum_j w_j D'_j D'_j^T + lam I symmetric and independent of Y,
//   b = sum_j w_j (Y_j - Ybar) D'_j,   Ybar = sum_j w_j Y_j,
// giving G_{k+1, j} = w_j (D'_j . bbar + alphabar - sum_i w_i D'_i . bbar) with bbar = A^{-1} alpha_xbar
// (one extra CG solve per level).  The terminal step adds sum_j G_{N, j} grad g(X_N^j) to x0bar.
#pragma once
#include "fbsde_kernels.hpp"

namespace fbsde {


// Level k of the adjoint, per point: finish G_k from the previous level's row pass
// (G_j += w^(k-1)_j (alphabar_{k-1} - tau_{k-1})), then the Newton adjoint cbar_j = G_j / F'(Y^j_k),
// alphabar_k = sum cbar, the coefficient of Zbar (Zbar = zc Z) and the f-parameter sums.
// init (k = 0): G = ubar / M (u is the particle mean).  terminal: only finish G_N.
__global__ void __launch_bounds__(256)
k_adj_newton(double* __restrict__ G, const double* __restrict__ w_prev, int64_t w_stride, const double* __restrict__ psc,
             int nchunk,
             const double* __restrict__ Yk, const double* __restrict__ tscal_k, int ns, FSpec f, double dt,
             int newton_iters, int M, const double* __restrict__ u_bar, double* __restrict__ cbar,
             double* __restrict__ adj, int init, int terminal, uint32_t* __restrict__ status) {
    __shared__ double lds[16];
    const int p = blockIdx.x;
    double* a = adj + (int64_t)p * A_NS;
    double* Gp = G + (int64_t)p * M;
    if (init) {
        const double g0 = u_bar[p] / (double)M;
        for (int j = threadIdx.x; j < M; j += blockDim.x) Gp[j] = g0;
        __syncthreads();
        if (threadIdx.x == 0)
            for (int i = 0; i < A_NS; ++i) a[i] = 0.0;
    } else {
        double tau = 0.0;
        for (int c = 0; c < nchunk; ++c) tau += psc[((int64_t)p * nchunk + c) * 4];
        const double corr = a[A_ABAR] - tau;
        const double* wp = w_prev + (int64_t)p * w_stride;   // stride 0: weights shared by the points
        for (int j = threadIdx.x; j < M; j += blockDim.x) Gp[j] += wp[j] * corr;
    }
    __syncthreads();
    if (terminal) return;
    const double alpha = tscal_k[(int64_t)p * ns + 5];
    const double zz = tscal_k[(int64_t)p * ns + 6], zs = tscal_k[(int64_t)p * ns + 8];
    uint32_t st = 0;
    double y0 = 0.0, Fp0;
    if (!Yk) y0 = newton_y(f, alpha, zz, zs, dt, newton_iters, Fp0, st);
    double sc = 0.0, s0 = 0.0, s1 = 0.0, z1 = 0.0;
    for (int j = threadIdx.x; j < M; j += blockDim.x) {
        const double y = Yk ? Yk[(int64_t)p * M + j] : y0;
        double fv, fy;
        f_and_fy(f, y, zz, zs, fv, fy);
        const double Fp = 1.0 - dt * fy;
        if (fabs(Fp) < 1e-12) st |= ST_NEWTON_FLAT;
        const double cb = Gp[j] / Fp;
        cbar[(int64_t)p * M + j] = cb;
        sc += cb;
        if (f.kind == F_ALLEN_CAHN) { s0 += cb * y; s1 -= cb * y * y * y; }
        else if (f.kind == F_HJB) { s0 -= cb * zz; }
        else if (f.kind == F_BURGERS) { s0 += cb * (y - f.p1) * zs; s1 -= cb * f.p0 * zs; z1 += cb * (y - f.p1); }
    }
    sc = block_sum(sc, lds);
    s0 = block_sum(s0, lds);
    s1 = block_sum(s1, lds);
    z1 = block_sum(z1, lds);
    if (threadIdx.x == 0) {
        a[A_ABAR] = sc;
        a[A_ZC] = (f.kind == F_HJB) ? -2.0 * f.p0 * dt * sc : 0.0;
        a[A_Z1] = (f.kind == F_BURGERS) ? f.p0 * dt * z1 : 0.0;
        a[A_FP + 0] += dt * s0;
        a[A_FP + 1] += dt * s1;
        if (st) atomicOr(&status[p], st);
    }
}

// Column sums sum_m cbar_m W^m_k over the particles of a block, fused with the forward
// regeneration W_{k+1} = W_k + sqrt(dt) xi_k (in place).  zero_state: k = 0, W_0 = 0.
template <typename S, int Q, int TEAM>
__global__ void __launch_bounds__((Geo<Q, TEAM>::BS))
k_adj_advance(S* __restrict__ W, int64_t ldw, int M, int rows_per_chunk, int nchunk, int d, int ld, int k,
              int zero_state, double sqdt, const double* __restrict__ cbar, uint32_t k0, uint32_t k1,
              uint32_t point_base, double* __restrict__ part) {
    using G = Geo<Q, TEAM>;
    using R = S;
    __shared__ double lds[(G::TPW > 1) ? G::TPW * 4 * Q * G::TL : 1];
    const int p = blockIdx.y, c = blockIdx.x;
    const int team = threadIdx.x / G::TL, L = threadIdx.x % G::TL;
    const int r0 = c * rows_per_chunk;
    const int r1 = min(M, r0 + rows_per_chunk);
    const uint32_t qs = point_base + (uint32_t)p;
    CSum<R> acc[Q][4];
    for (int j = r0 + team; j < r1; j += G::TPW) {
        S* row = W + ((int64_t)p * M + j) * ldw;
        const R cb = cbar ? (R)cbar[(int64_t)p * M + j] : (R)0;
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
#pragma unroll
                    for (int e = 0; e < 4; ++e) acc[q][e].add(cb * v[e]);
                }
                if (e0 < d) {
                    S z[4];
                    increment4<S>((uint32_t)g, (uint32_t)j, (uint32_t)k, qs, k0, k1, z);
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (e0 + e < d) v[e] = (S)((double)v[e] + sqdt * (double)z[e]);
                }
                store4(row + e0, v);
            }
        }
    }
    if (part) block_columns_out<Q, TEAM, R>(acc, lds, part + ((int64_t)p * nchunk + c) * ld, ld, team, L);
}

// alpha_xbar = s sum_m cbar_m W^m_k + s Zbar - alphabar s Wbar, then CG on A bbar = alpha_xbar; Zbar =
// zc Z + z1 (1, ..., 1) over the d coordinates (the pad stays 0).
// Cold (warm = 0): from bbar = 0.  Warm: the right-hand side goes to r, the previous level's bbar (in x)
// becomes the direction v of one CG product (pv, Wbar . v in scal[2]) that k_adj_warm_start turns into
// the start gamma v.
__global__ void __launch_bounds__(256)
k_adj_rhs_finish(const double* __restrict__ part, int nchunk, int vchunks, int ld, int d, double s, double lam,
                 const double* __restrict__ Wbar, const double* __restrict__ ax, const double* __restrict__ adj,
                 double* __restrict__ x, double* __restrict__ r, double* __restrict__ pv, double* __restrict__ scal,
                 int ns, int* __restrict__ iscal, int* active, int warm) {
    __shared__ double lds[16];
    const int p = blockIdx.x;
    const double* a = adj + (int64_t)p * A_NS;
    const double abar = a[A_ABAR], zc = a[A_ZC], z1 = a[A_Z1];
    const int64_t o = (int64_t)p * ld;
    double bb = 0.0, wv = 0.0;
    for (int i = threadIdx.x; i < ld; i += blockDim.x) {
        double cs = 0.0;
        for (int c = 0; c < vchunks; ++c) cs += part[((int64_t)p * nchunk + c) * ld + i];
        const double b = s * cs + s * s * zc * ax[o + i] + ((i < d) ? s * z1 : 0.0) - abar * s * Wbar[o + i];
        r[o + i] = b;
        bb += b * b;
        if (warm) {
            const double v = x[o + i];
            pv[o + i] = v;
            wv += Wbar[o + i] * v;
        } else {
            x[o + i] = 0.0;
            pv[o + i] = b;
            wv += Wbar[o + i] * b;
        }
    }
    bb = block_sum(bb, lds);
    wv = block_sum(wv, lds);
    if (threadIdx.x == 0) {
        scal[(int64_t)p * ns + 0] = bb;
        scal[(int64_t)p * ns + 1] = bb;
        scal[(int64_t)p * ns + 2] = wv;
        scal[(int64_t)p * ns + 3] = lam;
        iscal[p * 4 + 0] = 0;
        const int done = (!warm && bb == 0.0) ? 1 : 0;
        iscal[p * 4 + 1] = done;
        if (done) atomicSub(active, 1);
    }
}

// Warm start of the adjoint CG from the previous level's solution v: with q = A v from one CG product
// (per-chunk partials, summed like k_cg_update), the start gamma v with gamma = (b . v) / (v . A v)
// minimises the A-norm error along v (never worse than starting from 0); then r = b - gamma q, p = r.
__global__ void __launch_bounds__(256)
k_adj_warm_start(const double* __restrict__ part, const double* __restrict__ psc, int nchunk, int vchunks, int ld,
                 double s, const double* __restrict__ Wbar, double* __restrict__ x, double* __restrict__ r,
                 double* __restrict__ pv, double* __restrict__ qv, double* __restrict__ scal, int ns,
                 int* __restrict__ iscal, int* active) {
    __shared__ double lds[16];
    const int p = blockIdx.x;
    double* sc = scal + (int64_t)p * ns;
    const double lam = sc[3];
    double tau = 0.0;
    for (int c = 0; c < nchunk; ++c) tau += psc[(int64_t)p * nchunk + c];
    const int64_t o = (int64_t)p * ld;
    double vq = 0.0, bv = 0.0;
    for (int i = threadIdx.x; i < ld; i += blockDim.x) {
        double a = 0.0;
        for (int c = 0; c < vchunks; ++c) a += part[((int64_t)p * nchunk + c) * ld + i];
        const double q = s * (a - tau * Wbar[o + i]) + lam * pv[o + i];
        qv[o + i] = q;
        vq += pv[o + i] * q;
        bv += r[o + i] * pv[o + i];
    }
    vq = block_sum(vq, lds);
    bv = block_sum(bv, lds);
    const double gamma = (vq > 0.0) ? bv / vq : 0.0;
    double rr = 0.0, wv = 0.0;
    for (int i = threadIdx.x; i < ld; i += blockDim.x) {
        x[o + i] = gamma * pv[o + i];
        const double ri = r[o + i] - gamma * qv[o + i];
        r[o + i] = ri;
        pv[o + i] = ri;
        rr += ri * ri;
        wv += Wbar[o + i] * ri;
    }
    rr = block_sum(rr, lds);
    wv = block_sum(wv, lds);
    if (threadIdx.x == 0) {
        sc[0] = rr;
        sc[2] = wv;
        iscal[p * 4 + 0] = 0;
        const int done = (rr == 0.0) ? 1 : 0;
        iscal[p * 4 + 1] = done;
        if (done) atomicSub(active, 1);
    }
}

__global__ void k_set_int(int* a, int v) { if (threadIdx.x == 0 && blockIdx.x == 0) *a = v; }

// Wbar . bbar per point.
__global__ void __launch_bounds__(256)
k_adj_bbar(const double* __restrict__ x, const double* __restrict__ Wbar, int ld, double* __restrict__ adj) {
    __shared__ double lds[16];
    const int p = blockIdx.x;
    double v = 0.0;
    for (int i = threadIdx.x; i < ld; i += blockDim.x) v += Wbar[(int64_t)p * ld + i] * x[(int64_t)p * ld + i];
    v = block_sum(v, lds);
    if (threadIdx.x == 0) adj[(int64_t)p * A_NS + A_WB] = v;
}

// Row pass on W_{k+1}: t_j = D'_j . bbar = s (W_j . bbar - Wbar . bbar); G_j = w_j t_j and, per block,
// tau = sum_j w_j t_j (the term that makes the mean-response adjoint exact).
template <typename S, int Q, int TEAM>
__global__ void __launch_bounds__((Geo<Q, TEAM>::BS))
k_adj_rowdot(const S* __restrict__ W, int64_t ldw, int M, int rows_per_chunk, int nchunk, int ld, double s,
             const double* __restrict__ w, const double* __restrict__ x, const double* __restrict__ adj,
             double* __restrict__ G, double* __restrict__ psc) {
    using Gm = Geo<Q, TEAM>;
    // FP64 arithmetic on the state: bbar carries the ridge-only null-space component of its
    // right-hand side scaled by 1/lam, which the centred product W_j.bbar - Wbar.bbar cancels; in
    // FP32 the cancellation would leave eps32 |W| |bbar| of noise in t_j
    using R = double;
    __shared__ double red[2 * Gm::BS / 64];
    const int p = blockIdx.y, c = blockIdx.x;
    const int team = threadIdx.x / Gm::TL, L = threadIdx.x % Gm::TL;
    const int r0 = c * rows_per_chunk;
    const int r1 = min(M, r0 + rows_per_chunk);
    R v[Q][4];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int e0 = 4 * (L + q * Gm::TL);
#pragma unroll
        for (int e = 0; e < 4; ++e) v[q][e] = (e0 < ld) ? (R)x[(int64_t)p * ld + e0 + e] : (R)0;
    }
    const double wb = adj[(int64_t)p * A_NS + A_WB];
    double tau = 0.0;
    for (int jb = r0; jb < r1; jb += Gm::TPW) {
        const int j = jb + team;
        const bool valid = j < r1;
        CSum<R> dl;
        if (valid) {
            const S* row = W + ((int64_t)p * M + j) * ldw;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int e0 = 4 * (L + q * Gm::TL);
                if (e0 < ld) {
                    S xv[4];
                    load4(row + e0, xv);
#pragma unroll
                    for (int e = 0; e < 4; ++e) dl.add((R)xv[e] * v[q][e]);
                }
            }
        }
        double t = dl.get(), unused = 0.0;
        team_sum2<TEAM>(t, unused, red, team);
        if (valid) {
            const double tj = s * (t - wb);
            const double gj = w[(int64_t)p * M + j] * tj;
            tau += gj;
            if (L == 0) G[(int64_t)p * M + j] = gj;
        }
    }
    const double contrib = (L == 0) ? tau : 0.0;
    const double tot = block_sum(contrib, red);
    if (threadIdx.x == 0) psc[((int64_t)p * nchunk + c) * 4] = tot;
}

// Terminal adjoint on W_N: for radial g = h(|X|^2), grad g(X) = 2 h'(|X|^2) X with X = xc + s W
// (xc = x0 + mu T): accumulate sum_j G_j 2h'_j W_j (columns) and, per block, sum_j G_j 2h'_j,
// sum_j G_j dg/dgp0, sum_j G_j dg/dgp1, sum_j G_j.  qpre: the argument of g per particle ([P][M], |X|^2 or
// gvec . X) formed by the caller (a constant diffusion matrix, X = xc + sigma W); the columns stay sums
// over W.
template <typename S, int Q, int TEAM>
__global__ void __launch_bounds__((Geo<Q, TEAM>::BS))
k_adj_terminal(const S* __restrict__ W, int64_t ldw, int M, int rows_per_chunk, int nchunk, int d, int ld,
               const double* __restrict__ x0, const double* __restrict__ mu, const double* __restrict__ gvec,
               double s, double T, int g_kind, double ga, const double* __restrict__ G, double* __restrict__ part,
               double* __restrict__ psc, const double* __restrict__ qpre = nullptr) {
    using Gm = Geo<Q, TEAM>;
    using R = S;
    __shared__ double lds[(Gm::TPW > 1) ? Gm::TPW * 4 * Q * Gm::TL : 1];
    __shared__ double red[2 * Gm::BS / 64];
    const int p = blockIdx.y, c = blockIdx.x;
    const int team = threadIdx.x / Gm::TL, L = threadIdx.x % Gm::TL;
    const int r0 = c * rows_per_chunk;
    const int r1 = min(M, r0 + rows_per_chunk);
    double xc[Q][4];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int i = 4 * (L + q * Gm::TL) + e;
            xc[q][e] = (i < d) ? x0[(int64_t)p * d + i] + (mu ? mu[i] * T : 0.0) : 0.0;
        }
    CSum<R> acc[Q][4];
    double s1 = 0.0, g0 = 0.0, g1 = 0.0, sg = 0.0;
    for (int jb = r0; jb < r1; jb += Gm::TPW) {
        const int j = jb + team;
        const bool valid = j < r1;
        S xv[Q][4];
        double qsum = 0.0;
        if (valid) {
            const S* row = W + ((int64_t)p * M + j) * ldw;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int e0 = 4 * (L + q * Gm::TL);
                if (e0 < ld) load4(row + e0, xv[q]);
                else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) xv[q][e] = (S)0;
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const double X = xc[q][e] + s * (double)xv[q][e];
                    if (g_dot_arg(g_kind)) qsum += ((e0 + e < d) ? gvec[e0 + e] : 0.0) * X;
                    else qsum += X * X;
                }
            }
        }
        double unused = 0.0;
        team_sum2<TEAM>(qsum, unused, red, team);
        if (qpre && valid) qsum = qpre[(int64_t)p * M + j];
        if (valid) {
            const double gj = G[(int64_t)p * M + j];
            double hp = 0.0, d0 = 0.0, d1 = 0.0;
            if (g_kind == G_QUAD) { hp = ga / (double)d; d0 = qsum / (double)d; d1 = 1.0; }
            else if (g_kind == G_AC) { const double den = 2.0 + ga * qsum; hp = -ga / (den * den); d0 = -qsum / (den * den); }
            else if (g_kind == G_HJB_LOG) { const double den = 1.0 + ga * qsum; hp = ga / den; d0 = qsum / den; }
            else if (g_kind == G_LOGISTIC) { const double gv = 1.0 / (1.0 + exp(-(qsum + ga))); d0 = gv * (1.0 - gv); }
            else if (g_kind == G_HJ_GAUSS) {   // g = (1 + 4a)^(-d/2) e^(-q / (1 + 4a))
                const double a4 = 1.0 + 4.0 * ga, gv = g_of(G_HJ_GAUSS, ga, 0.0, qsum, d);
                hp = -gv / a4;
                d0 = gv * (-2.0 * (double)d / a4 + 4.0 * qsum / (a4 * a4));
            }
            else { d0 = 1.0; }
            const double phi = 2.0 * hp * gj;
            s1 += phi; g0 += gj * d0; g1 += gj * d1; sg += gj;
            const R cr = (R)phi;
#pragma unroll
            for (int q = 0; q < Q; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[q][e].add(cr * xv[q][e]);
        }
    }
    block_columns_out<Q, TEAM, R>(acc, lds, part + ((int64_t)p * nchunk + c) * ld, ld, team, L);
    const bool lead = (L == 0);
    const double t1 = block_sum(lead ? s1 : 0.0, red);
    const double t2 = block_sum(lead ? g0 : 0.0, red);
    const double t3 = block_sum(lead ? g1 : 0.0, red);
    const double t4 = block_sum(lead ? sg : 0.0, red);
    if (threadIdx.x == 0) {
        double* o = psc + ((int64_t)p * nchunk + c) * 4;
        o[0] = t1; o[1] = t2; o[2] = t3; o[3] = t4;
    }
}

// x0bar = (sum_j G_j 2h'_j) xc + s sum_j G_j 2h'_j W_j   (affine: (sum_j G_j) gvec; logistic:
// (sum_j G_j g'_j) gvec, which is the gp0 sum); per-point gp sums.
__global__ void __launch_bounds__(256)
k_adj_x0bar(const double* __restrict__ part, const double* __restrict__ psc, int nchunk, int vchunks, int d, int ld,
            const double* __restrict__ x0, const double* __restrict__ mu, const double* __restrict__ gvec,
            double s, double T, int g_kind, double* __restrict__ adj, double* __restrict__ x0_bar) {
    const int p = blockIdx.x;
    double S1 = 0.0, G0 = 0.0, G1 = 0.0, SG = 0.0;
    for (int c = 0; c < nchunk; ++c) {
        const double* o = psc + ((int64_t)p * nchunk + c) * 4;
        S1 += o[0]; G0 += o[1]; G1 += o[2]; SG += o[3];
    }
    for (int i = threadIdx.x; i < d; i += blockDim.x) {
        double v;
        if (g_kind == G_AFFINE) v = SG * gvec[i];
        else if (g_kind == G_LOGISTIC) v = G0 * gvec[i];
        else {
            double cs = 0.0;
            for (int c = 0; c < vchunks; ++c) cs += part[((int64_t)p * nchunk + c) * ld + i];
            const double xc = x0[(int64_t)p * d + i] + (mu ? mu[i] * T : 0.0);
            v = S1 * xc + s * cs;
        }
        x0_bar[(int64_t)p * d + i] = v;
    }
    if (threadIdx.x == 0) {
        double* a = adj + (int64_t)p * A_NS;
        a[A_GP + 0] = G0;
        a[A_GP + 1] = G1;
    }
}

// Parameter gradients summed over points in a fixed order.
__global__ void k_adj_params(const double* __restrict__ adj, int64_t P, double* __restrict__ gp_bar,
                             double* __restrict__ fp_bar) {
    const int t = threadIdx.x;
    if (t >= 8) return;
    const int slot = (t < 4) ? A_GP + t : A_FP + (t - 4);
    double v = 0.0;
    for (int64_t p = 0; p < P; ++p) v += adj[p * A_NS + slot];
    if (t < 4) gp_bar[t] = v;
    else fp_bar[t - 4] = v;
}

}  // namespace fbsde
