// Reverse mode of the per-point scheme under the affine diagonal coefficients mu(x) = mu0 x + mu1,
// sigma(x) = diag(sigma0 x + sigma1) (the problem class of Sec. 2.1 with eq. Xk's Euler-Maruyama particles),
// for L = sum_p ubar_p u(0, x0_p).
//
// With constant coefficients the regression design does not depend on x0; here it does, through three
// routes: the particles (coordinate-wise affine in x0, slope J_k = prod (1 + mu0 dt + sigma0 dW), the
// tangent state kept beside the displacement state D = X - m), the mean path m_k (slope A_k = (1 + mu0 dt)^k)
// and the cloud variance V_k of the moment recursion (bandwidth h^2 V and ridge ridge_rel V / d).  Per level
// k, walked k = 0 .. N-1 forward in time on the regenerated state (a = 1 + mu0 dt, level k's slope alpha_x,
// CG solution mu of the level's adjoint system, w the kernel weights of the cloud at t_{k+1}):
//   k_cadj_newton:  cbar_j = G_j / F'_j, alphabar = sum cbar, f's parameter sums, and the particle's
//                   weight of Zbar_j (HJB: Zbar_j = zw_j Z_j; Burgers: Zbar_j = zw_j (1, .., 1)).
//   k_cadj_advance: one row pass over (D_k, J_k): the columns of alpha_xbar = a sum cbar_j D_j +
//                   sum Zbar_j (sigma0 X_j + sigma1) and of the x0 adjoint of the level's positions,
//                   sum_j (J_j - A_k) Dbar_j + J_j sigma0 Zbar_j alpha_x (Dbar_j: Ebar_j = a cbar_j alpha_x plus
//                   the design adjoint of level k - 1), then the Euler-Maruyama step of D and J.
//   k_cadj_rhs:     alpha_xbar - alphabar Dbar as the right-hand side of the adjoint CG (cold start, the
//                   point's own ridge), and the position columns into the x0 accumulator.
//   k_cadj_rowdot:  one row pass over D_{k+1}: mu . D_j, alpha_x . D_j and |D_j|^2.
//   k_cadj_design:  per point, G_{k+1, j} = w_j (mu . D'_j + alphabar) and the design adjoint
//                   Dbar_j = c1_j mu + c2_j alpha_x + c3_j D_j, with c3 from the kernel weights' softmax, and
//                   the variance adjoint Vbar_{k+1} (weights and ridge).
// Then k_cadj_terminal adds the terminal value's gradient (J_j G_j grad g(X_j)) and the last design
// adjoint, and k_cadj_x0bar sums everything with sum_k Vbar_k dV_k/dx0 (the moment recursion's tangent).
#pragma once
#include "fbsde_adjoint.hpp"

namespace fbsde {

// Newton's adjoint at level k.  Yk == nullptr: level 0, where every particle sits at x0 with
// Z_0 = (sigma0 x0 + sigma1) * alpha_x, and y, F' come from one Newton solve per point; otherwise Y_k,
// 1 / F' and the particle's |Z|^2, sum Z from the tape.  init: G = ubar / M and the adjoint slots zeroed.
__global__ void __launch_bounds__(256)
k_cadj_newton(double* __restrict__ G, const double* __restrict__ Yk, const double* __restrict__ dydc,
              const double* __restrict__ zzp, const double* __restrict__ zsp, const double* __restrict__ tscal_k,
              int ns, const double* __restrict__ x0, const double* __restrict__ ax, int d, int ld, CoefArgs cf,
              FSpec f, double dt, int newton_iters, int M, const double* __restrict__ u_bar,
              double* __restrict__ cbar, double* __restrict__ zw, double* __restrict__ adj, int init,
              uint32_t* __restrict__ status) {
    __shared__ double lds[16];
    const int p = blockIdx.x, t = threadIdx.x;
    double* a = adj + (int64_t)p * A_NS;
    double* Gp = G + (int64_t)p * M;
    if (init) {
        const double g0 = u_bar[p] / (double)M;
        for (int j = t; j < M; j += blockDim.x) Gp[j] = g0;
        if (t == 0)
            for (int i = 0; i < A_NS; ++i) a[i] = 0.0;
    }
    __syncthreads();
    uint32_t st = 0;
    double y0 = 0.0, Fp0 = 1.0, zz0 = 0.0, zs0 = 0.0;
    if (!Yk) {
        double s1 = 0.0, s2 = 0.0;
        for (int i = t; i < d; i += blockDim.x) {
            const double zi = (cf.s0 * x0[(int64_t)p * d + i] + cf.s1) * ax[(int64_t)p * ld + i];
            s1 += zi * zi;
            s2 += zi;
        }
        zz0 = block_sum(s1, lds);
        zs0 = block_sum(s2, lds);
        y0 = newton_y(f, tscal_k[(int64_t)p * ns + 5], zz0, zs0, dt, newton_iters, Fp0, st);
    }
    double sc = 0.0, s0 = 0.0, s1 = 0.0;
    for (int j = t; j < M; j += blockDim.x) {
        const int64_t o = (int64_t)p * M + j;
        const double y = Yk ? Yk[o] : y0;
        const double zz = Yk ? zzp[o] : zz0, zs = Yk ? zsp[o] : zs0;
        const double cb = Gp[j] * (Yk ? dydc[o] : 1.0 / Fp0);
        double z = 0.0;
        if (f.kind == F_ALLEN_CAHN) { s0 += cb * y; s1 -= cb * y * y * y; }
        else if (f.kind == F_HJB) { z = -2.0 * f.p0 * dt * cb; s0 -= cb * zz; }
        else if (f.kind == F_BURGERS) {
            z = dt * f.p0 * cb * (y - f.p1);
            s0 += cb * (y - f.p1) * zs;
            s1 -= cb * f.p0 * zs;
        }
        cbar[o] = cb;
        zw[o] = z;
        sc += cb;
    }
    sc = block_sum(sc, lds);
    s0 = block_sum(s0, lds);
    s1 = block_sum(s1, lds);
    if (t == 0) {
        a[A_ABAR] = sc;
        a[A_FP + 0] += dt * s0;
        a[A_FP + 1] += dt * s1;
        if (st) atomicOr(&status[p], st);
    }
}

// One row pass over the displacement D_k and the tangent J_k of level k (cf.Aa, cf.Ba: A_k, B_k; the
// mean path m_k = x0 A_k + B_k), then D_{k+1} = a D_k + (sigma0 X_k + sigma1) dW_k, J_{k+1} =
// (a + sigma0 dW_k) J_k in place.  zero_state: level 0 (D_0 = 0, J_0 = 1; no design adjoint yet).
// part_ax: the columns of alpha_xbar; part_x0: the columns of the x0 adjoint of the level's positions.
// c1, c2, c3, mup, axp: the design adjoint of the previous level (on this state).
template <typename S, int Q, int TEAM>
__global__ void __launch_bounds__((Geo<Q, TEAM>::BS))
k_cadj_advance(S* __restrict__ W, S* __restrict__ J, int64_t ldw, int M, int rows_per_chunk, int nchunk, int d,
               int ld, int k, int zero_state, double sqdt, CoefArgs cf, int fkind, const double* __restrict__ x0,
               const double* __restrict__ ax, const double* __restrict__ axp, const double* __restrict__ mup,
               const double* __restrict__ cbar, const double* __restrict__ zw, const double* __restrict__ c1,
               const double* __restrict__ c2, const double* __restrict__ c3, uint32_t k0, uint32_t k1,
               uint32_t point_base, double* __restrict__ part_ax, double* __restrict__ part_x0) {
    using Gm = Geo<Q, TEAM>;
    // FP64 vectors and sums on either state: mu carries the ridge-only null-space component of its
    // right-hand side scaled by 1 / lam, which the sums over the cloud largely cancel
    using R = double;
    __shared__ double lds[(Gm::TPW > 1) ? Gm::TPW * 4 * Q * Gm::TL : 1];
    const int p = blockIdx.y, c = blockIdx.x;
    const int team = threadIdx.x / Gm::TL, L = threadIdx.x % Gm::TL;
    const int r0 = c * rows_per_chunk;
    const int r1 = min(M, r0 + rows_per_chunk);
    const uint32_t qs = point_base + (uint32_t)p;
    const double a = 1.0 + cf.mu0 * cf.dt, Ak = cf.Aa;
    R mk[Q][4], al[Q][4], alp[Q][4], mu[Q][4];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int i = 4 * (L + q * Gm::TL) + e;
            const bool in = i < d;
            mk[q][e] = in ? (R)(x0[(int64_t)p * d + i] * cf.Aa + cf.Ba) : (R)0;
            al[q][e] = in ? (R)ax[(int64_t)p * ld + i] : (R)0;
            alp[q][e] = (in && !zero_state) ? (R)axp[(int64_t)p * ld + i] : (R)0;
            mu[q][e] = (in && !zero_state) ? (R)mup[(int64_t)p * ld + i] : (R)0;
        }
    CSum<R> acc_a[Q][4], acc_x[Q][4];
    for (int j = r0 + team; j < r1; j += Gm::TPW) {
        const int64_t o = (int64_t)p * M + j;
        const double cb = cbar[o], zwj = zw[o];
        const double e1 = zero_state ? 0.0 : c1[o], e2 = zero_state ? 0.0 : c2[o], e3 = zero_state ? 0.0 : c3[o];
        S* row = W + o * ldw;
        S* jrow = J + o * ldw;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int g = L + q * Gm::TL;
            const int e0 = 4 * g;
            if (e0 < ld) {
                S v[4], jv[4];
                if (zero_state) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) { v[e] = (S)0; jv[e] = (S)1; }
                } else {
                    load4(row + e0, v);
                    load4(jrow + e0, jv);
                }
                if (e0 < d) {
                    S z[4];
                    increment4<S>((uint32_t)g, (uint32_t)j, (uint32_t)k, qs, k0, k1, z);
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        if (e0 + e < d) {
                            const double Dd = (double)v[e], Jv = (double)jv[e], alv = (double)al[q][e];
                            const double X = Dd + (double)mk[q][e];
                            const double sx = cf.s0 * X + cf.s1;
                            const double Zb = (fkind == F_HJB) ? zwj * sx * alv : (fkind == F_BURGERS) ? zwj : 0.0;
                            const double Dbar = a * cb * alv + e1 * (double)mu[q][e] + e2 * (double)alp[q][e] + e3 * Dd;
                            acc_x[q][e].add((R)((Jv - Ak) * Dbar + Jv * cf.s0 * Zb * alv));
                            acc_a[q][e].add((R)(a * cb * Dd + Zb * sx));
                            const double dW = sqdt * (double)z[e];
                            v[e] = (S)(a * Dd + sx * dW);
                            jv[e] = (S)((a + cf.s0 * dW) * Jv);
                        } else {
                            v[e] = (S)0;
                            jv[e] = (S)0;
                        }
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) { v[e] = (S)0; jv[e] = (S)0; }
                }
                store4(row + e0, v);
                store4(jrow + e0, jv);
            }
        }
    }
    block_columns_out<Q, TEAM, R>(acc_a, lds, part_ax + ((int64_t)p * nchunk + c) * ld, ld, team, L);
    block_columns_out<Q, TEAM, R>(acc_x, lds, part_x0 + ((int64_t)p * nchunk + c) * ld, ld, team, L);
}

// The adjoint CG's right-hand side alpha_xbar - alphabar Dbar (cold start: x = 0), the point's ridge
// ridge_rel V_{k+1} / d, and the level's position columns added to the x0 accumulator (first: set).
__global__ void __launch_bounds__(256)
k_cadj_rhs(const double* __restrict__ part_ax, const double* __restrict__ part_x0, int nchunk, int vchunks, int ld,
           const double* __restrict__ Dbar, const double* __restrict__ adj, const double* __restrict__ Vt, int vstride,
           double rho_d, double* __restrict__ x, double* __restrict__ r, double* __restrict__ pv,
           double* __restrict__ scal, int ns, int* __restrict__ iscal, int* active, double* __restrict__ x0acc,
           int first) {
    __shared__ double lds[16];
    const int p = blockIdx.x;
    const double abar = adj[(int64_t)p * A_NS + A_ABAR];
    const int64_t o = (int64_t)p * ld;
    double bb = 0.0, wv = 0.0;
    for (int i = threadIdx.x; i < ld; i += blockDim.x) {
        double ca = 0.0, cx = 0.0;
        for (int c = 0; c < vchunks; ++c) {
            ca += part_ax[((int64_t)p * nchunk + c) * ld + i];
            cx += part_x0[((int64_t)p * nchunk + c) * ld + i];
        }
        const double b = ca - abar * Dbar[o + i];
        r[o + i] = b;
        x[o + i] = 0.0;
        pv[o + i] = b;
        bb += b * b;
        wv += Dbar[o + i] * b;
        x0acc[o + i] = first ? cx : x0acc[o + i] + cx;
    }
    bb = block_sum(bb, lds);
    wv = block_sum(wv, lds);
    if (threadIdx.x == 0) {
        double* sc = scal + (int64_t)p * ns;
        sc[0] = bb;
        sc[1] = bb;
        sc[2] = wv;
        sc[3] = rho_d * Vt[(int64_t)p * vstride];
        iscal[p * 4 + 0] = 0;
        const int done = (bb == 0.0) ? 1 : 0;
        iscal[p * 4 + 1] = done;
        if (done) atomicSub(active, 1);
    }
}

// Row pass over D_{k+1}: mu . D_j, alpha_x . D_j, |D_j|^2 per particle (FP64 arithmetic on the state).
template <typename S, int Q, int TEAM>
__global__ void __launch_bounds__((Geo<Q, TEAM>::BS))
k_cadj_rowdot(const S* __restrict__ W, int64_t ldw, int M, int rows_per_chunk, int ld, const double* __restrict__ mu,
              const double* __restrict__ ax, double* __restrict__ pd, double* __restrict__ qd,
              double* __restrict__ n2) {
    using Gm = Geo<Q, TEAM>;
    __shared__ double red[2 * Gm::BS / 64];
    const int p = blockIdx.y, c = blockIdx.x;
    const int team = threadIdx.x / Gm::TL, L = threadIdx.x % Gm::TL;
    const int r0 = c * rows_per_chunk;
    const int r1 = min(M, r0 + rows_per_chunk);
    double mv[Q][4], av[Q][4];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int e0 = 4 * (L + q * Gm::TL);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            mv[q][e] = (e0 < ld) ? mu[(int64_t)p * ld + e0 + e] : 0.0;
            av[q][e] = (e0 < ld) ? ax[(int64_t)p * ld + e0 + e] : 0.0;
        }
    }
    for (int jb = r0; jb < r1; jb += Gm::TPW) {
        const int j = jb + team;
        const bool valid = j < r1;
        double sm = 0.0, sa = 0.0, sn = 0.0;
        if (valid) {
            const S* row = W + ((int64_t)p * M + j) * ldw;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int e0 = 4 * (L + q * Gm::TL);
                if (e0 < ld) {
                    S xv[4];
                    load4(row + e0, xv);
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const double v = (double)xv[e];
                        sm += v * mv[q][e];
                        sa += v * av[q][e];
                        sn += v * v;
                    }
                }
            }
        }
        team_sum2<TEAM>(sm, sa, red, team);
        double unused = 0.0;
        team_sum2<TEAM>(sn, unused, red, team);
        if (valid && L == 0) {
            const int64_t o = (int64_t)p * M + j;
            pd[o] = sm;
            qd[o] = sa;
            n2[o] = sn;
        }
    }
}

// Level k's regression adjoint per point (one block): the adjoint of Y_{k+1} and the design adjoint
// Dbar_j = c1_j mu + c2_j alpha_x + c3_j D_j of the cloud at t_{k+1}, with
//   p_j = mu . D'_j, q_j = alpha_x . D'_j, r_j = Y_j - Ybar (D' = D - Dbar centred by the weights),
//   G_j = w_j (p_j + alphabar),  c1_j = w_j (r_j - q_j),  c2_j = -w_j (p_j + alphabar),
//   wbar_j = p_j (r_j - q_j) + alphabar (Y_j - alpha_x . D_j),  lbar_j = w_j (wbar_j - sum_i w_i wbar_i),
//   c3_j = -2 lbar_j / (h^2 V),  Vbar_{k+1} = sum_j lbar_j |D_j|^2 / (h^2 V^2) - (mu . alpha_x) rho_d.
// h2 = 0: uniform weights (no weight or bandwidth term).
__global__ void __launch_bounds__(256)
k_cadj_design(const double* __restrict__ pd, const double* __restrict__ qd, const double* __restrict__ n2,
              const double* __restrict__ w, const double* __restrict__ Y, const double* __restrict__ tscal_k, int ns,
              const double* __restrict__ mu, const double* __restrict__ ax, const double* __restrict__ Dbar, int ld,
              const double* __restrict__ adj, const double* __restrict__ Vt, double* __restrict__ Vbar, int vstride,
              double h2, double rho_d, int M, double* __restrict__ G, double* __restrict__ c1,
              double* __restrict__ c2, double* __restrict__ c3) {
    __shared__ double lds[16];
    const int p = blockIdx.x, t = threadIdx.x;
    const int64_t o = (int64_t)p * ld;
    double md = 0.0, ad = 0.0, ma = 0.0;
    for (int i = t; i < ld; i += blockDim.x) {
        md += mu[o + i] * Dbar[o + i];
        ad += ax[o + i] * Dbar[o + i];
        ma += mu[o + i] * ax[o + i];
    }
    md = block_sum(md, lds);
    ad = block_sum(ad, lds);
    ma = block_sum(ma, lds);
    const double yb = tscal_k[(int64_t)p * ns + 4];
    const double abar = adj[(int64_t)p * A_NS + A_ABAR];
    const double V = Vt[(int64_t)p * vstride];
    double sw = 0.0;
    for (int j = t; j < M; j += blockDim.x) {
        const int64_t q = (int64_t)p * M + j;
        const double pj = pd[q] - md, qj = qd[q] - ad, y = Y[q];
        const double wb = pj * (y - yb - qj) + abar * (y - qd[q]);
        c3[q] = wb;   // held until the weighted mean of wbar is known
        sw += w[q] * wb;
    }
    sw = block_sum(sw, lds);
    double vs = 0.0;
    for (int j = t; j < M; j += blockDim.x) {
        const int64_t q = (int64_t)p * M + j;
        const double wj = w[q], pj = pd[q] - md, qj = qd[q] - ad;
        const double lb = (h2 > 0.0) ? wj * (c3[q] - sw) : 0.0;
        G[q] = wj * (pj + abar);
        c1[q] = wj * (Y[q] - yb - qj);
        c2[q] = -wj * (pj + abar);
        c3[q] = (h2 > 0.0) ? -2.0 * lb / (h2 * V) : 0.0;
        vs += lb * n2[q];
    }
    vs = block_sum(vs, lds);
    if (t == 0) Vbar[(int64_t)p * vstride] = ((h2 > 0.0) ? vs / (h2 * V * V) : 0.0) - ma * rho_d;
}

// Terminal adjoint on (D_N, J_N) (cf.Aa, cf.Ba: A_N, B_N): X_j = D_j + m_N, G_j the adjoint of Y_N.  Columns
// sum_j J_j G_j grad g(X_j) + (J_j - A_N) Dbar_j (the last level's design adjoint); per block the gp sums
// (psc[1], psc[2]) as k_adj_terminal.
template <typename S, int Q, int TEAM>
__global__ void __launch_bounds__((Geo<Q, TEAM>::BS))
k_cadj_terminal(const S* __restrict__ W, const S* __restrict__ J, int64_t ldw, int M, int rows_per_chunk, int nchunk,
                int d, int ld, const double* __restrict__ x0, const double* __restrict__ gvec, CoefArgs cf,
                int g_kind, double ga, const double* __restrict__ G, const double* __restrict__ mup,
                const double* __restrict__ axp, const double* __restrict__ c1, const double* __restrict__ c2,
                const double* __restrict__ c3, double* __restrict__ part, double* __restrict__ psc) {
    using Gm = Geo<Q, TEAM>;
    using R = double;   // as k_cadj_advance
    __shared__ double lds[(Gm::TPW > 1) ? Gm::TPW * 4 * Q * Gm::TL : 1];
    __shared__ double red[2 * Gm::BS / 64];
    const int p = blockIdx.y, c = blockIdx.x;
    const int team = threadIdx.x / Gm::TL, L = threadIdx.x % Gm::TL;
    const int r0 = c * rows_per_chunk;
    const int r1 = min(M, r0 + rows_per_chunk);
    const double AN = cf.Aa;
    const bool dot = g_dot_arg(g_kind);
    R mk[Q][4], mu[Q][4], al[Q][4], gv[Q][4];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int i = 4 * (L + q * Gm::TL) + e;
            const bool in = i < d;
            mk[q][e] = in ? (R)(x0[(int64_t)p * d + i] * cf.Aa + cf.Ba) : (R)0;
            mu[q][e] = in ? (R)mup[(int64_t)p * ld + i] : (R)0;
            al[q][e] = in ? (R)axp[(int64_t)p * ld + i] : (R)0;
            gv[q][e] = (in && dot) ? (R)gvec[i] : (R)0;
        }
    CSum<R> acc[Q][4];
    double g0 = 0.0, g1 = 0.0;
    for (int jb = r0; jb < r1; jb += Gm::TPW) {
        const int j = jb + team;
        const bool valid = j < r1;
        S xv[Q][4], jv[Q][4];
        double qsum = 0.0;
        if (valid) {
            const S* row = W + ((int64_t)p * M + j) * ldw;
            const S* jrow = J + ((int64_t)p * M + j) * ldw;
            load_row<S, Q, Gm::TL>(row, ld, L, xv);
            load_row<S, Q, Gm::TL>(jrow, ld, L, jv);
#pragma unroll
            for (int q = 0; q < Q; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const double X = (double)xv[q][e] + (double)mk[q][e];
                    qsum += dot ? (double)gv[q][e] * X : X * X;
                }
        }
        double unused = 0.0;
        team_sum2<TEAM>(qsum, unused, red, team);
        if (valid) {
            const int64_t o = (int64_t)p * M + j;
            const double gj = G[o];
            double hp = 0.0, d0 = 0.0, d1 = 0.0, gd = 0.0;
            if (g_kind == G_QUAD) { hp = ga / (double)d; d0 = qsum / (double)d; d1 = 1.0; }
            else if (g_kind == G_AC) { const double den = 2.0 + ga * qsum; hp = -ga / (den * den); d0 = -qsum / (den * den); }
            else if (g_kind == G_HJB_LOG) { const double den = 1.0 + ga * qsum; hp = ga / den; d0 = qsum / den; }
            else if (g_kind == G_LOGISTIC) { const double g = 1.0 / (1.0 + exp(-(qsum + ga))); d0 = g * (1.0 - g); gd = d0; }
            else if (g_kind == G_HJ_GAUSS) {
                const double a4 = 1.0 + 4.0 * ga, g = g_of(G_HJ_GAUSS, ga, 0.0, qsum, d);
                hp = -g / a4;
                d0 = g * (-2.0 * (double)d / a4 + 4.0 * qsum / (a4 * a4));
            }
            else { d0 = 1.0; gd = 1.0; }   // affine
            g0 += gj * d0;
            g1 += gj * d1;
            const double phi = 2.0 * hp * gj, psi = gd * gj;
            const double e1 = c1[o], e2 = c2[o], e3 = c3[o];
#pragma unroll
            for (int q = 0; q < Q; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const double Dd = (double)xv[q][e], Jv = (double)jv[q][e];
                    const double X = Dd + (double)mk[q][e];
                    const double gx = phi * X + psi * (double)gv[q][e];
                    const double Db = e1 * (double)mu[q][e] + e2 * (double)al[q][e] + e3 * Dd;
                    acc[q][e].add((R)(Jv * gx + (Jv - AN) * Db));
                }
        }
    }
    block_columns_out<Q, TEAM, R>(acc, lds, part + ((int64_t)p * nchunk + c) * ld, ld, team, L);
    const bool lead = (L == 0);
    const double t2 = block_sum(lead ? g0 : 0.0, red);
    const double t3 = block_sum(lead ? g1 : 0.0, red);
    if (threadIdx.x == 0) {
        double* o = psc + ((int64_t)p * nchunk + c) * 4;
        o[0] = 0.0; o[1] = t2; o[2] = t3; o[3] = 0.0;
    }
}

// x0bar = the position accumulator + the terminal columns + sum_{k=1..N} Vbar_k dV_k/dx0, with the moment
// recursion's tangent per coordinate: dv_{k+1} = dv_k (a^2 + dt sigma0^2) + dt (2 sigma0^2 m_k + 2 sigma0 sigma1) A_k;
// the gp sums into the adjoint slots.
__global__ void __launch_bounds__(256)
k_cadj_x0bar(const double* __restrict__ part, const double* __restrict__ psc, int nchunk, int vchunks, int d, int ld,
             const double* __restrict__ x0acc, const double* __restrict__ x0, CoefArgs cf, int N,
             const double* __restrict__ Vbar, int vstride, double* __restrict__ adj, double* __restrict__ x0_bar) {
    const int p = blockIdx.x;
    const double a = 1.0 + cf.mu0 * cf.dt;
    const double* vb = Vbar + (int64_t)p * vstride;
    for (int i = threadIdx.x; i < d; i += blockDim.x) {
        double v = x0acc[(int64_t)p * ld + i];
        for (int c = 0; c < vchunks; ++c) v += part[((int64_t)p * nchunk + c) * ld + i];
        double m = x0[(int64_t)p * d + i], A = 1.0, dv = 0.0;
        for (int k = 0; k < N; ++k) {
            dv = dv * (a * a + cf.dt * cf.s0 * cf.s0) + cf.dt * (2.0 * cf.s0 * cf.s0 * m + 2.0 * cf.s0 * cf.s1) * A;
            m = m + (cf.mu0 * m + cf.mu1) * cf.dt;
            A *= a;
            v += vb[k + 1] * dv;
        }
        x0_bar[(int64_t)p * d + i] = v;
    }
    if (threadIdx.x == 0) {
        double G0 = 0.0, G1 = 0.0;
        for (int c = 0; c < nchunk; ++c) {
            G0 += psc[((int64_t)p * nchunk + c) * 4 + 1];
            G1 += psc[((int64_t)p * nchunk + c) * 4 + 2];
        }
        double* ap = adj + (int64_t)p * A_NS;
        ap[A_GP + 0] = G0;
        ap[A_GP + 1] = G1;
    }
}

}  // namespace fbsde
