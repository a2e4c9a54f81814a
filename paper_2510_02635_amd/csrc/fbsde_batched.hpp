// Persistent batched launch: many evaluation points of many PDE instances (uneven d and M) in one
// kernel per geometry class.  Each workgroup pulls (instance, point) work items from an atomic queue
// and runs the whole chain of Algorithm 1 for that point by itself -- forward sweep, every level's
// weights, moments, conjugate-gradient solve (all reductions inside the workgroup, so no global
// synchronisation and no host round trip), particle reversal and Newton -- in a private slot of the
// workspace.  Work items are ordered by decreasing cost, so the queue balances uneven instances; the
// kernel ends when the queue is empty (every workgroup reaches that exit).
#pragma once
#include "fbsde_rowteam.hpp"

namespace fbsde {

struct BatchInst {
    int d, ld, M, N, P;
    double T, s, eps_h, ridge_rel, rtol2;
    int newton_iters, cg_maxit, g_kind, warm;
    FSpec f;
    double ga, gb;
    const double* mu;
    const double* gvec;
    uint32_t k0, k1, point_base;
    const double* x0;
    double* u;
    double* grad;
    uint32_t* status;
};

struct BatchItem { int inst, p; };

// Slot of one in-flight point (offsets in elements, computed by the host for the class maximum).
struct SlotLayout {
    size_t bytes;          // per slot
    size_t off_rn2, off_Y, off_w, off_c2, off_vec;   // byte offsets of the [M] arrays and the [6][ld] vectors
};

// R: arithmetic type of the row dots and column sums (FP64 on the FP32 state for a rank-deficient FP32C
// design, as in the single-instance path; otherwise the state's type).
template <typename S, typename R, int Q, int TEAM>
struct PointSolver {
    using G = Geo<Q, TEAM>;
    static constexpr int SPAN = 4 * Q * G::TL;

    const BatchInst& I;
    int p;
    S* W;
    double *rn2, *Y, *w, *c2, *x, *r, *pv, *qv, *Wbar, *tmp;
    double* lds;    // [TPW][SPAN] column combine
    double* red;    // [2 * waves] team reductions / [16] block sums
    int team, L;

    __device__ __forceinline__ void combine(CSum<R> (&acc)[Q][4], double* out) {
        block_columns_out<Q, TEAM, R>(acc, lds, out, I.ld, team, L);
        if constexpr (G::TPW == 1) __syncthreads();   // the per-lane stores must land before others read
    }

    __device__ void load_vec(const double* v, R (&dst)[Q][4]) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int e0 = 4 * (L + q * G::TL);
#pragma unroll
            for (int e = 0; e < 4; ++e) dst[q][e] = (e0 < I.ld) ? (R)v[e0 + e] : (R)0;
        }
    }

    __device__ void forward() {
        const double sqdt = sqrt(I.T / I.N);
        const uint32_t qs = I.point_base + (uint32_t)p;
        uint32_t st = 0;
        for (int jb = 0; jb < I.M; jb += G::TPW) {
            const int j = jb + team;
            const bool valid = j < I.M;
            double wv[Q][4];
#pragma unroll
            for (int q = 0; q < Q; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) wv[q][e] = 0.0;
            if (valid)
                for (int k = 0; k < I.N; ++k)
#pragma unroll 1
                    for (int q = 0; q < Q; ++q) {
                        const int g = L + q * G::TL;
                        if (4 * g < I.d) {
                            S z[4];
                            increment4<S>((uint32_t)g, (uint32_t)j, (uint32_t)k, qs, I.k0, I.k1, z);
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                if (4 * g + e < I.d) wv[q][e] += sqdt * (double)z[e];
                        }
                    }
            double n2 = 0.0, gq = 0.0;
            if (valid) {
                S* row = W + (int64_t)j * I.ld;
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int e0 = 4 * (L + q * G::TL);
                    if (e0 < I.ld) {
                        S v[4];
#pragma unroll
                        for (int e = 0; e < 4; ++e) v[e] = (S)wv[q][e];
                        store4(row + e0, v);
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const double ws = (double)v[e];
                            n2 += ws * ws;
                            const int i = e0 + e;
                            const double xc = (i < I.d) ? I.x0[(int64_t)p * I.d + i] + (I.mu ? I.mu[i] * I.T : 0.0) : 0.0;
                            const double X = xc + I.s * ws;
                            if (g_dot_arg(I.g_kind)) gq += ((e0 + e < I.d) ? I.gvec[e0 + e] : 0.0) * X;
                            else gq += X * X;
                        }
                    }
                }
            }
            team_sum2<TEAM>(n2, gq, red, team);
            if (valid && L == 0) {
                const double y = g_of(I.g_kind, I.ga, I.gb, gq, I.d);
                Y[j] = y;
                rn2[j] = n2;
                if (!isfinite(y)) st |= ST_NONFINITE;
            }
        }
        if (st) atomicOr(&I.status[p], st);
        __syncthreads();
    }

    // weights, Ybar, warm-start scale; c2 <- w (Y - Ybar).  Returns (Ybar, rho).
    __device__ void weights(int k, int warm, double& ybar, double& rho) {
        const double t_next = (double)(k + 1) * I.T / I.N;
        const double s2 = I.s * I.s;
        const double eps2 = (I.eps_h > 0.0) ? I.eps_h * I.eps_h * s2 * t_next * I.d : 0.0;
        double mn = INFINITY;
        for (int j = threadIdx.x; j < I.M; j += G::BS) mn = fmin(mn, rn2[j]);
        mn = block_min(mn, red);
        double se = 0.0;
        for (int j = threadIdx.x; j < I.M; j += G::BS) {
            const double e = (eps2 > 0.0) ? exp(-(s2 * rn2[j] - s2 * mn) / eps2) : 1.0;
            w[j] = e;
            se += e;
        }
        se = block_sum(se, red);
        double yb = 0.0, rh = 0.0;
        for (int j = threadIdx.x; j < I.M; j += G::BS) {
            const double wj = w[j] / se;
            w[j] = wj;
            yb += wj * Y[j];
            if (warm) rh += wj * c2[j];
        }
        ybar = block_sum(yb, red);
        rho = block_sum(rh, red);
        for (int j = threadIdx.x; j < I.M; j += G::BS) c2[j] = w[j] * (Y[j] - ybar);
        __syncthreads();
    }

    // moments and CG initialisation; returns |b|^2 and sets rr, wv.  Two passes over the state when warm:
    // (1) sum_j w_j W_j and sum_j w_j (Y_j - Ybar) W_j; (2) the pieces of A x0 -- two accumulators per pass
    // keep the register footprint of the persistent kernel low.
    __device__ void moments(int warm, double rho, double lam, double& rr, double& bb2, double& wvp) {
        double sig = 0.0, tau = 0.0;
        {
            CSum<R> a1[Q][4], a2[Q][4];
            for (int j = team; j < I.M; j += G::TPW) {
                const S* row = W + (int64_t)j * I.ld;
                const double wjd = w[j], cjd = c2[j];
                sig += cjd;
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int e0 = 4 * (L + q * G::TL);
                    if (e0 < I.ld) {
                        S xr[4];
                        load4(row + e0, xr);
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            a1[q][e].add((R)wjd * xr[e]);
                            a2[q][e].add((R)cjd * xr[e]);
                        }
                    }
                }
            }
            combine(a1, Wbar);
            combine(a2, tmp);
        }
        if (warm) {
            R v[Q][4];
            load_vec(x, v);
#pragma unroll
            for (int q = 0; q < Q; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) v[q][e] = (R)(rho * (double)v[q][e]);
            CSum<R> a3[Q][4];
            for (int jb = 0; jb < I.M; jb += G::TPW) {
                const int j = jb + team;
                const bool valid = j < I.M;
                S xr[Q][4];
                CSum<R> dl;
                if (valid) {
                    const S* row = W + (int64_t)j * I.ld;
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        const int e0 = 4 * (L + q * G::TL);
                        if (e0 < I.ld) load4(row + e0, xr[q]);
                        else {
#pragma unroll
                            for (int e = 0; e < 4; ++e) xr[q][e] = (S)0;
                        }
#pragma unroll
                        for (int e = 0; e < 4; ++e) dl.add(xr[q][e] * v[q][e]);
                    }
                }
                double t = dl.get(), unused = 0.0;
                team_sum2<TEAM>(t, unused, red, team);
                if (valid) {
                    const double ct = w[j] * t;
                    tau += ct;
#pragma unroll
                    for (int q = 0; q < Q; ++q)
#pragma unroll
                        for (int e = 0; e < 4; ++e) a3[q][e].add((R)ct * xr[q][e]);
                }
            }
            combine(a3, qv);
        }
        sig = block_sum((L == 0) ? sig : 0.0, red);
        tau = block_sum((L == 0) ? tau : 0.0, red);
        double rr_ = 0.0, bb_ = 0.0, wv_ = 0.0;
        for (int i = threadIdx.x; i < I.ld; i += G::BS) {
            const double wb = Wbar[i];
            const double b = I.s * (tmp[i] - sig * wb);
            double x0 = 0.0, res = b;
            if (warm) {
                x0 = rho * x[i];
                res = b - (I.s * I.s * (qv[i] - tau * wb) + lam * x0);
            }
            x[i] = x0;
            r[i] = res;
            pv[i] = res;
            rr_ += res * res;
            bb_ += b * b;
            wv_ += wb * res;
        }
        rr = block_sum(rr_, red);
        bb2 = block_sum(bb_, red);
        wvp = block_sum(wv_, red);
    }

    // one fused CG product q = A p (result in qv)
    __device__ void matvec(double wvp, double lam) {
        R v[Q][4];
        load_vec(pv, v);
        CSum<R> acc[Q][4];
        double tau = 0.0;
        for (int jb = 0; jb < I.M; jb += G::TPW) {
            const int j = jb + team;
            const bool valid = j < I.M;
            S xr[Q][4];
            CSum<R> dl;
            if (valid) {
                const S* row = W + (int64_t)j * I.ld;
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int e0 = 4 * (L + q * G::TL);
                    if (e0 < I.ld) load4(row + e0, xr[q]);
                    else {
#pragma unroll
                        for (int e = 0; e < 4; ++e) xr[q][e] = (S)0;
                    }
#pragma unroll
                    for (int e = 0; e < 4; ++e) dl.add(xr[q][e] * v[q][e]);
                }
            }
            double t = dl.get(), unused = 0.0;
            team_sum2<TEAM>(t, unused, red, team);
            if (valid) {
                const double cj = w[j] * I.s * (t - wvp);
                tau += cj;
                const R cr = (R)cj;
#pragma unroll
                for (int q = 0; q < Q; ++q)
#pragma unroll
                    for (int e = 0; e < 4; ++e) acc[q][e].add(cr * xr[q][e]);
            }
        }
        combine(acc, qv);
        tau = block_sum((L == 0) ? tau : 0.0, red);
        for (int i = threadIdx.x; i < I.ld; i += G::BS) qv[i] = I.s * (qv[i] - tau * Wbar[i]) + lam * pv[i];
        __syncthreads();
    }

    // reversal to level k (or W_0 = 0), Newton for Y_k, |W_k|^2, dY/dC
    __device__ void reverse(int k, double alpha, double zz, double zs) {
        const double dt = I.T / I.N, sqdt = sqrt(dt);
        const uint32_t qs = I.point_base + (uint32_t)p;
        R a[Q][4];
        load_vec(x, a);
        const FSpec f = I.f;
        uint32_t st = 0;
        for (int jb = 0; jb < I.M; jb += G::TPW) {
            const int j = jb + team;
            const bool valid = j < I.M;
            CSum<R> n2s, dots;
            if (valid) {
                S* row = W + (int64_t)j * I.ld;
#pragma unroll 1
                for (int q = 0; q < Q; ++q) {
                    const int g = L + q * G::TL;
                    const int e0 = 4 * g;
                    if (e0 < I.ld) {
                        S v[4];
                        load4(row + e0, v);
                        if (e0 < I.d) {
                            S z[4];
                            increment4<S>((uint32_t)g, (uint32_t)j, (uint32_t)k, qs, I.k0, I.k1, z);
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                if (e0 + e < I.d) v[e] = (S)((double)v[e] - sqdt * (double)z[e]);
                        }
                        store4(row + e0, v);
#pragma unroll
                        for (int e = 0; e < 4; ++e) { n2s.add(v[e] * v[e]); dots.add(a[q][e] * v[e]); }
                    }
                }
            }
            double n2 = n2s.get(), dd = dots.get();
            team_sum2<TEAM>(n2, dd, red, team);
            if (valid && L == 0) {
                double Fp;
                Y[j] = newton_y(f, alpha + I.s * dd, zz, zs, dt, I.newton_iters, Fp, st);
                rn2[j] = n2;
                c2[j] = 1.0 / Fp;
            }
        }
        if (st) atomicOr(&I.status[p], st);
        __syncthreads();
    }

    __device__ void run() {
        forward();
        const double dt = I.T / I.N;
        uint32_t st = 0;
        for (int k = I.N - 1; k >= 0; --k) {
            const int warm = (I.warm && k < I.N - 1) ? 1 : 0;
            double ybar, rho;
            weights(k, warm, ybar, rho);
            const double lam = I.ridge_rel * I.s * I.s * (double)(k + 1) * dt;
            double rr, bb2, wvp;
            moments(warm, rho, lam, rr, bb2, wvp);
            bool done = !(rr > 0.0);
            for (int it = 0; it < I.cg_maxit && !done; ++it) {
                matvec(wvp, lam);
                double pq = 0.0;
                for (int i = threadIdx.x; i < I.ld; i += G::BS) pq += pv[i] * qv[i];
                pq = block_sum(pq, red);
                const double al = (pq > 0.0) ? rr / pq : 0.0;
                double rr2 = 0.0;
                for (int i = threadIdx.x; i < I.ld; i += G::BS) {
                    x[i] += al * pv[i];
                    const double ri = r[i] - al * qv[i];
                    r[i] = ri;
                    rr2 += ri * ri;
                }
                rr2 = block_sum(rr2, red);
                if (!(pq > 0.0) || rr2 <= I.rtol2 * bb2) { done = true; break; }
                if (it + 1 >= I.cg_maxit) { st |= ST_CG_MAXIT; break; }
                const double beta = rr2 / rr;
                double wv_ = 0.0;
                for (int i = threadIdx.x; i < I.ld; i += G::BS) {
                    const double pi = r[i] + beta * pv[i];
                    pv[i] = pi;
                    wv_ += Wbar[i] * pi;
                }
                wvp = block_sum(wv_, red);
                rr = rr2;
            }
            double xw = 0.0, xx = 0.0, xs = 0.0;
            for (int i = threadIdx.x; i < I.ld; i += G::BS) { xw += x[i] * Wbar[i]; xx += x[i] * x[i]; xs += x[i]; }
            xw = block_sum(xw, red);
            xx = block_sum(xx, red);
            xs = block_sum(xs, red);
            const double alpha = ybar - I.s * xw;
            const double zz = I.s * I.s * xx, zs = I.s * xs;
            if (k > 0) {
                reverse(k, alpha, zz, zs);
            } else {
                double Fp;
                uint32_t s0 = 0;
                const double y = newton_y(I.f, alpha, zz, zs, dt, I.newton_iters, Fp, s0);
                st |= s0;
                if (threadIdx.x == 0) I.u[p] = y;
                if (I.grad)
                    for (int i = threadIdx.x; i < I.d; i += G::BS) I.grad[(int64_t)p * I.d + i] = x[i] / Fp;
            }
        }
        if (st && threadIdx.x == 0) atomicOr(&I.status[p], st);
        __syncthreads();
    }
};

template <typename S, typename R, int Q, int TEAM>
__global__ void __launch_bounds__((Geo<Q, TEAM>::BS))
k_batched(const BatchInst* __restrict__ insts, const BatchItem* __restrict__ items, int n_items, int* queue,
          char* __restrict__ slots, SlotLayout lay) {
    using G = Geo<Q, TEAM>;
    __shared__ double lds[(G::TPW > 1) ? G::TPW * 4 * Q * G::TL : 1];
    __shared__ double red[2 * G::BS / 64 + 16];
    __shared__ int item_s;
    char* slot = slots + (size_t)blockIdx.x * lay.bytes;
    for (;;) {
        if (threadIdx.x == 0) item_s = atomicAdd(queue, 1);
        __syncthreads();
        const int it = item_s;
        __syncthreads();
        if (it >= n_items) break;
        const BatchItem item = items[it];
        const BatchInst& I = insts[item.inst];
        double* vec = (double*)(slot + lay.off_vec);
        PointSolver<S, R, Q, TEAM> ps{I, item.p, (S*)slot, (double*)(slot + lay.off_rn2), (double*)(slot + lay.off_Y),
                                   (double*)(slot + lay.off_w), (double*)(slot + lay.off_c2), vec,
                                   vec + (size_t)I.ld, vec + 2 * (size_t)I.ld, vec + 3 * (size_t)I.ld,
                                   vec + 4 * (size_t)I.ld, vec + 5 * (size_t)I.ld, lds, red,
                                   (int)(threadIdx.x / G::TL), (int)(threadIdx.x % G::TL)};
        ps.run();
    }
}

}  // namespace fbsde
