// Scheme R under a constant invertible diffusion matrix sigma (Sec. 2.1's problem class with a matrix
// sigma; Z = sigma^T grad u).  The particles are X = x0 + mu t + sigma W.  The regression runs in the
// cloud's own metric: Gaussian weights exp(-D^T Sigma^{-1} D / (h^2 d)), Sigma = t sigma sigma^T, and the
// ridge on Z = sigma^T alpha_x.  In the coordinates W = sigma^{-1} (X - x0 - mu t) both become the
// isotropic weights and ridge of the scalar scheme at s = 1, the slope in W is Z itself and
// C = alpha + Z . W_k.  So the per-point path runs unchanged at s = 1, and only two steps see sigma:
//   the terminal values g(x0 + mu T + sigma W_N): sigma W_N on the matrix cores (GEMM), point chunk by
//     point chunk, then one wavefront per particle row forms the argument of g;
//   grad u(0, x0) = sigma^{-T} (grad in W): solved through sigma sigma^T (GEMM, blocked Cholesky) with
//     the right-hand sides sigma b.
#include "fbsde_host.hpp"
#include "fbsde_mfma.hpp"

using namespace fbsde;
using namespace fbsde::host;

namespace {

// Bytes of one chunk of sigma W_N rows at most (a chunk holds whole points).
constexpr int64_t SIGMA_CHUNK_BYTES = 512ll << 20;

struct SigmaLayout {
    size_t base;        // the per-point workspace (s = 1), with the tape when asked for
    size_t sig_off;     // sigma in the state's precision [d][d] (FP32C only)
    size_t t_off;       // sigma W_N of one chunk [Pc * M][d], state precision
    size_t k_off;       // sigma sigma^T [d][d] FP64
    size_t r_off;       // right-hand sides sigma b, or the W-column sums of the reverse mode [P][d] FP64
    size_t info_off;    // Cholesky status word
    size_t q_off;       // the reverse mode's argument of g per particle [P][M] FP64 (tape only)
    size_t total;
    int64_t pc;         // points per chunk
};

inline size_t up256(size_t b) { return (b + 255) / 256 * 256; }

int sigma_layout(const fbsde_problem* pb, int64_t P, int32_t flags, fbsde_problem& pbc, SigmaLayout& L) {
    int rc = check_problem(pb, P);
    if (rc) return rc;
    if (flags & ~FBSDE_WS_TAPE) return FBSDE_EINVAL;
    // one cloud per point; sources that read x and the Case 2 terminal value are not covered
    if (pb->shared_dw || per_point_forward_only(pb)) return FBSDE_EINVAL;
    pbc = *pb;
    pbc.s = 1.0;
    L.base = per_point_workspace_bytes(&pbc, P, flags);
    if (L.base == 0) return FBSDE_EINVAL;
    const size_t esz = (pb->prec == FBSDE_F64) ? 8 : 4;
    const int64_t row_bytes = (int64_t)pb->M * pb->d * (int64_t)esz;
    L.pc = std::max<int64_t>(1, std::min<int64_t>(std::max<int64_t>(P, 1), SIGMA_CHUNK_BYTES / row_bytes));
    size_t off = up256(L.base);
    L.sig_off = off;
    off += up256((size_t)pb->d * pb->d * esz);
    L.t_off = off;
    off += up256((size_t)L.pc * row_bytes);
    L.k_off = off;
    off += up256((size_t)pb->d * pb->d * 8);
    L.r_off = off;
    off += up256((size_t)std::max<int64_t>(P, 1) * pb->d * 8);
    L.info_off = off;
    off += 256;
    L.q_off = off;
    if (flags & FBSDE_WS_TAPE) off += up256((size_t)std::max<int64_t>(P, 1) * pb->M * 8);
    L.total = off;
    return FBSDE_OK;
}

__global__ void k_to_f32(const double* __restrict__ a, int64_t n, float* __restrict__ b) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

// Terminal values of `rows` particle rows (chunk rows r = (p - p0) M + j): X = x0_p + mu T + (sigma W_N)_r,
// Y[p0 M + r] = g(X), or (qout) the argument of g itself, qout[p0 M + r], for the reverse mode.  One
// wavefront per row; the argument of g (|X|^2 or gvec . X) is summed per lane and across the wavefront
// in a fixed order.
template <typename S>
__global__ void __launch_bounds__(256)
k_sigma_terminal(const S* __restrict__ T, int64_t rows, int M, int64_t p0, const double* __restrict__ x0,
                 const double* __restrict__ mu, double Tt, int d, int g_kind, double ga, double gb,
                 const double* __restrict__ gvec, double* __restrict__ Y, uint32_t* __restrict__ status,
                 double* __restrict__ qout) {
    const int64_t r = blockIdx.x * 4ll + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= rows) return;   // the whole wavefront leaves together
    const int64_t p = p0 + r / M;
    const S* t = T + r * (int64_t)d;
    const double* xp = x0 + p * d;
    const bool dot = g_dot_arg(g_kind);
    double q = 0.0;
    for (int i = lane; i < d; i += 64) {
        const double X = xp[i] + (mu ? mu[i] * Tt : 0.0) + (double)t[i];
        q += dot ? gvec[i] * X : X * X;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) q += __shfl_xor(q, off, 64);
    if (lane == 0 && qout) {
        qout[p0 * M + r] = q;
    } else if (lane == 0) {
        const double y = g_of(g_kind, ga, gb, q, d);
        Y[p0 * M + r] = y;
        if (!isfinite(y)) atomicOr(&status[p], (uint32_t)ST_NONFINITE);
    }
}

// grad u rows from the solved right-hand sides; a failed factorisation (sigma singular to working
// precision) or a non-finite entry marks the point.
__global__ void __launch_bounds__(256)
k_sigma_grad_out(const double* __restrict__ R, int d, const int* __restrict__ info, double* __restrict__ grad,
                 uint32_t* __restrict__ status) {
    __shared__ int bad;
    const int64_t p = blockIdx.x;
    if (threadIdx.x == 0) bad = (*info != 0);
    __syncthreads();
    int b = 0;
    for (int i = threadIdx.x; i < d; i += blockDim.x) {
        const double v = R[p * d + i];
        grad[p * d + i] = v;
        if (!isfinite(v)) b = 1;
    }
    if (b) atomicOr(&bad, 1);
    __syncthreads();
    if (threadIdx.x == 0 && bad) atomicOr(&status[p], (uint32_t)ST_NONFINITE);
}

// The W-column sums of the terminal adjoint, summed over their chunk slots: cs [P][d].
__global__ void __launch_bounds__(256)
k_sigma_colsum(const double* __restrict__ part, int nchunk, int vchunks, int ld, int d, double* __restrict__ cs) {
    const int64_t p = blockIdx.x;
    for (int i = threadIdx.x; i < d; i += blockDim.x) {
        double a = 0.0;
        for (int c = 0; c < vchunks; ++c) a += part[(p * nchunk + c) * ld + i];
        cs[p * d + i] = a;
    }
}

template <typename S>
int sigma_terminal(const fbsde_problem* pb, int64_t P, const double* x0, const S* sig, S* Tbuf, int64_t pc,
                   const void* Wv, int64_t ldw, double* Y, uint32_t* status, hipStream_t st, double* qout = nullptr) {
    const S* W = (const S*)Wv;
    const int M = (int)pb->M, d = (int)pb->d;
    for (int64_t p0 = 0; p0 < P; p0 += pc) {
        const int64_t np = std::min<int64_t>(pc, P - p0);
        const int64_t rows = np * M;
        // (sigma W_N)_r = row r of W_N sigma^T: A = the chunk's state rows, op(B) = sigma^T
        gemm<S, true>((int)rows, d, d, W + p0 * M * ldw, ldw, sig, d, EpiStore<S>{Tbuf, d, 1.0, 0.0, 0.0}, st);
        hipLaunchKernelGGL((k_sigma_terminal<S>), dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, Tbuf, rows,
                           M, p0, x0, pb->mu, pb->T, d, pb->g_kind, pb->gp[0], pb->gp[1], pb->gvec, Y, status,
                           qout);
        const int err = last_error();
        if (err) return err;
    }
    return FBSDE_OK;
}

}  // namespace

extern "C" {

int fbsde_sigma_workspace_size(const fbsde_problem* pb, int64_t P, int32_t flags, size_t* bytes) {
    if (!bytes) return FBSDE_EINVAL;
    fbsde_problem pbc;
    SigmaLayout L;
    const int rc = sigma_layout(pb, P, flags, pbc, L);
    if (rc) return rc;
    *bytes = L.total;
    return FBSDE_OK;
}

int fbsde_solve_sigma(const fbsde_problem* pb, const double* sigma, int64_t P, const double* x0, double* u,
                      double* grad, uint32_t* status, void* wsp, size_t ws_bytes, int32_t flags,
                      int32_t* cg_iters_out, fbsde_stream stream) {
    fbsde_problem pbc;
    SigmaLayout L;
    int rc = sigma_layout(pb, P, flags, pbc, L);
    if (rc) return rc;
    if (P == 0) {
        if (cg_iters_out)
            for (int64_t k = 0; k < pb->N; ++k) cg_iters_out[k] = 0;
        return FBSDE_OK;
    }
    if (!sigma || !x0 || !u || !status || !wsp) return FBSDE_EINVAL;
    if (L.total > ws_bytes) return FBSDE_ENOSPC;
    hipStream_t st = (hipStream_t)stream;
    char* base = (char*)wsp;
    const int d = (int)pb->d;
    const bool f64 = pb->prec == FBSDE_F64;
    if (!f64)
        hipLaunchKernelGGL(k_to_f32, dim3((unsigned)std::min<int64_t>(((int64_t)d * d + 255) / 256, 4096)), dim3(256),
                           0, st, sigma, (int64_t)d * d, (float*)(base + L.sig_off));
    const TerminalStep term = [&](const void* W, int64_t ldw, double* Y, hipStream_t s) -> int {
        if (f64)
            return sigma_terminal<double>(pb, P, x0, sigma, (double*)(base + L.t_off), L.pc, W, ldw, Y, status, s);
        return sigma_terminal<float>(pb, P, x0, (const float*)(base + L.sig_off), (float*)(base + L.t_off), L.pc, W,
                                     ldw, Y, status, s);
    };
    // the per-point solve at s = 1 in the coordinates W; grad (if asked) is the slope in W over F'
    if ((rc = solve_per_point_terminal(&pbc, P, x0, u, grad, status, wsp, L.base, flags, cg_iters_out, st, term)))
        return rc;
    if (!grad) return FBSDE_OK;
    // grad u = sigma^{-T} b: (sigma sigma^T) g = sigma b
    double* K = (double*)(base + L.k_off);
    double* R = (double*)(base + L.r_off);
    int* info = (int*)(base + L.info_off);
    set_int(info, 0, st);
    gemm<double, true>((int)P, d, d, grad, d, sigma, d, EpiStore<double>{R, d, 1.0, 0.0, 0.0}, st);
    gemm<double, true>(d, d, d, sigma, d, sigma, d, EpiStore<double>{K, d, 1.0, 0.0, 0.0}, st);
    cholesky<double>(K, d, d, info, st);
    cholesky_solve_rows<double>(K, d, d, R, d, (int)P, st);
    hipLaunchKernelGGL(k_sigma_grad_out, dim3((unsigned)P), dim3(256), 0, st, R, d, info, grad, status);
    return last_error();
}

int fbsde_solve_sigma_backward(const fbsde_problem* pb, const double* sigma, int64_t P, const double* x0,
                               const double* u_bar, double* x0_bar, double* gp_bar, double* fp_bar, uint32_t* status,
                               void* wsp, size_t ws_bytes, int32_t* cg_iters_out, fbsde_stream stream) {
    fbsde_problem pbc;
    SigmaLayout L;
    int rc = sigma_layout(pb, P, FBSDE_WS_TAPE, pbc, L);
    if (rc) return rc;
    if (!gp_bar || !fp_bar) return FBSDE_EINVAL;
    if (P > 0 && (!sigma || !wsp)) return FBSDE_EINVAL;
    if (P > 0 && L.total > ws_bytes) return FBSDE_ENOSPC;
    hipStream_t st = (hipStream_t)stream;
    char* base = (char*)wsp;
    const int d = (int)pb->d;
    const bool f64 = pb->prec == FBSDE_F64;
    if (P > 0 && !f64)
        hipLaunchKernelGGL(k_to_f32, dim3((unsigned)std::min<int64_t>(((int64_t)d * d + 255) / 256, 4096)), dim3(256),
                           0, st, sigma, (int64_t)d * d, (float*)(base + L.sig_off));
    double* qpre = (double*)(base + L.q_off);
    double* cs = (double*)(base + L.r_off);
    AdjTerminalHooks hooks;
    hooks.qpre = qpre;
    // the argument of g at X_N = x0 + mu T + sigma W_N for every particle, from the state W_N
    hooks.before = [&](const void* W, int64_t ldw, hipStream_t s) -> int {
        if (f64)
            return sigma_terminal<double>(pb, P, x0, sigma, (double*)(base + L.t_off), L.pc, W, ldw, nullptr, status,
                                          s, qpre);
        return sigma_terminal<float>(pb, P, x0, (const float*)(base + L.sig_off), (float*)(base + L.t_off), L.pc, W,
                                     ldw, nullptr, status, s, qpre);
    };
    // x0_bar += sigma (sum_j G_j 2 h'_j W_j): the W-column sums mapped to X by sigma
    hooks.after = [&](const double* part, int nchunk, int vchunks, int ld, double* xb, hipStream_t s) -> int {
        hipLaunchKernelGGL(k_sigma_colsum, dim3((unsigned)P), dim3(256), 0, s, part, nchunk, vchunks, ld, d, cs);
        gemm<double, true>((int)P, d, d, cs, d, sigma, d, EpiStore<double>{xb, d, 1.0, 1.0, 0.0}, s);
        return last_error();
    };
    return solve_per_point_backward_terminal(&pbc, P, x0, u_bar, x0_bar, gp_bar, fp_bar, status, wsp, L.base,
                                             cg_iters_out, st, hooks);
}

}  // extern "C"
