/*
 * fbsde.h -- C ABI of the MI355X (gfx950) library for the localized stochastic FBSDE /
 * local-linear-regression scheme for semilinear parabolic PDEs
 *
 *     (d_t + L) u + f(t, x, u, sigma^T grad u) = 0,   u(T, .) = g,
 *     L = 1/2 tr(sigma sigma^T Hess) + <mu, grad>            (paper Sec. 2.1, eq. mainprob)
 *
 * solved at evaluation points x0 through the FBSDE Y = u(t, X), Z = sigma^T grad u(t, X)
 * (eq. FBsyst), the implicit Euler step Y_k = E_k[Y_{k+1} + dt f(t_k, X_k, Y_k, Z_k)]
 * (eq. Ytkdiscrete), Euler-Maruyama particles (Sec. 2.3, eq. Xk), a kernel-weighted ridge
 * local linear regression for the gradient solved matrix-free (Sec. 2.4, eqs. leastsq, Dj,
 * normal-eq, the two-step matrix-free product and the ridge remark) and a scalar Newton
 * iteration for Y (Sec. 2.5, eqs. nonlinearf, NRiter), in the order of Algorithm 1.
 *
 * Scope of this ABI: sigma = s I (s > 0), constant drift mu, and built-in families for f and
 * g (device code cannot call host callbacks).  The scheme's readings of the paper:
 *   - level k regresses Y_{k+1} on the cloud at t_{k+1}: D_j = s W^j_{k+1}, the next-point
 *     form of Lemma 3.6 / 3.7, with weighted centring (Schur form of Lemma 3.7);
 *   - Gaussian kernel weights w_j ~ exp(-|D_j|^2 / eps_k^2), eps_k^2 = eps_h^2 s^2 t_{k+1} d,
 *     normalised over the cloud; eps_h = 0 gives uniform weights;
 *   - ridge only on the slope, lambda_k = ridge_rel s^2 t_{k+1};
 *   - E_k[Y_{k+1} | X^m_k] is the fitted linear model at the drift-transported particle,
 *     C^m_k = alpha + s alpha_x . W^m_k, and Z_k = s alpha_x;
 *   - Newton on F(y) = y - C - dt f(t_k, X, y, Z), newton_iters iterations from y = C;
 *   - u(0, x0) = mean_m Y^m_0 and grad u(0, x0) = (alpha_x + dt grad_x f) / F'(u) at level 0.
 * Particle increments are Philox4x32-10 (SC'11) normals regenerated on the fly:
 *   counter = (floor(i / 4), particle j, level k, point_base + p  | 0xFFFFFFFF if shared_dw),
 *   key     = (seed & 0xFFFFFFFF, (seed >> 32) ^ instance),
 *   Box-Muller on word pairs (0,1) and (2,3), u = (w + 1/2) 2^-32.
 *
 * Conventions for every entry point
 *   - Pointers named "device" are device memory of the current HIP device; the caller owns
 *     every buffer, including the workspace; the library allocates no device memory.  Its
 *     only process-wide state is the table of launch shapes chosen by fbsde_autotune, the
 *     optional launch timer (events kept once created) and the tiled batched schedule's pool of
 *     streams and events (created once per device and kept).
 *   - Calls enqueue work on `stream` (a hipStream_t; NULL = default stream) and return
 *     once it is enqueued, except where stated (the optional per-level CG iteration record of
 *     fbsde_solve, the tape checks of the reverse modes, the autotuner and the diagnostics return
 *     after their work has completed).  The CG iterations of
 *     a level run in one device-side loop, so no call waits for convergence on the host.
 *   - Return value: FBSDE_OK, or a negative code decided on the host before any launch
 *     (FBSDE_EINVAL, FBSDE_ENOSPC) or after a failed launch (FBSDE_EHIP).
 *   - Per-point numerical failures do not stop other points: they are OR-ed into
 *     status[p] (FBSDE_ST_* bits).
 *   - P = 0 (no evaluation points) is a valid call once the descriptor is valid: nothing is read
 *     or launched and the per-point pointers and the workspace may be NULL; cg_iters_out, when
 *     given, gets zeros, and the reverse modes write zeros into gp_bar and fp_bar (the gradient
 *     of an empty sum).  At most 65535 points per call (the batched call tiles larger instances).
 *   - Particle state layout: W[p][j][i] = W^j (Brownian displacement, X = x0 + t mu + s W)
 *     with a row pitch of fbsde_state_ld(pb) elements, padding kept at zero; element type
 *     double for FBSDE_F64, float for FBSDE_F32C.  In shared_dw mode the state is [M][ld].
 */
#ifndef FBSDE_H
#define FBSDE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* fbsde_stream;   /* hipStream_t */

enum { FBSDE_F64 = 0, FBSDE_F32C = 1 };       /* FP64 everywhere | FP32 state + compensated FP32
                                                 LLR sums, FP64 CG scalars, Newton and outputs */
enum { FBSDE_F_ZERO = 0,                      /* f = 0 (heat)                                  */
       FBSDE_F_ALLEN_CAHN = 1,                /* f = fp0 y - fp1 y^3 (Sec. 4.1 Case 1: 1, 1)  */
       FBSDE_F_HJB = 2,                       /* f = -fp0 |z|^2, z = sigma^T grad u            */
       FBSDE_F_BURGERS = 3,                   /* f = fp0 (y - fp1) sum_i z_i (Burgers type, Sec.
                                                 4; with fp0 = s/d, fp1 = d/s^2 + 1/2 and the
                                                 logistic g below, u = logistic(t + sum x / d)) */
       FBSDE_F_HJ_SINK = 4,                   /* f = S(t, x) - fp0 y |z|^2 / s^2: the Hamilton-
                                                 Jacobi-type equation of Sec. 4, sink kappa u
                                                 |grad u|^2 (kappa = fp0) and the source S that
                                                 makes v = (1+4t)^(-d/2) exp(-|x|^2/(1+4t)) exact
                                                 for v_t + (s^2/2) Lap v + f = 0 (with Lap v = v_t,
                                                 S = -(1 + s^2/2) v_t + kappa v |grad v|^2).  The
                                                 only family that depends on x: per-point solves
                                                 (fbsde_solve, _solve_step, _solve_noalloc, tiled
                                                 batches) only, forward only                      */
       FBSDE_F_LOG_POT = 5 };                 /* f = (fp0/2) ln((1+y)/(1-y)) - fp1 y - S2(t, x):
                                                 Allen-Cahn Case 2 (Sec. 4.1), log potential with
                                                 theta = fp0 < theta_c = fp1, and the source S2 that
                                                 makes v = fp2 cos(prod_j x_j) e^(cos t - |x|^2)
                                                 exact (amplitude fp2 < 1/e keeps |v| < 1).  Depends
                                                 on x: the same paths as FBSDE_F_HJ_SINK          */
enum { FBSDE_G_QUAD = 0,                      /* g = gp0 |x|^2 / d + gp1                       */
       FBSDE_G_AC = 1,                        /* g = 1 / (2 + gp0 |x|^2)   (Sec. 4.1 Case 1)   */
       FBSDE_G_HJB_LOG = 2,                   /* g = ln((1 + gp0 |x|^2) / 2)                   */
       FBSDE_G_AFFINE = 3,                    /* g = gvec . x + gp0                            */
       FBSDE_G_LOGISTIC = 4,                  /* g = 1 / (1 + exp(-(gvec . x + gp0)))          */
       FBSDE_G_HJ_GAUSS = 5,                  /* g = (1 + 4 gp0)^(-d/2) exp(-|x|^2 / (1 + 4 gp0)):
                                                 the HJ-type solution at time gp0 (= T)           */
       FBSDE_G_CASE2 = 6 };                   /* g = gp1 cos(prod_j x_j) e^(cos gp0 - |x|^2): the
                                                 Case 2 solution at time gp0 (= T)                */
enum { FBSDE_OK = 0, FBSDE_EINVAL = -1, FBSDE_ENOSPC = -2, FBSDE_EHIP = -3, FBSDE_ESTATE = -4 };
enum { FBSDE_ST_CG_MAXIT = 1, FBSDE_ST_NEWTON_FLAT = 2, FBSDE_ST_NONFINITE = 4,
       FBSDE_ST_WAIT_LIMIT = 8 };              /* a bounded device-side wait of the CG loop gave
                                                 up (internal error: the point's values are void) */
enum { FBSDE_WS_TAPE = 1 };                   /* workspace flag: keep the tape for the adjoint */

/* Problem descriptor (host memory).  Paper Algorithm 1 takes T, d, M, N, dt = T/N and the
 * target point; sigma, mu, f, g are the coefficients of Sec. 2.1. */
typedef struct fbsde_problem {
    int64_t d;               /* space dimension, 1 .. 16384 (FP64) or 32768 (FP32C): a point's */
                             /* row is held in the registers of one team of <= 16 wavefronts  */
    int64_t M;               /* particles per evaluation point, >= 2                          */
    int64_t N;               /* time steps, >= 1; dt = T / N                                  */
    double T;                /* horizon, > 0                                                  */
    double s;                /* sigma = s I, > 0                                              */
    const double* mu;        /* device [d] constant drift, or NULL for 0                      */
    int32_t f_kind;          /* FBSDE_F_*                                                     */
    int32_t g_kind;          /* FBSDE_G_*                                                     */
    double fp[4];            /* parameters of f                                               */
    double gp[4];            /* parameters of g                                               */
    const double* gvec;      /* device [d] slope of FBSDE_G_AFFINE / _LOGISTIC, else NULL     */
    double eps_h;            /* kernel bandwidth factor h >= 0 (0: uniform weights)           */
    double ridge_rel;        /* ridge factor >= 0; 0 needs M > d + 1                          */
    int32_t newton_iters;    /* Newton iterations per particle and level, >= 1                */
    int32_t cg_maxit;        /* CG iteration cap per level, >= 1                              */
    double cg_rtol;          /* CG stop: |r| <= cg_rtol |b|; FP32C with M <= d + 1 uses at     */
                             /* least 1e-7 (FP32 rounding in the ridge-only null space)        */
    int32_t cg_fixed_iters;  /* > 0: at most this many CG iterations per level (a point not   */
                             /* converged after them is flagged FBSDE_ST_CG_MAXIT); 0: the cap */
                             /* is cg_maxit                                                    */
    int32_t shared_dw;       /* 1: the same increments for every evaluation point             */
    uint64_t seed;           /* Philox key                                                     */
    uint32_t instance;       /* PDE instance id, folded into the key                          */
    uint32_t point_base;     /* global index of this call's point 0 (Philox counter word 3)   */
    int32_t prec;            /* FBSDE_F64 or FBSDE_F32C                                       */
    int32_t solver;          /* FBSDE_SOLVER_AUTO or FBSDE_SOLVER_CG (below)                  */
} fbsde_problem;

/* The level's ridge solve in the per-point form (fbsde_solve and the entry points built on it):
 * FBSDE_SOLVER_AUTO takes the direct dual solve where the design is rank-deficient and small
 * (d / 8 <= M <= d + 1, M <= FBSDE_DUAL_MAXM, ridge_rel > 0, cg_fixed_iters = 0): the M x M system
 * (W^1/2 D' D'^T W^1/2 + lambda I) c = W^1/2 (Y - Ybar), alpha_x = D'^T W^1/2 c (the push-through
 * identity of the normal equations, Sec. 2.4's system in its dual form), factored by Cholesky, with
 * cg_iters_out 0 for those levels; every other level, and every level with FBSDE_SOLVER_CG, runs the
 * matrix-free CG.  The reverse mode always runs CG. */
enum { FBSDE_SOLVER_AUTO = 0, FBSDE_SOLVER_CG = 1 };
#define FBSDE_DUAL_MAXM 128

/* Row pitch (elements) of the particle state for this problem (d rounded up so that rows
 * start on 128-byte boundaries).  Returns 0 for an invalid descriptor. */
int64_t fbsde_state_ld(const fbsde_problem* pb);

/* Workspace bytes needed by fbsde_solve / fbsde_solve_step / fbsde_solve_backward for P
 * points.  flags: FBSDE_WS_TAPE to keep what fbsde_solve_backward needs. */
int fbsde_workspace_size(const fbsde_problem* pb, int64_t P, int32_t flags, size_t* bytes);

/* Forward half of Algorithm 1 for P points (its first two loops): simulate the Brownian
 * displacements W^j_N = sum_k sqrt(dt) xi^j_k (eq. Xk) and set Y^j_N = g(x0 + mu T + s W^j_N).
 *   x0     device [P][d] evaluation points (row stride d)
 *   W      device [P][M][ldw] (shared_dw: [M][ldw]) output state at t_N, ldw >= fbsde_state_ld
 *   Y      device [P][M] output terminal values
 *   status device [P] cleared, then OR-ed with FBSDE_ST_NONFINITE on overflow */
int fbsde_terminal(const fbsde_problem* pb, int64_t P, const double* x0, void* W, int64_t ldw,
                   double* Y, uint32_t* status, fbsde_stream stream);

/* One backward level k (0 <= k < N) of Algorithm 1 on caller-owned state: the weighted ridge
 * regression of Y_{k+1} on the cloud W_{k+1} (matrix-free CG, eq. normal-eq and the ridge
 * remark), the particle reversal W_k = W_{k+1} - sqrt(dt) xi_k, and the Newton solve for Y_k.
 *   W       device state, in: W_{k+1}, out: W_k (layout as fbsde_terminal; not shared_dw)
 *   Y_next  device [P][M] in: Y_{k+1};   Y device [P][M] out: Y_k (may not alias Y_next)
 *   alpha   device [P] out: intercept;   alpha_x device [P][d] out: slope (row stride d)
 *   status  device [P] OR-ed with FBSDE_ST_* bits
 *   ws      device workspace of at least fbsde_workspace_size(pb, P, 0) bytes */
int fbsde_solve_step(const fbsde_problem* pb, int64_t P, int32_t k, const double* x0, void* W,
                     int64_t ldw, const double* Y_next, double* Y, double* alpha, double* alpha_x,
                     uint32_t* status, void* ws, size_t ws_bytes, fbsde_stream stream);

/* Algorithm 1 for P evaluation points: u(0, x0_p) and grad u(0, x0_p).
 *   x0     device [P][d];  u device [P];  grad device [P][d] or NULL;  status device [P]
 *   ws     device workspace, fbsde_workspace_size(pb, P, flags) bytes; with FBSDE_WS_TAPE it
 *          keeps the tape that fbsde_solve_backward reads (then do not reuse ws in between)
 *   cg_iters_out  host [N] or NULL: at each level k the largest CG iteration count over the points
 *                 (read back from the device after the level: one extra stream wait per level)
 * Each level's CG solve is one launch of a device-side loop: work items (iteration, point, chunk of
 * particle rows) are taken in order from a device counter, a point's next iteration starts when its
 * chunks' partial sums have been combined, and the point leaves the loop at |r| <= cg_rtol |b| or the
 * cap.  With cg_iters_out NULL the call returns once the work is enqueued. */
int fbsde_solve(const fbsde_problem* pb, int64_t P, const double* x0, double* u, double* grad,
                uint32_t* status, void* ws, size_t ws_bytes, int32_t flags, int32_t* cg_iters_out,
                fbsde_stream stream);
/* shared_dw = 1 (increments common to all points, the common-randomness remark after Lemma 3.7):
 * one cloud, one ridge system per level; the regressions of all points become dense MFMA
 * contractions with the inverse of the M x M dual matrix lam I + s^2 Dt Dt^T, Dt_j =
 * sqrt(w_j)(W_j - Wbar) (push-through form of the ridge solve; M > d: the d x d primal matrix),
 * formed once per level from its blocked Cholesky factor (blockwise inverse of the factor); no CG
 * (cg_iters_out gets 0).  flags = FBSDE_WS_TAPE keeps that inverse, the slopes and Y per level for
 * fbsde_solve_backward.  fbsde_terminal, fbsde_solve_step and fbsde_time_kernel return
 * FBSDE_EINVAL for shared_dw = 1. */

/* Reverse mode of fbsde_solve for the loss L = sum_p u_bar[p] u(0, x0_p): hand-written adjoint of
 * the whole backward chain (Newton by the implicit-function rule, the regression through one extra
 * CG solve per level with the same symmetric matrix, the terminal condition), regenerating the
 * particles from their Philox counters forward in time.
 *   Requires the immediately preceding fbsde_solve on the same pb, P, x0 and ws with
 *   flags = FBSDE_WS_TAPE (FBSDE_ESTATE otherwise).
 *   u_bar  device [P];  x0_bar device [P][d] out;  gp_bar, fp_bar device [4] out (summed
 *   over points);  status device [P] OR-ed;  cg_iters_out host [N] or NULL: the largest adjoint CG
 *   iteration count over the points at each level k.
 * With a rank-deficient centred design (M <= d + 1) the adjoint right-hand side reaches the
 * ridge-only null space, so in FP32C the CG product and the row dots of this pass use FP64
 * arithmetic on the FP32 state. */
int fbsde_solve_backward(const fbsde_problem* pb, int64_t P, const double* x0, const double* u_bar,
                         double* x0_bar, double* gp_bar, double* fp_bar, uint32_t* status,
                         void* ws, size_t ws_bytes, int32_t* cg_iters_out, fbsde_stream stream);

/* Diagnostic: the normals xi^j_k of point p (or the shared stream) for rows j0..j0+rows-1 of
 * level k, exactly as the kernels generate them in pb->prec (FP32C: the FP32 values, written as
 * doubles).  out device [rows][d]; words device [rows][ceil(d/4)][4] raw Philox output or NULL. */
int fbsde_normals(const fbsde_problem* pb, int64_t p, int32_t k, int64_t j0, int64_t rows,
                  double* out, uint32_t* words, fbsde_stream stream);

/* Diagnostic: the Box-Muller step alone on caller-given Philox words, exactly as the kernels apply
 * it in `prec` (FBSDE_F64, or FBSDE_F32C with its FP32 logarithm, hardware square root and sin/cos
 * on the exactly reduced angle; FP32 values written as doubles).  Lets a test reach the words that
 * counters rarely produce: 0, 2^32 - 1, the mantissa switch at sqrt(2), the octant boundaries.
 *   words device [n][4] (pairs (0,1) and (2,3) as in the normals above);  out device [n][4]. */
int fbsde_box_muller(int32_t prec, int64_t n, const uint32_t* words, double* out, fbsde_stream stream);

/* Diagnostic: average duration (host float, milliseconds) of one launch of a hot-path kernel at
 * this problem's launch geometry, timed with HIP events on `stream` over reps - 1 launches after
 * one warm-up launch; synchronises the stream.  which: 0 fused CG product (the dominant kernel),
 * 1 particle reversal + Newton, 2 weighted moments, 3 forward sweep + terminal, 4 a plain stream
 * over the same state bytes (16-byte non-temporal loads, nothing else): the read bandwidth the
 * hardware delivers on that buffer, the attainable ceiling for the CG product.  It runs on the
 * state and vectors left in ws by a preceding fbsde_solve with the same pb and P (flags 0) and
 * overwrites them: solve again before using ws for anything else. */
int fbsde_time_kernel(const fbsde_problem* pb, int64_t P, int32_t which, int32_t reps, void* ws,
                      size_t ws_bytes, float* avg_ms, fbsde_stream stream);

/* Many evaluation points of many PDE instances (uneven d, M, f, g, N, precision) in one call
 * (batching over points and instances goes beyond the paper; the per-point chain is Algorithm 1).
 * Two schedules, chosen by opts->mode:
 *  FBSDE_BATCH_TILED (default): the work items are (instance, point-tile) pairs.  Each tile runs the
 *    whole chain through the multi-block path of fbsde_solve (each point split over many workgroups
 *    along its particle rows, every level's CG on the device) on one of `streams` HIP streams, each
 *    with its own workspace arena, so tiles of different instances overlap on the chip.  The tiles are dealt to the streams before any is enqueued: largest expected time first
 *    (state bytes x levels x estimated passes, the CG count estimated from the design's condition),
 *    each to the stream with the least expected time so far.
 *    A tile holds as many points as fit `tile_bytes` of workspace (at least one, at most 65535), so
 *    memory is bounded by the tiles in flight, not by the batch.  Tile i of an instance covers its
 *    points [p0, p0 + np) with point_base + p0: results equal fbsde_solve of the whole instance up to
 *    the rounding order of the partial sums (same Philox streams, same CG test).
 *  FBSDE_BATCH_PERSISTENT: one persistent launch per geometry class (element type and row-team
 *    shape, decided by d); every workgroup owns a slot, pulls (instance, point) items from an atomic
 *    queue (largest M first) and runs the whole chain of its point alone, with workgroup reductions.
 *    Forward only.  Bounded by one compute unit's share of HBM per point: for points whose chain is
 *    long (large d and M) the tiled schedule is much faster.
 *   pbs     host [n_inst] descriptors (tiled: shared_dw allowed for the forward solve)
 *   P       host [n_inst] point counts (>= 0)
 *   x0, u, grad, status   host arrays of n_inst device pointers ([P_i][d_i], [P_i], [P_i][d_i] or
 *                         NULL, [P_i]); grad itself may be NULL
 *   opts    NULL for the defaults (tiled, 3 streams, 24 GiB tiles, 512 persistent slots; 3 streams
 *           because HIP gives a process four hardware queues by default and the caller's stream holds
 *           one, so a fourth pool stream would share a queue with another and wait behind it)
 *   ws      device workspace of fbsde_batched_workspace_size(pbs, n_inst, P, opts, adjoint) bytes
 * The tiled schedule forks from the caller's stream onto a pool of streams (created once per device and
 * kept for the life of the process), and the caller's stream waits for all of them: the call returns
 * once its work is enqueued (every level's CG is one device-side loop launch; the runtime may hold the
 * host back while a stream's command queue is full) and needs the calling
 * thread's current device to be the one holding the buffers.  Calls that overlap on one device from
 * several host threads queue their tiles on the same streams.  The persistent schedule synchronises
 * the stream once (after uploading its work tables), then runs asynchronously. */
enum { FBSDE_BATCH_TILED = 0, FBSDE_BATCH_PERSISTENT = 1 };
typedef struct fbsde_batch_opts {
    int32_t mode;         /* FBSDE_BATCH_TILED or FBSDE_BATCH_PERSISTENT                 */
    int32_t streams;      /* tiled: concurrent streams, 1..8 (0: 3)                       */
    int64_t tile_bytes;   /* tiled: workspace cap of one tile in bytes (0: 24 GiB)       */
    int32_t max_slots;    /* persistent: workgroups (points in flight) per class (0: 512) */
    int32_t reserved;     /* must be 0                                                   */
} fbsde_batch_opts;
int fbsde_batched_workspace_size(const fbsde_problem* pbs, int64_t n_inst, const int64_t* P,
                                 const fbsde_batch_opts* opts, int32_t adjoint, size_t* bytes);
int fbsde_solve_batched(const fbsde_problem* pbs, int64_t n_inst, const int64_t* P,
                        const double* const* x0, double* const* u, double* const* grad,
                        uint32_t* const* status, const fbsde_batch_opts* opts, void* ws,
                        size_t ws_bytes, fbsde_stream stream);
/* Batched forward + reverse mode (tiled schedule only): per instance, u [P_i] and the adjoints of
 * L_i = sum_p u_bar_i[p] u_i(0, x0_p): x0_bar [P_i][d_i], gp_bar [4], fp_bar [4] (device).  Each
 * tile runs fbsde_solve with the tape and fbsde_solve_backward in its arena; the parameter adjoints
 * of an instance are the sum of its tiles' sums in point order.  status ORs both passes.  Workspace:
 * fbsde_batched_workspace_size(..., adjoint = 1). */
int fbsde_solve_batched_backward(const fbsde_problem* pbs, int64_t n_inst, const int64_t* P,
                                 const double* const* x0, const double* const* u_bar, double* const* u,
                                 double* const* x0_bar, double* const* gp_bar, double* const* fp_bar,
                                 uint32_t* const* status, const fbsde_batch_opts* opts, void* ws,
                                 size_t ws_bytes, fbsde_stream stream);

/* Diagnostic: the algorithmic bytes that the CG products of the last tiled batched call (forward, or
 * forward + reverse with adjoint = 1) on this workspace streamed: for every product, the particle rows of
 * the points still iterating x d x element bytes (per-point tiles; shared-increment tiles have no CG).
 * pbs, n_inst, P, opts, adjoint: as in that call;  ws: its workspace;  *bytes host;  synchronises. */
int fbsde_batched_cg_bytes(const fbsde_problem* pbs, int64_t n_inst, const int64_t* P,
                           const fbsde_batch_opts* opts, int32_t adjoint, const void* ws, double* bytes,
                           fbsde_stream stream);

/* Dense helpers of the shared-increment form, exported for verification and reuse.
 * fbsde_gemm: C = alpha * A op(B) + beta * C on the matrix cores (v_mfma 16x16x4, FP64 or FP32
 *   operands by prec), A [m][lda] row-major (k contiguous); nt = 1: B [n][ldb] (op(B) = B^T),
 *   nt = 0: B [k][ldb] (op(B) = B); C [m][ldc]; all device memory.
 * fbsde_cholesky_solve: blocked Cholesky K = L L^T in place (lower triangle of the n x n SPD matrix
 *   K [n][ldk]) and, for P > 0, the solve X (L L^T) = R of the P right-hand sides stored as rows of
 *   R [P][ldr], in place; ws device scratch of fbsde_cholesky_workspace(prec, n, P) bytes; *info
 *   (host) is nonzero if a non-positive pivot was met; synchronises the stream. */
int fbsde_gemm(int32_t prec, int32_t nt, int64_t m, int64_t n, int64_t k, const void* A, int64_t lda,
               const void* B, int64_t ldb, void* C, int64_t ldc, double alpha, double beta,
               fbsde_stream stream);
size_t fbsde_cholesky_workspace(int32_t prec, int64_t n, int64_t P);
int fbsde_cholesky_solve(int32_t prec, int64_t n, void* K, int64_t ldk, int64_t P, void* R, int64_t ldr,
                         void* ws, size_t ws_bytes, int32_t* info, fbsde_stream stream);

/* Autotuner of the launch shape (beyond the paper: the tile and split choices are picked by
 * measurement).  For this problem's precision, d, M and this P it times the fused CG product -- the
 * kernel that dominates a solve -- over the candidate shapes: the split of a particle row over 1, 2
 * or 4 times the default team width of wavefronts (fewer coordinates per lane) and the split of a
 * point's particle rows over the default, half or a quarter of the default workgroups.  The timing
 * runs on the forward sweep of the given points x0 (device [P][d]) in ws (fbsde_workspace_size(pb, P,
 * 0) bytes, overwritten).  The fastest shape (a new one must win by 2 %) is recorded in a process-wide
 * table that every later plan with the same (precision, d, M, P) uses -- fbsde_solve, _step, _backward,
 * fbsde_time_kernel and the workspace sizes (never larger than before tuning).  This table and the
 * launch timer below are the library's only global state; fbsde_autotune_reset clears the table.  Thread-safe; synchronises the stream. */
typedef struct fbsde_tune_result {
    int32_t team;            /* wavefronts per particle row                        */
    int32_t q;               /* groups of four coordinates per lane                */
    int32_t nchunk;          /* workgroups per point                               */
    int32_t n_candidates;    /* shapes timed                                       */
    float best_ms;           /* one launch of the CG product at the chosen shape   */
    float default_ms;        /* the same at the default shape                      */
} fbsde_tune_result;
int fbsde_autotune(const fbsde_problem* pb, int64_t P, const double* x0, void* ws, size_t ws_bytes,
                   fbsde_tune_result* out, fbsde_stream stream);
int fbsde_autotune_reset(void);

/* Launch timer of the dominant kernels, for measuring them inside a caller's own timed region.
 * fbsde_launch_timer(1) clears the record and starts it; fbsde_launch_timer(0) stops it and keeps the
 * record.  While it runs, each timed launch on a stream that is not being captured is bracketed by two
 * HIP events on that stream, at a few microseconds of host time per launch. The timed launches are the
 * CG products of fbsde_solve and fbsde_solve_backward, and the Gram and anchor launches of
 * fbsde_solve_literal.
 * fbsde_launch_timer_read waits for the recorded launches. For the first `cap` of them, in launch
 * order, it writes the duration in milliseconds to `ms` (host) and the algorithmic work to `bytes`
 * (host, or NULL); it writes their total count to *n. The work unit depends on the kind:
 *   FBSDE_TIMED_CG_PRODUCT       bytes: points x particles x d x element bytes, the one read of the
 *                                state that each product needs
 *   FBSDE_TIMED_LITERAL_GRAM     FP64 flops: points x M (M + 1) x d (lower triangle of W W^T)
 *   FBSDE_TIMED_LITERAL_ANCHORS  FP64 flops: points x M x (2/3 (M + 1)^3 + 6 M^2) (bordered factorisation,
 *                                back substitution, system and quadratic-form assembly)
 * fbsde_launch_timer_kinds writes the kinds of the same records.  The events are created on first use
 * and kept for the life of the process.  Thread-safe; the record is process-wide. */
enum { FBSDE_TIMED_CG_PRODUCT = 0, FBSDE_TIMED_LITERAL_GRAM = 1, FBSDE_TIMED_LITERAL_ANCHORS = 2,
       FBSDE_TIMED_CG_LOOP = 3 };   /* the device-side CG loop of one level: its work is not known when
                                       it is launched (recorded as 0); fbsde_workspace_cg_rows gives the
                                       rows its products streamed */
int fbsde_launch_timer(int32_t on);
int fbsde_launch_timer_read(float* ms, double* bytes, int64_t cap, int64_t* n);
int fbsde_launch_timer_kinds(int32_t* kinds, int64_t cap, int64_t* n);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): fbsde_solve of the per-point form (shared_dw = 0, flags = 0, no
 * iteration record) with the workspace taken from a file-scope device array of
 * FBSDE_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on (until the process ends).
 * The caller still passes the inputs and outputs (x0, u, grad or NULL, status: device memory as in
 * fbsde_solve).  No device or host memory is allocated and no launch timer events are created.
 * FBSDE_ENOSPC if fbsde_workspace_size(pb, P, 0) exceeds that size, FBSDE_EINVAL for shared_dw = 1.
 * Every call on one GPU uses that GPU's one array: calls that overlap on one GPU (different streams or
 * host threads without ordering) race and must not be issued; calls on one stream are ordered.  The
 * array keeps the last call's contents; every value a solve reads is written by that solve first. */
#define FBSDE_NOALLOC_SCRATCH_BYTES (64ll << 20)
int fbsde_solve_noalloc(const fbsde_problem* pb, int64_t P, const double* x0, double* u, double* grad,
                        uint32_t* status, fbsde_stream stream);

/* Diagnostic: the particle rows that the CG products of the per-point path have streamed since the
 * start of the last fbsde_solve on this workspace (its backward pass included).  One row of a point is
 * d elements of the state, so rows x d x element bytes is the algorithmic read traffic of those
 * products.  ws: the device workspace of that solve; *rows host; synchronises the stream. */
int fbsde_workspace_cg_rows(const void* ws, int64_t* rows, fbsde_stream stream);

/* Captured solve, for callers that repeat one solve with the same problem, sizes and buffers
 * (serving loops, parameter sweeps that rewrite x0 in place): the launch sequence of fbsde_solve
 * (flags as there) is captured once into a HIP graph on a private stream that waits for `stream`,
 * and fbsde_graph_launch replays it with a single launch.  The graph binds every pointer given here
 * and in pb (mu, gvec): a replay reads x0 and writes u, grad, status and ws at these addresses, so
 * they must stay allocated until fbsde_graph_destroy.  Every level's CG solve is one device-side
 * loop, so any descriptor can be captured (with FBSDE_CG_HOST_LOOP=1 in the environment, the host-
 * polled diagnostic loop, the per-point form needs cg_fixed_iters > 0).
 * Status words and flags are cleared by kernels, so no memset node enters the graph.  Nothing is
 * launched by the capture itself. */
typedef struct fbsde_graph_s* fbsde_graph;
int fbsde_graph_capture(const fbsde_problem* pb, int64_t P, const double* x0, double* u, double* grad,
                        uint32_t* status, void* ws, size_t ws_bytes, int32_t flags, fbsde_graph* out,
                        fbsde_stream stream);
int fbsde_graph_launch(fbsde_graph graph, fbsde_stream stream);
int fbsde_graph_destroy(fbsde_graph graph);
/* fbsde_solve_batched (tiled schedule) captured into a graph the same way: the fork onto the stream pool
 * and the join back are recorded with the tiles, so one fbsde_graph_launch replays the whole batch.
 * Arguments as fbsde_solve_batched (opts->mode must be FBSDE_BATCH_TILED); every pointer, the
 * workspace included, is bound into the graph.  The graph replays on the pool's streams, so two
 * graphs (or a graph and an eager tiled call) of one device must not run at the same time. */
int fbsde_graph_capture_batched(const fbsde_problem* pbs, int64_t n_inst, const int64_t* P,
                                const double* const* x0, double* const* u, double* const* grad,
                                uint32_t* const* status, const fbsde_batch_opts* opts, void* ws,
                                size_t ws_bytes, fbsde_graph* out, fbsde_stream stream);

/* Paper-literal per-anchor scheme: Algorithm 1 as printed (Sec. 2.3 to 2.5), with none of the
 * readings that fbsde_solve takes for the regression.  At every level k and for every particle m:
 * the weighted ridge regression of eq. normal-eq (functional J_lambda of the ridge remark, intercept
 * penalised as printed) over D^m_j = X^j_k - X^m_k (eq. Dj), Gaussian weights with
 * eps_k^2 = eps_h^2 2 s^2 t_k d (uniform at k = 0 and for eps_h = 0), lambda_k = ridge_rel s^2 t_{k+1};
 * Z^m_k = s alpha_x; Y^m_k from pb->newton_iters Newton steps (eq. NRiter) on
 * y - Ybar - dt f(y, Z^m_k) started at the plain particle mean Ybar = (1/M) sum_j Y^j_{k+1}
 * (eq. discreteYkm).  The slope is identically zero at k = 0 (every particle starts at x0), so the
 * scheme gives no gradient.  Same particles (Philox counters) as fbsde_solve.
 * Each regression is solved through its M x M dual system, built from the Gram matrix of the
 * particles at level k; O(M^2 d + M^4 / 3) per level and point.
 *   Requires prec = FBSDE_F64, shared_dw = 0, 2 <= M <= 256, ridge_rel > 0 (FBSDE_EINVAL otherwise).
 *   k_stop   0 <= k_stop < N: the backward sweep runs levels N-1 .. k_stop
 *   x0       device [P][d];  u device [P] out: mean_m Y^m_{k_stop} (u(0, x0) for k_stop = 0)
 *   Y_out    device [P][M] out: Y^m_{k_stop}, or NULL
 *   z_stats  device [P][M][2] out: |Z^m_{k_stop}|^2 and sum_i Z^m_{k_stop,i}, or NULL
 *   status   device [P] cleared, then OR-ed with FBSDE_ST_NEWTON_FLAT / FBSDE_ST_NONFINITE
 *   ws       device workspace of fbsde_literal_workspace_size(pb, P) bytes (FBSDE_ENOSPC if smaller).  With
 *            at least fbsde_literal_workspace_size_stored(pb, P) bytes ((N + 1) P M d doubles and more) the
 *            forward sweep keeps the particles of every level and the backward sweep reads them, instead
 *            of reversing the path with regenerated increments; the results agree to rounding.
 * P = 0 returns FBSDE_OK without touching the pointers. */
int fbsde_literal_workspace_size(const fbsde_problem* pb, int64_t P, size_t* bytes);
int fbsde_literal_workspace_size_stored(const fbsde_problem* pb, int64_t P, size_t* bytes);
int fbsde_solve_literal(const fbsde_problem* pb, int64_t P, int32_t k_stop, const double* x0, double* u,
                        double* Y_out, double* z_stats, uint32_t* status, void* ws, size_t ws_bytes,
                        fbsde_stream stream);

/* The same printed scheme with x-dependent coefficients (the problem class of Sec. 2.1 allows mu(t, x)
 * and sigma(t, x)).  Affine diagonal family, componentwise: mu(x) = mu0 x + mu1, sigma(x) =
 * diag(sigma0 x + sigma1).  FBSDE_COEF_GEOMETRIC is its case mu1 = sigma1 = 0 (both must be 0);
 * FBSDE_COEF_AFFINE_DIAG takes all four (sigma0 = 0, mu0 < 0: an Ornstein-Uhlenbeck drift with additive
 * noise).  The particles follow the Euler-Maruyama step of eq. Xk,
 *   X_{k+1} = X_k + (mu0 X_k + mu1) dt + (sigma0 X_k + sigma1) * sqrt(dt) xi_k, X_0 = x0,
 * with the same increments xi as every other entry point.  Per level and particle m, as in
 * fbsde_solve_literal, except:
 *   Z^m_k = sigma(X^m_k)^T alpha_x = (sigma0 X^m_k + sigma1) * alpha_x (componentwise), from the explicit slope;
 *   eps_k^2 = eps_h^2 2 (1/M) sum_j |X^j_k - Xbar_k|^2, the cloud's own mean squared pairwise distance
 *     (uniform weights at k = 0);
 *   lambda_k = ridge_rel (sigma0^2 + sigma1^2) t_{k+1}.
 * The path is not reversible from its increments, so the displacements X_k - x0 of every level are
 * kept: the workspace holds (N + 1) P M d doubles.  pb->s is not used; pb->mu must be NULL.
 * Arguments, outputs, limits and errors as fbsde_solve_literal; coef host, reserved 0, finite
 * coefficients with sigma0^2 + sigma1^2 > 0 (FBSDE_EINVAL otherwise). */
enum { FBSDE_COEF_GEOMETRIC = 1, FBSDE_COEF_AFFINE_DIAG = 2 };
typedef struct fbsde_coef {
    int32_t kind;            /* FBSDE_COEF_GEOMETRIC or FBSDE_COEF_AFFINE_DIAG                */
    int32_t reserved;        /* must be 0                                                     */
    double mu0;              /* drift: mu(x) = mu0 x + mu1                                    */
    double sigma0;           /* volatility: sigma(x) = diag(sigma0 x + sigma1)                */
    double mu1;              /* 0 for FBSDE_COEF_GEOMETRIC                                    */
    double sigma1;           /* 0 for FBSDE_COEF_GEOMETRIC                                    */
} fbsde_coef;
int fbsde_literal_coef_workspace_size(const fbsde_problem* pb, const fbsde_coef* coef, int64_t P, size_t* bytes);
int fbsde_solve_literal_coef(const fbsde_problem* pb, const fbsde_coef* coef, int64_t P, int32_t k_stop,
                             const double* x0, double* u, double* Y_out, double* z_stats, uint32_t* status,
                             void* ws, size_t ws_bytes, fbsde_stream stream);

/* Scheme R (fbsde_solve: one weighted ridge regression per point and level, CG on the normal equations,
 * Newton for Y) under the same affine diagonal coefficients, mu(x) = mu0 x + mu1 and sigma(x) =
 * diag(sigma0 x + sigma1) componentwise.  The particles of point p follow the Euler-Maruyama step of
 * eq. Xk from x0[p] with fbsde_solve's increments; the regressor is the displacement D_k = X_k - m_k
 * from the mean path m_{k+1} = m_k + (mu0 m_k + mu1) dt (m_0 = x0), which makes every particle's
 * position a function of its own increments and lets the path run backwards in place (the step is
 * inverted, X_k = (X_{k+1} - mu1 dt - sigma1 dW_k) / (1 + mu0 dt + sigma0 dW_k)).  Per level k:
 *   weights exp(-|D_{k+1}|^2 / (eps_h^2 V_{k+1})) (uniform for eps_h = 0), V_k = E|X_k - m_k|^2 from
 *     the exact moment recursion of the step;
 *   ridge lambda_k = ridge_rel V_{k+1} / d;
 *   the fitted model taken at the drift-transported particle, C = alpha + (1 + mu0 dt) alpha_x . D_k;
 *   Z = (sigma0 X_k + sigma1) * alpha_x per particle (sigma(X)^T times the slope);
 *   grad u = ((1 + mu0 dt) alpha_x + dt sigma0 alpha_x * df/dz) / F'(u) at level 0.
 * pb->s is not used and pb->mu must be NULL; shared_dw, f kinds that read x and the Case 2 terminal
 * value are refused (FBSDE_EINVAL), as are coef kinds and values fbsde_solve_literal_coef refuses.  A
 * cloud whose spread vanishes (V = 0: sigma1 = 0 with x0 = 0) has no regression and is undefined.
 * Workspace: fbsde_coef_workspace_size bytes for the same flags (FBSDE_WS_TAPE: also the tape that
 * fbsde_solve_coef_backward reads, and the tangent state it regenerates).  u [P], grad [P][d] or NULL,
 * status [P] and cg_iters_out as fbsde_solve, on stream; cg_iters_out, when given, makes the call wait for
 * the stream once per level. */
int fbsde_coef_workspace_size(const fbsde_problem* pb, const fbsde_coef* coef, int64_t P, int32_t flags,
                              size_t* bytes);
int fbsde_solve_coef(const fbsde_problem* pb, const fbsde_coef* coef, int64_t P, const double* x0, double* u,
                     double* grad, uint32_t* status, void* ws, size_t ws_bytes, int32_t flags,
                     int32_t* cg_iters_out, fbsde_stream stream);

/* Reverse mode of fbsde_solve_coef for L = sum_p u_bar[p] u(0, x0_p), after fbsde_solve_coef with
 * FBSDE_WS_TAPE on the same workspace, problem, coefficients and points (else FBSDE_ESTATE).  Under these
 * coefficients x0 reaches u through every level's regression: the particles (X_k is coordinate-wise
 * affine in x0, with slope J_k = prod_i (1 + mu0 dt + sigma0 dW_i), regenerated beside the state), the mean
 * path (slope (1 + mu0 dt)^k) and the cloud variance V_k (bandwidth and ridge; its x0-derivative from
 * the moment recursion).  Per level the adjoint solves one more ridge system (CG) and differentiates the
 * design, the kernel weights (softmax) and the ridge; Z = sigma(X)^T alpha_x contributes per particle.
 * Outputs as fbsde_solve_backward: x0_bar [P][d], gp_bar [4], fp_bar [4] (summed over points), status
 * [P] (flags added).  The tape is consumed (a second call needs a new forward solve).  f kinds and terminal
 * values as fbsde_solve_coef.  With FBSDE_WS_TAPE, FBSDE_F32C and a rank-deficient design (M <= d + 1) the
 * taped forward and this call keep the state in FP64 (the adjoint's right-hand side reaches the design's
 * ridge-only null space, where FP32 rounding of the state comes back scaled by 1 / lambda); the workspace
 * size accounts for it. */
int fbsde_solve_coef_backward(const fbsde_problem* pb, const fbsde_coef* coef, int64_t P, const double* x0,
                              const double* u_bar, double* x0_bar, double* gp_bar, double* fp_bar,
                              uint32_t* status, void* ws, size_t ws_bytes, int32_t* cg_iters_out,
                              fbsde_stream stream);

/* Scheme R under a constant diffusion matrix (Sec. 2.1's problem class with matrix sigma; Z = sigma^T
 * grad u in the steps after the matrix-free solve): X_k = x0 + mu t_k + sigma W_k with sigma [d][d]
 * invertible (device, FP64, row-major) and pb->mu the constant drift (or NULL).  The regression of level k
 * uses the cloud's own metric: Gaussian weights exp(-D^T Sigma^{-1} D / (eps_h^2 d)) with Sigma =
 * t_{k+1} sigma sigma^T, the ridge lambda |sigma^T alpha_x|^2 with lambda = ridge_rel t_{k+1} on the
 * quantity the scheme uses (Z = sigma^T alpha_x), C = alpha + alpha_x . (X_k - x0 - mu t_k); both reduce
 * to fbsde_solve's at sigma = s I.  grad u(0, x0) = alpha_x / F'(u).  The library runs the per-point path in
 * the coordinates W = sigma^{-1} (X - x0 - mu t), where the weights and ridge are fbsde_solve's at s = 1
 * and the slope is Z; sigma enters the terminal values (sigma W_N on the matrix cores, point chunk by
 * chunk) and grad u = sigma^{-T} Z / F' (solved through sigma sigma^T, blocked Cholesky).
 * pb->s is not used; shared_dw, f kinds that read x and the Case 2 terminal value are refused
 * (FBSDE_EINVAL).  A sigma singular to working precision marks every point's status ST_NONFINITE
 * (grad NULL: not detected).  Workspace fbsde_sigma_workspace_size(pb, P, flags) bytes (the per-point
 * workspace plus at most 512 MiB of sigma W_N rows, the d x d factor and, with FBSDE_WS_TAPE, the
 * tape and P x M doubles for the reverse mode); flags 0 or FBSDE_WS_TAPE as fbsde_solve; u [P], grad [P][d]
 * or NULL, status [P], cg_iters_out as fbsde_solve, on stream.
 * fbsde_solve_sigma_backward: the reverse mode of L = sum_p u_bar[p] u_p (as fbsde_solve_backward, same
 * outputs and tape contract) after fbsde_solve_sigma with FBSDE_WS_TAPE on the same workspace and sigma.
 * x0 enters only through the terminal values, so x0_bar = sum_j G_j grad g(X^j_N) with G the adjoint of
 * the terminal values: the argument of g is formed again from sigma W_N (GEMM), and the W-column sums of
 * the radial terms are mapped to X by sigma (one more GEMM). */
int fbsde_sigma_workspace_size(const fbsde_problem* pb, int64_t P, int32_t flags, size_t* bytes);
int fbsde_solve_sigma(const fbsde_problem* pb, const double* sigma, int64_t P, const double* x0, double* u,
                      double* grad, uint32_t* status, void* ws, size_t ws_bytes, int32_t flags,
                      int32_t* cg_iters_out, fbsde_stream stream);
int fbsde_solve_sigma_backward(const fbsde_problem* pb, const double* sigma, int64_t P, const double* x0,
                               const double* u_bar, double* x0_bar, double* gp_bar, double* fp_bar,
                               uint32_t* status, void* ws, size_t ws_bytes, int32_t* cg_iters_out,
                               fbsde_stream stream);

/* Human-readable text of a return code. */
const char* fbsde_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* FBSDE_H */
