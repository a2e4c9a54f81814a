// Device-side conjugate-gradient loop of one backward level: every CG iteration of every point of the
// level in ONE launch, with no host round trip (the matrix-free product of the ridge normal equations,
// paper Sec. 2.4, matrix-free steps 1-2 fused into one read of the state, then the CG step).
//
// Work items are (point, chunk) pairs of the point's current iteration, kept in NQ <= 32 ring queues
// (point p in queue p mod NQ; block b's home queue is b mod NQ): the launch starts with every point's
// chunks of the first iteration in them, and the block that finishes a point's CG step enqueues that
// point's chunks of the next iteration (none once the point has converged).  A block streams its chunk of
// the point's particle rows (the same per-row work as k_matvec) and reports the chunk's partial column
// sums up a per-point arrival tree of fan-in CG_FAN.  The block that completes the root does the CG step
// of the point (the same arithmetic as k_cg_update, chunk partials summed in a fixed order) and publishes
// the point's new iteration count.
//
// Taking items: a block holds a ticket, an index of its home queue drawn with one fetch-and-add, and the
// item filled at that index is its next one.  Tickets may run ahead of the fill counter (the item comes
// with a later iteration).  A block whose ticket is not filled yet takes, now and then, an item nobody
// holds a ticket for (an index below a queue's fill counter, claimed with a compare-and-swap of the take
// counter), so the items of a queue whose home blocks are not resident (other kernels holding their
// compute units) still get done, and no block ever waits on a block that is not running.  Drawing
// tickets with fetch-and-add rather than claiming every item with compare-and-swap matters: with hundreds
// of blocks polling a few queues, the failed swaps of the losers delayed the winners (measured: 8 points
// at d = 5000, M = 4800 went 721 -> 369 ms per solve).  The loop is over when no point iterates any more:
// then no item can come (a point enqueues only while it iterates, and a point that iterates holds the
// count of iterating points above zero).  A queue holds a slot for every item the level can produce,
// (its points) x nchunk x (the iteration cap), each with a sequence number: slot j is free for index j when
// its number is j and filled when it is j + 1.  No slot is reused within a launch, and that is what keeps
// the loop free of deadlock: with a ring of (its points) x nchunk slots a producer had to wait until the
// index one lap earlier was taken, and that index could be the ticket of the producer itself (a block
// that took a stolen item while holding a ticket on the same queue, then completed that item's point) or
// of a block waiting, in turn, on this producer's own held ticket; both stalled until the wait bound
// (seen with 64 points of 6 chunks each, two points per queue).  Now a producer writes at once, and a
// block waits only for an item that a running producer is writing.  The waits are still bounded in
// wall-clock time (counted from the last time any queue counter moved): past the bound the loop winds
// down and the points still iterating are flagged FBSDE_ST_WAIT_LIMIT (an internal error, never
// expected).
//
// Coherence: the L2 caches of the XCDs are not coherent with each other within a kernel.  The data that
// blocks hand to one another inside the loop (chunk partials, the CG vectors and scalars of a point, the
// published state words) is therefore written and read only with agent-scope atomic accesses, which go to
// the coherence point, and a block publishes after every wave has waited for its own stores to complete
// (then a barrier, then the one atomic that hands over).  The streamed state, the weights and the vectors
// set before the launch are read with ordinary loads.  Agent-scope fences, which write back or invalidate
// a whole L2, are not used: measured, they cost more than the streaming itself.
#pragma once
#include "fbsde_rowteam.hpp"

namespace fbsde {

constexpr int CG_FAN = 8;                  // arrival-tree fan-in
enum { ST_WAIT_LIMIT = 8 };                // status bit: a bounded device-side wait gave up

// Control words of the device loop, in the workspace: the particle rows streamed by products since the
// last reset (algorithmic work for measurement), an error flag, and per queue its take and fill counters,
// each pair on a line of its own.
constexpr int CG_MAXQ = 32;
struct CgCtl {
    unsigned long long rows;
    unsigned long long bytes;            // the same rows x d x element bytes (algorithmic read traffic)
    int err;
    int pad[27];
    unsigned long long q[CG_MAXQ][16];   // [0] head (taken), [1] tail (filled)
};

// Number of arrival counters of one point (levels 1.. of the tree over nchunk leaves).
__host__ __device__ inline int cg_tree_counters(int nchunk) {
    int n = 0;
    for (int m = nchunk; m > 1;) {
        m = (m + CG_FAN - 1) / CG_FAN;
        n += m;
    }
    return n;
}

// coherent (agent-scope, relaxed) loads and stores of the data handed between blocks
__device__ __forceinline__ double ldc(const double* a) {
    return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void stc(double* a, double v) {
    __hip_atomic_store(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ldc(const int* a) {
    return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void stc(int* a, int v) {
    __hip_atomic_store(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Every wave's stores have completed at the coherence point, then the block meets: what one thread
// publishes after this is ordered after all of them.
__device__ __forceinline__ void stores_done_barrier() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __syncthreads();
}

// Before each loop: the queues filled with every point's chunks of the first iteration (slot j of queue
// q, at q * qcap + j, holds ((j + 1) << 32) | item, item = p * nchunk + c, j = (p / nq) * nchunk + c; a slot
// with no first item is free for index j: j << 32), no error, arrival counters 0, and the published state
// of each point (word 2 of iscal: iterations | done << 30) from the start kernel's done flag.
__global__ void __launch_bounds__(256)
k_cg_arm(CgCtl* ctl, unsigned long long* __restrict__ queue, int nq, int64_t qcap, int nchunk, int* __restrict__ cnt,
         int64_t ncnt_total, int* __restrict__ iscal, int64_t P, int reset_rows) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x, n = (int64_t)gridDim.x * blockDim.x;
    if (t == 0) {
        ctl->err = 0;
        if (reset_rows) {
            ctl->rows = 0ull;
            ctl->bytes = 0ull;
        }
        for (int q = 0; q < nq; ++q) {
            ctl->q[q][0] = 0ull;
            ctl->q[q][1] = (unsigned long long)(((P - q + nq - 1) / nq) * nchunk);
        }
    }
    for (int64_t i = t; i < (int64_t)nq * qcap; i += n) {
        const int64_t q = i / qcap, j = i - q * qcap;
        const int64_t p = q + (j / nchunk) * nq, c = j - (j / nchunk) * nchunk;
        queue[i] = (p < P) ? (((unsigned long long)(uint32_t)(j + 1) << 32) | (uint32_t)(p * nchunk + c))
                           : ((unsigned long long)(uint32_t)j << 32);
    }
    for (int64_t i = t; i < ncnt_total; i += n) cnt[i] = 0;
    for (int64_t p = t; p < P; p += n) iscal[p * 4 + 2] = iscal[p * 4 + 1] ? (1 << 30) : 0;
}

// Per-block combination of per-lane column accumulators into out[0..ld), written coherently (the
// counterpart of block_columns_out for partials another block reads within the same launch).
template <int Q, int TEAM, typename R>
__device__ __forceinline__ void block_columns_out_c(CSum<R> (&acc)[Q][4], double* lds, double* __restrict__ out,
                                                    int ld, int team, int L) {
    using G = Geo<Q, TEAM>;
    if constexpr (G::TPW == 1) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int e0 = 4 * (L + q * G::TL);
            if (e0 < ld) {
#pragma unroll
                for (int e = 0; e < 4; ++e) stc(out + e0 + e, acc[q][e].get());
            }
        }
    } else {
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
            stc(out + i, s);
        }
        __syncthreads();
    }
}

// Coherent loads that one thread issues back to back before it uses any of them: each loop below takes
// RU of its elements per round (RU2 where every element sums up to CG_FAN children), so a round costs
// one memory round trip instead of one per element.  Loads past the end of a vector or the last child
// re-read an element that exists and are not used.
// Kernels whose row registers already exceed what wider rounds take (eight groups of four per lane) use
// wider rounds, and 16-wave teams (128 registers at most) narrower ones: the rounds then add nothing to
// the kernel's register peak.
template <int Q, int TEAM> struct CgRounds {
    static constexpr int RU = (TEAM >= 16) ? 2 : (Q >= 8) ? 8 : 4;
    static constexpr int RU2 = (TEAM >= 16) ? 1 : (Q >= 8) ? 3 : 2;   // the same for sums of CG_FAN children
};

// The CG step of point p at iteration `it`, by the whole block, from the nchild partial vectors / tau
// partials at chunk slots k * stride (k < nchild, summed in that order).  Ends with the point's new state
// published (iterations | done << 30) and, while it iterates, its chunks of the next iteration enqueued.
template <int CG_RU, int CG_RU2>
__device__ __forceinline__ void cg_root_update(int p, int it, const double* __restrict__ part,
                                               const double* __restrict__ psc, int nchunk, int nchild, int stride,
                                               int ld, double s, const double* __restrict__ Wbar, double* __restrict__ x,
                                               double* __restrict__ r, double* __restrict__ pv, double* __restrict__ qv,
                                               double* __restrict__ scal, int ns, int* __restrict__ iscal, double rtol2,
                                               int maxit, int* active, uint32_t* __restrict__ status, double* lds,
                                               CgCtl* ctl, unsigned long long* __restrict__ queue,
                                               int nq, int64_t qcap, uint64_t wait_ticks) {
    double* sc = scal + (int64_t)p * ns;
    const double lam = sc[3];
    double tau = 0.0;
    {
        double t[CG_FAN];
#pragma unroll
        for (int k = 0; k < CG_FAN; ++k) t[k] = ldc(psc + (int64_t)p * nchunk + min(k, nchild - 1) * stride);
#pragma unroll
        for (int k = 0; k < CG_FAN; ++k)
            if (k < nchild) tau += t[k];
    }
    const int64_t o = (int64_t)p * ld;
    const int bs = blockDim.x;
    double pq = 0.0;
    for (int i0 = threadIdx.x; i0 < ld; i0 += CG_RU2 * bs) {
        double a[CG_RU2][CG_FAN], pw[CG_RU2];
#pragma unroll
        for (int u = 0; u < CG_RU2; ++u) {
            const int i = min(i0 + u * bs, ld - 1);
#pragma unroll
            for (int k = 0; k < CG_FAN; ++k)
                a[u][k] = ldc(part + ((int64_t)p * nchunk + min(k, nchild - 1) * stride) * ld + i);
            pw[u] = ldc(pv + o + i);
        }
#pragma unroll
        for (int u = 0; u < CG_RU2; ++u) {
            const int i = i0 + u * bs;
            if (i < ld) {
                double acc = 0.0;
#pragma unroll
                for (int k = 0; k < CG_FAN; ++k)
                    if (k < nchild) acc += a[u][k];
                const double q = s * (acc - tau * Wbar[o + i]) + lam * pw[u];
                stc(qv + o + i, q);
                pq += pw[u] * q;
            }
        }
    }
    pq = block_sum(pq, lds);
    const double rr = ldc(sc + 0);
    const double alpha = (pq > 0.0) ? rr / pq : 0.0;
    double rr2 = 0.0;
    for (int i0 = threadIdx.x; i0 < ld; i0 += CG_RU * bs) {
        double pw[CG_RU], xw[CG_RU], rw[CG_RU], qw[CG_RU];
#pragma unroll
        for (int u = 0; u < CG_RU; ++u) {
            const int i = min(i0 + u * bs, ld - 1);
            pw[u] = ldc(pv + o + i);
            xw[u] = ldc(x + o + i);
            rw[u] = ldc(r + o + i);
            qw[u] = ldc(qv + o + i);
        }
#pragma unroll
        for (int u = 0; u < CG_RU; ++u) {
            const int i = i0 + u * bs;
            if (i < ld) {
                stc(x + o + i, xw[u] + alpha * pw[u]);
                const double ri = rw[u] - alpha * qw[u];
                stc(r + o + i, ri);
                rr2 += ri * ri;
            }
        }
    }
    rr2 = block_sum(rr2, lds);
    const int itn = it + 1;
    int done = 0;
    uint32_t st = 0;
    if (!(pq > 0.0) || rr2 <= rtol2 * sc[1]) done = 1;
    else if (itn >= maxit) { done = 1; st = ST_CG_MAXIT; }
    double wv = 0.0;
    if (!done) {
        const double beta = rr2 / rr;
        for (int i0 = threadIdx.x; i0 < ld; i0 += CG_RU * bs) {
            double pw[CG_RU], rw[CG_RU];
#pragma unroll
            for (int u = 0; u < CG_RU; ++u) {
                const int i = min(i0 + u * bs, ld - 1);
                rw[u] = ldc(r + o + i);
                pw[u] = ldc(pv + o + i);
            }
#pragma unroll
            for (int u = 0; u < CG_RU; ++u) {
                const int i = i0 + u * bs;
                if (i < ld) {
                    const double pi = rw[u] + beta * pw[u];
                    stc(pv + o + i, pi);
                    wv += Wbar[o + i] * pi;
                }
            }
        }
        wv = block_sum(wv, lds);
    }
    if (threadIdx.x == 0) {
        stc(sc + 0, rr2);
        stc(sc + 2, wv);
        stc(iscal + p * 4 + 0, itn);
        stc(iscal + p * 4 + 1, done);
    }
    stores_done_barrier();
    __shared__ unsigned long long sh_base;
    const int qi = p % nq;
    if (threadIdx.x == 0) {
        if (st) atomicOr(&status[p], st);
        stc(iscal + p * 4 + 2, itn | (done << 30));
        if (done) atomicSub(active, 1);
        else sh_base = atomicAdd(&ctl->q[qi][1], (unsigned long long)nchunk);
    }
    if (!done) {
        // the point's chunks of the next iteration, after its new state is published (each slot is fresh:
        // the wait below ends at once unless the queue were too small, which the wait bound reports)
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        const unsigned long long b = sh_base;
        unsigned long long* qq = queue + (int64_t)qi * qcap;
        for (int k = threadIdx.x; k < nchunk; k += blockDim.x) {
            const unsigned long long j = b + (unsigned long long)k;
            unsigned long long* slot = qq + (j % (unsigned long long)qcap);
            const uint64_t t0 = wall_clock64();
            while ((uint32_t)(__hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> 32) !=
                   (uint32_t)j) {
                if (wall_clock64() - t0 > wait_ticks) {
                    atomicExch(&ctl->err, 1);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            __hip_atomic_store(slot, ((unsigned long long)(uint32_t)(j + 1) << 32) | (uint32_t)(p * nchunk + k),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// After the loop: the rows its products streamed (each point's iterations x M, summed per block, one atomic
// per block) and their bytes (row_bytes = d x element bytes), and, after a loop that gave up a bounded wait (an internal error), every point still
// iterating flagged.
__global__ void __launch_bounds__(256)
k_cg_check(CgCtl* ctl, const int* __restrict__ iscal, int64_t P, int64_t M, int64_t row_bytes,
           uint32_t* __restrict__ status) {
    __shared__ double lds[16];
    const int err = ctl->err;
    double rows = 0.0;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        rows += (double)iscal[p * 4 + 0] * (double)M;
        if (err && !(iscal[p * 4 + 2] >> 30)) status[p] |= (uint32_t)ST_WAIT_LIMIT;
    }
    rows = block_sum(rows, lds);
    if (threadIdx.x == 0 && rows > 0.0) {
        atomicAdd(&ctl->rows, (unsigned long long)rows);
        atomicAdd(&ctl->bytes, (unsigned long long)rows * (unsigned long long)row_bytes);
    }
}

// Waves per SIMD asked of the register allocator: the occupancy of the stand-alone product kernel
// where its row fits 128 registers without spilling (FP32 state and arithmetic, four groups per lane,
// one-wave teams: the d = 1000 shape).
template <typename S, typename R, int Q, int TEAM>
struct CgLoopWaves {
    static constexpr int value = (sizeof(S) == 4 && sizeof(R) == 4 && Q == 4 && TEAM == 1) ? 4 : 1;
};

template <typename S, typename R, int Q, int TEAM>
__global__ void __launch_bounds__((Geo<Q, TEAM>::BS)) __attribute__((amdgpu_waves_per_eu(CgLoopWaves<S, R, Q, TEAM>::value)))
k_cg_loop(const S* __restrict__ W, int64_t ldw, int M, int rows_per_chunk, int nchunk, int ld, double s,
          const double* __restrict__ w, const double* __restrict__ Wbar, double* __restrict__ x, double* __restrict__ r,
          double* __restrict__ pv, double* __restrict__ qv, double* __restrict__ scal, int ns, int* __restrict__ iscal,
          double* __restrict__ part, double* __restrict__ psc, CgCtl* ctl, unsigned long long* __restrict__ queue,
          int nq, int64_t qcap, int* active, int* __restrict__ cnt, int ncnt, double rtol2, int maxit,
          uint32_t* __restrict__ status, uint64_t wait_ticks) {
    using G = Geo<Q, TEAM>;
    __shared__ double lds[(G::TPW > 1) ? G::TPW * 4 * Q * G::TL : 1];
    __shared__ double red[2 * G::BS / 64 + 16];
    __shared__ int sh_flag;
    const int team0 = threadIdx.x / G::TL, L0 = threadIdx.x % G::TL;
    const int qi = blockIdx.x % nq;   // home queue
    long long tick = -1;               // the block's ticket on its home queue (wave 0), -1: none
    constexpr bool PF = G::BS < 1024 && !(sizeof(R) > sizeof(S) && Q == 8);
    for (;;) {
        // ------------------------------------------------------------ next work item
        if (threadIdx.x < 64) {
            // Wave 0 finds the block's next item.  The block holds a ticket, an index of its home queue
            // taken with one fetch-and-add (no retries however many blocks share the queue): the item
            // filled at that index is the block's.  A ticket may run ahead of the fill counter (the item
            // comes with a later iteration of a point of that queue); while it waits, the block takes
            // items nobody holds a ticket for (indices below a queue's fill counter, claimed with a
            // compare-and-swap of the take counter), so items of a queue whose blocks are not resident
            // still get done.  The loop is over when no point iterates any more: then no item can come
            // (a point enqueues only while it iterates, and a point that iterates holds the count above
            // zero).  The wait bound counts from the last time any queue counter moved.
            const int lane = threadIdx.x;
            int item = -1;   // -1: leave
            uint64_t t0 = wall_clock64();
            unsigned long long seen = ~0ull;
            for (int k = 0;; ++k) {
                if (tick < 0) {
                    unsigned long long t = 0;
                    if (lane == 0) t = atomicAdd(&ctl->q[qi][0], 1ull);
                    tick = (long long)__shfl(t, 0, 64);
                }
                unsigned long long* myslot = queue + (int64_t)qi * qcap + (int64_t)((unsigned long long)tick % (unsigned long long)qcap);
                const unsigned long long v = __hip_atomic_load(myslot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const int err = ldc(&ctl->err);
                const int act = ldc(active);
                if ((uint32_t)(v >> 32) == (uint32_t)(tick + 1)) {
                    item = (int)(uint32_t)v;
                    // taken: the slot is free for the index one ring later
                    if (lane == 0)
                        __hip_atomic_store(myslot, (unsigned long long)(uint32_t)(tick + qcap) << 32, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    tick = -1;
                    break;
                }
                if (err != 0) break;
                // every fourth round: lane q reads queue q's counters (one round trip for all queues), then
                // the block claims an unticketed item if there is one, home queue first
                if ((k & 3) == 3) {
                    unsigned long long h = 0, tl = 0;
                    if (lane < nq) {
                        h = __hip_atomic_load(&ctl->q[lane][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        tl = __hip_atomic_load(&ctl->q[lane][1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                    unsigned long long moved = 0, n = 0;
                    int qt = -1;
                    for (int j = 0; j < nq; ++j) {
                        const int q = (qi + j) % nq;
                        const unsigned long long hq = __shfl(h, q, 64);
                        const unsigned long long tq = __shfl(tl, q, 64);
                        moved += hq + tq;
                        if (qt < 0 && hq < tq) {
                            unsigned long long got = 0;
                            if (lane == 0) got = (atomicCAS(&ctl->q[q][0], hq, hq + 1ull) == hq) ? 1ull : 0ull;
                            if (__shfl(got, 0, 64)) {
                                n = hq;
                                qt = q;
                            }
                        }
                    }
                    if (qt >= 0) {
                        // below the fill counter: the producer has reserved the index and fills it shortly
                        if (lane == 0) {
                            unsigned long long* slot = queue + (int64_t)qt * qcap + (int64_t)(n % (unsigned long long)qcap);
                            const uint32_t want = (uint32_t)(n + 1);
                            const uint64_t t1 = wall_clock64();
                            for (;;) {
                                const unsigned long long w = __hip_atomic_load(slot, __ATOMIC_RELAXED,
                                                                               __HIP_MEMORY_SCOPE_AGENT);
                                if ((uint32_t)(w >> 32) == want) {
                                    item = (int)(uint32_t)w;
                                    __hip_atomic_store(slot,
                                                       (unsigned long long)(uint32_t)(n + (unsigned long long)qcap) << 32,
                                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                    break;
                                }
                                if (wall_clock64() - t1 > wait_ticks) {
                                    atomicExch(&ctl->err, 1);
                                    break;
                                }
                                __builtin_amdgcn_s_sleep(1);
                            }
                        }
                        item = __shfl(item, 0, 64);
                        break;
                    }
                    if (moved != seen) {
                        seen = moved;
                        t0 = wall_clock64();
                    } else if (wall_clock64() - t0 > wait_ticks) {
                        if (lane == 0) atomicExch(&ctl->err, 1);
                        break;
                    }
                }
                if (act <= 0) break;   // the level is over
                if (k < 16) __builtin_amdgcn_s_sleep(1);
                else __builtin_amdgcn_s_sleep(4);
            }
            if (lane == 0) sh_flag = item;
        }
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(sh_flag);
        if (item < 0) break;
        const int p = item / nchunk;
        const int c = item - p * nchunk;
        // the point's current iteration (stable while its items are outstanding); a point that had
        // converged before the loop started has its first items skipped
        const int sw = __builtin_amdgcn_readfirstlane(ldc(&iscal[p * 4 + 2]));
        if (sw >> 30) {
            __syncthreads();
            continue;
        }
        const int it = sw & 0x3FFFFFFF;
        // ------------------------------------------------------------ the chunk's share of the product
        // the lane's coordinates are re-derived per work item: an opaque copy keeps the compiler from
        // hoisting the per-lane addresses out of the loop, where they would hold registers throughout
        int team = team0, L = L0;
        asm volatile("" : "+v"(team), "+v"(L));
        const int r0 = c * rows_per_chunk;
        const int r1 = min(M, r0 + rows_per_chunk);
        R v[Q][4];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int e0 = 4 * (L + q * G::TL);
#pragma unroll
            for (int e = 0; e < 4; ++e) v[q][e] = (e0 < ld) ? (R)ldc(pv + (int64_t)p * ld + e0 + e) : (R)0;
        }
        const double wvp = ldc(scal + (int64_t)p * ns + 2);
        CSum<R> acc[Q][4];
        double tau = 0.0;
        const S* base = W + (int64_t)p * M * ldw;
        if constexpr (TEAM > 1 && G::BS <= 256) {
            // A team of two or four waves per row: every row's dot needs a team reduction (two barriers).
            // Two rows per step share one reduction, and both rows' loads are in flight together; the
            // rows and the sums keep the one-row order, so the result is the same.  Measured at 64
            // points: d = 5000 (four-wave teams) 3.9-4.25 -> 4.3-4.5 TB/s in the loop; with eight-wave
            // teams (d = 10^4, 512-thread blocks) the second row's registers cost more than the barrier
            // saves (4.2 -> 3.0 TB/s), so those keep one row per step.
            for (int jb = r0; jb < r1; jb += 2 * G::TPW) {
                const int j0 = jb + team, j1 = jb + G::TPW + team;
                const bool v0 = j0 < r1, v1 = j1 < r1;
                S xa[Q][4], xb[Q][4];
                if (v0) load_row<S, Q, G::TL>(base + (int64_t)j0 * ldw, ld, L, xa);
                if (v1) load_row<S, Q, G::TL>(base + (int64_t)j1 * ldw, ld, L, xb);
                CSum<R> d0, d1;
                if (v0) {
#pragma unroll
                    for (int q = 0; q < Q; ++q)
#pragma unroll
                        for (int e = 0; e < 4; ++e) d0.add((R)xa[q][e] * v[q][e]);
                }
                if (v1) {
#pragma unroll
                    for (int q = 0; q < Q; ++q)
#pragma unroll
                        for (int e = 0; e < 4; ++e) d1.add((R)xb[q][e] * v[q][e]);
                }
                double t0 = d0.get(), t1 = d1.get();
                team_sum2<TEAM>(t0, t1, red, team);
                if (v0) {
                    const double cj = w[(int64_t)p * M + j0] * s * (t0 - wvp);
                    tau += cj;
                    const R cr = (R)cj;
#pragma unroll
                    for (int q = 0; q < Q; ++q)
#pragma unroll
                        for (int e = 0; e < 4; ++e) acc[q][e].add(cr * (R)xa[q][e]);
                }
                if (v1) {
                    const double cj = w[(int64_t)p * M + j1] * s * (t1 - wvp);
                    tau += cj;
                    const R cr = (R)cj;
#pragma unroll
                    for (int q = 0; q < Q; ++q)
#pragma unroll
                        for (int e = 0; e < 4; ++e) acc[q][e].add(cr * (R)xb[q][e]);
                }
            }
        } else {
        S xr[Q][4];
        if (PF && r0 + team < r1) load_row<S, Q, G::TL>(base + (int64_t)(r0 + team) * ldw, ld, L, xr);
        for (int jb = r0; jb < r1; jb += G::TPW) {
            const int j = jb + team;
            const bool valid = j < r1;
            S xn[Q][4];
            if (PF) {
                if (j + G::TPW < r1) load_row<S, Q, G::TL>(base + (int64_t)(j + G::TPW) * ldw, ld, L, xn);
            } else if (valid) {
                load_row<S, Q, G::TL>(base + (int64_t)j * ldw, ld, L, xr);
            }
            CSum<R> dl;
            if (valid) {
#pragma unroll
                for (int q = 0; q < Q; ++q)
#pragma unroll
                    for (int e = 0; e < 4; ++e) dl.add((R)xr[q][e] * v[q][e]);
            }
            double tt = dl.get(), unused = 0.0;
            team_sum2<TEAM>(tt, unused, red, team);
            if (valid) {
                const double cj = w[(int64_t)p * M + j] * s * (tt - wvp);
                tau += cj;
                const R cr = (R)cj;
#pragma unroll
                for (int q = 0; q < Q; ++q)
#pragma unroll
                    for (int e = 0; e < 4; ++e) acc[q][e].add(cr * (R)xr[q][e]);
            }
            if (PF) {
#pragma unroll
                for (int q = 0; q < Q; ++q)
#pragma unroll
                    for (int e = 0; e < 4; ++e) xr[q][e] = xn[q][e];
            }
        }
        }
        block_columns_out_c<Q, TEAM, R>(acc, lds, part + ((int64_t)p * nchunk + c) * ld, ld, team, L);
        const double tot = block_sum((L == 0) ? tau : 0.0, red);
        if (threadIdx.x == 0) stc(psc + (int64_t)p * nchunk + c, tot);
        // ------------------------------------------------------------ climb the arrival tree
        int node = c, n_l = nchunk, base_c = 0, stride = 1;
        for (;;) {
            stores_done_barrier();   // this block's partials are complete before it reports them
            if (n_l == 1) {          // a single chunk: this block holds the whole product
                cg_root_update<CgRounds<Q, TEAM>::RU, CgRounds<Q, TEAM>::RU2>(p, it, part, psc, nchunk, 1, stride, ld, s, Wbar, x, r, pv, qv, scal, ns, iscal,
                               rtol2, maxit, active, status, red, ctl, queue, nq, qcap, wait_ticks);
                break;
            }
            const int parent = node / CG_FAN;
            const int nchild = min(CG_FAN, n_l - parent * CG_FAN);
            if (threadIdx.x == 0) {
                int* ctr = cnt + (int64_t)p * ncnt + base_c + parent;
                const int old = atomicAdd(ctr, 1);
                const int last = (old == nchild - 1) ? 1 : 0;
                if (last) stc(ctr, 0);   // ready for the next iteration (reached only after this update)
                sh_flag = last;
            }
            __syncthreads();
            if (!__builtin_amdgcn_readfirstlane(sh_flag)) break;
            const int n_up = (n_l + CG_FAN - 1) / CG_FAN;
            const int cstride = stride;                  // children at slots (parent * FAN + k) * cstride
            const int pslot = parent * CG_FAN * cstride;
            if (n_up == 1) {
                cg_root_update<CgRounds<Q, TEAM>::RU, CgRounds<Q, TEAM>::RU2>(p, it, part + (int64_t)pslot * ld, psc + pslot, nchunk, nchild, cstride, ld, s,
                               Wbar, x, r, pv, qv, scal, ns, iscal, rtol2, maxit, active, status, red, ctl, queue,
                               nq, qcap, wait_ticks);
                break;
            }
            // sum the children into the first child's slot, which is the parent's slot one level up
            double* dst = part + ((int64_t)p * nchunk + pslot) * ld;
            constexpr int CG_RU2 = CgRounds<Q, TEAM>::RU2;
            for (int i0 = threadIdx.x; i0 < ld; i0 += CG_RU2 * (int)blockDim.x) {
                double a[CG_RU2][CG_FAN];
#pragma unroll
                for (int u = 0; u < CG_RU2; ++u) {
                    const int i = min(i0 + u * (int)blockDim.x, ld - 1);
#pragma unroll
                    for (int k = 0; k < CG_FAN; ++k) a[u][k] = ldc(dst + (int64_t)min(k, nchild - 1) * cstride * ld + i);
                }
#pragma unroll
                for (int u = 0; u < CG_RU2; ++u) {
                    const int i = i0 + u * (int)blockDim.x;
                    if (i < ld) {
                        double acc = 0.0;
#pragma unroll
                        for (int k = 0; k < CG_FAN; ++k)
                            if (k < nchild) acc += a[u][k];
                        stc(dst + i, acc);
                    }
                }
            }
            if (threadIdx.x == 0) {
                double a = 0.0;
                for (int k = 0; k < nchild; ++k) a += ldc(psc + (int64_t)p * nchunk + pslot + k * cstride);
                stc(psc + (int64_t)p * nchunk + pslot, a);
            }
            node = parent;
            base_c += n_up;
            n_l = n_up;
            stride *= CG_FAN;
        }
        __syncthreads();
    }
}

}  // namespace fbsde
