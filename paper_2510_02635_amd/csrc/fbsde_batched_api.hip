// Host side of the batched solve of many instances.
//  Tiled (default): the work items are (instance, point-tile) pairs, each run through the whole level
//    chain by the multi-block path of fbsde_solve (every point split over many workgroups along its
//    particle rows), dealt to a pool of HIP streams that each own a workspace arena.  Tiles are sized to
//    the arena, taken largest first, and overlap on the chip across the streams; the call only enqueues.
//  Persistent: one launch per geometry class; every workgroup pulls (instance, point) items from an
//    atomic queue and runs the whole chain of its point alone.
#include "fbsde_host.hpp"
#include "fbsde_batched.hpp"

#include <algorithm>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

using namespace fbsde;
using namespace fbsde::host;

namespace {

// ------------------------------------------------------------------ persistent batched launch
SlotLayout slot_layout(int64_t M, int ld, size_t esz) {
    SlotLayout lay;
    size_t off = (size_t)round_up((int64_t)(M * ld * esz), 256);
    lay.off_rn2 = off; off += (size_t)round_up(M * 8, 256);
    lay.off_Y = off; off += (size_t)round_up(M * 8, 256);
    lay.off_w = off; off += (size_t)round_up(M * 8, 256);
    lay.off_c2 = off; off += (size_t)round_up(M * 8, 256);
    lay.off_vec = off; off += (size_t)round_up(6 * (int64_t)ld * 8, 256);
    lay.bytes = off;
    return lay;
}

// The persistent kernel keeps a whole point's chain in one function, so its registers are sized by the
// largest phase: prefer wider teams over more groups per lane (at most 4 groups of 4 per lane).
void batch_geometry(Plan& pl) {
    while (pl.Q > 4 && pl.TEAM < 16) {
        pl.TEAM *= 2;
        const int groups = pl.ld / 4;
        const int q = (groups + 64 * pl.TEAM - 1) / (64 * pl.TEAM);
        pl.Q = (q <= 1) ? 1 : (q <= 2) ? 2 : (q <= 4) ? 4 : 8;
    }
    pl.BS = 64 * std::max(pl.TEAM, 4);
    pl.TPW = pl.BS / (64 * pl.TEAM);
}

struct BatchClass {
    int prec, Q, TEAM;
    bool r64 = false;         // FP32C with a rank-deficient centred design (M <= d + 1): FP64 arithmetic
    std::vector<int> insts;   // instance indices, by decreasing per-point cost
    int64_t items = 0;
    int64_t maxM = 0;
    int ld = 0;
};

int batch_classes(const fbsde_problem* pbs, int64_t n_inst, const int64_t* P, std::vector<BatchClass>& out) {
    std::map<std::tuple<int, int, int, int, int>, BatchClass> cls;
    for (int64_t i = 0; i < n_inst; ++i) {
        int rc = check_problem(&pbs[i], P[i]);
        if (rc) return rc;
        if (pbs[i].shared_dw || per_point_forward_only(&pbs[i])) return FBSDE_EINVAL;
        Plan pl;
        if ((rc = make_plan(&pbs[i], 1, pl))) return rc;
        batch_geometry(pl);
        const bool r64 = pbs[i].prec == FBSDE_F32C && pbs[i].M <= pbs[i].d + 1;
        const auto key = std::make_tuple(pbs[i].prec, (int)r64, pl.Q, pl.TEAM, pl.ld);
        BatchClass& c = cls[key];
        c.prec = pbs[i].prec; c.Q = pl.Q; c.TEAM = pl.TEAM; c.ld = pl.ld; c.r64 = r64;
        c.insts.push_back((int)i);
        c.items += P[i];
        c.maxM = std::max<int64_t>(c.maxM, pbs[i].M);
    }
    for (auto& kv : cls) {
        BatchClass& c = kv.second;
        std::stable_sort(c.insts.begin(), c.insts.end(), [&](int a, int b) { return pbs[a].M > pbs[b].M; });
        out.push_back(c);
    }
    return FBSDE_OK;
}

size_t batch_header_bytes(int64_t n_inst, int64_t total_items) {
    return (size_t)round_up(n_inst * (int64_t)sizeof(BatchInst), 256) +
           (size_t)round_up(total_items * (int64_t)sizeof(BatchItem), 256) + 256;
}

template <typename S>
void launch_batched_class(const BatchClass& c, const BatchInst* d_insts, const BatchItem* d_items, int n_items,
                          int* queue, char* slots, const SlotLayout& lay, int nslots, hipStream_t st) {
    set_int(queue, 0, st);
    dispatch<S>(c.Q, c.TEAM, [&](auto qc, auto tc) {
        constexpr int QQ = decltype(qc)::value, TT = decltype(tc)::value;
        if (c.r64)
            hipLaunchKernelGGL((k_batched<S, double, QQ, TT>), dim3(nslots), dim3(Geo<QQ, TT>::BS), 0, st, d_insts,
                               d_items, n_items, queue, slots, lay);
        else
            hipLaunchKernelGGL((k_batched<S, S, QQ, TT>), dim3(nslots), dim3(Geo<QQ, TT>::BS), 0, st, d_insts,
                               d_items, n_items, queue, slots, lay);
    });
}


// ------------------------------------------------------------------ tiled scheduler
struct TileUnit {
    int inst;
    int64_t p0, np;
    double cost;
};

struct Opts {
    int mode, streams, max_slots;
    size_t tile_bytes;
};

int read_opts(const fbsde_batch_opts* o, Opts& r) {
    r.mode = o ? o->mode : FBSDE_BATCH_TILED;
    // three streams by default: with HIP's default of four hardware queues per process and one taken by
    // the caller's stream, a fourth pool stream shares a queue and waits behind another (measured on
    // 64 uneven instances x 8 points, forward: 13.7 s on three streams, 14.8 s on four)
    r.streams = (o && o->streams) ? o->streams : 3;
    r.max_slots = (o && o->max_slots) ? o->max_slots : 512;
    r.tile_bytes = (o && o->tile_bytes) ? (size_t)o->tile_bytes : ((size_t)24 << 30);
    if (r.mode != FBSDE_BATCH_TILED && r.mode != FBSDE_BATCH_PERSISTENT) return FBSDE_EINVAL;
    if (r.streams < 1 || r.streams > 8 || r.max_slots < 1 || (o && o->tile_bytes < 0)) return FBSDE_EINVAL;
    if (o && o->reserved != 0) return FBSDE_EINVAL;
    return FBSDE_OK;
}

// Expected time of a tile, in state bytes streamed: per level the moments pass, the reversal (read and
// write) and the CG products.  The CG iteration count is estimated from the condition number of the
// centred ridge system of an isotropic cloud: the Marchenko-Pastur edges (1 -+ sqrt(r))^2 with
// r = min(d, M) / max(d, M), the smallest eigenvalue held above a floor set by the ridge (relative to the
// spread s^2 t of the cloud); CG reaches a relative residual rtol in about sqrt(kappa) ln(2 / rtol) / 2 iterations.
double tile_cost(const fbsde_problem& pb, const Plan& pl, int64_t m) {
    const double r = (double)std::min(pb.d, pb.M) / (double)std::max(pb.d, pb.M);
    const double hi = (1.0 + std::sqrt(r)) * (1.0 + std::sqrt(r));
    // the floor is four times the ridge: with the ridge itself the estimate overshot the measured CG
    // counts of near-square designs about twice (0.44-0.57 of it, against 0.7-0.8 elsewhere; 64 HJB
    // instances x 8 points), which skewed the dealing (forward 13.7-13.8 s, with the floor 13.6 s)
    const double lo = std::max((1.0 - std::sqrt(r)) * (1.0 - std::sqrt(r)), 4.0 * std::max(pb.ridge_rel, 1e-6));
    const double rtol = std::max(cg_rtol_of(&pb), 1e-16);
    const double iters = std::min((double)pb.cg_maxit, 3.0 + 0.5 * std::sqrt(hi / lo) * std::log(2.0 / rtol));
    return (double)m * (double)pb.M * (double)pl.ld * (double)pl.esz * (double)pb.N * (3.0 + iters);
}

// Point tiles of every instance: the largest tile whose workspace fits the arena cap (at least one
// point, at most 65535), then equal tiles; largest cost (points x particle rows x row bytes) first.
int plan_tiles(const fbsde_problem* pbs, int64_t n_inst, const int64_t* P, const Opts& o, int32_t flags,
               std::vector<TileUnit>& units, size_t& arena) {
    units.clear();
    arena = 0;
    for (int64_t i = 0; i < n_inst; ++i) {
        int rc = check_problem(&pbs[i], 0);
        if (rc) return rc;
        if (P[i] < 0) return FBSDE_EINVAL;
        if (P[i] == 0) continue;
        auto ws_of = [&](int64_t np, size_t& b) { return fbsde_workspace_size(&pbs[i], np, flags, &b); };
        int64_t lo = 1, hi = std::min<int64_t>(P[i], 65535);
        size_t b = 0;
        if ((rc = ws_of(hi, b))) return rc;
        if (b > o.tile_bytes) {
            while (lo < hi) {   // largest np in [1, hi) that fits
                const int64_t mid = (lo + hi + 1) / 2;
                if ((rc = ws_of(mid, b))) return rc;
                if (b <= o.tile_bytes) lo = mid; else hi = mid - 1;
            }
            hi = lo;
        }
        const int64_t ntiles = (P[i] + hi - 1) / hi;
        const int64_t np = (P[i] + ntiles - 1) / ntiles;
        Plan pl;
        if ((rc = make_plan(&pbs[i], 1, pl))) return rc;
        for (int64_t p0 = 0; p0 < P[i]; p0 += np) {
            const int64_t m = std::min<int64_t>(np, P[i] - p0);
            if ((rc = ws_of(m, b))) return rc;
            arena = std::max(arena, (size_t)round_up((int64_t)b, 256));
            units.push_back(TileUnit{(int)i, p0, m, tile_cost(pbs[i], pl, m)});
        }
    }
    std::stable_sort(units.begin(), units.end(), [](const TileUnit& a, const TileUnit& b) { return a.cost > b.cost; });
    return FBSDE_OK;
}

// Header of the tiled schedule's workspace: per tile its 8 parameter adjoints, then one counter per stream
// of the algorithmic bytes its tiles' CG products streamed.
size_t tiled_header_bytes(size_t n_units) {
    return (size_t)round_up((int64_t)(n_units * 8 * sizeof(double) + 8 * sizeof(unsigned long long)), 256);
}
unsigned long long* tiled_cg_counters(char* base, size_t n_units) {
    return (unsigned long long*)(base + n_units * 8 * sizeof(double));
}

__global__ void k_zero_u64(unsigned long long* a, int n) {
    if (threadIdx.x < n) a[threadIdx.x] = 0ull;
}
__global__ void k_add_u64(unsigned long long* acc, const unsigned long long* v) {
    if (threadIdx.x == 0) *acc += *v;
}

int tiled_size(const fbsde_problem* pbs, int64_t n_inst, const int64_t* P, const Opts& o, int32_t flags,
               size_t* bytes, std::vector<TileUnit>* keep = nullptr, size_t* arena_out = nullptr, int* nw_out = nullptr) {
    std::vector<TileUnit> units;
    size_t arena = 0;
    int rc = plan_tiles(pbs, n_inst, P, o, flags, units, arena);
    if (rc) return rc;
    const int nw = (int)std::min<int64_t>(o.streams, std::max<int64_t>(1, (int64_t)units.size()));
    *bytes = tiled_header_bytes(units.size()) + (size_t)nw * arena;
    if (keep) *keep = std::move(units);
    if (arena_out) *arena_out = arena;
    if (nw_out) *nw_out = nw;
    return FBSDE_OK;
}

// Parameter adjoints of an instance: the sum of its tiles' sums, in tile order.  The tile indices come
// as a kernel argument (so a captured graph holds them): up to TILE_LIST per launch, later launches of
// the same instance adding to the first.
constexpr int TILE_LIST = 30;
struct TileList {
    int n;
    int idx[TILE_LIST];
};
__global__ void k_sum_tiles(const double* __restrict__ part, TileList tl, int accumulate, double* gp_bar,
                            double* fp_bar) {
    const int t = threadIdx.x;
    if (t >= 8) return;
    double* out = (t < 4) ? gp_bar + t : fp_bar + (t - 4);
    double v = accumulate ? *out : 0.0;
    for (int k = 0; k < tl.n; ++k) v += part[(int64_t)tl.idx[k] * 8 + t];
    *out = v;
}

// The streams and events the tiled schedule forks onto, created once per device and kept for the life of
// the process (a captured graph can then fork onto them too).  A mutex serialises the enqueueing of
// concurrent calls on one device; their tiles then queue up on the same streams.
constexpr int POOL_STREAMS = 8;
struct TiledPool {
    hipStream_t s[POOL_STREAMS];
    hipEvent_t fork;
    hipEvent_t join[POOL_STREAMS];
};
std::mutex g_pool_mu;
std::map<int, TiledPool> g_pool;

int tiled_pool(int dev, TiledPool*& out) {   // call with g_pool_mu held
    auto it = g_pool.find(dev);
    if (it != g_pool.end()) {
        out = &it->second;
        return FBSDE_OK;
    }
    TiledPool tp;
    if (hipEventCreateWithFlags(&tp.fork, hipEventDisableTiming) != hipSuccess) return FBSDE_EHIP;
    for (int w = 0; w < POOL_STREAMS; ++w)
        if (hipStreamCreateWithFlags(&tp.s[w], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&tp.join[w], hipEventDisableTiming) != hipSuccess)
            return FBSDE_EHIP;
    out = &(g_pool[dev] = tp);
    return FBSDE_OK;
}

struct TiledArgs {
    const fbsde_problem* pbs;
    const double* const* x0;
    double* const* u;
    double* const* grad;
    uint32_t* const* status;
    const double* const* u_bar;      // adjoint only
    double* const* x0_bar;
    double* const* gp_bar;
    double* const* fp_bar;
};

// Enqueue the whole tiled schedule: the pool's streams wait for the caller's stream, each takes its tiles
// in turn (every level's CG one device-side loop launch, so no call waits for the device), and the
// caller's stream then waits for every stream.  Nothing synchronises with the host: the call returns once
// the work is enqueued, and it can be captured into a graph.
int run_tiled(const TiledArgs& a, int64_t n_inst, const int64_t* P, const Opts& o, bool adjoint, void* wsp,
              size_t ws_bytes, hipStream_t caller) {
    const int32_t flags = adjoint ? FBSDE_WS_TAPE : 0;
    std::vector<TileUnit> units;
    size_t need = 0, arena = 0;
    int nw = 1;
    int rc = tiled_size(a.pbs, n_inst, P, o, flags, &need, &units, &arena, &nw);
    if (rc) return rc;
    if (need > ws_bytes) return FBSDE_ENOSPC;
    if (units.empty()) {   // every instance is empty: its parameter adjoints are zero sums
        if (adjoint)
            for (int64_t i = 0; i < n_inst; ++i)
                hipLaunchKernelGGL(k_sum_tiles, dim3(1), dim3(64), 0, caller, nullptr, TileList{0, {}}, 0,
                                   a.gp_bar[i], a.fp_bar[i]);
        return last_error();
    }
    char* base = (char*)wsp;
    double* tpart = (double*)base;   // [units][8]: gp_bar, fp_bar of each tile
    unsigned long long* cgc = tiled_cg_counters(base, units.size());
    char* arenas = base + tiled_header_bytes(units.size());
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return FBSDE_EHIP;
    std::lock_guard<std::mutex> lk(g_pool_mu);
    TiledPool* pool = nullptr;
    if ((rc = tiled_pool(dev, pool))) return rc;
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, caller, cgc, 8);
    if (hipEventRecord(pool->fork, caller) != hipSuccess) return FBSDE_EHIP;
    // The tiles are dealt to the streams up front: largest expected time first, each to the stream with
    // the least time so far.
    std::vector<std::vector<int>> deal((size_t)nw);
    {
        std::vector<double> load((size_t)nw, 0.0);
        for (size_t k = 0; k < units.size(); ++k) {
            const size_t w = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
            deal[w].push_back((int)k);
            load[w] += units[k].cost;
        }
    }
    // the streams' CG loops share the chip instead of each asking for all of it: each asks for half
    // (measured on 64 uneven instances x 8 points over four streams: a quarter 20.2 s, half 15.2 s,
    // all 18.0 s; blocks of a loop that cannot start wait until another stream's loop ends)
    struct ShareScope {
        explicit ShareScope(int n) { loop_share = n; }
        ~ShareScope() { loop_share = 1; }
    } share_scope(std::min(nw, 2));
    for (int w = 0; w < nw; ++w)
        if (hipStreamWaitEvent(pool->s[w], pool->fork, 0) != hipSuccess) return FBSDE_EHIP;
    // Tiles are enqueued round-robin over the streams, one tile per stream in turn: a launch blocks the
    // host once its stream holds as many commands as the runtime queues, and enqueueing one stream's
    // whole list first kept the other streams empty meanwhile (measured on 64 uneven instances x 8 points
    // over four streams: 20.1 s stream by stream, 15.4 s round-robin, forward).
    size_t rounds = 0;
    for (const auto& l : deal) rounds = std::max(rounds, l.size());
    for (size_t r = 0; r < rounds; ++r)
        for (int w = 0; w < nw; ++w) {
            if (r >= deal[(size_t)w].size()) continue;
            hipStream_t s = pool->s[w];
            char* ar = arenas + (size_t)w * arena;
            const int k = deal[(size_t)w][r];
            const TileUnit& t = units[(size_t)k];
            const int i = t.inst;
            fbsde_problem pb = a.pbs[i];
            pb.point_base = (uint32_t)(pb.point_base + (uint32_t)t.p0);
            const int64_t d = pb.d;
            const double* x0 = a.x0[i] + t.p0 * d;
            double* u = a.u[i] + t.p0;
            double* g = a.grad && a.grad[i] ? a.grad[i] + t.p0 * d : nullptr;
            uint32_t* st = a.status[i] + t.p0;
            int e = solve_tile(&pb, t.np, x0, u, g, st, ar, arena, flags, true, s);
            if (!e && adjoint)
                e = solve_backward_after_forward(&pb, t.np, x0, a.u_bar[i] + t.p0, a.x0_bar[i] + t.p0 * d,
                                                 tpart + (size_t)k * 8, tpart + (size_t)k * 8 + 4, st, ar, arena, s);
            // the tile's CG traffic (forward and reverse), counted in the arena's loop control
            if (!e && !pb.shared_dw) hipLaunchKernelGGL(k_add_u64, dim3(1), dim3(64), 0, s, cgc + w, cg_bytes_counter(ar));
            if (e) return e;
        }
    for (int w = 0; w < nw; ++w)
        if (hipEventRecord(pool->join[w], pool->s[w]) != hipSuccess ||
            hipStreamWaitEvent(caller, pool->join[w], 0) != hipSuccess)
            return FBSDE_EHIP;
    if (adjoint) {
        // per instance, its tiles in point order, summed by launches that carry the indices
        std::vector<std::vector<std::pair<int64_t, int>>> by_inst((size_t)n_inst);
        for (size_t k = 0; k < units.size(); ++k) by_inst[(size_t)units[k].inst].emplace_back(units[k].p0, (int)k);
        for (int64_t i = 0; i < n_inst; ++i) {
            auto& v = by_inst[(size_t)i];
            std::sort(v.begin(), v.end());
            size_t k0 = 0;
            do {
                TileList tl{0, {}};
                for (; k0 < v.size() && tl.n < TILE_LIST; ++k0) tl.idx[tl.n++] = v[k0].second;
                hipLaunchKernelGGL(k_sum_tiles, dim3(1), dim3(64), 0, caller, tpart, tl,
                                   (k0 > (size_t)tl.n) ? 1 : 0, a.gp_bar[i], a.fp_bar[i]);
            } while (k0 < v.size());
        }
    }
    return last_error();
}

int persistent_size(const fbsde_problem* pbs, int64_t n_inst, const int64_t* P, int32_t max_slots, size_t* bytes) {
    std::vector<BatchClass> cls;
    int rc = batch_classes(pbs, n_inst, P, cls);
    if (rc) return rc;
    int64_t total = 0;
    size_t slot_max = 0;
    for (const auto& c : cls) {
        total += c.items;
        const SlotLayout lay = slot_layout(c.maxM, c.ld, c.prec == FBSDE_F64 ? 8 : 4);
        slot_max = std::max(slot_max, lay.bytes * (size_t)std::min<int64_t>(c.items, max_slots));
    }
    *bytes = batch_header_bytes(n_inst, total) + slot_max;
    return FBSDE_OK;
}

int run_persistent(const fbsde_problem* pbs, int64_t n_inst, const int64_t* P, const double* const* x0,
                   double* const* u, double* const* grad, uint32_t* const* status, int32_t max_slots, void* wsp,
                   size_t ws_bytes, hipStream_t st) {
    std::vector<BatchClass> cls;
    int rc = batch_classes(pbs, n_inst, P, cls);
    if (rc) return rc;
    size_t need = 0;
    if ((rc = persistent_size(pbs, n_inst, P, max_slots, &need))) return rc;
    if (need > ws_bytes) return FBSDE_ENOSPC;
    for (int64_t i = 0; i < n_inst; ++i)
        if (P[i] > 0 && (!x0[i] || !u[i] || !status[i])) return FBSDE_EINVAL;
    // descriptor table and the work items of every class (device copies in the workspace header)
    std::vector<BatchInst> hi((size_t)n_inst);
    for (int64_t i = 0; i < n_inst; ++i) {
        const fbsde_problem* pb = &pbs[i];
        Plan pl;
        make_plan(pb, 1, pl);
        batch_geometry(pl);
        const Keys ky = keys_of(pb);
        BatchInst& b = hi[(size_t)i];
        b.d = (int)pb->d; b.ld = pl.ld; b.M = (int)pb->M; b.N = (int)pb->N; b.P = (int)P[i];
        b.T = pb->T; b.s = pb->s; b.eps_h = pb->eps_h; b.ridge_rel = pb->ridge_rel;
        b.rtol2 = cg_rtol_of(pb) * cg_rtol_of(pb);
        b.newton_iters = pb->newton_iters;
        b.cg_maxit = pb->cg_fixed_iters > 0 ? pb->cg_fixed_iters : pb->cg_maxit;
        b.g_kind = pb->g_kind;
        b.warm = (pb->M > pb->d + 1) ? 1 : 0;
        b.f = fspec_of(pb);
        b.ga = pb->gp[0]; b.gb = pb->gp[1];
        b.mu = pb->mu; b.gvec = pb->gvec;
        b.k0 = ky.k0; b.k1 = ky.k1; b.point_base = pb->point_base;
        b.x0 = x0[i]; b.u = u[i]; b.grad = grad ? grad[i] : nullptr; b.status = status[i];
        clear_status(status[i], P[i], st);
    }
    std::vector<BatchItem> items;
    std::vector<std::pair<int64_t, int64_t>> ranges;   // per class: [first item, count)
    for (const auto& c : cls) {
        const int64_t first = (int64_t)items.size();
        for (int i : c.insts)
            for (int64_t p = 0; p < P[i]; ++p) items.push_back(BatchItem{i, (int)p});
        ranges.emplace_back(first, (int64_t)items.size() - first);
    }
    char* base = (char*)wsp;
    BatchInst* d_insts = (BatchInst*)base;
    BatchItem* d_items = (BatchItem*)(base + round_up(n_inst * (int64_t)sizeof(BatchInst), 256));
    int* queue = (int*)(base + batch_header_bytes(n_inst, (int64_t)items.size()) - 256);
    char* slots = base + batch_header_bytes(n_inst, (int64_t)items.size());
    if (hipMemcpyAsync(d_insts, hi.data(), hi.size() * sizeof(BatchInst), hipMemcpyHostToDevice, st) != hipSuccess)
        return FBSDE_EHIP;
    if (!items.empty() &&
        hipMemcpyAsync(d_items, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice, st) != hipSuccess)
        return FBSDE_EHIP;
    // the host tables must outlive the copies
    if (hipStreamSynchronize(st) != hipSuccess) return FBSDE_EHIP;
    for (size_t ci = 0; ci < cls.size(); ++ci) {
        const BatchClass& c = cls[ci];
        if (ranges[ci].second == 0) continue;
        const SlotLayout lay = slot_layout(c.maxM, c.ld, c.prec == FBSDE_F64 ? 8 : 4);
        const int nslots = (int)std::min<int64_t>(ranges[ci].second, max_slots);
        if (c.prec == FBSDE_F64)
            launch_batched_class<double>(c, d_insts, d_items + ranges[ci].first, (int)ranges[ci].second, queue, slots,
                                         lay, nslots, st);
        else
            launch_batched_class<float>(c, d_insts, d_items + ranges[ci].first, (int)ranges[ci].second, queue, slots,
                                        lay, nslots, st);
        if ((rc = last_error())) return rc;
    }
    return FBSDE_OK;
}

}  // namespace

extern "C" {

int fbsde_batched_workspace_size(const fbsde_problem* pbs, int64_t n_inst, const int64_t* P,
                                 const fbsde_batch_opts* opts, int32_t adjoint, size_t* bytes) {
    if (!pbs || !P || !bytes || n_inst < 1 || (adjoint != 0 && adjoint != 1)) return FBSDE_EINVAL;
    Opts o;
    int rc = read_opts(opts, o);
    if (rc) return rc;
    if (o.mode == FBSDE_BATCH_PERSISTENT) {
        if (adjoint) return FBSDE_EINVAL;
        return persistent_size(pbs, n_inst, P, o.max_slots, bytes);
    }
    return tiled_size(pbs, n_inst, P, o, adjoint ? FBSDE_WS_TAPE : 0, bytes);
}

int fbsde_solve_batched(const fbsde_problem* pbs, int64_t n_inst, const int64_t* P, const double* const* x0,
                        double* const* u, double* const* grad, uint32_t* const* status, const fbsde_batch_opts* opts,
                        void* wsp, size_t ws_bytes, fbsde_stream stream) {
    if (!pbs || !P || !x0 || !u || !status || !wsp || n_inst < 1) return FBSDE_EINVAL;
    Opts o;
    int rc = read_opts(opts, o);
    if (rc) return rc;
    for (int64_t i = 0; i < n_inst; ++i)
        if (P[i] > 0 && (!x0[i] || !u[i] || !status[i])) return FBSDE_EINVAL;
    if (o.mode == FBSDE_BATCH_PERSISTENT)
        return run_persistent(pbs, n_inst, P, x0, u, grad, status, o.max_slots, wsp, ws_bytes, (hipStream_t)stream);
    TiledArgs a{pbs, x0, u, grad, status, nullptr, nullptr, nullptr, nullptr};
    return run_tiled(a, n_inst, P, o, false, wsp, ws_bytes, (hipStream_t)stream);
}

int fbsde_solve_batched_backward(const fbsde_problem* pbs, int64_t n_inst, const int64_t* P,
                                 const double* const* x0, const double* const* u_bar, double* const* u,
                                 double* const* x0_bar, double* const* gp_bar, double* const* fp_bar,
                                 uint32_t* const* status, const fbsde_batch_opts* opts, void* wsp, size_t ws_bytes,
                                 fbsde_stream stream) {
    if (!pbs || !P || !x0 || !u_bar || !u || !x0_bar || !gp_bar || !fp_bar || !status || !wsp || n_inst < 1)
        return FBSDE_EINVAL;
    Opts o;
    int rc = read_opts(opts, o);
    if (rc) return rc;
    if (o.mode != FBSDE_BATCH_TILED) return FBSDE_EINVAL;
    for (int64_t i = 0; i < n_inst; ++i)
        if ((P[i] > 0 && (!x0[i] || !u_bar[i] || !u[i] || !x0_bar[i] || !status[i])) || !gp_bar[i] || !fp_bar[i])
            return FBSDE_EINVAL;
    TiledArgs a{pbs, x0, u, nullptr, status, u_bar, x0_bar, gp_bar, fp_bar};
    return run_tiled(a, n_inst, P, o, true, wsp, ws_bytes, (hipStream_t)stream);
}

int fbsde_graph_capture_batched(const fbsde_problem* pbs, int64_t n_inst, const int64_t* P, const double* const* x0,
                                double* const* u, double* const* grad, uint32_t* const* status,
                                const fbsde_batch_opts* opts, void* wsp, size_t ws_bytes, fbsde_graph* out,
                                fbsde_stream stream) {
    if (!out) return FBSDE_EINVAL;
    *out = nullptr;
    if (!pbs || !P || !x0 || !u || !status || !wsp || n_inst < 1) return FBSDE_EINVAL;
    Opts o;
    int rc = read_opts(opts, o);
    if (rc) return rc;
    if (o.mode != FBSDE_BATCH_TILED) return FBSDE_EINVAL;   // the persistent schedule uploads host tables
    for (int64_t i = 0; i < n_inst; ++i) {
        if (P[i] > 0 && (!x0[i] || !u[i] || !status[i])) return FBSDE_EINVAL;
        // the host-driven CG loop (a diagnostic alternative) polls the device, which a graph cannot do
        if (!pbs[i].shared_dw && pbs[i].cg_fixed_iters <= 0 && std::getenv("FBSDE_CG_HOST_LOOP") &&
            std::getenv("FBSDE_CG_HOST_LOOP")[0] == '1')
            return FBSDE_EINVAL;
    }
    size_t need = 0;
    if ((rc = tiled_size(pbs, n_inst, P, o, 0, &need))) return rc;
    if (need > ws_bytes) return FBSDE_ENOSPC;
    TiledArgs a{pbs, x0, u, grad, status, nullptr, nullptr, nullptr, nullptr};
    return capture_graph([&](hipStream_t cap) { return run_tiled(a, n_inst, P, o, false, wsp, ws_bytes, cap); },
                         (hipStream_t)stream, out);
}

int fbsde_batched_cg_bytes(const fbsde_problem* pbs, int64_t n_inst, const int64_t* P, const fbsde_batch_opts* opts,
                           int32_t adjoint, const void* wsp, double* bytes, fbsde_stream stream) {
    if (!pbs || !P || !wsp || !bytes || n_inst < 1 || (adjoint != 0 && adjoint != 1)) return FBSDE_EINVAL;
    Opts o;
    int rc = read_opts(opts, o);
    if (rc) return rc;
    if (o.mode != FBSDE_BATCH_TILED) return FBSDE_EINVAL;
    std::vector<TileUnit> units;
    size_t need = 0, arena = 0;
    int nw = 1;
    if ((rc = tiled_size(pbs, n_inst, P, o, adjoint ? FBSDE_WS_TAPE : 0, &need, &units, &arena, &nw))) return rc;
    *bytes = 0.0;
    if (units.empty()) return FBSDE_OK;
    unsigned long long c[8] = {};
    const unsigned long long* cgc = tiled_cg_counters((char*)wsp, units.size());
    if (hipMemcpyAsync(c, cgc, sizeof(c), hipMemcpyDeviceToHost, (hipStream_t)stream) != hipSuccess ||
        hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
        return FBSDE_EHIP;
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += (double)c[w];
    *bytes = t;
    return FBSDE_OK;
}

}  // extern "C"
