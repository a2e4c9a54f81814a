// Host side of the persistent batched launch: geometry classes, work tables, one persistent kernel per class.
#include "fbsde_host.hpp"
#include "fbsde_batched.hpp"

#include <map>
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
    std::vector<int> insts;   // instance indices, by decreasing per-point cost
    int64_t items = 0;
    int64_t maxM = 0;
    int ld = 0;
};

int batch_classes(const fbsde_problem* pbs, int64_t n_inst, const int64_t* P, std::vector<BatchClass>& out) {
    std::map<std::tuple<int, int, int, int>, BatchClass> cls;
    for (int64_t i = 0; i < n_inst; ++i) {
        int rc = check_problem(&pbs[i], P[i]);
        if (rc) return rc;
        if (pbs[i].shared_dw) return FBSDE_EINVAL;
        Plan pl;
        if ((rc = make_plan(&pbs[i], 1, pl))) return rc;
        batch_geometry(pl);
        const auto key = std::make_tuple(pbs[i].prec, pl.Q, pl.TEAM, pl.ld);
        BatchClass& c = cls[key];
        c.prec = pbs[i].prec; c.Q = pl.Q; c.TEAM = pl.TEAM; c.ld = pl.ld;
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
        hipLaunchKernelGGL((k_batched<S, QQ, TT>), dim3(nslots), dim3(Geo<QQ, TT>::BS), 0, st, d_insts, d_items,
                           n_items, queue, slots, lay);
    });
}

}  // namespace

extern "C" {

int fbsde_batched_workspace_size(const fbsde_problem* pbs, int64_t n_inst, const int64_t* P, int32_t max_slots,
                                 size_t* bytes) {
    if (!pbs || !P || !bytes || n_inst < 1 || max_slots < 1) return FBSDE_EINVAL;
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

int fbsde_solve_batched(const fbsde_problem* pbs, int64_t n_inst, const int64_t* P, const double* const* x0,
                        double* const* u, double* const* grad, uint32_t* const* status, int32_t max_slots, void* wsp,
                        size_t ws_bytes, fbsde_stream stream) {
    if (!pbs || !P || !x0 || !u || !status || !wsp || n_inst < 1 || max_slots < 1) return FBSDE_EINVAL;
    std::vector<BatchClass> cls;
    int rc = batch_classes(pbs, n_inst, P, cls);
    if (rc) return rc;
    size_t need = 0;
    if ((rc = fbsde_batched_workspace_size(pbs, n_inst, P, max_slots, &need))) return rc;
    if (need > ws_bytes) return FBSDE_ENOSPC;
    for (int64_t i = 0; i < n_inst; ++i)
        if (P[i] > 0 && (!x0[i] || !u[i] || !status[i])) return FBSDE_EINVAL;
    hipStream_t st = (hipStream_t)stream;
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
        b.rtol2 = pb->cg_rtol * pb->cg_rtol;
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

}  // extern "C"
