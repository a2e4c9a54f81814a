"""GPU parity of the batched solve (fbsde_solve_batched, fbsde_solve_batched_backward) against the FP64
oracle and the single-instance path.

Instances of uneven d (several geometry classes, team widths 1..16 waves), M, f, g and precision run in
one call.  Persistent schedule: fewer workgroup slots than points, so slots are reused through the work
queue.  Tiled schedule: a small tile cap splits instances into several point tiles spread over three
streams.  Each instance must equal the oracle at the precision bar (FP64 1e-10, FP32C 1e-5).
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_2510_02635_amd as F  # noqa: E402
from oracle import scheme as OS  # noqa: E402
from paper_2510_02635_amd import workloads  # noqa: E402

from _convert import problems, rel_err  # noqa: E402

DEV = "cuda"


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    F._native.load()


INSTANCES = [
    (dict(d=37, M=100, N=3, T=0.5, f_kind=F.F_HJB, fp=(0.8, 0, 0, 0), g_kind=F.G_HJB_LOG, gp=(1.0, 0, 0, 0), seed=7,
          instance=0), "uniform", 5),
    (dict(d=37, M=150, N=3, T=0.3, f_kind=F.F_ALLEN_CAHN, fp=(1, 1, 0, 0), g_kind=F.G_AC, gp=(0.4, 0, 0, 0),
          instance=1), "normal:0.3", 3),
    (dict(d=600, M=130, N=2, T=0.3, f_kind=F.F_ALLEN_CAHN, fp=(1, 1, 0, 0), g_kind=F.G_AC, gp=(0.4, 0, 0, 0),
          instance=2), "normal:0.2", 2),
    (dict(d=1500, M=70, N=2, T=0.3, f_kind=F.F_ZERO, g_kind=F.G_QUAD, prec=F.F32C, instance=3), "normal:0.5", 2),
    (dict(d=3000, M=64, N=2, T=1.0, f_kind=F.F_HJB, fp=(1.3, 0, 0, 0), g_kind=F.G_HJB_LOG, gp=(1.0, 0, 0, 0),
          instance=4), "uniform", 1),
    (dict(d=200, M=400, N=4, T=0.3, f_kind=F.F_ALLEN_CAHN, fp=(1, 1, 0, 0), g_kind=F.G_AC, gp=(0.4, 0, 0, 0),
          instance=5), "normal_over_sqrt_d", 3),   # M > d + 1: warm-started CG
    (dict(d=80, M=200, N=3, T=0.5, f_kind=F.F_BURGERS, fp=(2 ** 0.5 / 80, 40.5, 0, 0), g_kind=F.G_LOGISTIC,
          gp=(0.5, 0, 0, 0), gvec=np.ones(80) / 80, instance=7), "normal:0.5", 2),
]


SCHEDULES = [dict(mode="persistent", max_slots=3), dict(mode="persistent", max_slots=64),
             dict(mode="tiled", streams=3, tile_bytes=1 << 20), dict(mode="tiled")]


@pytest.mark.parametrize("sched", SCHEDULES, ids=["persistent3", "persistent64", "tiled_small", "tiled"])
def test_batched_matches_oracle(sched):
    hps, ops, xs = [], [], []
    for kw, xkind, P in INSTANCES:
        hp, op = problems(**kw)
        hps.append(hp)
        ops.append(op)
        xs.append(workloads.points(xkind, P, kw["d"], 21 + kw["instance"]))
    _say(f"[batched] {len(hps)} instances, {sched}")
    us, gs, sts = F.solve_batched(hps, [torch.tensor(x, device=DEV) for x in xs], **sched)
    torch.cuda.synchronize()
    for i, (hp, op, x) in enumerate(zip(hps, ops, xs)):
        tol = 1e-10 if hp.prec == F.F64 else 1e-5
        u, g, st = us[i].cpu().numpy(), gs[i].cpu().numpy(), sts[i].cpu().numpy()
        for p in range(x.shape[0]):
            ref = OS.solve_point(op, x[p], p)
            eu = abs(u[p] - ref["u"]) / abs(ref["u"])
            eg = rel_err(g[p], ref["grad"])
            _say(f"  inst {i} d={hp.d} M={hp.M} p={p} rel_u={eu:.2e} rel_grad={eg:.2e}")
            assert st[p] == 0
            assert eu <= tol and eg <= tol


def test_batched_equals_single_solve():
    kw, xkind, P = INSTANCES[5]
    hp, _ = problems(**kw)
    x = torch.tensor(workloads.points(xkind, P, kw["d"], 99), device=DEV)
    _say("[batched] persistent vs single")
    us, gs, _ = F.solve_batched([hp], [x], mode="persistent", max_slots=2)
    u1, g1, _ = F.solve(hp, x)
    torch.cuda.synchronize()
    assert torch.allclose(us[0], u1, rtol=1e-12, atol=0)
    assert torch.allclose(gs[0], g1, rtol=1e-10, atol=1e-14)
    # one tile holding the whole instance runs the very same launches: identical bits
    _say("[batched] tiled (one tile) vs single")
    ut, gt, _ = F.solve_batched([hp], [x], mode="tiled", streams=2)
    torch.cuda.synchronize()
    assert torch.equal(ut[0], u1) and torch.equal(gt[0], g1)
    # one point per tile: other chunk splits, same streams and test
    _say("[batched] tiled (one point per tile) vs single")
    w1 = F.workspace_size(hp, 1)
    ut, gt, _ = F.solve_batched([hp], [x], mode="tiled", streams=2, tile_bytes=w1)
    torch.cuda.synchronize()
    assert torch.allclose(ut[0], u1, rtol=1e-12, atol=0)
    assert torch.allclose(gt[0], g1, rtol=1e-10, atol=1e-14)


ADJ = [
    (dict(d=37, M=100, N=3, T=0.5, f_kind=F.F_HJB, fp=(0.8, 0, 0, 0), g_kind=F.G_HJB_LOG, gp=(1.0, 0, 0, 0), seed=7,
          instance=0), "uniform", 5),
    (dict(d=200, M=400, N=4, T=0.3, f_kind=F.F_ALLEN_CAHN, fp=(1, 1, 0, 0), g_kind=F.G_AC, gp=(0.4, 0, 0, 0),
          instance=5), "normal_over_sqrt_d", 3),
    (dict(d=700, M=96, N=2, T=0.3, f_kind=F.F_ALLEN_CAHN, fp=(1, 1, 0, 0), g_kind=F.G_AC, gp=(0.4, 0, 0, 0),
          prec=F.F32C, instance=6), "normal:0.2", 2),
    (dict(d=80, M=200, N=3, T=0.5, f_kind=F.F_BURGERS, fp=(2 ** 0.5 / 80, 40.5, 0, 0), g_kind=F.G_LOGISTIC,
          gp=(0.5, 0, 0, 0), gvec=np.ones(80) / 80, instance=7), "normal:0.5", 2),
]


@pytest.mark.parametrize("tile_small", [False, True], ids=["one_tile", "point_tiles"])
def test_batched_backward_matches_single_and_oracle(tile_small):
    hps, ops, xs, ubs = [], [], [], []
    for kw, xkind, P in ADJ:
        hp, op = problems(**kw)
        hps.append(hp)
        ops.append(op)
        xs.append(torch.tensor(workloads.points(xkind, P, kw["d"], 5 + kw["instance"]), device=DEV))
        ubs.append(torch.linspace(0.5, 1.5, P, dtype=torch.float64, device=DEV))
    tb = max(F.workspace_size(hp, 1, tape=True) for hp in hps) if tile_small else 0
    _say(f"[batched-adjoint] {len(hps)} instances, tile_bytes={tb}")
    us, xbs, gps, fps, sts = F.solve_batched_backward(hps, xs, ubs, streams=3, tile_bytes=tb)
    torch.cuda.synchronize()
    for i, (hp, op) in enumerate(zip(hps, ops)):
        tol = 1e-10 if hp.prec == F.F64 else 1e-5
        assert int(sts[i].abs().sum().item()) == 0
        ws = F.workspace(hp, xs[i].shape[0], tape=True, device=DEV)
        u1, _, _ = F.solve(hp, xs[i], tape=True, ws=ws)
        xb1, gp1, fp1, _ = F.solve_backward(hp, xs[i], ubs[i], ws)
        torch.cuda.synchronize()
        _say(f"  inst {i}: |du|={float((us[i] - u1).abs().max()):.2e} |dx0bar|={float((xbs[i] - xb1).abs().max()):.2e}")
        if not tile_small:
            assert torch.equal(us[i], u1) and torch.equal(xbs[i], xb1)
        assert torch.allclose(us[i], u1, rtol=1e-12, atol=0)
        assert torch.allclose(xbs[i], xb1, rtol=1e-9, atol=1e-13)
        assert torch.allclose(gps[i], gp1, rtol=1e-9, atol=1e-13)
        assert torch.allclose(fps[i], fp1, rtol=1e-9, atol=1e-13)
        # oracle on the first point: x0_bar of ubar_0 u_0
        x = xs[i].cpu().numpy()
        ref = OS.adjoint_point(op, x[0], 0, ubar=float(ubs[i][0]))
        e = rel_err(xbs[i][0].cpu().numpy(), ref["x0bar"])
        _say(f"  inst {i}: oracle rel_err x0bar[0] = {e:.2e}")
        assert e <= tol


def test_persistent_rank_deficient_fp32c_matches_oracle():
    # the uneven-instance set's smallest-M instance of the d = 1000 class (HJB, T = 1, M <= d + 1): the persistent
    # schedule runs its rows with FP64 arithmetic on the FP32 state, as the single-instance path does
    it = min((i for i in workloads.batched_instances(64) if i["d"] == 1000), key=lambda i: i["M"])
    hp, op = problems(d=it["d"], M=it["M"], N=20, T=1.0, f_kind=F.F_HJB, fp=(it["lam"], 0, 0, 0),
                      g_kind=F.G_HJB_LOG, gp=(1.0, 0, 0, 0), prec=F.F32C, seed=0, instance=it["instance"])
    x = workloads.points("uniform", 2, it["d"], 100 + it["instance"])
    _say(f"[batched persistent] rank-deficient FP32C d={it['d']} M={it['M']}")
    us, gs, sts = F.solve_batched([hp], [torch.tensor(x, device=DEV)], mode="persistent", max_slots=8)
    torch.cuda.synchronize()
    for p in range(2):
        ref = OS.solve_point(op, x[p], p)
        eu = abs(us[0][p].item() - ref["u"]) / abs(ref["u"])
        eg = rel_err(gs[0][p].cpu().numpy(), ref["grad"])
        _say(f"  p={p} rel_u={eu:.2e} rel_grad={eg:.2e}")
        assert int(sts[0][p].item()) == 0 and eu <= 1e-5 and eg <= 1e-5
