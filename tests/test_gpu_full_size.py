"""GPU parity at the full sizes of the five workload configurations, in the launch shapes the
benchmark times, on sampled outputs the FP64 oracle computes point by point, and through
properties that hold at any size where the oracle is too slow.

  C0  d=100, one point x0=0, T=0.3, N=5, M=512, Allen-Cahn, FP64: the whole configuration.
  C1  d=1000, 1024 points x0 ~ N(0, 0.25 I), T=0.3, N=20, M=4096, Allen-Cahn and heat, FP32C and FP64:
      oracle on points 0 and 1023.
  C2  uneven HJB instances (T=1, N=20, FP32C): the smallest-M instance of the d = 100, 500, 1000 classes
      against the oracle; the largest (d, M) of the d = 5000 and 10^4 classes through the batched call
      equal, bit for bit, to the single-instance solve of the same points (one tile each); the nearly
      square designs (d = 5000 with M = 4800 and 5376, d = 10^4 with M = 8192) at two levels, forward and
      adjoint, against the oracle.
  C3  d=10^4, 128 points x0 ~ N(0, I/d), T=0.3, N=20, M=1024, Allen-Cahn: forward + adjoint in FP32C and
      FP64 against the oracle's reverse mode on point 0.
  C4  shared increments, d=10^4, 4096 points, M=2048, N=20, T=0.3, Allen-Cahn, FP32C: the forward against
      the oracle on point 0; the adjoint in FP64 against central differences of the FP64 forward along
      a random direction, and the FP32C adjoint against the FP64 one.
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
AC = dict(f_kind=F.F_ALLEN_CAHN, fp=(1.0, 1.0, 0, 0), g_kind=F.G_AC, gp=(0.4, 0, 0, 0))


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    F._native.load()
    F.autotune_reset()


def _check(u, g, st, refs, tol, tag):
    for p, ref in refs.items():
        eu = abs(u[p] - ref["u"]) / abs(ref["u"])
        eg = rel_err(g[p], ref["grad"])
        _say(f"  {tag} p={p} rel_u={eu:.2e} rel_grad={eg:.2e}")
        assert st[p] == 0
        assert eu <= tol and eg <= tol


def test_c0_whole_configuration():
    hp, op = problems(d=100, M=512, N=5, T=0.3, seed=0, instance=0, **AC)
    x0 = np.zeros((1, 100))
    _say("[C0] d=100 P=1 M=512 N=5 fp64")
    u, g, st = F.solve(hp, torch.tensor(x0, device=DEV))
    torch.cuda.synchronize()
    ref = OS.solve_point(op, x0[0], 0)
    _check(u.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy(), {0: ref}, 1e-10, "C0")


@pytest.mark.parametrize("kind", ["allen_cahn", "heat"])
def test_c1_full_size_sampled(kind):
    fk = AC if kind == "allen_cahn" else dict(f_kind=F.F_ZERO, g_kind=F.G_QUAD, gp=(1.0, 0.0, 0, 0))
    P = 1024
    x0 = workloads.points("normal:0.5", P, 1000, seed=1)
    xt = torch.tensor(x0, device=DEV)
    refs = None
    for prec, tol in ((F.F32C, 1e-5), (F.F64, 1e-10)):
        hp, op = problems(d=1000, M=4096, N=20, T=0.3, seed=0, instance=1, prec=prec, **fk)
        _say(f"[C1 {kind}] d=1000 P=1024 M=4096 N=20 prec={prec}")
        u, g, st = F.solve(hp, xt)
        torch.cuda.synchronize()
        if refs is None:
            refs = {p: OS.solve_point(op, x0[p], p) for p in (0, P - 1)}
        _check(u.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy(), refs, tol, f"C1 {kind} prec={prec}")
        assert int((st != 0).sum().item()) == 0
        del u, g, st
        torch.cuda.empty_cache()


def _c2_problem(it, P):
    return problems(d=it["d"], M=it["M"], N=20, T=1.0, f_kind=F.F_HJB, fp=(it["lam"], 0, 0, 0), g_kind=F.G_HJB_LOG,
                    gp=(1.0, 0, 0, 0), prec=F.F32C, seed=0, instance=it["instance"])


def test_c2_instances_full_size():
    insts = workloads.batched_instances(64)
    by_d = {}
    for it in insts:
        by_d.setdefault(it["d"], []).append(it)
    small = [min(by_d[d], key=lambda it: it["M"]) for d in (100, 500, 1000)]
    large = [max(by_d[d], key=lambda it: it["M"]) for d in (5000, 10000)]
    # oracle classes: 256 points each, oracle on point 0
    hps, ops, xs = [], [], []
    for it in small:
        hp, op = _c2_problem(it, 256)
        hps.append(hp)
        ops.append(op)
        xs.append(workloads.points("uniform", 256, it["d"], seed=100 + it["instance"]))
    _say(f"[C2] batched: {[(it['d'], it['M']) for it in small]} x 256 points")
    us, gs, sts = F.solve_batched(hps, [torch.tensor(x, device=DEV) for x in xs])
    torch.cuda.synchronize()
    for i, op in enumerate(ops):
        ref = OS.solve_point(op, xs[i][0], 0)
        _check(us[i].cpu().numpy(), gs[i].cpu().numpy(), sts[i].cpu().numpy(), {0: ref}, 1e-5, f"C2 d={op.d}")
        assert int((sts[i] != 0).sum().item()) == 0
    # the largest instances: batched (one tile each) equals the single-instance solve bit for bit
    hps = [_c2_problem(it, 8)[0] for it in large]
    xl = [torch.tensor(workloads.points("uniform", 8, it["d"], seed=100 + it["instance"]), device=DEV) for it in large]
    _say(f"[C2] batched vs single: {[(it['d'], it['M']) for it in large]} x 8 points")
    us, gs, sts = F.solve_batched(hps, xl)
    torch.cuda.synchronize()
    for i, hp in enumerate(hps):
        u1, g1, st1 = F.solve(hp, xl[i])
        torch.cuda.synchronize()
        assert torch.equal(us[i], u1) and torch.equal(gs[i], g1) and torch.equal(sts[i], st1)
        assert int((st1 != 0).sum().item()) == 0


@pytest.mark.parametrize("d,M", [(5000, 4800), (5000, 5376), (10000, 8192)])
def test_c2_near_square_instances_against_oracle(d, M):
    # The nearly square designs of the uneven HJB set (FP32C, T = 1), where CG needs the most iterations and
    # FP32 rounding in CG matters most, at their full d and M through the batched forward and forward +
    # adjoint calls, on 4 points; the oracle's cost bounds the levels to N = 2 (the per-level shape the batch
    # runs 20 times).  Point 0 against the oracle's reverse mode, u and grad u and x0_bar at the FP32C bar.
    it = next(i for i in workloads.batched_instances(64) if i["d"] == d and i["M"] == M)
    P, N = 4, 2
    hp, op = problems(d=d, M=M, N=N, T=1.0, f_kind=F.F_HJB, fp=(it["lam"], 0, 0, 0), g_kind=F.G_HJB_LOG,
                      gp=(1.0, 0, 0, 0), prec=F.F32C, seed=0, instance=it["instance"])
    x = workloads.points("uniform", P, d, seed=100 + it["instance"])
    xt = torch.tensor(x, device=DEV)
    ub = torch.ones(P, dtype=torch.float64, device=DEV)
    _say(f"[C2 near-square] d={d} M={M} P={P} N={N} fp32c batched forward and forward + adjoint")
    us, gs, sts = F.solve_batched([hp], [xt])
    ub_, xbs, gps, fps, sts2 = F.solve_batched_backward([hp], [xt], [ub])
    torch.cuda.synchronize()
    u, g, xb = us[0].cpu().numpy(), gs[0].cpu().numpy(), xbs[0].cpu().numpy()
    assert int((sts[0] != 0).sum().item()) == 0 and int((sts2[0] != 0).sum().item()) == 0
    assert torch.allclose(ub_[0], us[0], rtol=1e-12, atol=0)
    ref = OS.adjoint_point(op, x[0], 0, ubar=1.0)
    eu = abs(u[0] - ref["u"]) / abs(ref["u"])
    eg = rel_err(g[0], ref["grad"])
    ex = rel_err(xb[0], ref["x0bar"])
    _say(f"  p=0 rel_u={eu:.2e} rel_grad={eg:.2e} rel_x0bar={ex:.2e}")
    assert eu <= 1e-5 and eg <= 1e-5 and ex <= 1e-5


def test_c3_forward_adjoint_full_size():
    P = 128
    x0 = workloads.points("normal_over_sqrt_d", P, 10000, seed=3)
    xt = torch.tensor(x0, device=DEV)
    ubar = torch.ones(P, dtype=torch.float64, device=DEV)
    ref = None
    for prec, tol in ((F.F32C, 1e-5), (F.F64, 1e-10)):
        hp, op = problems(d=10000, M=1024, N=20, T=0.3, seed=0, instance=3, prec=prec, **AC)
        _say(f"[C3] d=10000 P=128 M=1024 N=20 prec={prec} forward + adjoint")
        ws = F.workspace(hp, P, tape=True)
        u, g, st = F.solve(hp, xt, tape=True, ws=ws)
        x0b, gpb, fpb, st2 = F.solve_backward(hp, xt, ubar, ws)
        torch.cuda.synchronize()
        if ref is None:
            ref = OS.adjoint_point(op, x0[0], 0, ubar=1.0)
        _check(u.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy(), {0: ref}, tol, f"C3 prec={prec}")
        e = rel_err(x0b[0].cpu().numpy(), ref["x0bar"])
        _say(f"  C3 prec={prec} rel_x0bar[0]={e:.2e}")
        assert e <= tol
        assert int((st2 != 0).sum().item()) == 0
        del ws, u, g, x0b
        torch.cuda.empty_cache()


def test_c4_shared_full_size():
    P = 4096
    x0 = workloads.points("normal_over_sqrt_d", P, 10000, seed=7)
    xt = torch.tensor(x0, device=DEV)
    hp32, op = problems(d=10000, M=2048, N=20, T=0.3, seed=0, instance=4, shared_dw=1, prec=F.F32C, **AC)
    _say("[C4] shared d=10000 P=4096 M=2048 N=20 fp32c forward + adjoint")
    ws32 = F.workspace(hp32, P, tape=True)
    u32, g32, st32 = F.solve(hp32, xt, tape=True, ws=ws32)
    ubar = torch.ones(P, dtype=torch.float64, device=DEV)
    xb32, _, _, _ = F.solve_backward(hp32, xt, ubar, ws32)
    torch.cuda.synchronize()
    u32n, g32n, st32n = u32.cpu().numpy(), g32.cpu().numpy(), st32.cpu().numpy()
    xb32 = xb32.cpu().numpy()
    del ws32
    torch.cuda.empty_cache()
    ref = OS.solve_point(op, x0[0], 0)
    _check(u32n, g32n, st32n, {0: ref}, 1e-5, "C4 fp32c")
    assert int((st32 != 0).sum().item()) == 0
    # FP64 adjoint against central differences of the FP64 forward along a random direction
    hp64, _ = problems(d=10000, M=2048, N=20, T=0.3, seed=0, instance=4, shared_dw=1, prec=F.F64, **AC)
    _say("[C4] shared fp64 adjoint vs central differences")
    ws64 = F.workspace(hp64, P, tape=True)
    u64, g64, _ = F.solve(hp64, xt, tape=True, ws=ws64)
    xb64, _, _, _ = F.solve_backward(hp64, xt, ubar, ws64)
    torch.cuda.synchronize()
    del ws64
    torch.cuda.empty_cache()
    _check(u64.cpu().numpy(), g64.cpu().numpy(), np.zeros(P, dtype=np.int32), {0: ref}, 1e-10, "C4 fp64")
    # one unit direction per point: sum_p x0bar_p . v_p against the central difference of sum_p u_p
    rng = np.random.default_rng(11)
    v = rng.standard_normal((P, 10000))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    vt = torch.tensor(v, device=DEV)
    h = 1e-4
    up, _, _ = F.solve(hp64, xt + h * vt)
    um, _, _ = F.solve(hp64, xt - h * vt)
    torch.cuda.synchronize()
    fd = float((up - um).sum().item()) / (2 * h)
    ad = float((xb64 * vt).sum().item())
    _say(f"  C4 fp64 directional: adjoint={ad:.12g} fd={fd:.12g} rel={abs(ad - fd) / abs(fd):.2e}")
    assert abs(ad - fd) <= 1e-5 * abs(fd)
    e = rel_err(xb32, xb64.cpu().numpy())
    _say(f"  C4 fp32c adjoint vs fp64 adjoint: rel {e:.2e}")
    assert e <= 1e-5
