"""GPU edge cases of the C ABI against the FP64 oracle: empty inputs, the smallest problems, the widest rows
each precision supports, the most points one call takes (and a batched instance larger than that), and the
per-point status flags on degenerate inputs (a flat Newton derivative, overflow, the CG cap).

Bar: FP64 <= 1e-10 and FP32C <= 1e-5 relative error against the oracle, as in the parity tests; status bits
equal to the oracle's where the oracle defines them (it solves the regression directly, so it has no CG cap).
"""
import ctypes
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_2510_02635_amd as F  # noqa: E402
from paper_2510_02635_amd import _native as N  # noqa: E402
from oracle import scheme as OS  # noqa: E402
from paper_2510_02635_amd import workloads  # noqa: E402

from _convert import problems, rel_err  # noqa: E402

DEV = "cuda"
AC = dict(f_kind=F.F_ALLEN_CAHN, fp=(1.0, 1.0, 0, 0), g_kind=F.G_AC, gp=(0.4, 0, 0, 0))
TOL = {F.F64: 1e-10, F.F32C: 1e-5}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    N.load()


def _against_oracle(u, g, st, op, x0, pts, tol, tag):
    u, g, st = u.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy()
    for p in pts:
        ref = OS.solve_point(op, x0[p], p)
        eu = abs(u[p] - ref["u"]) / max(abs(ref["u"]), 1e-300)
        eg = rel_err(g[p], ref["grad"])
        _say(f"  {tag} p={p} rel_u={eu:.2e} rel_grad={eg:.2e} status={st[p]}")
        assert st[p] == ref["status"] == 0
        assert eu <= tol and eg <= tol, (p, eu, eg)


# ------------------------------------------------------------------ empty inputs
@pytest.mark.parametrize("shared", [0, 1])
@pytest.mark.parametrize("prec", [F.F64, F.F32C])
def test_zero_points(prec, shared):
    hp, _ = problems(d=12, M=40, N=3, T=0.3, prec=prec, shared_dw=shared, **AC)
    x0 = torch.empty((0, 12), dtype=torch.float64, device=DEV)
    _say(f"[empty] prec={prec} shared={shared}")
    u, g, st, iters = F.solve(hp, x0, tape=True, return_iters=True)
    assert u.shape == (0,) and g.shape == (0, 12) and st.shape == (0,) and iters == [0, 0, 0]
    # the reverse mode through the C ABI with sentinel-filled parameter adjoints: zeros come back
    lib = N.load()
    gp = torch.full((4,), float("nan"), dtype=torch.float64, device=DEV)
    fp = torch.full((4,), float("nan"), dtype=torch.float64, device=DEV)
    it = (ctypes.c_int32 * 3)(7, 7, 7)
    rc = lib.fbsde_solve_backward(ctypes.byref(hp.c()), 0, None, None, None, gp.data_ptr(), fp.data_ptr(), None,
                                  None, 0, ctypes.cast(it, ctypes.c_void_p),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert rc == 0 and list(it) == [0, 0, 0]
    assert torch.all(gp == 0) and torch.all(fp == 0)
    # autograd over an empty set of points
    xg = x0.clone().requires_grad_(True)
    gpt = torch.tensor([0.4, 0, 0, 0], dtype=torch.float64, requires_grad=True)
    fpt = torch.tensor([1.0, 1, 0, 0], dtype=torch.float64, requires_grad=True)
    ua, _, _ = F.solve_autograd(hp, xg, gpt, fpt)
    ua.sum().backward()
    torch.cuda.synchronize()
    assert xg.grad.shape == (0, 12) and torch.all(gpt.grad == 0) and torch.all(fpt.grad == 0)


def _batched_backward_raw(hps, xs, ubs):
    """fbsde_solve_batched_backward with NaN-filled parameter adjoints, so an unwritten one shows."""
    n = len(hps)
    cps = (N.CProblem * n)(*[hp.c() for hp in hps])
    Ps = (ctypes.c_int64 * n)(*[int(x.shape[0]) for x in xs])
    opts = N.CBatchOpts(N.BATCH_TILED, 2, 0, 512, 0)
    us = [torch.empty(x.shape[0], dtype=torch.float64, device=DEV) for x in xs]
    xbs = [torch.empty_like(x) for x in xs]
    gps = [torch.full((4,), float("nan"), dtype=torch.float64, device=DEV) for _ in xs]
    fps = [torch.full((4,), float("nan"), dtype=torch.float64, device=DEV) for _ in xs]
    sts = [torch.empty(x.shape[0], dtype=torch.int32, device=DEV) for x in xs]
    size = ctypes.c_size_t(0)
    lib = N.load()
    assert lib.fbsde_batched_workspace_size(cps, n, ctypes.cast(Ps, ctypes.c_void_p), ctypes.byref(opts), 1,
                                            ctypes.byref(size)) == 0
    ws = torch.empty(max(int(size.value), 1), dtype=torch.uint8, device=DEV)

    def ptrs(ts):
        return (ctypes.c_void_p * n)(*[t.data_ptr() for t in ts])

    rc = lib.fbsde_solve_batched_backward(cps, n, ctypes.cast(Ps, ctypes.c_void_p), ptrs(xs), ptrs(ubs), ptrs(us),
                                          ptrs(xbs), ptrs(gps), ptrs(fps), ptrs(sts), ctypes.byref(opts),
                                          ws.data_ptr(), ws.numel(),
                                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert rc == 0
    return us, xbs, gps, fps, sts


def test_batched_with_empty_instances():
    hp0, _ = problems(d=12, M=40, N=3, T=0.3, instance=0, **AC)
    hp1, _ = problems(d=20, M=64, N=3, T=0.3, instance=1, **AC)
    x0e = torch.empty((0, 12), dtype=torch.float64, device=DEV)
    x1 = torch.tensor(workloads.points("normal:0.3", 3, 20, 4), device=DEV)
    _say("[empty batched] instances of 0 and 3 points, forward")
    us, gs, sts = F.solve_batched([hp0, hp1], [x0e, x1])
    torch.cuda.synchronize()
    u1, g1, st1 = F.solve(hp1, x1)
    torch.cuda.synchronize()
    assert us[0].shape == (0,) and torch.equal(us[1], u1) and torch.equal(gs[1], g1) and torch.equal(sts[1], st1)
    _say("[empty batched] backward, one empty instance")
    ub = [torch.empty(0, dtype=torch.float64, device=DEV), torch.ones(3, dtype=torch.float64, device=DEV)]
    _, xbs, gps, fps, _ = _batched_backward_raw([hp0, hp1], [x0e, x1], ub)
    ws = F.workspace(hp1, 3, tape=True)
    F.solve(hp1, x1, tape=True, ws=ws)
    xb1, gp1, fp1, _ = F.solve_backward(hp1, x1, ub[1], ws)
    torch.cuda.synchronize()
    assert torch.all(gps[0] == 0) and torch.all(fps[0] == 0)
    assert torch.equal(xbs[1], xb1) and torch.equal(gps[1], gp1) and torch.equal(fps[1], fp1)
    _say("[empty batched] backward, every instance empty")
    _, _, gps, fps, _ = _batched_backward_raw([hp0, hp1], [x0e, torch.empty((0, 20), dtype=torch.float64,
                                                                                device=DEV)], [ub[0], ub[0]])
    assert all(torch.all(t == 0) for t in gps + fps)


# ------------------------------------------------------------------ smallest problems
@pytest.mark.parametrize("prec", [F.F64, F.F32C])
@pytest.mark.parametrize("d,M", [(1, 2), (1, 3), (2, 2)])
def test_smallest_problems(d, M, prec):
    kw = dict(d=d, M=M, N=1, T=0.4, f_kind=F.F_ALLEN_CAHN, fp=(0.7, 0.3, 0, 0), g_kind=F.G_QUAD,
              gp=(1.0, 0.2, 0, 0), seed=5)
    if M > d + 1:
        kw["ridge_rel"] = 0.0          # full-rank design: the unregularised fit
    hp, op = problems(prec=prec, **kw)
    x0 = workloads.points("normal:0.5", 3, d, 9)
    xt = torch.tensor(x0, device=DEV)
    _say(f"[smallest] d={d} M={M} N=1 prec={prec}")
    ws = F.workspace(hp, 3, tape=True)
    u, g, st = F.solve(hp, xt, tape=True, ws=ws)
    ub = torch.tensor([1.0, -0.5, 2.0], dtype=torch.float64, device=DEV)
    xb, gpb, fpb, st2 = F.solve_backward(hp, xt, ub, ws)
    torch.cuda.synchronize()
    tol = TOL[prec]
    _against_oracle(u, g, st, op, x0, range(3), tol, "per-point")
    xb = xb.cpu().numpy()
    gp_ref, fp_ref = np.zeros(4), np.zeros(4)
    for p in range(3):
        ref = OS.adjoint_point(op, x0[p], p, ubar=float(ub[p]))
        e = rel_err(xb[p], ref["x0bar"])
        _say(f"  adjoint p={p} rel_x0bar={e:.2e}")
        assert e <= tol
        gp_ref += ref["gpbar"]
        fp_ref += ref["fpbar"]
    assert rel_err(gpb.cpu().numpy(), gp_ref) <= tol and rel_err(fpb.cpu().numpy(), fp_ref) <= tol
    assert int((st2 != 0).sum().item()) == 0
    # the shared form on the same sizes (primal for M > d, dual for M <= d)
    hs, os_ = problems(prec=prec, shared_dw=1, **kw)
    us, gs, sts = F.solve(hs, xt)
    torch.cuda.synchronize()
    _against_oracle(us, gs, sts, os_, x0, range(3), tol, "shared")


# ------------------------------------------------------------------ widest rows
@pytest.mark.parametrize("prec,d", [(F.F64, 16384), (F.F32C, 32768)])
def test_widest_rows(prec, d):
    hp, op = problems(d=d, M=64, N=2, T=0.3, prec=prec, seed=2, **AC)
    x0 = workloads.points("normal_over_sqrt_d", 2, d, 6)
    xt = torch.tensor(x0, device=DEV)
    _say(f"[widest] d={d} M=64 N=2 P=2 prec={prec} forward + adjoint")
    ws = F.workspace(hp, 2, tape=True)
    u, g, st = F.solve(hp, xt, tape=True, ws=ws)
    xb, _, _, st2 = F.solve_backward(hp, xt, torch.ones(2, dtype=torch.float64, device=DEV), ws)
    torch.cuda.synchronize()
    _against_oracle(u, g, st, op, x0, range(2), TOL[prec], "widest")
    ref = OS.adjoint_point(op, x0[1], 1, ubar=1.0)
    e = rel_err(xb[1].cpu().numpy(), ref["x0bar"])
    _say(f"  adjoint p=1 rel_x0bar={e:.2e}")
    assert e <= TOL[prec] and int((st2 != 0).sum().item()) == 0


# ------------------------------------------------------------------ most points
@pytest.mark.parametrize("prec", [F.F64, F.F32C])
def test_most_points_per_call(prec):
    P = 65535
    hp, op = problems(d=4, M=16, N=2, T=0.3, prec=prec, seed=3, **AC)
    x0 = workloads.points("normal:0.5", P, 4, 8)
    _say(f"[most points] P={P} d=4 M=16 N=2 prec={prec}")
    u, g, st = F.solve(hp, torch.tensor(x0, device=DEV))
    torch.cuda.synchronize()
    assert int((st != 0).sum().item()) == 0 and bool(torch.isfinite(u).all())
    _against_oracle(u, g, st, op, x0, (0, 1, P // 2, P - 1), TOL[prec], "most points")


def test_batched_instance_larger_than_one_call():
    P = 70000
    hp, op = problems(d=4, M=16, N=2, T=0.3, seed=3, instance=2, point_base=100, **AC)
    x0 = workloads.points("normal:0.5", P, 4, 10)
    _say(f"[batched over the per-call maximum] P={P} d=4 M=16 N=2 point_base=100")
    us, gs, sts = F.solve_batched([hp], [torch.tensor(x0, device=DEV)], streams=2)
    torch.cuda.synchronize()
    assert int((sts[0] != 0).sum().item()) == 0
    # the oracle's point p is global point point_base + p; the tiles split the instance at P / 2
    _against_oracle(us[0], gs[0], sts[0], op, x0, (0, P // 2 - 1, P // 2, P - 1), 1e-10, "batched")


# ------------------------------------------------------------------ status flags
def test_flat_newton_derivative_flags_like_the_oracle():
    # f = c1 y with c1 = N / T makes F'(y) = 1 - dt c1 exactly 0: Newton flags it and the values overflow
    kw = dict(d=6, M=32, N=1, T=0.5, f_kind=F.F_ALLEN_CAHN, fp=(2.0, 0.0, 0, 0), g_kind=F.G_QUAD,
              gp=(1.0, 0.5, 0, 0), seed=1)
    hp, op = problems(**kw)
    x0 = workloads.points("normal:0.5", 2, 6, 2)
    _say("[flat Newton] d=6 M=32 N=1 c1=N/T")
    u, g, st = F.solve(hp, torch.tensor(x0, device=DEV))
    torch.cuda.synchronize()
    st = st.cpu().numpy()
    with np.errstate(all="ignore"):
        refs = [OS.solve_point(op, x0[p], p)["status"] for p in range(2)]
    _say(f"  status gpu={list(st)} oracle={refs}")
    assert list(st) == refs
    assert all(s & F.ST_NEWTON_FLAT and s & F.ST_NONFINITE for s in refs)


def test_overflow_flags_one_point_only():
    hp, op = problems(d=8, M=48, N=2, T=0.3, f_kind=F.F_ZERO, g_kind=F.G_QUAD, gp=(1.0, 0, 0, 0), seed=4)
    x0 = workloads.points("normal:0.5", 3, 8, 3)
    x0[1, :] = 1e200            # |x|^2 overflows in g
    _say("[overflow] point 1 of 3 overflows in g")
    u, g, st = F.solve(hp, torch.tensor(x0, device=DEV))
    torch.cuda.synchronize()
    stn = st.cpu().numpy()
    _say(f"  status={list(stn)}")
    assert stn[1] & F.ST_NONFINITE
    _against_oracle(u, g, st, op, x0, (0, 2), 1e-10, "overflow neighbours")


def test_cg_cap_flags_every_point():
    hp, op = problems(d=20, M=200, N=2, T=0.3, seed=6, cg_maxit=2, cg_rtol=1e-14, **AC)
    x0 = workloads.points("normal:0.3", 4, 20, 5)
    _say("[CG cap] d=20 M=200 cg_maxit=2")
    u, g, st, iters = F.solve(hp, torch.tensor(x0, device=DEV), return_iters=True)
    torch.cuda.synchronize()
    stn = st.cpu().numpy()
    _say(f"  status={list(stn)} iters={iters}")
    assert iters == [2, 2]
    assert all(s == F.ST_CG_MAXIT for s in stn)
    assert bool(torch.isfinite(u).all()) and bool(torch.isfinite(g).all())
