"""GPU parity of the paper-literal per-anchor scheme (Algorithm 1 as printed) against the FP64 oracle.

Every case compares u = mean_m Y^m_{k_stop}, Y^m_{k_stop} for every anchor m and (|Z^m|^2, sum_i Z^m_i)
at level k_stop element by element. The tolerance is FP64's 1e-10 relative; |Z|^2 gets 1e-8 of its
largest value, since it is a quadratic form of an ill-conditioned ridge solve (condition number up to
about 2e3 d). The cases cover:
* each register layout of the anchor factorisation (one wavefront for M + 1 <= 56; four wavefronts
  for M + 1 <= 80, 112, 144; eight for M + 1 <= 224; sixteen for M + 1 <= 257) and the boundaries
  between them;
* every f family, including z-dependent ones (HJB, Burgers-type), and the affine and logistic
  terminal conditions;
* uniform weights (h = 0) and the first, a middle and the last backward level;
* the edge cases M = 2, d = 1, P = 0 and the largest M (256);
* d = 1000 (rank-deficient designs, M << d).
"""
import numpy as np
import pytest
import torch

import paper_2510_02635_amd as F
from oracle import literal as OL
from oracle import scheme as OS

pytestmark = pytest.mark.gpu


def _x0(P, d, seed):
    rng = np.random.default_rng(seed)
    return 0.3 * rng.normal(size=(P, d))


def _run(kw, P, k_stop=0, seed=1, points=None):
    x0 = _x0(P, kw["d"], seed)
    okw = dict(kw)
    gkw = dict(kw)
    if kw.get("gvec") is not None:
        gkw["gvec"] = torch.tensor(kw["gvec"], device="cuda")
    pb = F.Problem(**gkw)
    xt = torch.tensor(x0, device="cuda")
    print(f"[literal] d={kw['d']} M={kw['M']} N={kw['N']} P={P} k_stop={k_stop}", flush=True)
    u, st, Y, zs = F.solve_literal(pb, xt, k_stop=k_stop, want_Y=True, want_zstats=True)
    torch.cuda.synchronize()
    u, st, Y, zs = u.cpu().numpy(), st.cpu().numpy(), Y.cpu().numpy(), zs.cpu().numpy()
    opb = OS.Problem(**okw)
    for p in (range(P) if points is None else points):
        ref = OL.solve_point(opb, x0[p], p, k_stop=k_stop, tape=True)
        assert int(st[p]) == ref["status"] == 0
        scale = max(1.0, abs(ref["u"]))
        assert abs(u[p] - ref["u"]) <= 1e-10 * scale, (p, u[p], ref["u"])
        ys = max(1.0, np.max(np.abs(ref["Y"])))
        assert np.max(np.abs(Y[p] - ref["Y"])) <= 1e-10 * ys, (p, np.max(np.abs(Y[p] - ref["Y"])))
        zz_ref, zs_ref = ref["zz"][k_stop], ref["zs"][k_stop]
        assert np.max(np.abs(zs[p, :, 0] - zz_ref)) <= 1e-8 * max(1e-300, np.max(np.abs(zz_ref))) + 1e-300
        assert np.max(np.abs(zs[p, :, 1] - zs_ref)) <= 1e-8 * max(1e-300, np.max(np.abs(zs_ref))) + 1e-300
    return u, Y, zs


HJB = dict(f_kind=OS.F_HJB, fp=(1.0, 0.0, 0.0, 0.0), g_kind=OS.G_HJB_LOG, gp=(1.0, 0.0, 0.0, 0.0))
AC = dict(f_kind=OS.F_ALLEN_CAHN, fp=(1.0, 1.0, 0.0, 0.0), g_kind=OS.G_AC, gp=(0.4, 0.0, 0.0, 0.0))


@pytest.mark.parametrize("M", [2, 16, 55, 56, 79, 80, 100, 111, 112, 143, 144, 200, 223, 224])
def test_literal_hjb_every_layout(M):
    kw = dict(d=24, M=M, N=3, T=0.5, s=np.sqrt(2.0), ridge_rel=1e-2, seed=M, **HJB)
    _run(kw, P=2)               # u(0, x0)
    _run(kw, P=2, k_stop=1)     # every anchor's Y and Z at a level where they differ


@pytest.mark.parametrize("k_stop", [0, 2, 4])
def test_literal_levels_burgers_logistic(k_stop):
    d = 30
    kw = dict(d=d, M=40, N=5, T=0.4, s=1.0, f_kind=OS.F_BURGERS, fp=(1.0 / d, d + 0.5, 0.0, 0.0), g_kind=OS.G_LOGISTIC,
              gp=(0.0, 0.0, 0.0, 0.0), gvec=np.full(d, 1.0 / d), ridge_rel=1e-3, seed=7)
    _run(kw, P=3, k_stop=k_stop)


def test_literal_allen_cahn_case1_shape():
    kw = dict(d=100, M=100, N=4, T=0.3, s=np.sqrt(2.0), ridge_rel=1e-3, seed=3, **AC)
    u, Y, zs = _run(kw, P=2, points=[0, 1])
    # f does not depend on z: every particle's Y is the same below the terminal level
    assert np.ptp(Y[0]) <= 1e-14


def test_literal_affine_uniform_weights_d1():
    kw = dict(d=1, M=33, N=4, T=1.0, s=0.8, eps_h=0.0, ridge_rel=5e-2, f_kind=OS.F_HJB, fp=(0.5, 0.0, 0.0, 0.0),
              g_kind=OS.G_AFFINE, gp=(0.1, 0.0, 0.0, 0.0), gvec=np.array([1.5]), seed=4)
    _run(kw, P=2, k_stop=1)


def test_literal_rank_deficient_d1000():
    kw = dict(d=1000, M=64, N=3, T=0.3, s=np.sqrt(2.0), ridge_rel=1e-3, seed=9, **HJB)
    _run(kw, P=2)


def test_literal_largest_M():
    kw = dict(d=12, M=256, N=2, T=0.3, s=1.0, ridge_rel=1e-2, seed=5, **HJB)
    _run(kw, P=1)


def test_literal_empty_and_errors():
    pb = F.Problem(d=8, M=16, N=3, T=0.3)
    x = torch.empty((0, 8), dtype=torch.float64, device="cuda")
    u, st, Y, zs = F.solve_literal(pb, x, want_Y=True, want_zstats=True)
    assert u.numel() == 0 and Y.numel() == 0
    x = torch.zeros((2, 8), dtype=torch.float64, device="cuda")
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(F.FbsdeError):
        F.solve_literal(pb, x, ws=ws)
    with pytest.raises(F.FbsdeError):
        F.solve_literal(F.Problem(d=8, M=300, N=3, T=0.3), x)


def test_literal_launch_timer_records_gram_and_anchor_launches():
    d, M, N, P = 40, 30, 3, 2
    pb = F.Problem(d=d, M=M, N=N, T=0.3, ridge_rel=1e-2, **HJB)
    x = torch.zeros((P, d), dtype=torch.float64, device="cuda")
    F.launch_timer(True)
    F.solve_literal(pb, x)
    torch.cuda.synchronize()
    F.launch_timer(False)
    ms, work = F.launch_timer_read(with_bytes=True)
    kinds = F.launch_timer_kinds()
    assert list(kinds) == [F.TIMED_LITERAL_GRAM, F.TIMED_LITERAL_ANCHORS] * N
    assert np.all(ms > 0)
    assert np.all(work[kinds == F.TIMED_LITERAL_GRAM] == P * M * (M + 1.0) * d)
    ref = P * M * (2.0 / 3.0 * (M + 1.0) ** 3 + 6.0 * M * M)
    assert np.allclose(work[kinds == F.TIMED_LITERAL_ANCHORS], ref, rtol=1e-12)


@pytest.mark.parametrize("M,N", [(100, 6), (200, 3)])
def test_literal_full_size_burgers_d10000(M, N):
    # the benchmarked shape (d = 10^4, M = 100 or 200, dt = 0.003) in the bench's launch configuration
    # (64 points), fewer levels; sampled points against the oracle one by one
    d, P = 10000, 64
    s = float(np.sqrt(2.0))
    kw = dict(d=d, M=M, N=N, T=0.003 * N, s=s, f_kind=OS.F_BURGERS, fp=(s / d, d / 2 + 0.5, 0.0, 0.0),
              g_kind=OS.G_LOGISTIC, gp=(0.3, 0.0, 0.0, 0.0), gvec=np.full(d, 1.0 / d), ridge_rel=1e-3, seed=0,
              instance=6)
    gkw = dict(kw, gvec=torch.tensor(kw["gvec"], device="cuda"))
    print(f"[literal full size] d={d} M={M} N={N} P={P}", flush=True)
    u, st, Y, zs = F.solve_literal(F.Problem(**gkw), torch.zeros((P, d), dtype=torch.float64, device="cuda"),
                                   want_Y=True)
    torch.cuda.synchronize()
    u, st, Y = u.cpu().numpy(), st.cpu().numpy(), Y.cpu().numpy()
    assert np.all(st == 0)
    opb = OS.Problem(**kw)
    for p in ((0, P - 1) if M == 100 else (P - 1,)):
        ref = OL.solve_point(opb, np.zeros(d), p)
        assert abs(u[p] - ref["u"]) <= 1e-10 * abs(ref["u"]), (p, u[p], ref["u"])
        assert np.max(np.abs(Y[p] - ref["Y"])) <= 1e-10 * np.max(np.abs(ref["Y"]))



@pytest.mark.parametrize("M", [40, 100])
def test_literal_stored_path(M):
    # a workspace that holds every level: the backward sweep reads the stored particles instead of reversing
    # the path; against the oracle at 1e-10 and against the reversing form to rounding
    kw = dict(d=300, M=M, N=5, T=0.5, s=np.sqrt(2.0), ridge_rel=1e-2, seed=2, **HJB)
    P = 3
    x0 = _x0(P, kw["d"], 4)
    pb = F.Problem(**kw)
    xt = torch.tensor(x0, device="cuda")
    print(f"[literal stored] M={M}", flush=True)
    u1, st1, Y1, _ = F.solve_literal(pb, xt, want_Y=True, stored=True)
    u0, st0, Y0, _ = F.solve_literal(pb, xt, want_Y=True)
    torch.cuda.synchronize()
    u1, Y1, u0, Y0 = u1.cpu().numpy(), Y1.cpu().numpy(), u0.cpu().numpy(), Y0.cpu().numpy()
    assert np.max(np.abs(Y1 - Y0)) <= 1e-12 * np.max(np.abs(Y0))
    opb = OS.Problem(**kw)
    for p in range(P):
        ref = OL.solve_point(opb, x0[p], p)
        assert abs(u1[p] - ref["u"]) <= 1e-10 * max(1.0, abs(ref["u"]))
