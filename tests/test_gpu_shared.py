"""GPU parity of the shared-increment form (every point uses the same Philox stream 0xFFFFFFFF, the
common-randomness remark after Lemma 3.7): the dense MFMA contractions, the blocked Cholesky of the dual
ridge matrix and the per-point Newton epilogues against the FP64 oracle run with shared increments,
plus direct checks of the exported GEMM / Cholesky helpers against float64 references.
FP64 <= 1e-10, FP32C <= 1e-5 (relative, u and grad u).
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


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("m,n,k", [(16, 16, 4), (129, 70, 33), (300, 257, 1000), (64, 2048, 17), (200, 130, 1500),
                                   (70, 300, 3001)])
@pytest.mark.parametrize("nt", [True, False])
def test_gemm_matches_reference(dtype, m, n, k, nt):
    _say(f"[gemm] {dtype} m={m} n={n} k={k} nt={nt}")
    g = torch.Generator().manual_seed(m * 7 + n + k)
    A = torch.randn((m, k), generator=g, dtype=torch.float64)
    B = torch.randn((n, k) if nt else (k, n), generator=g, dtype=torch.float64)
    C0 = torch.randn((m, n), generator=g, dtype=torch.float64)
    ref = 0.5 * (A @ (B.T if nt else B)) - 2.0 * C0
    C = C0.to(dtype).to(DEV)
    F.gemm(A.to(dtype).to(DEV), B.to(dtype).to(DEV), nt=nt, C=C, alpha=0.5, beta=-2.0)
    torch.cuda.synchronize()
    err = (C.double().cpu() - ref).abs().max().item() / (1.0 + ref.abs().max().item())
    tol = 1e-13 if dtype == torch.float64 else 2e-5
    assert err < tol, err


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n,P", [(64, 3), (200, 130), (517, 40)])
def test_blocked_cholesky_solve(dtype, n, P):
    _say(f"[cholesky] {dtype} n={n} P={P}")
    g = torch.Generator().manual_seed(n + P)
    X = torch.randn((n, 3 * n), generator=g, dtype=torch.float64)
    K = X @ X.T / (3 * n) + 0.5 * torch.eye(n, dtype=torch.float64)
    R = torch.randn((P, n), generator=g, dtype=torch.float64)
    ref_L = torch.linalg.cholesky(K)
    ref_X = torch.linalg.solve(K, R.T).T
    Kd = K.to(dtype).to(DEV).contiguous()
    Rd = R.to(dtype).to(DEV).contiguous()
    info = F.cholesky_solve(Kd, Rd)
    assert info == 0
    L = torch.tril(Kd.double().cpu())
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    assert (L - ref_L).abs().max().item() < tol
    assert (Rd.double().cpu() - ref_X).abs().max().item() / ref_X.abs().max().item() < 10 * tol


SHARED_CASES = [
    ("ac_d37_P5", dict(d=37, M=100, N=3, T=0.3, f_kind=F.F_ALLEN_CAHN, fp=(1, 1, 0, 0), g_kind=F.G_AC,
                       gp=(0.4, 0, 0, 0)), "normal:0.3", 5),
    ("hjb_d300_P130_ragged", dict(d=300, M=200, N=2, T=0.5, f_kind=F.F_HJB, fp=(0.9, 0, 0, 0), g_kind=F.G_HJB_LOG,
                                  gp=(1.0, 0, 0, 0), seed=3), "uniform", 130),
    ("heat_d1000_M64", dict(d=1000, M=64, N=2, T=0.3, f_kind=F.F_ZERO, g_kind=F.G_QUAD, gp=(1.0, 0.5, 0, 0)),
     "normal:0.5", 3),
    ("ac_d2000_M300", dict(d=2000, M=300, N=3, T=0.3, f_kind=F.F_ALLEN_CAHN, fp=(1, 1, 0, 0), g_kind=F.G_AC,
                           gp=(0.4, 0, 0, 0)), "normal_over_sqrt_d", 4),
    ("burgers_logistic_d60_primal", dict(d=60, M=150, N=3, T=0.5, f_kind=F.F_BURGERS, fp=(2 ** 0.5 / 60, 30.5, 0, 0),
                                         g_kind=F.G_LOGISTIC, gp=(0.5, 0, 0, 0),
                                         gvec=np.linspace(-1.0, 2.0, 60) / 60), "normal:0.5", 6),
    ("burgers_logistic_d300_dual", dict(d=300, M=120, N=2, T=0.5, f_kind=F.F_BURGERS,
                                        fp=(2 ** 0.5 / 300, 150.5, 0, 0), g_kind=F.G_LOGISTIC, gp=(0.5, 0, 0, 0),
                                        gvec=np.ones(300) / 300), "normal:0.5", 4),
]


def _shared_case(kw, xkind, P, prec, tol, sample=None):
    hp, op = problems(shared_dw=1, prec=prec, **kw)
    x0 = workloads.points(xkind, P, kw["d"], 13)
    _say(f"[shared] d={kw['d']} M={kw['M']} N={kw['N']} P={P} prec={prec}")
    u, g, st = F.solve(hp, torch.tensor(x0, device=DEV))
    torch.cuda.synchronize()
    u, g, st = u.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy()
    idx = range(P) if sample is None else sample
    for p in idx:
        ref = OS.solve_point(op, x0[p], p)
        eu = abs(u[p] - ref["u"]) / abs(ref["u"])
        eg = rel_err(g[p], ref["grad"])
        _say(f"  p={p} u={u[p]:.12g} ref={ref['u']:.12g} rel_u={eu:.2e} rel_grad={eg:.2e}")
        assert st[p] == 0
        assert eu <= tol and eg <= tol


@pytest.mark.parametrize("name,kw,xkind,P", SHARED_CASES, ids=[c[0] for c in SHARED_CASES])
def test_shared_fp64_matches_oracle(name, kw, xkind, P):
    _shared_case(kw, xkind, P, F.F64, 1e-10, sample=[0, 1, P - 1] if P > 5 else None)


@pytest.mark.parametrize("name,kw,xkind,P", SHARED_CASES, ids=[c[0] for c in SHARED_CASES])
def test_shared_fp32c_matches_fp64_oracle(name, kw, xkind, P):
    _shared_case(kw, xkind, P, F.F32C, 1e-5, sample=[0, P - 1])


def test_shared_affine_closed_form():
    d, M, N, T, c1, b = 12, 60, 4, 0.5, 0.6, 0.3
    rng = np.random.default_rng(5)
    a = rng.standard_normal(d)
    hp, _ = problems(gvec=a, shared_dw=1, d=d, M=M, N=N, T=T, s=1.2, f_kind=F.F_ALLEN_CAHN, fp=(c1, 0, 0, 0),
                     g_kind=F.G_AFFINE, gp=(b, 0, 0, 0), ridge_rel=0.0)
    x0 = rng.standard_normal((7, d))
    _say("[shared affine]")
    u, g, st = F.solve(hp, torch.tensor(x0, device=DEV))
    torch.cuda.synchronize()
    fac = (1 - c1 * T / N) ** N
    for p in range(7):
        assert abs(u[p].item() - (a @ x0[p] + b) / fac) <= 1e-11 * max(1, abs((a @ x0[p] + b) / fac))
        assert rel_err(g[p].cpu().numpy(), a / fac) <= 1e-10


def _shared_adjoint_case(kw, xkind, P, prec, tol, sample):
    hp, op = problems(shared_dw=1, prec=prec, **kw)
    x0 = workloads.points(xkind, P, kw["d"], 17)
    ubar = np.linspace(0.5, 1.5, P)
    _say(f"[shared-adjoint] d={kw['d']} M={kw['M']} N={kw['N']} P={P} prec={prec}")
    xt = torch.tensor(x0, device=DEV)
    ws = F.workspace(hp, P, tape=True)
    u, g, st = F.solve(hp, xt, tape=True, ws=ws)
    x0b, gpb, fpb, st2 = F.solve_backward(hp, xt, torch.tensor(ubar, device=DEV), ws)
    torch.cuda.synchronize()
    x0b = x0b.cpu().numpy()
    gp_ref, fp_ref = np.zeros(4), np.zeros(4)
    for p in range(P):
        ref = OS.adjoint_point(op, x0[p], p, ubar=ubar[p])
        gp_ref += ref["gpbar"]
        fp_ref += ref["fpbar"]
        if p in sample:
            e = rel_err(x0b[p], ref["x0bar"])
            _say(f"  p={p} rel_x0bar={e:.2e}")
            assert e <= tol
    for got, ref, name in ((gpb.cpu().numpy(), gp_ref, "gp"), (fpb.cpu().numpy(), fp_ref, "fp")):
        for i in range(4):
            if ref[i] != 0.0 or got[i] != 0.0:
                err = abs(got[i] - ref[i]) / max(abs(ref[i]), 1e-300)
                _say(f"  {name}[{i}] got={got[i]:.12g} ref={ref[i]:.12g} rel={err:.2e}")
                assert err <= tol, (name, i)
    assert np.all(st.cpu().numpy() == 0) and np.all(st2.cpu().numpy() == 0)


@pytest.mark.parametrize("name,kw,xkind,P", SHARED_CASES, ids=[c[0] for c in SHARED_CASES])
def test_shared_adjoint_fp64_matches_oracle(name, kw, xkind, P):
    _shared_adjoint_case(kw, xkind, P, F.F64, 1e-10, sample=[0, 1, P - 1])


@pytest.mark.parametrize("name,kw,xkind,P", SHARED_CASES, ids=[c[0] for c in SHARED_CASES])
def test_shared_adjoint_fp32c_matches_fp64_oracle(name, kw, xkind, P):
    _shared_adjoint_case(kw, xkind, P, F.F32C, 1e-5, sample=[0, P - 1])


def test_shared_adjoint_affine_closed_form():
    """Affine g with f = c1 y: u(0, x) = (a.x + b) / (1 - c1 dt)^N exactly, so the adjoint of
    sum_p ubar_p u_p is x0bar_p = ubar_p a / (1 - c1 dt)^N and gpbar_0 = sum_p ubar_p / (1 - c1 dt)^N."""
    d, M, N, T, c1, b = 12, 60, 4, 0.5, 0.6, 0.3
    rng = np.random.default_rng(5)
    a = rng.standard_normal(d)
    hp, _ = problems(gvec=a, shared_dw=1, d=d, M=M, N=N, T=T, s=1.2, f_kind=F.F_ALLEN_CAHN, fp=(c1, 0, 0, 0),
                     g_kind=F.G_AFFINE, gp=(b, 0, 0, 0), ridge_rel=0.0)
    P = 7
    x0 = torch.tensor(rng.standard_normal((P, d)), device=DEV)
    ubar = torch.linspace(1.0, 2.0, P, dtype=torch.float64, device=DEV)
    _say("[shared affine adjoint]")
    ws = F.workspace(hp, P, tape=True)
    F.solve(hp, x0, tape=True, ws=ws)
    x0b, gpb, fpb, st = F.solve_backward(hp, x0, ubar, ws)
    torch.cuda.synchronize()
    fac = (1 - c1 * T / N) ** N
    for p in range(P):
        assert rel_err(x0b[p].cpu().numpy(), ubar[p].item() * a / fac) <= 1e-10
    assert abs(gpb[0].item() - ubar.sum().item() / fac) <= 1e-10 * abs(ubar.sum().item() / fac)


def test_shared_adjoint_against_central_differences():
    kw = dict(d=150, M=120, N=3, T=0.3, f_kind=F.F_HJB, fp=(0.7, 0, 0, 0), g_kind=F.G_HJB_LOG, gp=(1.0, 0, 0, 0))
    hp, _ = problems(shared_dw=1, **kw)
    P = 3
    x0 = torch.tensor(workloads.points("uniform", P, 150, 3), device=DEV)
    ubar = torch.ones(P, dtype=torch.float64, device=DEV)
    _say("[shared adjoint] central differences")
    ws = F.workspace(hp, P, tape=True)
    F.solve(hp, x0, tape=True, ws=ws)
    x0b, _, _, _ = F.solve_backward(hp, x0, ubar, ws)
    torch.cuda.synchronize()
    h = 1e-4
    for p, i in [(0, 0), (1, 77), (2, 149)]:
        xp, xm = x0.clone(), x0.clone()
        xp[p, i] += h
        xm[p, i] -= h
        up, _, _ = F.solve(hp, xp)
        um, _, _ = F.solve(hp, xm)
        fd = (up.sum().item() - um.sum().item()) / (2 * h)
        _say(f"  p={p} i={i} adjoint={x0b[p, i].item():.10g} fd={fd:.10g}")
        assert abs(x0b[p, i].item() - fd) <= 1e-6 * max(1.0, abs(fd))
