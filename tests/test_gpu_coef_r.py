"""GPU parity of scheme R under x-dependent coefficients mu(x) = mu0 x + mu1, sigma(x) = diag(sigma0 x + sigma1)
(Sec. 2.1's problem class; eq. Xk's Euler-Maruyama particles) against the FP64 oracle on identical seeded inputs.

The state is the displacement from the Euler-Maruyama mean path; the reversal inverts the step from the
regenerated increments; bandwidth and ridge follow the exact moment recursion per point; Z = sigma(X)^T alpha_x
per particle.  Covered: the geometric, Ornstein-Uhlenbeck and mixed families; Allen-Cahn, HJB (Z in f) and
Burgers; FP64 (1e-10) and FP32C (1e-5); full-rank and rank-deficient designs (both precisions); a two-wave team (d = 2000); the
d = 1000, M = 4096 shape on one sampled point; the constant-coefficient reduction to fbsde_solve; the affine
closed form (f = 0, affine g, no ridge: u = gvec . m_N + b exactly); refusals.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_2510_02635_amd as F  # noqa: E402
from oracle import scheme as OS  # noqa: E402

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


GEO, OU, MIX = (0.1, 0.3, 0.0, 0.0), (-0.8, 0.0, 0.2, 0.5), (0.05, 0.2, -0.1, 0.4)
FAM = {"ac": (F.F_ALLEN_CAHN, (1.0, 1.0, 0, 0)), "hjb": (F.F_HJB, (0.7, 0, 0, 0)),
       "burgers": (F.F_BURGERS, (0.2, 1.5, 0, 0))}

CASES = [
    # (d, M, N, T, P, prec, f, coef, tol)
    (20, 384, 4, 0.3, 3, F.F64, "ac", GEO, 1e-10),       # full rank, warm-started CG
    (60, 40, 3, 0.3, 2, F.F64, "hjb", OU, 1e-10),        # rank-deficient (dual) design, Z in f
    (2000, 256, 2, 0.05, 2, F.F64, "burgers", MIX, 1e-10),  # a two-wave team per row
    (20, 512, 4, 0.3, 3, F.F32C, "ac", MIX, 1e-5),       # FP32 state, FP64 Newton
    (40, 300, 3, 0.3, 2, F.F32C, "hjb", GEO, 1e-5),
    # rank-deficient designs on the FP32 state (untaped): the direct dual solve (M >= d / 8) and the CG with
    # FP64 arithmetic (M < d / 8)
    (80, 64, 3, 0.3, 2, F.F32C, "burgers", OU, 1e-5),
    (600, 64, 3, 0.3, 2, F.F32C, "hjb", MIX, 1e-5),
]


def _x0(P, d, seed):
    return np.random.default_rng(seed).uniform(0.5, 1.5, size=(P, d)) / np.sqrt(d / 20.0)


@pytest.mark.parametrize("case", CASES, ids=[f"d{c[0]}_M{c[1]}_{c[6]}_{'f64' if c[5] == F.F64 else 'f32c'}"
                                             for c in CASES])
def test_coef_against_oracle(case):
    d, M, N, T, P, prec, fam, coef, tol = case
    fk, fp = FAM[fam]
    hp, op = problems(d=d, M=M, N=N, T=T, prec=prec, f_kind=fk, fp=fp, g_kind=F.G_AC, gp=(0.4, 0, 0, 0),
                      seed=4, instance=5)
    x0 = _x0(P, d, d + M)
    _say(f"[coef] d={d} M={M} N={N} T={T} P={P} prec={prec} f={fam} coef={coef}")
    u, g, st, it = F.solve_coef(hp, torch.tensor(x0, device=DEV), *coef, return_iters=True)
    torch.cuda.synchronize()
    u, g, st = u.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy()
    _say(f"  cg iterations per level {it}")
    for p in range(P):
        ref = OS.solve_point_coef(op, x0[p], p, coef)
        eu = abs(u[p] - ref["u"]) / abs(ref["u"])
        eg = rel_err(g[p], ref["grad"])
        _say(f"  p={p} u={u[p]:.12g} ref={ref['u']:.12g} rel_u={eu:.2e} rel_grad={eg:.2e}")
        assert st[p] == 0 and ref["status"] == 0
        assert eu <= tol and eg <= tol


def test_coef_d1000_M4096_sampled_point():
    # the Allen-Cahn shape d = 1000, M = 4096 (FP32C) at three levels; the oracle takes one point of four
    d, M, N, T, P = 1000, 4096, 3, 0.3, 4
    hp, op = problems(d=d, M=M, N=N, T=T, prec=F.F32C, f_kind=F.F_ALLEN_CAHN, fp=(1.0, 1.0, 0, 0), g_kind=F.G_AC,
                      gp=(0.4, 0, 0, 0), seed=8, instance=1)
    x0 = _x0(P, d, 3)
    _say(f"[coef full] d={d} M={M} N={N} P={P}")
    u, g, st = F.solve_coef(hp, torch.tensor(x0, device=DEV), *MIX)
    torch.cuda.synchronize()
    ref = OS.solve_point_coef(op, x0[2], 2, MIX)
    eu = abs(u[2].item() - ref["u"]) / abs(ref["u"])
    eg = rel_err(g[2].cpu().numpy(), ref["grad"])
    _say(f"  u={u[2].item():.12g} ref={ref['u']:.12g} rel_u={eu:.2e} rel_grad={eg:.2e}")
    assert eu <= 1e-5 and eg <= 1e-5
    assert not st.cpu().numpy().any()


@pytest.mark.parametrize("fam", ["ac", "hjb"])
def test_constant_coefficients_reduce_to_solve(fam):
    # mu0 = sigma0 = 0: the Euler-Maruyama particles are x0 + mu1 t + sigma1 W, the constant-coefficient scheme
    d, M, N, T, P = 24, 256, 3, 0.3, 3
    fk, fp = FAM[fam]
    mu1, s1 = 0.2, 1.3
    hp, _ = problems(d=d, M=M, N=N, T=T, s=s1, mu=np.full(d, mu1), f_kind=fk, fp=fp, g_kind=F.G_AC,
                     gp=(0.4, 0, 0, 0), seed=3, instance=2)
    hc, _ = problems(d=d, M=M, N=N, T=T, s=9.0, f_kind=fk, fp=fp, g_kind=F.G_AC, gp=(0.4, 0, 0, 0), seed=3,
                     instance=2)
    x0 = torch.tensor(_x0(P, d, 7), device=DEV)
    _say(f"[coef const] f={fam}")
    u0, g0, s0 = F.solve(hp, x0)
    u1, g1, s1_ = F.solve_coef(hc, x0, 0.0, 0.0, mu1, s1)
    torch.cuda.synchronize()
    assert rel_err(u1.cpu().numpy(), u0.cpu().numpy()) <= 1e-11
    assert rel_err(g1.cpu().numpy(), g0.cpu().numpy()) <= 1e-10
    assert not s0.any() and not s1_.any()


@pytest.mark.parametrize("coef", [GEO, OU, MIX], ids=["geometric", "ou", "mixed"])
@pytest.mark.parametrize("prec,tol", [(F.F64, 1e-11), (F.F32C, 1e-5)], ids=["f64", "f32c"])
def test_affine_closed_form(coef, prec, tol):
    # f = 0, g affine and no ridge: every level's regression is exact, u(0, x0) = gvec . m_N(x0) + b and
    # grad u = gvec (1 + mu0 dt)^N, for any increments
    d, M, N, T, P = 12, 200, 4, 0.6, 3
    rng = np.random.default_rng(2)
    gvec = rng.normal(size=d)
    hp, op = problems(d=d, M=M, N=N, T=T, prec=prec, g_kind=F.G_AFFINE, gp=(0.3, 0, 0, 0), gvec=gvec,
                      ridge_rel=0.0, eps_h=1.0, seed=11, instance=0)
    x0 = _x0(P, d, 9)
    _say(f"[coef affine] coef={coef} prec={prec}")
    u, g, st = F.solve_coef(hp, torch.tensor(x0, device=DEV), *coef)
    torch.cuda.synchronize()
    u, g = u.cpu().numpy(), g.cpu().numpy()
    for p in range(P):
        ms, _ = OS.coef_moments(op, x0[p], coef)
        exact = float(gvec @ ms[N]) + 0.3
        assert abs(u[p] - exact) <= tol * max(abs(exact), 1.0)
        assert rel_err(g[p], gvec * (1.0 + coef[0] * T / N) ** N) <= tol
    assert not st.cpu().numpy().any()


def test_coef_refusals_and_empty():
    d, M, N, T = 16, 64, 2, 0.2
    hp, _ = problems(d=d, M=M, N=N, T=T, f_kind=F.F_ALLEN_CAHN, fp=(1.0, 1.0, 0, 0), g_kind=F.G_AC,
                     gp=(0.4, 0, 0, 0))
    x0 = torch.full((2, d), 0.5, dtype=torch.float64, device=DEV)
    for bad in [(0.0, 0.0, 0.0, 0.0), (float("nan"), 0.3, 0.0, 0.0)]:
        with pytest.raises(F.FbsdeError):
            F.solve_coef(hp, x0, *bad)
    hm, _ = problems(d=d, M=M, N=N, T=T, mu=np.full(d, 0.1))   # the family's drift replaces mu
    with pytest.raises(F.FbsdeError):
        F.solve_coef(hm, x0, *GEO)
    hs, _ = problems(d=d, M=M, N=N, T=T, shared_dw=1)
    with pytest.raises(F.FbsdeError):
        F.solve_coef(hs, x0, *GEO)
    hj, _ = problems(d=d, M=M, N=N, T=T, f_kind=F.F_HJ_SINK, fp=(0.1, 0, 0, 0), g_kind=F.G_HJ_GAUSS,
                     gp=(T, 0, 0, 0))
    with pytest.raises(F.FbsdeError):
        F.solve_coef(hj, x0, *GEO)
    # the geometric kind with a nonzero affine part is refused at the boundary
    lib = F._native.load()
    import ctypes
    bad = F._native.CCoef(F._native.COEF_GEOMETRIC, 0, 0.1, 0.3, 0.2, 0.0)
    out = ctypes.c_size_t(0)
    assert lib.fbsde_coef_workspace_size(ctypes.byref(hp.c()), ctypes.byref(bad), 2, 0, ctypes.byref(out)) != 0
    # P = 0 touches nothing
    u, g, st = F.solve_coef(hp, torch.empty((0, d), dtype=torch.float64, device=DEV), *GEO)
    assert u.numel() == 0
