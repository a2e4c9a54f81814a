"""GPU parity of the reverse mode of scheme R under x-dependent coefficients mu(x) = mu0 x + mu1,
sigma(x) = diag(sigma0 x + sigma1) (Sec. 2.1's problem class, eq. Xk's particles): fbsde_solve_coef_backward
after a taped fbsde_solve_coef, against the oracle's reverse mode on identical seeded inputs.

Here x0 moves the regression design, the kernel weights and the ridge of every level.  Covered: the
geometric, Ornstein-Uhlenbeck and mixed families; Allen-Cahn, HJB (Z per particle in f) and Burgers; FP64
(1e-9) and FP32C (1e-5); full-rank and rank-deficient designs (FP32C ones taped with the FP64 state); uniform
weights; a two-wave team (d = 2000);
central differences of the GPU forward; the constant-coefficient reduction to fbsde_solve_backward; the
affine closed form; the tape's checks and the empty call.
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
    # (name, d, M, N, T, P, prec, f, coef, eps_h, tol)
    ("ac_full_rank_f64", 20, 384, 4, 0.3, 3, F.F64, "ac", GEO, 1.0, 1e-9),
    ("hjb_rank_deficient_f64", 60, 40, 3, 0.3, 2, F.F64, "hjb", OU, 1.0, 1e-9),
    ("burgers_mixed_f64", 16, 200, 3, 0.3, 2, F.F64, "burgers", MIX, 1.0, 1e-9),
    ("hjb_uniform_weights_f64", 12, 150, 3, 0.3, 2, F.F64, "hjb", MIX, 0.0, 1e-9),
    ("burgers_two_wave_f64", 2000, 256, 2, 0.05, 2, F.F64, "burgers", MIX, 1.0, 1e-9),
    ("ac_mixed_f32c", 20, 512, 4, 0.3, 3, F.F32C, "ac", MIX, 1.0, 1e-5),
    ("hjb_geometric_f32c", 40, 300, 3, 0.3, 2, F.F32C, "hjb", GEO, 1.0, 1e-5),
    # rank-deficient in FP32C: the taped solve and the reverse mode keep the state in FP64 (below)
    ("burgers_rank_deficient_f32c", 80, 64, 3, 0.3, 2, F.F32C, "burgers", OU, 1.0, 1e-5),
    # the smallest problem (d = 1, M = 2, one level) and the widest team (d = 10^4: 16-wave rows)
    ("ac_smallest_f64", 1, 2, 1, 0.3, 2, F.F64, "ac", MIX, 1.0, 1e-9),
    ("hjb_d10000_team16_f32c", 10000, 64, 2, 0.05, 1, F.F32C, "hjb", MIX, 1.0, 1e-5),
]


def test_rank_deficient_fp32c_tape_keeps_fp64_state():
    # the adjoint's right-hand side reaches the ridge-only null space of a rank-deficient design, where FP32
    # rounding of the state would come back scaled by 1 / lambda (1.6e-5 measured on the case above): the
    # taped solve sizes and runs the FP64 state there, and only there
    kw = dict(N=3, T=0.3, f_kind=F.F_BURGERS, fp=(0.2, 1.5, 0, 0), g_kind=F.G_AC, gp=(0.4, 0, 0, 0))
    for d, M, fp64_state in ((80, 64, True), (80, 81, True), (80, 82, False)):
        h32, _ = problems(d=d, M=M, prec=F.F32C, **kw)
        h64, _ = problems(d=d, M=M, prec=F.F64, **kw)
        taped32 = F.coef_workspace_size(h32, 4, *OU, tape=True)
        assert (taped32 == F.coef_workspace_size(h64, 4, *OU, tape=True)) == fp64_state
        assert F.coef_workspace_size(h32, 4, *OU) < F.coef_workspace_size(h64, 4, *OU)


def _x0(P, d, seed):
    return np.random.default_rng(seed).uniform(0.5, 1.5, size=(P, d)) / np.sqrt(d / 20.0)


def _forward_backward(hp, x0, coef, ubar):
    ws = torch.empty(max(F.coef_workspace_size(hp, x0.shape[0], *coef, tape=True), 1), dtype=torch.uint8,
                     device=DEV)
    u, g, st = F.solve_coef(hp, x0, *coef, ws=ws, tape=True)
    xb, gpb, fpb, stb, it = F.solve_coef_backward(hp, x0, ubar, ws, *coef, return_iters=True)
    torch.cuda.synchronize()
    return u, xb, gpb, fpb, st, stb, it


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_coef_adjoint_against_oracle(case):
    name, d, M, N, T, P, prec, fam, coef, eps_h, tol = case
    fk, fp = FAM[fam]
    hp, op = problems(d=d, M=M, N=N, T=T, prec=prec, f_kind=fk, fp=fp, g_kind=F.G_AC, gp=(0.4, 0, 0, 0),
                      eps_h=eps_h, seed=4, instance=5)
    x0 = _x0(P, d, d + M)
    ubar = np.linspace(0.5, 1.5, P)
    _say(f"[coef adjoint] {name}: d={d} M={M} N={N} P={P} prec={prec} coef={coef}")
    u, xb, gpb, fpb, st, stb, it = _forward_backward(hp, torch.tensor(x0, device=DEV), coef,
                                                     torch.tensor(ubar, device=DEV))
    _say(f"  adjoint cg iterations per level {it}")
    xb, gpb, fpb = xb.cpu().numpy(), gpb.cpu().numpy(), fpb.cpu().numpy()
    gp_ref, fp_ref = np.zeros(4), np.zeros(4)
    for p in range(P):
        ref = OS.adjoint_point_coef(op, x0[p], p, coef, ubar=ubar[p])
        e = rel_err(xb[p], ref["x0bar"])
        _say(f"  p={p} rel_x0bar={e:.2e}")
        assert e <= tol
        gp_ref += ref["gpbar"]
        fp_ref += ref["fpbar"]
    eg, ef = rel_err(gpb[:2], gp_ref[:2]), rel_err(fpb[:2], fp_ref[:2])
    _say(f"  gp_bar {gpb[:2]} ref {gp_ref[:2]} ({eg:.2e}); fp_bar {fpb[:2]} ref {fp_ref[:2]} ({ef:.2e})")
    assert eg <= tol and ef <= tol
    assert not st.cpu().numpy().any() and not stb.cpu().numpy().any()


def test_coef_adjoint_against_central_differences():
    # the GPU forward itself, differenced in x0 (FP64, CG at 1e-13): an independent check of the reverse mode
    d, M, N, T, P = 6, 256, 3, 0.3, 2
    fk, fp = FAM["hjb"]
    hp, _ = problems(d=d, M=M, N=N, T=T, f_kind=fk, fp=fp, g_kind=F.G_AC, gp=(0.4, 0, 0, 0), seed=2, instance=1)
    x0 = torch.tensor(_x0(P, d, 5), device=DEV)
    _say("[coef adjoint fd]")
    _, xb, gpb, fpb, *_ = _forward_backward(hp, x0, MIX, torch.ones(P, dtype=torch.float64, device=DEV))
    h = 1e-5
    fd = torch.empty_like(x0)
    for i in range(d):
        e = torch.zeros_like(x0)
        e[:, i] = h
        up = F.solve_coef(hp, x0 + e, *MIX)[0]
        um = F.solve_coef(hp, x0 - e, *MIX)[0]
        fd[:, i] = (up - um) / (2 * h)
    torch.cuda.synchronize()
    e = rel_err(xb.cpu().numpy(), fd.cpu().numpy())
    _say(f"  rel err against central differences {e:.2e}")
    assert e <= 1e-7


@pytest.mark.parametrize("prec,tol", [(F.F64, 1e-10), (F.F32C, 1e-6)], ids=["f64", "f32c"])
def test_constant_coefficients_reduce_to_backward(prec, tol):
    d, M, N, T, P = 24, 256, 3, 0.3, 3
    fk, fp = FAM["hjb"]
    mu1, s1 = 0.2, 1.3
    hp, _ = problems(d=d, M=M, N=N, T=T, prec=prec, s=s1, mu=np.full(d, mu1), f_kind=fk, fp=fp, g_kind=F.G_AC,
                     gp=(0.4, 0, 0, 0), seed=3, instance=2)
    hc, _ = problems(d=d, M=M, N=N, T=T, prec=prec, s=9.0, f_kind=fk, fp=fp, g_kind=F.G_AC, gp=(0.4, 0, 0, 0),
                     seed=3, instance=2)
    x0 = torch.tensor(_x0(P, d, 7), device=DEV)
    ub = torch.tensor([0.3, 1.0, -0.7], dtype=torch.float64, device=DEV)
    _say(f"[coef adjoint const] prec={prec}")
    ws0 = torch.empty(F.workspace_size(hp, P, tape=True), dtype=torch.uint8, device=DEV)
    F.solve(hp, x0, ws=ws0, tape=True)
    x_ref, gp_ref, fp_ref, _ = F.solve_backward(hp, x0, ub, ws0)
    _, xb, gpb, fpb, *_ = _forward_backward(hc, x0, (0.0, 0.0, mu1, s1), ub)
    for a, b in [(xb, x_ref), (gpb[:2], gp_ref[:2]), (fpb[:2], fp_ref[:2])]:
        assert rel_err(a.cpu().numpy(), b.cpu().numpy()) <= tol


@pytest.mark.parametrize("coef", [GEO, OU, MIX], ids=["geometric", "ou", "mixed"])
def test_affine_closed_form(coef):
    # f = 0, affine g, no ridge: u(0, x0) = gvec . m_N(x0) + b, so d u / d x0 = gvec (1 + mu0 dt)^N
    d, M, N, T, P = 12, 200, 4, 0.6, 3
    gvec = np.random.default_rng(2).normal(size=d)
    hp, _ = problems(d=d, M=M, N=N, T=T, g_kind=F.G_AFFINE, gp=(0.3, 0, 0, 0), gvec=gvec, ridge_rel=0.0,
                     eps_h=1.0, seed=11, instance=0)
    x0 = torch.tensor(_x0(P, d, 9), device=DEV)
    _say(f"[coef adjoint affine] coef={coef}")
    _, xb, gpb, _, *_ = _forward_backward(hp, x0, coef, torch.ones(P, dtype=torch.float64, device=DEV))
    exact = np.tile(gvec * (1.0 + coef[0] * T / N) ** N, (P, 1))
    assert rel_err(xb.cpu().numpy(), exact) <= 1e-10
    assert abs(gpb[0].item() - P) <= 1e-10 * P


def test_tape_checks_and_empty():
    d, M, N, T, P = 8, 64, 2, 0.2, 2
    fk, fp = FAM["ac"]
    hp, _ = problems(d=d, M=M, N=N, T=T, f_kind=fk, fp=fp, g_kind=F.G_AC, gp=(0.4, 0, 0, 0))
    x0 = torch.full((P, d), 0.5, dtype=torch.float64, device=DEV)
    ub = torch.ones(P, dtype=torch.float64, device=DEV)
    ws = torch.empty(F.coef_workspace_size(hp, P, *MIX, tape=True), dtype=torch.uint8, device=DEV)
    F.solve_coef(hp, x0, *MIX, ws=ws)            # no tape
    with pytest.raises(F.FbsdeError):
        F.solve_coef_backward(hp, x0, ub, ws, *MIX)
    F.solve_coef(hp, x0, *MIX, ws=ws, tape=True)
    with pytest.raises(F.FbsdeError):           # another family's tape
        F.solve_coef_backward(hp, x0, ub, ws, *GEO)
    F.solve_coef(hp, x0, *MIX, ws=ws, tape=True)
    F.solve_coef_backward(hp, x0, ub, ws, *MIX)
    with pytest.raises(F.FbsdeError):           # the tape is consumed
        F.solve_coef_backward(hp, x0, ub, ws, *MIX)
    # a plain tape (same buffer) is not a coefficient family's
    F.solve(hp, x0, ws=ws, tape=True)
    with pytest.raises(F.FbsdeError):
        F.solve_coef_backward(hp, x0, ub, ws, *MIX)
    e = torch.empty((0, d), dtype=torch.float64, device=DEV)
    xb, gpb, fpb, _ = F.solve_coef_backward(hp, e, torch.empty(0, dtype=torch.float64, device=DEV), ws, *MIX)
    torch.cuda.synchronize()
    assert xb.numel() == 0 and not gpb.any() and not fpb.any()


def test_coef_adjoint_d1000_M4096_sampled_point():
    # the Allen-Cahn shape d = 1000, M = 4096 (FP32C) at three levels; the oracle takes one point of four
    d, M, N, T, P = 1000, 4096, 3, 0.3, 4
    fk, fp = FAM["ac"]
    hp, op = problems(d=d, M=M, N=N, T=T, prec=F.F32C, f_kind=fk, fp=fp, g_kind=F.G_AC, gp=(0.4, 0, 0, 0), seed=8,
                      instance=1)
    x0 = _x0(P, d, 3)
    _say(f"[coef adjoint full] d={d} M={M} N={N} P={P}")
    _, xb, _, _, st, stb, it = _forward_backward(hp, torch.tensor(x0, device=DEV), MIX,
                                                 torch.ones(P, dtype=torch.float64, device=DEV))
    ref = OS.adjoint_point_coef(op, x0[2], 2, MIX)
    e = rel_err(xb[2].cpu().numpy(), ref["x0bar"])
    _say(f"  adjoint cg iterations {it}; rel_x0bar={e:.2e}")
    assert e <= 1e-5
    assert not st.cpu().numpy().any() and not stb.cpu().numpy().any()


def test_autograd_matches_the_entry_points():
    # solve_coef_autograd: torch.autograd through the hand-written reverse mode, equal to the direct calls
    d, M, N, T, P = 10, 200, 3, 0.3, 3
    fk, fp = FAM["burgers"]
    hp, _ = problems(d=d, M=M, N=N, T=T, f_kind=fk, fp=fp, g_kind=F.G_AC, gp=(0.4, 0, 0, 0), seed=6, instance=2)
    x0 = torch.tensor(_x0(P, d, 4), device=DEV, requires_grad=True)
    gp = torch.tensor(hp.gp, dtype=torch.float64, requires_grad=True)
    fpt = torch.tensor(hp.fp, dtype=torch.float64, requires_grad=True)
    w = torch.tensor([0.5, -1.0, 2.0], dtype=torch.float64, device=DEV)
    _say("[coef autograd]")
    u, _, st = F.solve_coef_autograd(hp, x0, *MIX, gp=gp, fp=fpt)
    (u * w).sum().backward()
    _, xb, gpb, fpb, *_ = _forward_backward(hp, x0.detach(), MIX, w)
    assert torch.equal(x0.grad, xb)
    assert torch.equal(gp.grad, gpb.cpu()) and torch.equal(fpt.grad, fpb.cpu())
    assert not st.any()
