"""The direct dual solve of small rank-deficient clouds (d / 8 <= M <= d + 1, M <= FBSDE_DUAL_MAXM): the level's ridge
system (D'^T W D' + lambda I) alpha_x = D'^T W (Y - Ybar) solved through its M x M dual form (the
push-through identity), one Cholesky factorisation per point, instead of the matrix-free CG.

Covered: FP64 (1e-10) and FP32C (1e-5) against the FP64 oracle (whose own solve is the direct dual form for
M <= d); Allen-Cahn, HJB, Burgers, the HJ-type and Case 2 families (f depends on x); M = d + 1, M = 128 and
M = 2; x-dependent coefficients; one level on caller state; the CG (SOLVER_CG) on the same problem agreeing;
zero CG iterations reported for the dual levels.
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


AC = dict(f_kind=F.F_ALLEN_CAHN, fp=(1.0, 1.0, 0, 0), g_kind=F.G_AC, gp=(0.4, 0, 0, 0))
HJB = dict(f_kind=F.F_HJB, fp=(0.7, 0, 0, 0), g_kind=F.G_HJB_LOG, gp=(1.0, 0, 0, 0))
BURG = dict(f_kind=F.F_BURGERS, fp=(0.2, 1.5, 0, 0), g_kind=F.G_AC, gp=(0.4, 0, 0, 0))
HJ = dict(f_kind=F.F_HJ_SINK, fp=(0.1, 0, 0, 0), g_kind=F.G_HJ_GAUSS, gp=(0.5, 0, 0, 0))
C2 = dict(f_kind=F.F_LOG_POT, fp=(0.8, 1.6, 0.25, 0), g_kind=F.G_CASE2, gp=(0.5, 0.25, 0, 0))

CASES = [
    # (name, d, M, N, T, P, prec, family, x0 kind, tol)
    ("ac_d60_M40", 60, 40, 3, 0.3, 3, F.F64, AC, "normal:0.3", 1e-10),
    ("hjb_d200_M100", 200, 100, 3, 0.3, 2, F.F64, HJB, "normal_over_sqrt_d", 1e-10),
    ("burgers_d100_M101", 100, 101, 3, 0.3, 2, F.F64, BURG, "normal:0.2", 1e-10),   # M = d + 1
    ("ac_d300_M128", 300, 128, 2, 0.3, 2, F.F64, AC, "normal:0.2", 1e-10),         # the largest M
    ("ac_d10_M2", 10, 2, 3, 0.3, 2, F.F64, AC, "normal:0.3", 1e-10),               # the smallest M
    ("hj_d500_M100", 500, 100, 4, 0.5, 2, F.F64, HJ, "zero", 1e-10),
    ("case2_d60_M40", 60, 40, 10, 0.5, 2, F.F64, C2, "uniform", 1e-10),
    ("ac_d600_M100_f32c", 600, 100, 3, 0.3, 2, F.F32C, AC, "normal_over_sqrt_d", 1e-5),
    ("hjb_d80_M64_f32c", 80, 64, 3, 0.3, 3, F.F32C, HJB, "normal:0.3", 1e-5),
]


def _x0(kind, P, d, seed):
    if kind == "zero":
        return np.zeros((P, d))
    if kind == "tenth":
        return np.full((P, d), 0.1)
    return workloads.points(kind, P, d, seed)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_dual_against_oracle_and_cg(case):
    name, d, M, N, T, P, prec, fam, xk, tol = case
    hp, op = problems(d=d, M=M, N=N, T=T, prec=prec, seed=2, instance=3, **fam)
    hc, _ = problems(d=d, M=M, N=N, T=T, prec=prec, seed=2, instance=3, solver=F.SOLVER_CG, **fam)
    x0 = _x0(xk, P, d, d + M)
    xt = torch.tensor(x0, device=DEV)
    _say(f"[dual] {name}")
    u, g, st, it = F.solve(hp, xt, return_iters=True)
    uc, gc, stc, itc = F.solve(hc, xt, return_iters=True)
    torch.cuda.synchronize()
    _say(f"  iterations: dual {it} cg {itc}")
    assert it == [0] * N and min(itc) > 0
    u, g = u.cpu().numpy(), g.cpu().numpy()
    for p in range(P):
        ref = OS.solve_point(op, x0[p], p)
        eu = abs(u[p] - ref["u"]) / max(abs(ref["u"]), 1e-300)
        eg = rel_err(g[p], ref["grad"])
        _say(f"  p={p} u={u[p]:.12g} ref={ref['u']:.12g} rel_u={eu:.2e} rel_grad={eg:.2e}")
        assert ref["status"] == 0 and eu <= tol and eg <= tol
    assert not st.cpu().numpy().any() and not stc.cpu().numpy().any()
    # the two solves of the same regression agree to the CG tolerance
    assert rel_err(u, uc.cpu().numpy()) <= tol and rel_err(g, gc.cpu().numpy()) <= 10 * tol


def test_dual_with_x_dependent_coefficients():
    d, M, N, T, P = 120, 60, 3, 0.3, 2
    coef = (0.05, 0.2, -0.1, 0.4)
    hp, op = problems(d=d, M=M, N=N, T=T, seed=4, instance=5, **AC)
    x0 = np.random.default_rng(1).uniform(0.5, 1.5, size=(P, d)) / np.sqrt(d / 20.0)
    _say("[dual coef]")
    u, g, st, it = F.solve_coef(hp, torch.tensor(x0, device=DEV), *coef, return_iters=True)
    torch.cuda.synchronize()
    assert it == [0] * N
    for p in range(P):
        ref = OS.solve_point_coef(op, x0[p], p, coef)
        assert abs(u[p].item() - ref["u"]) <= 1e-10 * abs(ref["u"])
        assert rel_err(g[p].cpu().numpy(), ref["grad"]) <= 1e-10
    assert not st.cpu().numpy().any()


def test_dual_one_level_on_caller_state():
    d, M, N, T, P, k = 40, 30, 3, 0.3, 2, 1
    hp, op = problems(d=d, M=M, N=N, T=T, seed=2, instance=3, **AC)
    x0 = workloads.points("normal:0.4", P, d, seed=11)
    xt = torch.tensor(x0, device=DEV)
    rng = np.random.default_rng(5)
    Wn = rng.normal(size=(P, M, d)) * np.sqrt((k + 1) * T / N)
    ld = F.state_ld(hp)
    Wt = torch.zeros((P, M, ld), dtype=torch.float64, device=DEV)
    Wt[:, :, :d] = torch.tensor(Wn, device=DEV)
    Yn = rng.uniform(0.2, 0.9, size=(P, M))
    _say("[dual step]")
    Y, alpha, alpha_x, st = F.solve_step(hp, k, Wt, torch.tensor(Yn, device=DEV), x0=xt)
    torch.cuda.synchronize()
    Wk = Wt[:, :, :d].cpu().numpy()
    for p in range(P):
        ref = OS.level_step(op, k, Wn[p], Wk[p], Yn[p], x0=x0[p])
        assert rel_err(Y[p].cpu().numpy(), ref["Y"]) <= 1e-10
        assert rel_err(alpha_x[p].cpu().numpy(), ref["alpha_x"]) <= 1e-10
    assert not st.any()


def test_thin_cloud_keeps_cg():
    # M < d / 8: the CG converges in a few iterations there and stays the level's solver
    d, M, N = 1000, 100, 2
    hp, _ = problems(d=d, M=M, N=N, T=0.3, seed=2, instance=3, **AC)
    xt = torch.tensor(workloads.points("normal_over_sqrt_d", 2, d, 4), device=DEV)
    _, _, st, it = F.solve(hp, xt, return_iters=True)
    torch.cuda.synchronize()
    assert min(it) > 0 and not st.any()
