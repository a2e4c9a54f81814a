"""GPU parity of Allen-Cahn Case 2 (Sec. 4.1: log potential f(u) = (theta/2) ln((1+u)/(1-u)) - theta_c u and
the re-derived source that makes a cos(prod_j x_j) e^(cos t - |x|^2) exact) against the FP64 oracle.

The source depends on every coordinate of x through prod_j x_j and sum_i prod_{j != i} x_j^2: the reversal
forms them per particle (per lane, then across the team), the forward sweep forms prod_j x_j for the terminal
value, and the level-0 outputs form the products of the coordinates other than k for d/dx_k of the source.
Steps are small enough (dt <= 0.025 at small d) that Newton stays inside the potential's domain |u| < 1.  Covered:
FP64 (1e-10) at small d where the products are of order one (one coordinate exactly zero, a drift),
a rank-deficient design, a two-wave team (d = 2000), FP32C (1e-5), and the paper's d = 100 evaluation points
x = 0 and x = (0.1, ..., 0.1) with T = 1.  The paths that do not evaluate these families refuse them.
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
TH, THC, AMP = 0.8, 1.6, 0.25


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    F._native.load()


def _c2(d, M, N, T, **kw):
    return problems(d=d, M=M, N=N, T=T, f_kind=F.F_LOG_POT, fp=(TH, THC, AMP, 0), g_kind=F.G_CASE2,
                    gp=(T, AMP, 0, 0), **kw)


def _x0(kind, P, d, seed):
    if kind == "uniform_zero":   # coordinates of order one, one of them exactly zero
        x = workloads.points("uniform", P, d, seed)
        x[:, d // 2] = 0.0
        return x
    if kind == "tenth":
        return np.full((P, d), 0.1)
    return workloads.points(kind, P, d, seed)


CASES = [
    # (d, M, N, T, P, prec, x0 kind, mu, tol)
    (3, 512, 20, 0.5, 3, F.F64, "uniform", False, 1e-10),
    (5, 384, 10, 0.5, 2, F.F64, "uniform_zero", True, 1e-10),
    (60, 40, 10, 0.5, 2, F.F64, "uniform", False, 1e-10),       # rank-deficient (dual) design
    (2000, 256, 2, 0.05, 2, F.F64, "normal:0.1", False, 1e-10),  # a two-wave team per row
    (4, 512, 20, 0.5, 3, F.F32C, "uniform", True, 1e-5),
    # the paper's evaluation points at d = 100, T = 1 (dt = 0.0005: the source's -2d term makes coarser
    # steps leave the potential's domain at x = 0)
    (100, 100, 2000, 1.0, 1, F.F64, "zero", False, 1e-10),
    (100, 100, 2000, 1.0, 1, F.F64, "tenth", False, 1e-10),
]


@pytest.mark.parametrize("case", CASES, ids=[f"d{c[0]}_M{c[1]}_{c[6]}_{'f64' if c[5] == F.F64 else 'f32c'}"
                                             f"{'_mu' if c[7] else ''}" for c in CASES])
def test_case2_against_oracle(case):
    d, M, N, T, P, prec, kind, with_mu, tol = case
    mu = (0.2 * np.cos(np.arange(d))) if with_mu else None
    hp, op = _c2(d, M, N, T, prec=prec, mu=mu, seed=6, instance=7)
    x0 = _x0(kind, P, d, seed=d + M)
    _say(f"[case2] d={d} M={M} N={N} T={T} P={P} prec={prec} x0={kind} mu={with_mu}")
    u, g, st = F.solve(hp, torch.tensor(x0, device=DEV))
    torch.cuda.synchronize()
    u, g, st = u.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy()
    for p in range(P):
        ref = OS.solve_point(op, x0[p], p)
        eu = abs(u[p] - ref["u"]) / abs(ref["u"])
        eg = rel_err(g[p], ref["grad"])
        ex = float(OS.case2_exact(AMP, 0.0, x0[p][None])[0])
        _say(f"  p={p} u={u[p]:.12g} ref={ref['u']:.12g} exact={ex:.6g} rel_u={eu:.2e} rel_grad={eg:.2e}")
        assert st[p] == 0 and ref["status"] == 0
        assert eu <= tol and eg <= tol


def test_case2_refused_where_not_evaluated():
    d, M, N, T = 8, 64, 2, 0.2
    hp, _ = _c2(d, M, N, T)
    x0 = torch.zeros((2, d), dtype=torch.float64, device=DEV)
    ws = F.workspace(hp, 2, tape=True)
    F.solve(hp, x0, tape=True, ws=ws)
    with pytest.raises(F.FbsdeError):
        F.solve_backward(hp, x0, torch.ones(2, dtype=torch.float64, device=DEV), ws)
    with pytest.raises(F.FbsdeError):
        F.solve_literal(hp, x0)
    with pytest.raises(F.FbsdeError):
        F.solve_batched([hp], [x0], mode="persistent")
    # the Case 2 terminal value alone (with an f the shared form evaluates) is refused there too
    hg, _ = problems(d=d, M=M, N=N, T=T, f_kind=F.F_ALLEN_CAHN, fp=(1.0, 1.0, 0, 0), g_kind=F.G_CASE2,
                     gp=(T, AMP, 0, 0), shared_dw=1)
    with pytest.raises(F.FbsdeError):
        F.solve(hg, x0)
