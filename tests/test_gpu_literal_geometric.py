"""GPU parity of the paper-literal scheme under x-dependent coefficients (the affine diagonal family
mu(x) = mu0 x + mu1, sigma(x) = diag(sigma0 x + sigma1); geometric when mu1 = sigma1 = 0) against the FP64 oracle.

Every case compares u, every particle's Y and (|Z|^2, sum Z) at level k_stop element by element, at 1e-10.
|Z|^2 and sum Z get 1e-8 of their largest values plus a floor of 1e-12 |Y|^2 and 1e-10 |Y|: with M << d the
slope is small beside the response, and its error is about eps kappa |Y| with the ridge solve's condition
number kappa (about 1e6 at d = 600), i.e. 1e-10 |Y|. Z = sigma(X^m)^T alpha_x needs the explicit slope. The
cases cover: the first, a middle and the last level; HJB, Burgers-type with logistic g, and Allen-Cahn at
M = 100; uniform weights at d = 1; M = 150 (the tiled Gram path); M = 256; d = 600 (M << d).
"""
import numpy as np
import pytest
import torch

import paper_2510_02635_amd as F
from oracle import literal as OL
from oracle import scheme as OS

pytestmark = pytest.mark.gpu


def _run(kw, P, mu0, s0, k_stop=0, seed=1, mu1=0.0, s1=0.0):
    rng = np.random.default_rng(seed)
    x0 = 1.0 + 0.3 * rng.normal(size=(P, kw["d"]))
    gkw = dict(kw)
    if kw.get("gvec") is not None:
        gkw["gvec"] = torch.tensor(kw["gvec"], device="cuda")
    pb = F.Problem(**gkw)
    print(f"[literal-geometric] d={kw['d']} M={kw['M']} N={kw['N']} P={P} k_stop={k_stop}", flush=True)
    u, st, Y, zs = F.solve_literal_geometric(pb, torch.tensor(x0, device="cuda"), mu0, s0, k_stop=k_stop,
                                             want_Y=True, want_zstats=True, mu1=mu1, sigma1=s1)
    torch.cuda.synchronize()
    u, st, Y, zs = u.cpu().numpy(), st.cpu().numpy(), Y.cpu().numpy(), zs.cpu().numpy()
    opb = OS.Problem(**kw)
    for p in range(P):
        ref = OL.solve_point_geometric(opb, x0[p], p, mu0, s0, k_stop=k_stop, tape=True, mu1=mu1, sigma1=s1)
        assert int(st[p]) == ref["status"] == 0
        assert abs(u[p] - ref["u"]) <= 1e-10 * max(1.0, abs(ref["u"])), (p, u[p], ref["u"])
        assert np.max(np.abs(Y[p] - ref["Y"])) <= 1e-10 * max(1.0, np.max(np.abs(ref["Y"])))
        # Z carries the ridge solve's conditioning relative to the response's scale, so beside 1e-8 of
        # their largest value |Z|^2 and sum Z get a floor in the units of Y: eps kappa ~ 1e-10 at d = 600
        ymax = np.max(np.abs(ref["Y"]))
        for c, key, floor in ((0, "zz", 1e-12 * ymax ** 2), (1, "zs", 1e-10 * ymax)):
            r = ref[key][k_stop]
            assert np.max(np.abs(zs[p, :, c] - r)) <= 1e-8 * np.max(np.abs(r)) + floor, (key, p)


HJB = dict(f_kind=OS.F_HJB, fp=(0.8, 0, 0, 0), g_kind=OS.G_QUAD, gp=(1.0, 0.1, 0, 0))


@pytest.mark.parametrize("k_stop", [0, 2, 3])
def test_geometric_hjb_levels(k_stop):
    _run(dict(d=6, M=20, N=4, T=0.6, ridge_rel=1e-2, seed=3, **HJB), P=3, mu0=0.2, s0=0.5, k_stop=k_stop)


def test_geometric_burgers_logistic():
    d = 10
    kw = dict(d=d, M=40, N=3, T=0.3, f_kind=OS.F_BURGERS, fp=(0.2, 1.5, 0, 0), g_kind=OS.G_LOGISTIC,
              gp=(0.1, 0, 0, 0), gvec=np.full(d, 1.0 / d), ridge_rel=1e-3, seed=5)
    _run(kw, P=2, mu0=-0.1, s0=0.3, k_stop=1)


def test_geometric_allen_cahn_M100():
    kw = dict(d=50, M=100, N=3, T=0.3, f_kind=OS.F_ALLEN_CAHN, fp=(1.0, 1.0, 0, 0), g_kind=OS.G_AC,
              gp=(0.4, 0, 0, 0), ridge_rel=1e-3, seed=6)
    _run(kw, P=2, mu0=0.05, s0=0.2, k_stop=0)


def test_geometric_uniform_weights_d1():
    _run(dict(d=1, M=17, N=3, T=1.0, eps_h=0.0, ridge_rel=5e-2, seed=7, **HJB), P=2, mu0=0.3, s0=0.6, k_stop=1)


def test_geometric_tiled_gram_M150():
    _run(dict(d=8, M=150, N=2, T=0.4, ridge_rel=1e-2, seed=8, **HJB), P=1, mu0=0.1, s0=0.4, k_stop=1)


def test_geometric_rank_deficient_d600():
    _run(dict(d=600, M=48, N=3, T=0.3, ridge_rel=1e-3, seed=9, **HJB), P=2, mu0=0.1, s0=0.3, k_stop=1)


def test_geometric_errors():
    pb = F.Problem(d=8, M=16, N=3, T=0.3, mu=torch.zeros(8, dtype=torch.float64, device="cuda"))
    x = torch.ones((2, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(F.FbsdeError):   # the family's drift replaces the constant one
        F.solve_literal_geometric(pb, x, 0.1, 0.3)
    with pytest.raises(F.FbsdeError):
        F.solve_literal_geometric(F.Problem(d=8, M=16, N=3, T=0.3), x, 0.1, 0.0)
    u, st, _, _ = F.solve_literal_geometric(F.Problem(d=8, M=16, N=3, T=0.3),
                                            torch.empty((0, 8), dtype=torch.float64, device="cuda"), 0.1, 0.3)
    assert u.numel() == 0


def test_geometric_full_size_d1000_M100():
    # the benchmarked shape (d = 1000, M = 100, dt = 0.01, mu0 = 0.05, sigma0 = 0.2) in the bench's launch
    # configuration (64 points), fewer levels; sampled points against the oracle one by one
    d, M, N, P = 1000, 100, 5, 64
    kw = dict(d=d, M=M, N=N, T=0.01 * N, f_kind=OS.F_HJB, fp=(1.0, 0, 0, 0), g_kind=OS.G_HJB_LOG, gp=(1.0, 0, 0, 0),
              ridge_rel=1e-3, seed=0, instance=7)
    print(f"[literal-geometric full size] d={d} M={M} N={N} P={P}", flush=True)
    x0 = np.ones((P, d))
    u, st, Y, zs = F.solve_literal_geometric(F.Problem(**kw), torch.tensor(x0, device="cuda"), 0.05, 0.2,
                                             want_Y=True, want_zstats=True)
    torch.cuda.synchronize()
    u, st, Y = u.cpu().numpy(), st.cpu().numpy(), Y.cpu().numpy()
    assert np.all(st == 0)
    opb = OS.Problem(**kw)
    for p in (0, 31, P - 1):
        ref = OL.solve_point_geometric(opb, x0[p], p, 0.05, 0.2)
        assert abs(u[p] - ref["u"]) <= 1e-10 * abs(ref["u"]), (p, u[p], ref["u"])
        assert np.max(np.abs(Y[p] - ref["Y"])) <= 1e-10 * np.max(np.abs(ref["Y"]))


def test_geometric_largest_M():
    # M = 256: the slice of all displacements needs more than 64 KB of LDS (raised per launch)
    _run(dict(d=40, M=256, N=2, T=0.4, ridge_rel=1e-2, seed=10, **HJB), P=1, mu0=0.1, s0=0.3, k_stop=1)



@pytest.mark.parametrize("mu0,mu1,s0,s1", [(-0.8, 0.2, 0.0, 0.5), (-0.3, 0.1, 0.2, 0.3)])
def test_affine_diag_ou_and_mixed(mu0, mu1, s0, s1):
    # Ornstein-Uhlenbeck drift with additive noise (sigma0 = 0), and all four coefficients at once
    _run(dict(d=10, M=30, N=4, T=0.6, ridge_rel=1e-2, seed=11, **HJB), P=2, mu0=mu0, s0=s0, k_stop=1, mu1=mu1, s1=s1)
    _run(dict(d=10, M=30, N=4, T=0.6, ridge_rel=1e-2, seed=11, **HJB), P=2, mu0=mu0, s0=s0, k_stop=0, mu1=mu1, s1=s1)
