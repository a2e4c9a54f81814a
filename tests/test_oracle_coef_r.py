"""Pins of the oracle's scheme R under x-dependent coefficients mu = mu0 x + mu1, sigma = diag(sigma0 x + sigma1)
(Sec. 2.1's problem class; eq. Xk's Euler-Maruyama particles): CPU only.

* Constant coefficients (mu0 = sigma0 = 0): solve_point_coef equals the constant-coefficient scheme
  (solve_point with mu = mu1, s = sigma1) to rounding, for Allen-Cahn and HJB (whose Z enters f).
* Affine closed form: f = 0 and an affine g make every level's regression exact (ridge 0, M > d + 1), so
  u(0, x0) = gvec . m_N(x0) + b with the Euler-Maruyama mean m_N, and grad u = gvec (1 + mu0 dt)^N, to rounding,
  for every M and seed (geometric, Ornstein-Uhlenbeck and mixed coefficients).
* The moment recursion behind the bandwidth and ridge: the particles' sample mean and mean squared
  deviation at t_N match m_N and V_N within four standard errors (d = 3, 20000 particles).
"""
import numpy as np
import pytest

from oracle import scheme as OS


@pytest.mark.parametrize("fk,fp", [(OS.F_ALLEN_CAHN, (1.0, 1.0, 0, 0)), (OS.F_HJB, (0.7, 0, 0, 0)),
                                   (OS.F_BURGERS, (0.2, 1.5, 0, 0))])
def test_constant_coefficients_reduce_to_scheme_r(fk, fp):
    d, M, N = 6, 64, 3
    pb = OS.Problem(d=d, M=M, N=N, T=0.3, s=1.3, mu=np.full(d, 0.2), f_kind=fk, fp=fp, g_kind=OS.G_AC,
                    gp=(0.4, 0, 0, 0), seed=3)
    x0 = np.linspace(-0.3, 0.4, d)
    r0 = OS.solve_point(pb, x0, 1)
    r1 = OS.solve_point_coef(pb.copy(mu=None, s=9.0), x0, 1, (0.0, 0.0, 0.2, 1.3))
    assert abs(r0["u"] - r1["u"]) <= 1e-14 * abs(r0["u"])
    assert np.max(np.abs(r0["grad"] - r1["grad"])) <= 1e-13 * np.max(np.abs(r0["grad"]))


@pytest.mark.parametrize("coef", [(0.1, 0.3, 0.0, 0.0), (-0.8, 0.0, 0.2, 0.5), (0.05, 0.2, -0.1, 0.4)])
def test_affine_closed_form(coef):
    d, M, N, T = 5, 40, 4, 0.6
    rng = np.random.default_rng(2)
    gvec = rng.normal(size=d)
    pb = OS.Problem(d=d, M=M, N=N, T=T, g_kind=OS.G_AFFINE, gp=(0.3, 0, 0, 0), gvec=gvec, ridge_rel=0.0,
                    eps_h=1.0, seed=11)
    x0 = rng.uniform(0.5, 1.5, size=d)
    ms, _ = OS.coef_moments(pb, x0, coef)
    mu0 = coef[0]
    for p in range(2):
        r = OS.solve_point_coef(pb, x0, p, coef)
        exact = float(gvec @ ms[N]) + 0.3
        assert abs(r["u"] - exact) <= 1e-11 * max(abs(exact), 1.0)
        assert np.allclose(r["grad"], gvec * (1.0 + mu0 * T / N) ** N, rtol=1e-10, atol=1e-12)


def test_moment_recursion_matches_the_particles():
    d, M, N, T = 3, 20000, 8, 0.8
    coef = (0.3, 0.25, -0.2, 0.4)
    pb = OS.Problem(d=d, M=M, N=N, T=T, seed=5)
    x0 = np.array([0.8, -0.5, 1.2])
    X = OS.coef_path(pb, x0, 0, coef)
    ms, Vs = OS.coef_moments(pb, x0, coef)
    XN = X[N]
    mean = XN.mean(axis=0)
    se = XN.std(axis=0) / np.sqrt(M)
    assert np.all(np.abs(mean - ms[N]) <= 4.0 * se)
    dev2 = np.einsum("ij,ij->i", XN - ms[N][None, :], XN - ms[N][None, :])
    assert abs(dev2.mean() - Vs[N]) <= 4.0 * dev2.std() / np.sqrt(M)
