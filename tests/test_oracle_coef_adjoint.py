"""Pins of the oracle's reverse mode under x-dependent coefficients mu = mu0 x + mu1, sigma = diag(sigma0 x + sigma1)
(Sec. 2.1's problem class, eq. Xk's particles; the design, the kernel weights and the ridge then depend on x0):
CPU only.

* Central differences of the oracle's forward solve in x0 (every coordinate), in gp0 and in fp0, for Allen-Cahn,
  HJB (Z per particle in f) and Burgers, for geometric, Ornstein-Uhlenbeck and mixed coefficients; on a
  full-rank and a rank-deficient design (M < d, the dual solve); with uniform weights (h = 0).
* Constant coefficients (mu0 = sigma0 = 0): equals the constant-coefficient reverse mode (adjoint_point with
  mu = mu1, s = sigma1), whose design does not depend on x0.
* Affine closed form: f = 0, affine g, no ridge: u(0, x0) = gvec . m_N(x0) + b exactly, so
  d u / d x0 = gvec (1 + mu0 dt)^N for every draw of the increments.
"""
import numpy as np
import pytest

from oracle import scheme as OS

AC = (OS.F_ALLEN_CAHN, (1.0, 1.0, 0, 0))
HJB = (OS.F_HJB, (0.7, 0, 0, 0))
BURG = (OS.F_BURGERS, (0.2, 1.5, 0, 0))
COEFS = {"geometric": (0.1, 0.3, 0.0, 0.0), "ou": (-0.8, 0.0, 0.2, 0.5), "mixed": (0.05, 0.2, -0.1, 0.4)}


def _pb(fam, d=4, M=30, N=3, eps_h=1.0, ridge=1e-3):
    fk, fp = fam
    return OS.Problem(d=d, M=M, N=N, T=0.4, f_kind=fk, fp=fp, g_kind=OS.G_AC, gp=(0.4, 0, 0, 0), eps_h=eps_h,
                      ridge_rel=ridge, seed=3)


def _central(fun, x, h=1e-6):
    x = np.asarray(x, dtype=np.float64)
    out = np.empty(x.size)
    for i in range(x.size):
        e = np.zeros(x.size)
        e[i] = h
        out[i] = (fun(x + e) - fun(x - e)) / (2.0 * h)
    return out


def _check_fd(pb, coef, x0, p=1, tol=1e-7):
    r = OS.adjoint_point_coef(pb, x0, p, coef, ubar=1.0)
    fd = _central(lambda z: OS.solve_point_coef(pb, z, p, coef)["u"], x0)
    assert np.max(np.abs(r["x0bar"] - fd)) <= tol * np.max(np.abs(fd))
    h = 1e-6
    gpp = lambda dg: pb.copy(gp=(pb.gp[0] + dg,) + tuple(pb.gp[1:]))
    fdg = (OS.solve_point_coef(gpp(h), x0, p, coef)["u"] - OS.solve_point_coef(gpp(-h), x0, p, coef)["u"]) / (2 * h)
    assert abs(r["gpbar"][0] - fdg) <= tol * max(abs(fdg), 1e-3)
    fpp = lambda df: pb.copy(fp=(pb.fp[0] + df,) + tuple(pb.fp[1:]))
    fdf = (OS.solve_point_coef(fpp(h), x0, p, coef)["u"] - OS.solve_point_coef(fpp(-h), x0, p, coef)["u"]) / (2 * h)
    assert abs(r["fpbar"][0] - fdf) <= tol * max(abs(fdf), 1e-2)


@pytest.mark.parametrize("coef", list(COEFS.values()), ids=list(COEFS))
@pytest.mark.parametrize("fam", [AC, HJB, BURG], ids=["ac", "hjb", "burgers"])
def test_central_differences(fam, coef):
    _check_fd(_pb(fam), coef, np.linspace(0.3, 0.9, 4))


def test_central_differences_rank_deficient_and_uniform_weights():
    _check_fd(_pb(AC, d=6, M=3), COEFS["mixed"], np.linspace(0.3, 0.9, 6))
    _check_fd(_pb(HJB, eps_h=0.0), COEFS["mixed"], np.linspace(0.3, 0.9, 4))


@pytest.mark.parametrize("fam", [AC, HJB, BURG], ids=["ac", "hjb", "burgers"])
def test_constant_coefficients_reduce_to_scheme_r(fam):
    d = 5
    pb = _pb(fam, d=d, M=40)
    x0 = np.linspace(-0.3, 0.4, d)
    r0 = OS.adjoint_point(pb.copy(s=1.3, mu=np.full(d, 0.2)), x0, 1, ubar=0.7)
    r1 = OS.adjoint_point_coef(pb.copy(s=9.0), x0, 1, (0.0, 0.0, 0.2, 1.3), ubar=0.7)
    for key in ("x0bar", "gpbar", "fpbar"):
        scale = max(np.max(np.abs(r0[key])), 1e-300)
        assert np.max(np.abs(r0[key] - r1[key])) <= 1e-12 * scale, key


@pytest.mark.parametrize("coef", list(COEFS.values()), ids=list(COEFS))
def test_affine_closed_form(coef):
    d, M, N, T = 5, 40, 4, 0.6
    rng = np.random.default_rng(2)
    gvec = rng.normal(size=d)
    pb = OS.Problem(d=d, M=M, N=N, T=T, g_kind=OS.G_AFFINE, gp=(0.3, 0, 0, 0), gvec=gvec, ridge_rel=0.0,
                    eps_h=1.0, seed=11)
    x0 = rng.uniform(0.5, 1.5, size=d)
    r = OS.adjoint_point_coef(pb, x0, 0, coef, ubar=1.0)
    exact = gvec * (1.0 + coef[0] * T / N) ** N
    assert np.max(np.abs(r["x0bar"] - exact)) <= 1e-10 * np.max(np.abs(exact))
    assert abs(r["gpbar"][0] - 1.0) <= 1e-12


def test_moment_tangents_against_differences():
    d = 3
    pb = OS.Problem(d=d, M=8, N=6, T=0.6, seed=1)
    coef = COEFS["mixed"]
    x0 = np.array([0.7, -0.4, 1.1])
    _, dVs = OS.coef_moment_tangents(pb, x0, coef)
    for k in (1, 3, 6):
        fd = _central(lambda z: OS.coef_moments(pb, z, coef)[1][k], x0)
        assert np.max(np.abs(dVs[k] - fd)) <= 1e-8 * np.max(np.abs(fd))
