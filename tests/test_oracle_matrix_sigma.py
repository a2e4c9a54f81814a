"""Pins of the oracle's scheme R under a constant diffusion matrix sigma (Sec. 2.1's problem class,
Z = sigma^T grad u): CPU only.

* sigma = s I reduces to the scalar scheme (solve_point) to rounding, with a drift, for Allen-Cahn, HJB
  (Z in f) and Burgers.
* Rotation: sigma = s Q with Q orthogonal, x0 = 0, no drift and a radial g give the scalar scheme's u
  exactly in law and here exactly (the kernel metric, the ridge metric and Z are all invariant), with
  grad u rotated by Q.
* General linear map: sigma = s L (L invertible, non-symmetric) with g(x) = gvec_A . x + b equals the
  scalar scheme with g(x) = (L^T gvec_A) . x + b at a point of the same g-value, for nonlinear f and a
  positive ridge: u equal, grad u mapped by L^{-T}.  This pins the kernel metric (Sigma^{-1}), the ridge
  metric (sigma sigma^T, not sigma^T sigma) and Z = sigma^T alpha_x against the scalar scheme.
* Affine closed form: f = 0, g affine and no ridge make every regression exact, u = gvec . (x0 + mu T) + b
  and grad u = gvec, for a non-symmetric sigma.
* The path: the cloud's sample covariance at t_N matches T sigma sigma^T within sampling error.
"""
import numpy as np
import pytest

from oracle import scheme as OS


def _rand_sigma(d, seed, s=1.2):
    rng = np.random.default_rng(seed)
    return s * (np.eye(d) + 0.25 * rng.normal(size=(d, d)) / np.sqrt(d))


@pytest.mark.parametrize("fk,fp", [(OS.F_ALLEN_CAHN, (1.0, 1.0, 0, 0)), (OS.F_HJB, (0.7, 0, 0, 0)),
                                   (OS.F_BURGERS, (0.2, 1.5, 0, 0))])
def test_scalar_sigma_reduces_to_scheme_r(fk, fp):
    d, M, N, s = 6, 64, 3, 1.3
    pb = OS.Problem(d=d, M=M, N=N, T=0.3, s=s, mu=np.full(d, 0.2), f_kind=fk, fp=fp, g_kind=OS.G_AC,
                    gp=(0.4, 0, 0, 0), seed=3)
    x0 = np.linspace(-0.3, 0.4, d)
    r0 = OS.solve_point(pb, x0, 1)
    r1 = OS.solve_point_matrix_sigma(pb.copy(s=9.0), x0, 1, s * np.eye(d))
    assert abs(r0["u"] - r1["u"]) <= 1e-13 * abs(r0["u"])
    assert np.max(np.abs(r0["grad"] - r1["grad"])) <= 1e-12 * np.max(np.abs(r0["grad"]))


@pytest.mark.parametrize("fk,fp", [(OS.F_ALLEN_CAHN, (1.0, 1.0, 0, 0)), (OS.F_HJB, (0.7, 0, 0, 0))])
def test_rotated_sigma_is_invariant(fk, fp):
    d, M, N, s = 8, 96, 3, 1.1
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(rng.normal(size=(d, d)))
    pb = OS.Problem(d=d, M=M, N=N, T=0.4, s=s, f_kind=fk, fp=fp, g_kind=OS.G_AC, gp=(0.4, 0, 0, 0), seed=6)
    x0 = np.zeros(d)
    r0 = OS.solve_point(pb, x0, 2)
    r1 = OS.solve_point_matrix_sigma(pb, x0, 2, s * Q)
    # X = s Q W: the same cloud rotated, with the same weights, ridge and Z
    assert abs(r0["u"] - r1["u"]) <= 1e-12 * abs(r0["u"])
    assert np.max(np.abs(Q @ r0["grad"] - r1["grad"])) <= 1e-10 * max(np.max(np.abs(r0["grad"])), 1e-300)


@pytest.mark.parametrize("fk,fp", [(OS.F_ALLEN_CAHN, (1.0, 1.0, 0, 0)), (OS.F_HJB, (0.7, 0, 0, 0)),
                                   (OS.F_BURGERS, (0.2, 1.5, 0, 0))])
def test_general_linear_map_equivariance(fk, fp):
    d, M, N, s, T = 6, 48, 3, 1.2, 0.4
    rng = np.random.default_rng(9)
    L = np.eye(d) + 0.4 * rng.normal(size=(d, d)) / np.sqrt(d)
    assert np.max(np.abs(L - L.T)) > 0.1
    ga = rng.normal(size=d) * 0.5
    gb = L.T @ ga
    mua = rng.normal(size=d) * 0.2
    mub = gb * (ga @ mua) / (gb @ gb)
    x0a = rng.uniform(-0.5, 0.5, size=d)
    x0b = gb * (ga @ x0a) / (gb @ gb)
    common = dict(d=d, M=M, N=N, T=T, f_kind=fk, fp=fp, g_kind=OS.G_LOGISTIC, gp=(0.1, 0, 0, 0), seed=12)
    pa = OS.Problem(s=7.0, mu=mua, gvec=ga, **common)
    pb = OS.Problem(s=s, mu=mub, gvec=gb, **common)
    ra = OS.solve_point_matrix_sigma(pa, x0a, 1, s * L)
    rb = OS.solve_point(pb, x0b, 1)
    assert abs(ra["u"] - rb["u"]) <= 1e-12 * abs(rb["u"])
    ref = np.linalg.solve(L.T, rb["grad"])
    assert np.max(np.abs(ra["grad"] - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_affine_closed_form_nonsymmetric_sigma():
    d, M, N, T = 5, 40, 4, 0.6
    rng = np.random.default_rng(2)
    gvec = rng.normal(size=d)
    mu = rng.normal(size=d) * 0.3
    sigma = _rand_sigma(d, 7)
    assert np.max(np.abs(sigma - sigma.T)) > 0.05
    pb = OS.Problem(d=d, M=M, N=N, T=T, mu=mu, g_kind=OS.G_AFFINE, gp=(0.3, 0, 0, 0), gvec=gvec, ridge_rel=0.0,
                    eps_h=1.0, seed=11)
    x0 = rng.uniform(-1, 1, size=d)
    for p in range(2):
        r = OS.solve_point_matrix_sigma(pb, x0, p, sigma)
        exact = float(gvec @ (x0 + mu * T)) + 0.3
        assert abs(r["u"] - exact) <= 1e-12 * max(abs(exact), 1.0)
        assert np.allclose(r["grad"], gvec, rtol=1e-11, atol=1e-12)


def test_path_covariance():
    d, M, N, T = 3, 20000, 4, 0.8
    sigma = _rand_sigma(d, 1, s=0.9)
    pb = OS.Problem(d=d, M=M, N=N, T=T, mu=np.array([0.1, -0.2, 0.3]), seed=5)
    x0 = np.array([0.5, -0.5, 1.0])
    X = OS.matrix_sigma_path(pb, x0, 0, sigma)
    D = X[N] - (x0 + pb.mu * T)[None, :]
    cov = D.T @ D / M
    ref = T * sigma @ sigma.T
    # each entry's standard error is at most sqrt(2 / M) times the product of the two diagonal scales
    se = np.sqrt(np.outer(np.diag(ref), np.diag(ref)) * 2.0 / M)
    assert np.all(np.abs(cov - ref) <= 5.0 * se)
    assert np.all(np.abs(D.mean(axis=0)) <= 5.0 * np.sqrt(np.diag(ref) / M))
