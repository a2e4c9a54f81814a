"""Pins of the oracle's paper-literal per-anchor scheme (Algorithm 1 as printed, Sec. 2.3 to 2.5).

* Each anchor's fit is checked against scikit-learn's weighted ridge regression on the design [1, D]
  with no separate intercept. That is the functional J_lambda of the ridge remark, intercept
  included. Both forms (primal and dual) are checked.
* The kernel weights are checked against the weight-ratio identity of the kernel remark. They are
  uniform at level 0 and largest at the anchor itself.
* For an f that does not depend on z (Allen-Cahn), every particle's Y is the same below the terminal
  level. u is then N implicit steps of the scalar equation y = c + dt f(y), started from the mean of
  g over the cloud; each step's root is checked against bisection.
* HJB (f = -lam |z|^2) and the Burgers-type f = c (y - kappa) sum z are checked at the first backward
  level. Y^m has closed forms there, in the slope that scikit-learn fits. This pins Z = s alpha_x and
  the sign of f.
* At level 0 the design is zero, so the slope is exactly zero.
* Affine diagonal family (mu = mu0 x + mu1, sigma = diag(sigma0 x + sigma1); geometric for mu1 = sigma1 = 0),
  an x-dependent-coefficient case of the paper's problem class:
  - the Euler-Maruyama cloud against its exact first and second moments, per coordinate, by z-tests;
  - the first level against scikit-learn's ridge, with Z = sigma(X^m)^T alpha_x and the cloud bandwidth.
"""
import numpy as np
import pytest
from scipy.optimize import brentq
from sklearn.linear_model import Ridge

from oracle import literal as L
from oracle import scheme as S


def _sk_fit(pb, Xk, Y, m, k):
    D = Xk - Xk[m][None, :]
    w = L.anchor_weights(pb, D, k)
    A = np.hstack([np.ones((Xk.shape[0], 1)), D])
    r = Ridge(alpha=L.ridge_lambda(pb, k), fit_intercept=False, solver="cholesky")
    r.fit(A, Y, sample_weight=w)
    return r.coef_


@pytest.mark.parametrize("M,d,form", [(12, 5, "primal"), (12, 5, "dual"), (6, 10, "dual"), (6, 10, "primal"),
                                      (30, 3, None)])
def test_anchor_fit_matches_sklearn_ridge(M, d, form):
    rng = np.random.default_rng(M * 31 + d)
    pb = S.Problem(d=d, M=M, N=6, T=0.6, s=1.3, ridge_rel=3e-2, eps_h=0.8)
    k = 3
    Xk = rng.normal(size=(M, d)) * np.sqrt(k * pb.T / pb.N) * pb.s + 0.4
    Y = np.sin(Xk @ rng.normal(size=d)) + 0.1 * rng.normal(size=M)
    for m in (0, M // 2, M - 1):
        a, _ = L.anchor_fit(pb, Xk, Y, m, k, form)
        ref = _sk_fit(pb, Xk, Y, m, k)
        assert np.max(np.abs(a - ref)) <= 1e-9 * max(1.0, np.max(np.abs(ref)))


def test_primal_and_dual_agree():
    rng = np.random.default_rng(5)
    for M, d in ((9, 4), (5, 12), (20, 19)):
        pb = S.Problem(d=d, M=M, N=4, T=1.0, ridge_rel=1e-3)
        Xk = rng.normal(size=(M, d))
        Y = rng.normal(size=M)
        a1, _ = L.anchor_fit(pb, Xk, Y, 1, 2, "primal")
        a2, _ = L.anchor_fit(pb, Xk, Y, 1, 2, "dual")
        assert np.max(np.abs(a1 - a2)) <= 1e-9 * np.max(np.abs(a1))


def test_weights_ratio_identity_uniform_at_level0():
    rng = np.random.default_rng(8)
    pb = S.Problem(d=7, M=15, N=5, T=0.5, s=1.1, eps_h=1.3)
    k = 2
    X = rng.normal(size=(15, 7))
    D = X - X[4][None, :]
    w = L.anchor_weights(pb, D, k)
    eps2 = pb.eps_h ** 2 * 2 * pb.s ** 2 * (k * pb.T / pb.N) * pb.d
    n2 = np.sum(D * D, axis=1)
    for i, j in ((0, 1), (3, 9), (4, 14)):
        assert w[j] / w[i] == pytest.approx(np.exp(-(n2[j] - n2[i]) / eps2), rel=1e-12)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.argmax(w) == 4
    w0 = L.anchor_weights(pb, np.zeros((15, 7)), 0)
    assert np.all(w0 == 1.0 / 15)
    assert np.all(L.anchor_weights(pb.copy(eps_h=0.0), D, k) == 1.0 / 15)


def test_allen_cahn_regression_drops_out():
    pb = S.Problem(d=6, M=10, N=4, T=0.3, f_kind=S.F_ALLEN_CAHN, fp=(1.0, 1.0, 0.0, 0.0), g_kind=S.G_AC,
                   gp=(0.4, 0.0, 0.0, 0.0), ridge_rel=1e-2, seed=3)
    x0 = np.linspace(-0.5, 0.5, 6)
    out = L.solve_point(pb, x0, 0)
    W = S.brownian_path(pb, 0)
    gN, _, _ = S.g_eval(pb, S.positions(pb, x0, W[pb.N], pb.N))
    c = gN.mean()
    dt = pb.T / pb.N
    for _ in range(pb.N):
        c = brentq(lambda y: y - c - dt * (y - y ** 3), c - 1.0, c + 1.0, xtol=1e-15)
    assert out["u"] == pytest.approx(c, abs=1e-14)
    assert np.ptp(out["Y"]) == 0.0


@pytest.mark.parametrize("f_kind", [S.F_HJB, S.F_BURGERS])
def test_first_level_closed_forms(f_kind):
    d, M, N = 5, 9, 3
    fp = (0.7, 0.0, 0.0, 0.0) if f_kind == S.F_HJB else (0.4, 2.0, 0.0, 0.0)
    pb = S.Problem(d=d, M=M, N=N, T=0.9, s=1.2, f_kind=f_kind, fp=fp, g_kind=S.G_QUAD, gp=(1.0, 0.3, 0.0, 0.0),
                   ridge_rel=2e-2, eps_h=1.0, seed=11)
    x0 = np.full(d, 0.2)
    k = N - 1
    out = L.solve_point(pb, x0, 0, k_stop=k)
    W = S.brownian_path(pb, 0)
    YN, _, _ = S.g_eval(pb, S.positions(pb, x0, W[N], N))
    Xk = S.positions(pb, x0, W[k], k)
    Ybar = YN.mean()
    dt = pb.T / N
    for m in range(M):
        ax = _sk_fit(pb, Xk, YN, m, k)[1:]
        if f_kind == S.F_HJB:
            ref = Ybar - dt * fp[0] * pb.s ** 2 * (ax @ ax)
        else:
            zs = pb.s * ax.sum()
            ref = (Ybar - dt * fp[0] * fp[1] * zs) / (1.0 - dt * fp[0] * zs)
        assert out["Y"][m] == pytest.approx(ref, rel=1e-10, abs=1e-13)


def test_level0_slope_is_zero():
    pb = S.Problem(d=4, M=6, N=2, T=0.2, ridge_rel=1e-2)
    X0 = np.tile(np.array([0.1, -0.2, 0.3, 0.0]), (6, 1))
    a, w = L.anchor_fit(pb, X0, np.arange(6.0), 2, 0)
    assert np.all(a[1:] == 0.0)
    assert np.all(w == 1.0 / 6)


# ---------------------------------------------------------------- geometric (x-dependent) coefficients
def test_geometric_path_second_moment():
    # E X_{k+1,i}^2 = X_{k,i}^2 ((1 + mu0 dt)^2 + sigma0^2 dt) for the Euler-Maruyama step with mu = mu0 x,
    # sigma = sigma0 diag(x): a z-test of the cloud's mean over 4000 particles and 3 coordinates
    mu0, s0 = 0.3, 0.4
    pb = S.Problem(d=3, M=4000, N=5, T=1.0, seed=2)
    x0 = np.array([1.0, -0.5, 2.0])
    X = L.geometric_path(pb, x0, 0, mu0, s0)
    dt = pb.T / pb.N
    fac = ((1 + mu0 * dt) ** 2 + s0 ** 2 * dt) ** pb.N
    for i in range(3):
        v = X[pb.N, :, i] ** 2
        z = (v.mean() - x0[i] ** 2 * fac) / (v.std() / np.sqrt(v.size))
        assert abs(z) < 4.5, (i, z)
    # the mean follows (1 + mu0 dt)^N
    m = X[pb.N].mean(axis=0)
    se = X[pb.N].std(axis=0) / np.sqrt(pb.M)
    assert np.all(np.abs(m - x0 * (1 + mu0 * dt) ** pb.N) < 4.5 * se)


def test_geometric_first_level_hjb_closed_form():
    d, M, N, mu0, s0 = 4, 11, 3, 0.2, 0.5
    pb = S.Problem(d=d, M=M, N=N, T=0.9, f_kind=S.F_HJB, fp=(0.6, 0, 0, 0), g_kind=S.G_QUAD, gp=(1.0, 0.2, 0, 0),
                   ridge_rel=2e-2, eps_h=1.0, seed=4)
    x0 = np.array([0.8, 1.2, -0.6, 1.0])
    k = N - 1
    out = L.solve_point_geometric(pb, x0, 0, mu0, s0, k_stop=k, tape=True)
    X = L.geometric_path(pb, x0, 0, mu0, s0)
    YN, _, _ = S.g_eval(pb, X[N])
    Xk = X[k]
    C = Xk - Xk.mean(axis=0)
    eps2 = 2.0 * np.sum(C * C) / M
    dt = pb.T / N
    for m in range(M):
        D = Xk - Xk[m]
        n2 = np.sum(D * D, axis=1)
        w = np.exp(-n2 / eps2)
        w /= w.sum()
        r = Ridge(alpha=pb.ridge_rel * s0 ** 2 * (k + 1) * dt, fit_intercept=False, solver="cholesky")
        r.fit(np.hstack([np.ones((M, 1)), D]), YN, sample_weight=w)
        Z = s0 * Xk[m] * r.coef_[1:]
        assert out["zz"][k][m] == pytest.approx(Z @ Z, rel=1e-8)
        assert out["Y"][m] == pytest.approx(YN.mean() - dt * 0.6 * (Z @ Z), rel=1e-10, abs=1e-13)


def test_geometric_fit_primal_equals_dual():
    rng = np.random.default_rng(12)
    for M, d in ((9, 4), (6, 15)):
        X = 1.0 + 0.2 * rng.normal(size=(M, d))
        Y = rng.normal(size=M)
        a1, _ = L.anchor_fit_eps(X, Y, 2, 0.7, 3e-3, "primal")
        a2, _ = L.anchor_fit_eps(X, Y, 2, 0.7, 3e-3, "dual")
        assert np.max(np.abs(a1 - a2)) <= 1e-9 * np.max(np.abs(a1))


def test_affine_diag_path_moments():
    # exact moments of the Euler-Maruyama recursion for mu = mu0 x + mu1, sigma = diag(sigma0 x + sigma1):
    # E X' = a E X + mu1 dt and E X'^2 = a^2 E X^2 + 2 a mu1 dt E X + mu1^2 dt^2
    #        + dt (sigma0^2 E X^2 + 2 sigma0 sigma1 E X + sigma1^2), with a = 1 + mu0 dt
    mu0, mu1, s0, s1 = -0.8, 0.3, 0.2, 0.5
    pb = S.Problem(d=3, M=4000, N=5, T=1.0, seed=6)
    x0 = np.array([1.0, -0.5, 2.0])
    X = L.geometric_path(pb, x0, 0, mu0, s0, mu1, s1)
    dt = pb.T / pb.N
    a = 1 + mu0 * dt
    m1, m2 = x0.copy(), x0 ** 2
    for _ in range(pb.N):
        m1, m2 = (a * m1 + mu1 * dt,
                  a * a * m2 + 2 * a * mu1 * dt * m1 + mu1 ** 2 * dt ** 2 + dt * (s0 ** 2 * m2 + 2 * s0 * s1 * m1 + s1 ** 2))
    for i in range(3):
        v1, v2 = X[pb.N, :, i], X[pb.N, :, i] ** 2
        assert abs(v1.mean() - m1[i]) < 4.5 * v1.std() / np.sqrt(pb.M), i
        assert abs(v2.mean() - m2[i]) < 4.5 * v2.std() / np.sqrt(pb.M), i


def test_affine_diag_first_level_hjb_closed_form():
    d, M, N, mu0, mu1, s0, s1 = 4, 13, 3, -0.5, 0.2, 0.3, 0.4
    pb = S.Problem(d=d, M=M, N=N, T=0.9, f_kind=S.F_HJB, fp=(0.6, 0, 0, 0), g_kind=S.G_QUAD, gp=(1.0, 0.2, 0, 0),
                   ridge_rel=2e-2, eps_h=1.0, seed=9)
    x0 = np.array([0.8, 1.2, -0.6, 1.0])
    k = N - 1
    out = L.solve_point_geometric(pb, x0, 0, mu0, s0, k_stop=k, tape=True, mu1=mu1, sigma1=s1)
    X = L.geometric_path(pb, x0, 0, mu0, s0, mu1, s1)
    YN, _, _ = S.g_eval(pb, X[N])
    Xk = X[k]
    C = Xk - Xk.mean(axis=0)
    eps2 = 2.0 * np.sum(C * C) / M
    dt = pb.T / N
    for m in range(M):
        D = Xk - Xk[m]
        w = np.exp(-np.sum(D * D, axis=1) / eps2)
        w /= w.sum()
        r = Ridge(alpha=pb.ridge_rel * (s0 ** 2 + s1 ** 2) * (k + 1) * dt, fit_intercept=False, solver="cholesky")
        r.fit(np.hstack([np.ones((M, 1)), D]), YN, sample_weight=w)
        Z = (s0 * Xk[m] + s1) * r.coef_[1:]
        assert out["Y"][m] == pytest.approx(YN.mean() - dt * 0.6 * (Z @ Z), rel=1e-10, abs=1e-13)
