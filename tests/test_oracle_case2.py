"""Pins of the oracle's Allen-Cahn Case 2 family (log potential, Sec. 4.1 Case 2): CPU only.

* leave_one_out_products against the products of np.delete'd coordinates.
* case2_source (re-derived, a reading: the printed manufactured solution cos(prod x) e^(cos t - |x|^2)
  reaches e > 1, outside the log potential's domain, so it carries an amplitude a < 1/e) makes
  a cos(prod x) e^(cos t - |x|^2) exact: the residual u_t + (s^2/2) Lap u + f(t, x, u) of the PDE of Sec. 2.1
  with sigma = s I, every derivative by central differences of case2_exact, vanishes to the differences'
  accuracy (d = 1, 2, 3, 5, coordinates of order one so that the product terms matter).
* case2_source_grad (behind f_grad_x) and the terminal gradient match central differences; d f / d y is
  the log potential's derivative, checked by differences.
* The scheme converges at first order in dt to the manufactured solution: with uniform weights (h = 0) the
  errors of u(0, x0) fall at first order and the Richardson value 2 u(2N) - u(N) is within 2% of v(0, x0)
  (d = 2, M = 4096, 4 seeds; the Monte Carlo error of the mean is about 0.5%).
"""
import math

import numpy as np
import pytest

from oracle import scheme as OS

TH, THC, AMP = 0.8, 1.6, 0.25


def _v(t, x):
    return float(OS.case2_exact(AMP, t, np.asarray(x)[None, :])[0])


def test_leave_one_out_products():
    rng = np.random.default_rng(1)
    for d in (1, 2, 5, 9):
        X = rng.normal(size=(3, d))
        X[0, d // 2] = 0.0
        ref = np.array([[np.prod(np.delete(X[m], i)) for i in range(d)] for m in range(3)])
        assert np.allclose(OS.leave_one_out_products(X), ref, rtol=1e-14, atol=0.0)


@pytest.mark.parametrize("d", [1, 2, 3, 5])
@pytest.mark.parametrize("s", [math.sqrt(2.0), 0.9])
def test_source_makes_the_manufactured_solution_exact(d, s):
    rng = np.random.default_rng(10 + d)
    pb = OS.Problem(d=d, M=2, N=1, T=1.0, s=s, f_kind=OS.F_LOG_POT, fp=(TH, THC, AMP, 0))
    ht, hx = 1e-5, 1e-4
    for _ in range(5):
        t = float(rng.uniform(0.0, 1.0))
        x = rng.uniform(-1.1, 1.1, size=d)
        v = _v(t, x)
        vt = (_v(t + ht, x) - _v(t - ht, x)) / (2 * ht)
        lap = 0.0
        for i in range(d):
            e = np.zeros(d)
            e[i] = hx
            lap += (_v(t, x + e) - 2 * v + _v(t, x - e)) / (hx * hx)
        f, _, _, _, _ = OS.f_eval(pb, t, np.array([v]), np.zeros(d), x[None, :])
        res = vt + 0.5 * s * s * lap + f[0]
        scale = abs(vt) + 0.5 * s * s * abs(lap) + abs(f[0]) + abs(v)
        assert abs(res) <= 2e-6 * scale, (t, x, res, scale)


def test_derivatives_match_differences():
    rng = np.random.default_rng(4)
    h = 1e-6
    for d in (1, 3, 6):
        pb = OS.Problem(d=d, M=2, N=1, T=1.0, s=1.2, f_kind=OS.F_LOG_POT, fp=(TH, THC, AMP, 0))
        x = rng.uniform(-1.0, 1.0, size=d)
        t = 0.3
        y = np.array([0.2, -0.4])
        f, fy, _, _, _ = OS.f_eval(pb, t, y, np.zeros(d), np.stack([x, x]))
        fp_, _, _, _, _ = OS.f_eval(pb, t, y + h, np.zeros(d), np.stack([x, x]))
        fm_, _, _, _, _ = OS.f_eval(pb, t, y - h, np.zeros(d), np.stack([x, x]))
        assert np.allclose(fy, (fp_ - fm_) / (2 * h), rtol=1e-7)
        gx = OS.f_grad_x(pb, t, y[:1], np.zeros(d), x)
        for k in range(d):
            e = np.zeros(d)
            e[k] = h
            fp_, _, _, _, _ = OS.f_eval(pb, t, y[:1], np.zeros(d), (x + e)[None, :])
            fm_, _, _, _, _ = OS.f_eval(pb, t, y[:1], np.zeros(d), (x - e)[None, :])
            assert abs(gx[k] - (fp_[0] - fm_[0]) / (2 * h)) <= 1e-6 * (abs(gx[k]) + 1e-2)
        pg = OS.Problem(d=d, M=2, N=1, T=0.7, g_kind=OS.G_CASE2, gp=(0.7, AMP, 0, 0))
        g, gxx, _ = OS.g_eval(pg, x[None, :])
        assert abs(g[0] - _v(0.7, x)) <= 1e-15
        for k in range(d):
            e = np.zeros(d)
            e[k] = h
            fd = (_v(0.7, x + e) - _v(0.7, x - e)) / (2 * h)
            assert abs(gxx[0, k] - fd) <= 1e-7 * (abs(fd) + 1e-2)


def test_scheme_converges_at_first_order_to_the_manufactured_solution():
    d, M, T = 2, 4096, 1.0
    x0 = np.array([0.5, -0.4])
    exact = _v(0.0, x0)
    means = {}
    for N in (20, 40, 80):
        us = []
        for seed in range(4):
            pb = OS.Problem(d=d, M=M, N=N, T=T, f_kind=OS.F_LOG_POT, fp=(TH, THC, AMP, 0), g_kind=OS.G_CASE2,
                            gp=(T, AMP, 0, 0), eps_h=0.0, seed=seed)
            r = OS.solve_point(pb, x0, 0)
            assert r["status"] == 0
            us.append(r["u"])
        means[N] = float(np.mean(us))
    e20, e40, e80 = (means[n] - exact for n in (20, 40, 80))
    assert e20 > e40 > e80 > 0.0
    assert 1.6 <= e20 / e40 <= 4.5 and 1.6 <= e40 / e80 <= 4.5
    assert abs(2.0 * means[80] - means[40] - exact) <= 0.02 * exact
