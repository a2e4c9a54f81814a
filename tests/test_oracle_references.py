"""Pins of the oracle's independent reference solutions against closed forms (CPU only).

* colehopf.radial_expectation, both branches of its chi^2_{d-1} quadrature (generalized Gauss-Laguerre for
  d - 1 < 200, Gauss-Legendre on the Gamma law for d - 1 >= 200), against moments and the moment generating
  function of the non-central chi-square law: for X = x + sigma Z in R^d with |x| = r,
  E|X|^2 = r^2 + sigma^2 d, E|X|^4 = (r^2 + sigma^2 d)^2 + 2 sigma^4 d + 4 sigma^2 r^2 and
  E exp(-c |X|^2) = (1 + 2 c sigma^2)^(-d/2) exp(-c r^2 / (1 + 2 c sigma^2)).
* colehopf.hjb_log_cole_hopf at lam -> the linear limit: -ln E[exp(-2 lam g)] / (2 lam) -> E[g] as lam -> 0,
  and for a = 0 the constant terminal value ln(1/2).
* radial_pde.radial_solution against exact solutions of the radial PDE v_t + (s^2/2)(v_rr + (d-1) v_r / r)
  + f(v) = 0: g = r^2 with f = 0 gives v(0, r) = r^2 + s^2 d T; with f = c v it gives e^{cT}(r^2 + s^2 d T)
  (both reproduced exactly by the central differences and Crank-Nicolson, so checked at the grid nodes to
  rounding); g = exp(-b r^2) with f = 0 gives the Gaussian heat kernel's closed form, reached at second order
  in the grid spacing.
"""
import math

import numpy as np
import pytest

from oracle import colehopf as CH
from oracle import radial_pde as RP


@pytest.mark.parametrize("d", [200, 201, 1000, 5000])
@pytest.mark.parametrize("r,sig", [(0.0, 0.8), (1.3, 0.8), (3.0, 1.5)])
def test_radial_expectation_moments_and_mgf(d, r, sig):
    m1 = CH.radial_expectation(lambda q: q, r, d, sig)
    m2 = CH.radial_expectation(lambda q: q * q, r, d, sig)
    e1 = r * r + sig * sig * d
    e2 = e1 * e1 + 2.0 * sig ** 4 * d + 4.0 * sig * sig * r * r
    assert abs(m1 / e1 - 1.0) <= 1e-11
    assert abs(m2 / e2 - 1.0) <= 1e-11
    for c in (0.3 / (sig * sig * d), 2.0 / (sig * sig * d)):
        m3 = CH.radial_expectation(lambda q: np.exp(-c * q), r, d, sig)
        e3 = (1.0 + 2.0 * c * sig * sig) ** (-d / 2.0) * math.exp(-c * r * r / (1.0 + 2.0 * c * sig * sig))
        assert abs(m3 / e3 - 1.0) <= 1e-11


def test_quadrature_branches_agree_across_switch():
    # d - 1 = 199 (Laguerre) and 200 (Legendre) integrate the same smooth function to nearby values; the
    # step from one to the other is the change of d alone (checked through the closed form of E|X|^2)
    h = lambda q: np.log1p(q)
    for d in (200, 201):
        v = CH.radial_expectation(h, 0.7, d, 0.9)
        assert math.isfinite(v)
    a = CH.radial_expectation(lambda q: q, 0.7, 200, 0.9)
    b = CH.radial_expectation(lambda q: q, 0.7, 201, 0.9)
    assert abs((b - a) - 0.81) <= 1e-10


@pytest.mark.parametrize("d", [10, 200, 1000])
def test_cole_hopf_limits(d):
    rng = np.random.default_rng(d)
    x0 = 0.3 * rng.standard_normal(d) / math.sqrt(d)
    T, s = 0.4, math.sqrt(2.0)
    # a = 0: g = ln(1/2) everywhere, for any lam
    assert abs(CH.hjb_log_cole_hopf(x0, T, 1.3, s=s, a=0.0) - math.log(0.5)) <= 1e-13
    # lam -> 0: u -> E[g(x + s W_T)]; the first correction is -lam Var[g], so the gap shrinks linearly
    r = float(np.linalg.norm(x0))
    eg = CH.radial_expectation(lambda q: np.log((1.0 + q) / 2.0), r, d, s * math.sqrt(T))
    gaps = [abs(CH.hjb_log_cole_hopf(x0, T, lam, s=s) - eg) for lam in (1e-3, 5e-4)]
    assert gaps[1] < gaps[0]
    assert abs(gaps[0] / gaps[1] - 2.0) <= 0.02


@pytest.mark.parametrize("d", [1, 2, 10, 100])
def test_radial_solution_quadratic_exact(d):
    s, T = math.sqrt(2.0), 0.3
    r, v = RP.radial_solution(d, T, s, lambda v: 0.0 * v, lambda r: r * r, n=1200, steps=600)
    m = r <= 2.0   # away from the zero-flux edge at r_max = 12, which the exact solution does not satisfy
    assert np.max(np.abs(v[m] - (r[m] ** 2 + s * s * d * T))) <= 1e-9
    c = 0.7
    r, v = RP.radial_solution(d, T, s, lambda v: c * v, lambda r: r * r, n=1200, steps=600)
    exact = math.exp(c * T) * (r[m] ** 2 + s * s * d * T)
    # Heun's half steps of the linear reaction carry an O(dt^3) local error per step
    assert np.max(np.abs(v[m] - exact) / exact) <= 1e-8


@pytest.mark.parametrize("d", [1, 3])
def test_radial_solution_gaussian_second_order(d):
    s, T, b = math.sqrt(2.0), 0.3, 0.8
    sig2 = s * s * T
    errs = []
    for n in (600, 1200):
        r, v = RP.radial_solution(d, T, s, lambda v: 0.0 * v, lambda r: np.exp(-b * r * r), n=n, steps=400)
        m = r <= 3.0
        exact = (1.0 + 2.0 * b * sig2) ** (-d / 2.0) * np.exp(-b * r[m] ** 2 / (1.0 + 2.0 * b * sig2))
        errs.append(float(np.max(np.abs(v[m] - exact))))
    assert errs[1] <= 2e-5
    assert 3.0 <= errs[0] / errs[1] <= 5.0
