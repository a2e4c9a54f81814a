"""Independent reference values for the scheme's chain tests.  Test infrastructure only.

* Heat case (f = 0, g = a |x|^2/d + b, sigma = s I, drift mu): u(t, x) = E[g(x + mu tau + s W_tau)]
  with tau = T - t, i.e. a (|x + mu tau|^2 + s^2 tau d)/d + b, grad u = 2a (x + mu tau)/d.
* HJB case f(z) = -lam |z|^2 with z = sigma^T grad u (paper eq. mainprob, f takes sigma^T grad u):
  with v = exp(-2 lam u) the PDE becomes the backward heat equation d_t v + (s^2/2) Lap v = 0,
  so u(0, x) = -ln E[exp(-2 lam g(x + s W_T))] / (2 lam)  (Cole-Hopf).
  For radial g the expectation is a 2-D integral: |x + sigma Z|^2 = (|x| + sigma Z_1)^2 + sigma^2 C
  with Z_1 ~ N(0, 1) and C ~ chi^2_{d-1} independent, sigma = s sqrt(T).  Z_1 is integrated by
  Gauss-Hermite; C by generalized Gauss-Laguerre for small d - 1 and by Gauss-Legendre on
  +-60 standard deviations of the Gamma(k/2, 2) law (log-density via lgamma) for large d - 1.
* Burgers-type case (derived here; the printed Burgers PDE of the paper's Sec. 4 loses a coefficient):
  u(t, x) = phi(t + sum_i x_i / d) with the logistic phi(a) = 1 / (1 + e^-a) solves
  d_t u + (s^2/2) Lap u + c (u - kappa) sum_i z_i = 0, z = s grad u, for c = s / d and
  kappa = d / s^2 + 1/2: with phi' = phi (1 - phi) and phi'' = phi' (1 - 2 phi) the left side is
  phi' [1 + s^2 (1 - 2 phi) / (2d) + c s (phi - kappa)], zero for all phi exactly at those c, kappa.
  The terminal condition is the logistic g with gvec = 1/d and offset T.
"""
import numpy as np
from numpy.polynomial.hermite_e import hermegauss
from scipy.special import gammaln, roots_genlaguerre


def heat_quadratic(x0, T, s=np.sqrt(2.0), a=1.0, b=0.0, mu=None):
    x0 = np.asarray(x0, dtype=np.float64)
    d = x0.shape[-1]
    xt = x0 if mu is None else x0 + T * np.asarray(mu)
    u = a * (np.sum(xt * xt, axis=-1) + s * s * T * d) / d + b
    return u, 2.0 * a * xt / d


def _chi2_nodes(k, n):
    """Nodes/weights integrating against the chi^2_k density."""
    if k <= 0:
        return np.zeros(1), np.ones(1)
    alpha = k / 2.0 - 1.0
    if k < 200:
        y, w = roots_genlaguerre(n, alpha)
        w = w / np.exp(gammaln(k / 2.0))
        return 2.0 * y, w
    mean, sd = k / 2.0, np.sqrt(k / 2.0)
    t, wt = np.polynomial.legendre.leggauss(n)
    lo = max(mean - 60.0 * sd, 1e-300)
    hi = mean + 60.0 * sd
    y = 0.5 * (hi - lo) * t + 0.5 * (hi + lo)
    logpdf = alpha * np.log(y) - y - gammaln(k / 2.0)
    w = 0.5 * (hi - lo) * wt * np.exp(logpdf)
    return 2.0 * y, w


def radial_expectation(h, r, d, sigma, n_herm=160, n_chi=None):
    """E[h(|x + sigma Z|^2)] for |x| = r, Z ~ N(0, I_d)."""
    z, wz = hermegauss(n_herm)
    wz = wz / np.sqrt(2.0 * np.pi)
    if n_chi is None:
        n_chi = 80 if d - 1 < 200 else 400
    c, wc = _chi2_nodes(d - 1, n_chi)
    q = (r + sigma * z)[:, None] ** 2 + sigma ** 2 * c[None, :]
    return float(np.sum(wz[:, None] * wc[None, :] * h(q)))


def hjb_log_cole_hopf(x0, T, lam, s=np.sqrt(2.0), a=1.0, **kw):
    """u(0, x0) for f = -lam |z|^2, g = ln((1 + a|x|^2)/2), sigma = s I, no drift."""
    x0 = np.asarray(x0, dtype=np.float64)
    r = float(np.sqrt(x0 @ x0))
    sigma = s * np.sqrt(T)
    h = lambda q: np.exp(-2.0 * lam * np.log((1.0 + a * q) / 2.0))
    return -np.log(radial_expectation(h, r, x0.shape[0], sigma, **kw)) / (2.0 * lam)


def burgers_coefficients(d, s=np.sqrt(2.0)):
    """(c, kappa) of the Burgers-type nonlinearity c (y - kappa) sum_i z_i whose solution is logistic."""
    return s / d, d / (s * s) + 0.5


def burgers_logistic(x0, t):
    """u(t, x) = phi(t + sum_i x_i / d) and its gradient phi'(.) / d (every coordinate)."""
    x0 = np.asarray(x0, dtype=np.float64)
    d = x0.shape[-1]
    a = t + np.sum(x0, axis=-1) / d
    u = 1.0 / (1.0 + np.exp(-a))
    g = (u * (1.0 - u) / d)[..., None] * np.ones_like(x0)
    return u, g
