"""Finite-difference reference solution of the PDE itself, independent of the scheme.  Test infrastructure only.

For sigma = s I, zero drift, a radial terminal condition g(|x|) and an f that depends on u alone
(Allen-Cahn), the solution is radial: u(t, x) = v(t, |x|) with

    v_t + (s^2/2) (v_rr + (d - 1) v_r / r) + f(v) = 0,   v(T, r) = g(r),   v_r(0) = 0

(the Laplacian of a radial function; paper eq. mainprob with L = (s^2/2) Lap).  It is solved backward in
time on the cell-centred grid r_i = (i + 1/2) h, i < n, of [0, r_max]: the symmetry condition mirrors the
first cell, a zero-flux condition closes the far edge (far from the evaluation points the solution is
flat), diffusion by Crank-Nicolson and the reaction by two half steps of Heun's method around it
(Strang splitting, second order in time and space).
"""
import numpy as np
from scipy.linalg import solve_banded


def radial_solution(d, T, s, f, g, r_max=12.0, n=2400, steps=6000):
    """Grid r [n] and v(0, r) [n] for the problem above; f, g vectorised callables."""
    h = r_max / n
    r = (np.arange(n) + 0.5) * h
    dt = T / steps
    a = 0.5 * s * s
    lower = a * (1.0 / h ** 2 - (d - 1) / (2.0 * h * r))   # coefficient of v_{i-1}
    upper = a * (1.0 / h ** 2 + (d - 1) / (2.0 * h * r))   # coefficient of v_{i+1}
    diag = np.full(n, -2.0 * a / h ** 2)
    diag[0] += lower[0]            # v_{-1} = v_0 (mirror at r = 0)
    diag[-1] += upper[-1]          # v_n = v_{n-1} (zero flux at r_max)
    lower[0] = 0.0
    upper[-1] = 0.0

    def apply(v):
        out = diag * v
        out[1:] += lower[1:] * v[:-1]
        out[:-1] += upper[:-1] * v[1:]
        return out

    band = np.zeros((3, n))
    band[0, 1:] = -0.5 * dt * upper[:-1]
    band[1] = 1.0 - 0.5 * dt * diag
    band[2, :-1] = -0.5 * dt * lower[1:]

    def react(v, tau):
        k1 = f(v)
        return v + 0.5 * tau * (k1 + f(v + tau * k1))

    v = g(r)
    for _ in range(steps):
        v = react(v, 0.5 * dt)
        v = solve_banded((1, 1), band, v + 0.5 * dt * apply(v))
        v = react(v, 0.5 * dt)
    return r, v


def radial_value(d, T, s, f, g, radius, **kw):
    """v(0, radius) by linear interpolation on the grid."""
    r, v = radial_solution(d, T, s, f, g, **kw)
    return float(np.interp(radius, r, v))
