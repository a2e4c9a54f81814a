"""Pins of the oracle's hand-written reverse mode.

* Central finite differences (step 1e-4, common random numbers: the Philox stream does not
  depend on x0 or the parameters) for every f / g family, on x0 directions and parameters.
* Taylor remainder |L(x0 + e v) - L - e x0bar.v| = O(e^2).
* Affine case: x0bar equals the closed-form gradient a / (1 - c1 dt)^N.
"""
import numpy as np
import pytest

from oracle import scheme as S

CASES = [
    dict(f_kind=S.F_ALLEN_CAHN, fp=(1.0, 1.0, 0, 0), g_kind=S.G_AC, gp=(0.4, 0, 0, 0)),
    dict(f_kind=S.F_HJB, fp=(0.7, 0, 0, 0), g_kind=S.G_HJB_LOG, gp=(1.0, 0, 0, 0)),
    dict(f_kind=S.F_ZERO, fp=(0, 0, 0, 0), g_kind=S.G_QUAD, gp=(1.3, 0.2, 0, 0)),
    dict(f_kind=S.F_ALLEN_CAHN, fp=(0.5, 2.0, 0, 0), g_kind=S.G_HJB_LOG, gp=(0.6, 0, 0, 0)),
    dict(f_kind=S.F_BURGERS, fp=(0.3, 1.2, 0, 0), g_kind=S.G_LOGISTIC, gp=(0.4, 0, 0, 0)),
]


def _gvec(case, d):
    # the logistic g takes a slope vector; the other families ignore it
    return np.linspace(-0.5, 1.0, d) if CASES[case]["g_kind"] == S.G_LOGISTIC else None


def _u(pb, x0):
    return S.solve_point(pb, x0, 0)["u"]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("M,d", [(48, 6), (10, 16)])
def test_adjoint_vs_central_fd(case, M, d):
    rng = np.random.default_rng(10 + case)
    pb = S.Problem(d=d, M=M, N=4, T=0.3, eps_h=1.0, ridge_rel=1e-2, seed=case, gvec=_gvec(case, d), **CASES[case])
    x0 = 0.3 * rng.normal(size=d)
    adj = S.adjoint_point(pb, x0, 0, ubar=1.0)
    h = 1e-4
    for _ in range(3):
        v = rng.normal(size=d)
        v /= np.linalg.norm(v)
        fd = (_u(pb, x0 + h * v) - _u(pb, x0 - h * v)) / (2 * h)
        assert abs(fd - adj["x0bar"] @ v) <= 1e-6 * max(abs(fd), 1e-3)
    for which in ("gp", "fp"):
        base = getattr(pb, which)
        for i in range(2):
            if base[i] == 0.0:
                continue
            up = list(base); up[i] += h
            dn = list(base); dn[i] -= h
            fd = (_u(pb.copy(**{which: tuple(up)}), x0) - _u(pb.copy(**{which: tuple(dn)}), x0)) / (2 * h)
            got = adj[which + "bar"][i]
            assert abs(fd - got) <= 1e-6 * max(abs(fd), 1e-3), (which, i, fd, got)


def test_taylor_remainder_is_second_order():
    rng = np.random.default_rng(3)
    pb = S.Problem(d=8, M=40, N=5, T=0.3, eps_h=1.0, ridge_rel=1e-2, **CASES[0])
    x0 = 0.5 * rng.normal(size=8)
    v = rng.normal(size=8)
    adj = S.adjoint_point(pb, x0, 0)
    L0 = adj["u"]
    rem = [abs(_u(pb, x0 + e * v) - L0 - e * (adj["x0bar"] @ v)) for e in (1e-2, 5e-3)]
    assert 3.0 < rem[0] / rem[1] < 5.0


def test_affine_adjoint_equals_closed_form():
    rng = np.random.default_rng(4)
    d, M, N, T, c1 = 4, 30, 5, 0.5, 0.6
    a = rng.normal(size=d)
    pb = S.Problem(d=d, M=M, N=N, T=T, s=1.1, f_kind=S.F_ALLEN_CAHN, fp=(c1, 0, 0, 0), g_kind=S.G_AFFINE,
                   gp=(0.1, 0, 0, 0), gvec=a, ridge_rel=0.0)
    adj = S.adjoint_point(pb, rng.normal(size=d), 0)
    np.testing.assert_allclose(adj["x0bar"], a / (1 - c1 * T / N) ** N, rtol=1e-11)
