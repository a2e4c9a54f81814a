"""Pins of the oracle's local linear regression (paper Sec. 2.4) and Newton step (Sec. 2.5).

LLR: against a dense stacked least-squares solve (numpy.linalg.lstsq) of the penalised functional,
with the weights computed straight from eq. Dj (no minimum shift); exact recovery of affine data;
primal vs dual (push-through) forms; the full (d+1) normal equations vs the Schur-decoupled
solve of Lemma 3.7; uniform weights for h = 0; the kernel weight-ratio identity.
Newton: f = 0 gives y = C; an f that does not depend on y gives the explicit update after one
step; the Allen-Cahn root against bisection (scipy brentq).
"""
import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import scheme as S


def _weights_from_definition(D, eps2):
    K = np.exp(-np.einsum("ij,ij->i", D, D) / eps2)
    return K / K.sum()


def _stacked_lstsq(D, Y, w, lam):
    M, d = D.shape
    sw = np.sqrt(w)
    A = np.vstack([np.hstack([sw[:, None], sw[:, None] * D]),
                   np.hstack([np.zeros((d, 1)), np.sqrt(lam) * np.eye(d)])])
    rhs = np.concatenate([sw * Y, np.zeros(d)])
    sol = np.linalg.lstsq(A, rhs, rcond=None)[0]
    return sol[0], sol[1:]


@pytest.mark.parametrize("M,d,lam_rel,h", [(7, 3, 1e-2, 1.0), (3, 5, 1e-1, 1.0), (9, 4, 0.0, 0.7),
                                           (5, 5, 3e-2, 2.0), (40, 12, 1e-3, 1.0)])
def test_llr_matches_stacked_lstsq(M, d, lam_rel, h):
    rng = np.random.default_rng(M * 100 + d)
    k, N, T, s = 2, 5, 0.5, 1.3
    pb = S.Problem(d=d, M=M, N=N, T=T, s=s, eps_h=h, ridge_rel=lam_rel)
    W = rng.normal(size=(M, d)) * np.sqrt((k + 1) * T / N)
    Y = rng.normal(size=M)
    fit = S.llr(pb, W, Y, k)
    D = s * W
    t_next = (k + 1) * T / N
    w = _weights_from_definition(D, h * h * s * s * t_next * d)
    np.testing.assert_allclose(fit["w"], w, rtol=1e-12)
    a_ref, ax_ref = _stacked_lstsq(D, Y, w, lam_rel * s * s * t_next)
    np.testing.assert_allclose(fit["alpha_x"], ax_ref, rtol=1e-9, atol=1e-11)
    assert abs(fit["alpha"] - a_ref) < 1e-10 * max(1.0, abs(a_ref))


def test_weight_ratio_identity():
    rng = np.random.default_rng(2)
    D = rng.normal(size=(30, 8))
    pb = S.Problem(d=8, M=30, N=4, T=1.0, s=1.0, eps_h=0.8)
    t_next = 0.75
    w = S.kernel_weights(pb, D, t_next)
    eps2 = 0.8 ** 2 * t_next * 8
    n2 = (D * D).sum(1)
    for i, j in [(0, 1), (5, 9), (29, 3)]:
        assert abs(w[j] / w[i] - np.exp(-(n2[j] - n2[i]) / eps2)) < 1e-13 * np.exp(-(n2[j] - n2[i]) / eps2)
    assert abs(w.sum() - 1.0) < 1e-15
    np.testing.assert_allclose(S.kernel_weights(pb.copy(eps_h=0.0), D, t_next), np.full(30, 1 / 30), rtol=1e-15)


def test_affine_data_recovered_exactly():
    rng = np.random.default_rng(3)
    M, d = 25, 6
    pb = S.Problem(d=d, M=M, N=3, T=0.9, s=0.8, eps_h=1.0, ridge_rel=0.0)
    W = rng.normal(size=(M, d))
    a, c = rng.normal(size=d), 0.37
    Y = c + (pb.s * W) @ a
    fit = S.llr(pb, W, Y, 1)
    np.testing.assert_allclose(fit["alpha_x"], a, rtol=1e-12, atol=1e-13)
    assert abs(fit["alpha"] - c) < 1e-13


def test_primal_equals_dual():
    rng = np.random.default_rng(4)
    for M, d in [(12, 7), (7, 12)]:
        Dc = rng.normal(size=(M, d))
        w = rng.uniform(0.2, 1.0, size=M)
        w /= w.sum()
        Dc -= w @ Dc
        lam = 0.05
        P = S.RidgeSystem(Dc, w, lam, mode="primal")
        Q = S.RidgeSystem(Dc, w, lam, mode="dual")
        v = rng.normal(size=d)
        r = rng.normal(size=M)
        np.testing.assert_allclose(P.solve(v), Q.solve(v), rtol=1e-11, atol=1e-12)
        np.testing.assert_allclose(P.solve_rhs_weighted(r), Q.solve_rhs_weighted(r), rtol=1e-11, atol=1e-12)


def test_full_system_equals_schur_decoupled():
    # Lemma 3.7: [[S0, S^T], [S, Gamma + lam I]] (alpha, alpha_x) = (sum w Y, sum w Y D)
    rng = np.random.default_rng(6)
    M, d, k = 30, 5, 0
    pb = S.Problem(d=d, M=M, N=2, T=1.0, s=1.1, eps_h=1.2, ridge_rel=0.02)
    W = rng.normal(size=(M, d)) * np.sqrt(0.5)
    Y = np.sin(W.sum(1)) + 0.1 * rng.normal(size=M)
    fit = S.llr(pb, W, Y, k)
    D = pb.s * W
    w = fit["w"]
    lam = pb.ridge_rel * pb.s ** 2 * 0.5
    S0, Sv, G = w.sum(), w @ D, D.T @ (w[:, None] * D)
    A = np.block([[np.array([[S0]]), Sv[None, :]], [Sv[:, None], G + lam * np.eye(d)]])
    rhs = np.concatenate([[w @ Y], D.T @ (w * Y)])
    sol = np.linalg.solve(A, rhs)
    np.testing.assert_allclose(fit["alpha_x"], sol[1:], rtol=1e-10, atol=1e-12)
    assert abs(fit["alpha"] - sol[0]) < 1e-11


def test_uniform_weights_give_ordinary_least_squares():
    rng = np.random.default_rng(7)
    M, d = 20, 4
    pb = S.Problem(d=d, M=M, N=2, T=1.0, s=1.0, eps_h=0.0, ridge_rel=0.0)
    W = rng.normal(size=(M, d))
    Y = rng.normal(size=M)
    fit = S.llr(pb, W, Y, 0)
    X = np.hstack([np.ones((M, 1)), W])
    sol = np.linalg.lstsq(X, Y, rcond=None)[0]
    np.testing.assert_allclose(fit["alpha_x"], sol[1:], rtol=1e-11, atol=1e-12)
    assert abs(fit["alpha"] - sol[0]) < 1e-12


def test_newton_special_cases_and_bisection():
    rng = np.random.default_rng(8)
    C = rng.normal(size=50) * 0.5
    Z = rng.normal(size=6)
    pb = S.Problem(d=6, M=50, N=10, T=1.0)
    y, Fp, st = S.newton(pb.copy(f_kind=S.F_ZERO), 3, C, Z)
    assert np.array_equal(y, C) and st == 0 and np.all(Fp == 1.0)
    lam = 0.8
    y, _, _ = S.newton(pb.copy(f_kind=S.F_HJB, fp=(lam, 0, 0, 0)), 3, C, Z)
    np.testing.assert_allclose(y, C - 0.1 * lam * (Z @ Z), rtol=0, atol=1e-15)
    pbac = pb.copy(f_kind=S.F_ALLEN_CAHN, fp=(1.0, 1.0, 0, 0))
    y, _, _ = S.newton(pbac, 3, C, Z)
    dt = 0.1
    for m in range(C.size):
        F = lambda v: v - C[m] - dt * (v - v ** 3)
        root = brentq(F, C[m] - 1.0, C[m] + 1.0, xtol=1e-17, rtol=9e-16)
        assert abs(y[m] - root) <= 2e-15 * max(1.0, abs(root))
        assert abs(F(y[m])) <= 4 * np.finfo(float).eps * max(1.0, abs(y[m]))
        assert abs(y[m] - C[m]) <= 2 * dt * abs(C[m] - C[m] ** 3) + 1e-14
