"""Pins of the oracle's proximal operators and conjugates against independent numerics:
bisection on the optimality condition, the Moreau identity with the primal prox, a
numerical supremum for the conjugate, and constrained brute-force minimisation."""
import math

import numpy as np
import pytest
from scipy.optimize import minimize, minimize_scalar

from oracle import prox as P


def _bisect_kl_dual(w, sb):
    """Root of h(z) = z - w + sb / (1 - z) on (-inf, 1): the optimality condition of
    argmin_z (z - v)^2 / (2 sigma) + phi*(z) with w = v + sigma r, sb = sigma b > 0."""
    lo, hi = min(w, 0.0) - 1.0, 1.0
    while lo - w + sb / (1 - lo) > 0:
        lo = 2 * lo - 1
    for _ in range(2000):
        mid = 0.5 * (lo + hi)
        if mid == lo or mid == hi:
            break
        if mid - w + sb / (1 - mid) > 0:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)


def test_kl_dual_prox_vs_bisection():
    rng = np.random.default_rng(0)
    for _ in range(400):
        sigma = 10 ** rng.uniform(-4, 4)
        b = float(rng.integers(1, 40))
        r = 10 ** rng.uniform(-3, 1)
        v = rng.normal() * 10 ** rng.uniform(-2, 5)
        z = P.prox_kl_dual(v, sigma, b, r)
        ref = _bisect_kl_dual(v + sigma * r, sigma * b)
        assert abs(z - ref) <= 1e-13 * max(1.0, abs(ref)) + 1e-15


def test_kl_dual_prox_literal_form_agrees_where_accurate():
    rng = np.random.default_rng(1)
    v = rng.normal(size=1000)
    sigma = 10 ** rng.uniform(-1, 1, size=1000)
    b = rng.integers(0, 20, size=1000).astype(float)
    r = rng.uniform(0.01, 2, size=1000)
    np.testing.assert_allclose(P.prox_kl_dual(v, sigma, b, r),
                               P.prox_kl_dual_literal(v, sigma, b, r), rtol=1e-12, atol=1e-13)


def test_kl_dual_prox_zero_counts_and_bound():
    w = np.linspace(-5, 5, 101)
    np.testing.assert_allclose(P.prox_kl_dual(w, 0.7, 0.0, 0.0), np.minimum(w, 1.0), rtol=0, atol=1e-15)
    z = P.prox_kl_dual(np.linspace(-50, 5e4, 999), 0.3, 2.0, 0.1)
    assert np.all(z < 1.0)


def _primal_kl_prox(a, tau, b, r):
    """prox_{tau phi}(a): u - a + tau (1 - b / (u + r)) = 0, u + r = s > 0 solves
    s^2 - (a + r - tau) s - tau b = 0."""
    c = a + r - tau
    s = 0.5 * (c + math.sqrt(c * c + 4 * tau * b))
    return s - r


def test_moreau_identity():
    rng = np.random.default_rng(2)
    for _ in range(200):
        sigma = 10 ** rng.uniform(-2, 2)
        b = float(rng.integers(1, 30))
        r = rng.uniform(0.05, 3)
        v = rng.normal() * 5
        lhs = P.prox_kl_dual(v, sigma, b, r)
        rhs = v - sigma * _primal_kl_prox(v / sigma, 1 / sigma, b, r)
        assert lhs == pytest.approx(rhs, rel=1e-10, abs=1e-10)


def test_conjugate_by_numerical_supremum():
    rng = np.random.default_rng(3)
    for _ in range(30):
        b = float(rng.integers(1, 20))
        r = rng.uniform(0.1, 2)
        y = rng.uniform(-3, 0.9)
        res = minimize_scalar(lambda u: -(y * u - float(P.phi(u, b, r))),
                              bounds=(-r + 1e-12, 1e4), method="bounded",
                              options=dict(xatol=1e-12))
        assert float(P.phi_conj(y, b, r)) == pytest.approx(-res.fun, rel=1e-7, abs=1e-7)
    assert math.isinf(float(P.phi_conj(1.5, 1.0, 1.0)))


def test_phi_zero_iff_data_matched():
    """D(Pu) >= 0 with equality iff Pu + r = b (Section 1.2)."""
    b = np.array([3.0, 0.0, 7.0])
    r = np.array([0.5, 0.2, 1.0])
    assert np.allclose(P.phi(b - r, b, r), 0.0, atol=1e-14)
    assert np.all(P.phi(b - r + 0.3, b, r) > 0)
    assert math.isinf(float(P.phi(-2.0, 1.0, 0.5)))


def test_l2_ball_projection_vs_brute_force():
    rng = np.random.default_rng(4)
    for _ in range(40):
        v = rng.normal(size=3) * 2
        alpha = rng.uniform(0.1, 3)
        got = P.project_l2_ball(v[:, None], alpha)[:, 0]
        res = minimize(lambda z: np.sum((z - v) ** 2), np.zeros(3), method="SLSQP",
                       constraints=[dict(type="ineq", fun=lambda z: alpha ** 2 - z @ z)],
                       options=dict(ftol=1e-14, maxiter=500))
        np.testing.assert_allclose(got, res.x, atol=1e-6)
        np.testing.assert_allclose(P.project_l2_ball(got[:, None], alpha)[:, 0], got, rtol=1e-15)
    inside = np.array([[0.1], [0.2], [-0.1]])
    np.testing.assert_array_equal(P.project_l2_ball(inside, 1.0), inside)
    np.testing.assert_array_equal(P.project_l2_ball(np.zeros((3, 1)), 1.0), np.zeros((3, 1)))


def test_nonneg_prox_vs_brute_force():
    x = np.linspace(-2, 2, 9)
    for xi in x:
        res = minimize_scalar(lambda z: 0.5 * (z - xi) ** 2, bounds=(0, 10), method="bounded",
                              options=dict(xatol=1e-12))
        assert P.prox_nonneg(xi) == pytest.approx(res.x, abs=1e-8)


def _soft_threshold(v, t):
    """prox of t ||.||_1: sign(v) max(|v| - t, 0) (the textbook shrinkage)."""
    return np.sign(v) * np.maximum(np.abs(v) - t, 0.0)


def test_linf_ball_projection_vs_brute_force_and_moreau():
    """aTV's dual prox (Section 4.3): the prox of the conjugate of alpha ||.||_1, i.e. the
    projection onto the box |p_c| <= alpha, against (a) a bound-constrained minimiser of
    1/2 ||z - v||^2 and (b) the Moreau identity v = prox_{f*}(v) + prox_f(v) with the
    soft-thresholding prox of f = alpha ||.||_1."""
    rng = np.random.default_rng(5)
    for _ in range(40):
        v = rng.normal(size=3) * 2
        alpha = rng.uniform(0.1, 3)
        got = P.clip_linf_ball(v, alpha)
        res = minimize(lambda z: 0.5 * np.sum((z - v) ** 2), np.zeros(3), method="L-BFGS-B",
                       bounds=[(-alpha, alpha)] * 3, jac=lambda z: z - v,
                       options=dict(ftol=1e-15, gtol=1e-12, maxiter=500))
        np.testing.assert_allclose(got, res.x, atol=1e-7)
        np.testing.assert_allclose(got + _soft_threshold(v, alpha), v, rtol=0, atol=1e-14)
    np.testing.assert_array_equal(P.clip_linf_ball(np.array([0.5, -0.25, 0.0]), 1.0),
                                  [0.5, -0.25, 0.0])
    np.testing.assert_array_equal(P.clip_linf_ball(np.array([2.0, -3.0, 0.9]), 1.0),
                                  [1.0, -1.0, 0.9])
