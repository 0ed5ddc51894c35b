"""Pins for the oracle's Matern covariance (eq. 2) and dense likelihood (eq. 1).

Independent references: the exponential closed form at nu = 1/2 stated in
Section 2.2, the (1 + x) e^-x form at nu = 3/2, exact rational arithmetic on
the float64-rounded covariance (determinant by fraction elimination and the
Leibniz expansion, exact solve for the quadratic form), Hadamard's bound, and
the white-noise limit where the covariance is exactly diagonal.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle.dense import covariance_matrix, dense_loglik, loglik_from_matrix
from oracle.matern import matern_correlation
from paper_1709_04419_amd import workloads as wl


def test_matern_exponential_and_three_halves():
    x = np.logspace(-6, 2.5, 80)
    np.testing.assert_allclose(matern_correlation(x, 0.5), np.exp(-x), rtol=3e-15, atol=1e-300)
    np.testing.assert_allclose(matern_correlation(x, 1.5), (1 + x) * np.exp(-x), rtol=3e-15,
                               atol=1e-300)
    np.testing.assert_allclose(matern_correlation(x, 2.5), (1 + x + x * x / 3) * np.exp(-x),
                               rtol=5e-15, atol=1e-300)


def test_matern_at_zero_and_monotone():
    for nu in (0.325, 0.5, 1.0):
        assert matern_correlation(np.array([0.0]), nu)[0] == 1.0
        v = matern_correlation(np.logspace(-5, 1, 50), nu)
        assert np.all(np.diff(v) < 0) and np.all(v <= 1.0)


def test_covariance_diagonal_and_symmetry():
    P = wl.uniform_square(50, 3)
    C = covariance_matrix(P, (2.0, 0.2, 0.325), 1e-3)
    assert np.array_equal(C, C.T)
    np.testing.assert_array_equal(np.diag(C), 2.0 + 1e-3)


def _frac_elimination(C, z):
    """Exact determinant and z^T C^{-1} z of the float64 matrix C (rationals)."""
    n = len(C)
    A = [[Fraction(float(C[i, j])) for j in range(n)] + [Fraction(float(z[i]))] for i in range(n)]
    det = Fraction(1)
    for k in range(n):
        piv = A[k][k]
        assert piv != 0
        det *= piv
        for i in range(k + 1, n):
            f = A[i][k] / piv
            if f:
                for j in range(k, n + 1):
                    A[i][j] -= f * A[k][j]
    x = [Fraction(0)] * n
    for i in reversed(range(n)):
        s = A[i][n] - sum(A[i][j] * x[j] for j in range(i + 1, n))
        x[i] = s / A[i][i]
    quad = sum(Fraction(float(z[i])) * x[i] for i in range(n))
    return det, quad


def _log_fraction(f):
    # log of a positive rational without overflow
    return math.log(f.numerator) - math.log(f.denominator)


@pytest.mark.parametrize("nu", [0.5, 0.325])
def test_dense_against_exact_rational(nu):
    n = 20
    P = wl.uniform_square(n, 7)
    theta = (1.3, 0.25, nu)
    C = covariance_matrix(P, theta, 1e-2)
    z = wl.standard_normal(n, 1, 8)[:, 0]
    det, quad = _frac_elimination(C, z)
    ll, logdet, q = loglik_from_matrix(C, z)
    exact_logdet = _log_fraction(det)
    exact_quad = float(quad)
    assert abs(logdet[0] - exact_logdet) <= 1e-12 * max(1.0, abs(exact_logdet))
    assert abs(q[0] - exact_quad) <= 1e-11 * abs(exact_quad)
    exact_ll = -0.5 * n * math.log(2 * math.pi) - 0.5 * exact_logdet - 0.5 * exact_quad
    assert abs(ll[0] - exact_ll) <= 1e-11 * abs(exact_ll)


def test_dense_leibniz_n5():
    P = wl.uniform_square(5, 9)
    C = covariance_matrix(P, (1.0, 0.3, 1.0), 0.05)
    det = Fraction(0)
    for perm in itertools.permutations(range(5)):
        sign = 1
        for i in range(5):
            for j in range(i + 1, 5):
                if perm[i] > perm[j]:
                    sign = -sign
        term = Fraction(sign)
        for i in range(5):
            term *= Fraction(float(C[i, perm[i]]))
        det += term
    _, logdet, _ = loglik_from_matrix(C, np.ones(5))
    assert abs(logdet[0] - _log_fraction(det)) < 1e-13


def test_hadamard_bound_and_negative_logdet():
    P = wl.uniform_square(300, 5)
    _, logdet, _ = dense_loglik(P, np.ones(300), (1.0, 0.1, 0.5), 1e-6)
    # Hadamard: log|C| <= sum log C_ii = n log(sigma^2 + tau^2)
    assert logdet[0] <= 300 * math.log(1.0 + 1e-6)


def test_white_noise_limit():
    # points 1e4 ell apart: every off-diagonal entry underflows to exactly 0
    n = 40
    P = np.stack([np.arange(n) * 1000.0, np.zeros(n)], axis=1)
    Z = wl.standard_normal(n, 2, 4)
    s2, tau2 = 1.7, 0.3
    ll, logdet, quad = dense_loglik(P, Z, (s2, 0.1, 0.7), tau2)
    exp_logdet = n * math.log(s2 + tau2)
    exp_quad = np.sum(Z * Z, axis=0) / (s2 + tau2)
    np.testing.assert_allclose(logdet, exp_logdet, rtol=1e-14)
    np.testing.assert_allclose(quad, exp_quad, rtol=1e-14)
    np.testing.assert_allclose(ll, -0.5 * n * math.log(2 * math.pi) - 0.5 * exp_logdet
                               - 0.5 * exp_quad, rtol=1e-14)


def test_not_spd_reports_nan():
    # duplicate point, no nugget -> singular covariance
    P = np.array([[0.1, 0.1], [0.1, 0.1], [0.5, 0.2]])
    ll, logdet, quad = dense_loglik(P, np.ones(3), (1.0, 0.2, 0.5), 0.0)
    assert np.isnan(ll[0]) and np.isnan(logdet[0]) and np.isnan(quad[0])
