"""Pins for the oracle's K_nu (integral representation, trapezoidal rule).

Pinned against: closed forms at half-integer order, mpmath at 40 digits, the
three-term recurrence K_{nu+1} = K_{nu-1} + (2 nu / x) K_nu, and the small-x
limit x^nu K_nu(x) -> 2^(nu-1) Gamma(nu).  None of these re-evaluates the
oracle's own quadrature.
"""
import math

import mpmath
import numpy as np
import pytest

from oracle.besselk import kv, kve

XS = np.concatenate([np.logspace(-8, 2.8, 60), [0.5, 1.0, 2.0, 2.0000001, 5.0, 30.0]])


def test_half_integer_closed_forms():
    x = XS
    base = np.sqrt(np.pi / (2 * x))
    np.testing.assert_allclose(kve(0.5, x), base, rtol=2e-15, atol=0)
    np.testing.assert_allclose(kve(1.5, x), base * (1 + 1 / x), rtol=2e-15, atol=0)
    np.testing.assert_allclose(kve(2.5, x), base * (1 + 3 / x + 3 / x ** 2), rtol=4e-15, atol=0)


@pytest.mark.parametrize("nu", [0.1, 0.22, 0.325, 0.9, 1.0, 1.7])
def test_against_mpmath(nu):
    mpmath.mp.dps = 40
    x = XS
    ref = np.array([float(mpmath.besselk(nu, mpmath.mpf(float(v))) * mpmath.exp(mpmath.mpf(float(v))))
                    for v in x])
    np.testing.assert_allclose(kve(nu, x), ref, rtol=3e-15, atol=0)


@pytest.mark.parametrize("nu", [0.325, 0.8, 1.3])
def test_recurrence(nu):
    x = np.logspace(-2, 2, 40)
    lhs = kve(nu + 1, x)
    rhs = kve(nu - 1, x) + (2 * nu / x) * kve(nu, x)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-14)


@pytest.mark.parametrize("nu", [0.2, 0.5, 1.5])
def test_small_x_limit(nu):
    x = np.array([1e-12, 1e-10])
    val = x ** nu * kv(nu, x)
    lim = 2 ** (nu - 1) * math.gamma(nu)
    # next term of the expansion is O(x^(2 nu)) relative
    np.testing.assert_allclose(val, lim, rtol=5 * 1e-10 ** (2 * nu) + 1e-14)


def test_even_in_order():
    x = np.array([0.3, 3.0])
    np.testing.assert_allclose(kve(-0.7, x), kve(0.7, x), rtol=0)


def test_rejects_nonpositive():
    with pytest.raises(ValueError):
        kve(0.5, np.array([0.0]))
