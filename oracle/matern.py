"""Matern covariance for the oracle, eq. (2) of Section 2.2, plus the nugget.

    C(h; theta) = sigma^2 / (2^(nu-1) Gamma(nu)) * (h/ell)^nu * K_nu(h/ell),
    theta = (sigma^2, ell, nu),

read exactly as printed: the argument of K_nu is h/ell with no sqrt(2 nu)
factor.  At h = 0 the function is continued by its limit, C(0) = sigma^2
(x^nu K_nu(x) -> 2^(nu-1) Gamma(nu) as x -> 0).  The nugget tau^2 of the
remark in Section 2.4 is added on the diagonal i = j only (coincident but
distinct locations get sigma^2 without the nugget).

Parity pins: nu = 1/2 gives the exponential model exp(-h/ell) (Section 2.2);
nu = 3/2 gives (1 + x) exp(-x); the value at 0 is sigma^2 (tests/test_oracle_dense.py).
"""
from __future__ import annotations

import math

import numpy as np

from .besselk import kve


def matern_correlation(x, nu: float) -> np.ndarray:
    """M_nu(x) = x^nu K_nu(x) / (2^(nu-1) Gamma(nu)), with M_nu(0) = 1."""
    x = np.asarray(x, dtype=np.float64)
    out = np.ones_like(x)
    pos = x > 0
    if np.any(pos):
        xp = x[pos]
        norm = 2.0 ** (nu - 1.0) * math.gamma(nu)
        out[pos] = np.power(xp, nu) * kve(nu, xp) * np.exp(-xp) / norm
    return out


def pair_distance(P: np.ndarray, rows, cols) -> np.ndarray:
    """Euclidean distances ||s_i - s_j|| for i in rows, j in cols (2-D points)."""
    a = P[np.asarray(rows)]
    b = P[np.asarray(cols)]
    dx = a[:, None, 0] - b[None, :, 0]
    dy = a[:, None, 1] - b[None, :, 1]
    return np.sqrt(dx * dx + dy * dy)


def covariance_block(P: np.ndarray, rows, cols, theta, nugget: float) -> np.ndarray:
    """Entries C_ij = sigma^2 M_nu(||s_i - s_j|| / ell) + tau^2 [i == j] for
    the given index lists (indices refer to rows of P)."""
    sigma2, ell, nu = theta
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    C = sigma2 * matern_correlation(pair_distance(P, rows, cols) / ell, nu)
    if nugget:
        C = C + nugget * (rows[:, None] == cols[None, :])
    return C
