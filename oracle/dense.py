"""Exact (dense) Gaussian log-likelihood, eq. (1) of Section 1.

    L(theta) = -n/2 log(2 pi) - 1/2 log|C(theta)| - 1/2 Z^T C(theta)^{-1} Z

evaluated through the Cholesky factor C = L L^T: log|C| = 2 sum log L_ii and
Z^T C^{-1} Z = v^T v with L v = Z.  This is the plain definition of the
quantity the H-matrix method approximates; it is O(n^3) and used for n up to
a few thousand in tests.

A non-positive pivot means C is not numerically SPD; the oracle then reports
NaN for all three parts, as the device path does.

Parity pins (tests/test_oracle_dense.py): exact rational determinant and
solve of the float64-rounded matrix (fraction arithmetic) at small n, the
Leibniz expansion at n = 5, Hadamard's bound, and the white-noise closed form.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg

from .matern import covariance_block


def covariance_matrix(P, theta, nugget):
    n = len(P)
    idx = np.arange(n)
    return covariance_block(P, idx, idx, theta, nugget)


def loglik_from_matrix(C: np.ndarray, Z: np.ndarray):
    """Returns (loglik, logdet, quadform) arrays over the columns of Z."""
    Z = np.asarray(Z, dtype=np.float64)
    if Z.ndim == 1:
        Z = Z[:, None]
    n = C.shape[0]
    try:
        L = np.linalg.cholesky(C)
    except np.linalg.LinAlgError:
        nan = np.full(Z.shape[1], np.nan)
        return nan, nan, nan
    logdet = 2.0 * np.sum(np.log(np.diag(L)))
    v = scipy.linalg.solve_triangular(L, Z, lower=True)
    quad = np.sum(v * v, axis=0)
    ll = -0.5 * n * math.log(2.0 * math.pi) - 0.5 * logdet - 0.5 * quad
    return ll, np.full(Z.shape[1], logdet), quad


def dense_loglik(P, Z, theta, nugget):
    """Eq. (1) for locations P (n x 2), data Z (n or n x r), theta = (sigma2, ell, nu)."""
    return loglik_from_matrix(covariance_matrix(P, theta, nugget), Z)


def dense_factor(P, theta, nugget):
    """Lower Cholesky factor of the dense covariance (used to simulate data Z = L W)."""
    return np.linalg.cholesky(covariance_matrix(P, theta, nugget))
