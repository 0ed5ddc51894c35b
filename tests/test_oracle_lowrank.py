"""Pins for the oracle's ACA and SVD truncation (Section 2.1, Remark 2.4).

References: exact recovery of separable (exactly rank-r) matrices, the
Eckart-Young optimum of numpy's SVD of the explicit product, and the
definition of the fixed-rank class H(T, k) (Definition 2.1).
"""
import numpy as np
import pytest

from oracle.lowrank import K_MAX, aca, truncate
from oracle.matern import covariance_block


def _fns(M):
    return (lambda i: M[i, :].copy()), (lambda j: M[:, j].copy())


@pytest.mark.parametrize("r", [1, 3, 7])
def test_aca_exact_on_separable(r):
    rng = np.random.default_rng(r)
    m, n = 90, 70
    A = rng.standard_normal((m, r))
    B = rng.standard_normal((n, r))
    M = A @ B.T
    U, V = aca(*_fns(M), m, n, 1e-12, 64)
    # r pivots reproduce M; at most one more (noise) step to confirm convergence
    assert r <= U.shape[1] <= r + 1
    np.testing.assert_allclose(U @ V.T, M, atol=1e-12 * np.abs(M).max())


def test_aca_fixed_rank_steps():
    rng = np.random.default_rng(0)
    M = rng.standard_normal((40, 30))
    U, V = aca(*_fns(M), 40, 30, 0.0, 5)
    assert U.shape == (40, 5) and V.shape == (30, 5)


def test_aca_zero_block():
    M = np.zeros((10, 12))
    U, V = aca(*_fns(M), 10, 12, 1e-8, 10)
    assert U.shape[1] == 0


def test_aca_on_admissible_matern_block():
    rng = np.random.default_rng(5)
    P = np.concatenate([rng.random((120, 2)) * 0.2, rng.random((100, 2)) * 0.2 + [0.6, 0.0]])
    M = covariance_block(P, np.arange(120), np.arange(120, 220), (1.0, 0.1, 0.5), 0.0)
    U, V = aca(*_fns(M), 120, 100, 1e-8, 64)
    err = np.linalg.norm(M - U @ V.T, 2) / np.linalg.norm(M, 2)
    assert err < 1e-6     # Frobenius-estimate stop: within a modest factor of eps
    assert U.shape[1] < 40


@pytest.mark.parametrize("eps", [1e-3, 1e-7, 1e-10])
def test_truncate_matches_svd(eps):
    rng = np.random.default_rng(11)
    m, n, r = 80, 60, 25
    s = np.logspace(0, -14, r)
    X = np.linalg.qr(rng.standard_normal((m, r)))[0] * s
    Y = np.linalg.qr(rng.standard_normal((n, r)))[0]
    X = X @ np.linalg.qr(rng.standard_normal((r, r)))[0]   # mix columns
    Y = Y @ np.linalg.qr(rng.standard_normal((r, r)))[0]
    M = X @ Y.T
    sv = np.linalg.svd(M, compute_uv=False)
    U, V = truncate(X, Y, eps, 0)
    k = int(np.count_nonzero(sv > eps * sv[0]))
    assert U.shape[1] == k
    err = np.linalg.norm(M - U @ V.T, 2)
    # Eckart-Young: the optimal rank-k error is sv[k]
    assert err <= sv[k] * (1 + 1e-6) + 1e-14 * sv[0]


def test_truncate_fixed_rank_and_cap():
    rng = np.random.default_rng(12)
    X = rng.standard_normal((50, 30))
    Y = rng.standard_normal((40, 30))
    U, V = truncate(X, Y, 0.0, 4)
    assert U.shape[1] == 4
    sv = np.linalg.svd(X @ Y.T, compute_uv=False)
    assert abs(np.linalg.norm(X @ Y.T - U @ V.T, 2) - sv[4]) < 1e-9 * sv[0]
    X = rng.standard_normal((300, 200))
    Y = rng.standard_normal((300, 200))
    U, _ = truncate(X, Y, 1e-16, 0)
    assert U.shape[1] == K_MAX


def test_truncate_zero():
    U, V = truncate(np.zeros((5, 2)), np.ones((4, 2)), 1e-8, 0)
    assert U.shape == (5, 0) and V.shape == (4, 0)


@pytest.mark.parametrize("eps,k", [(1e-6, 0), (1e-12, 0), (0.0, 5)])
def test_truncate_dense_eckart_young(eps, k):
    from oracle.lowrank import truncate_dense
    rng = np.random.default_rng(3)
    D = rng.standard_normal((40, 30)) @ np.diag(np.logspace(0, -14, 30)) @ rng.standard_normal((30, 33))
    U, V = truncate_dense(D, eps, k)
    sv = np.linalg.svd(D, compute_uv=False)
    kk = k if k else int(np.count_nonzero(sv > eps * sv[0]))
    assert U.shape[1] == kk
    assert np.linalg.norm(D - U @ V.T, 2) <= sv[kk] * (1 + 1e-6) + 1e-14 * sv[0]
    # same best approximation as the factored truncation of D = D * I
    from oracle.lowrank import truncate
    U2, V2 = truncate(D, np.eye(33), eps, k)
    assert np.allclose(U @ V.T, U2 @ V2.T, atol=1e-12 * sv[0])
