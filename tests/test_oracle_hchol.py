"""Pins for the oracle's H-Cholesky likelihood, eq. (4), against the dense
definition, eq. (1).

  * eta = 0 admits no low-rank block: the H-Cholesky is then an exact blocked
    Cholesky and must equal the dense oracle to rounding ("the full rank gives
    an exact representation", Section 1).
  * With low-rank blocks at tiny eps the H value converges to the dense one.
  * Theorem 1 (Section 3.2): |L~ - L| <= n/2 (-log(1 - e)) + 1/2 |z|^2
    max(|C^-1|, |C~^-1|) e with e = || I - (L~ L~^T)^{-1} C ||_2 computed densely
    (the statement's C~^-1 and the proof's C^-1 differ; the larger is used).
  * || C~ - L~ L~^T ||_2 / || C~ ||_2 = O(eps) for the formatted factor.
  * a forced breakdown (duplicate points, no nugget) reports not SPD.
"""
import math

import numpy as np
import pytest

from oracle.dense import covariance_matrix, dense_loglik
from oracle.hchol import HLikelihood, h_loglik
from paper_1709_04419_amd import workloads as wl


@pytest.fixture(scope="module")
def case600():
    n = 600
    P = wl.uniform_square(n, 21)
    theta = (1.0, 0.1, 0.5)
    nug = 1e-6
    C = covariance_matrix(P, theta, nug)
    L = np.linalg.cholesky(C)
    W = wl.standard_normal(n, 2, 22)
    Z = L @ W
    return P, theta, nug, C, Z


def test_eta_zero_equals_dense(case600):
    P, theta, nug, C, Z = case600
    d = dense_loglik(P, Z, theta, nug)
    h = h_loglik(P, Z, theta, nug, n_min=32, eta=0.0, eps=1e-8)
    np.testing.assert_allclose(h["logdet"], d[1], rtol=1e-13)
    np.testing.assert_allclose(h["quadform"], d[2], rtol=1e-10)
    np.testing.assert_allclose(h["loglik"], d[0], rtol=1e-12)


def test_tiny_eps_converges(case600):
    P, theta, nug, C, Z = case600
    d = dense_loglik(P, Z, theta, nug)
    h = h_loglik(P, Z, theta, nug, n_min=32, eta=2.0, eps=1e-14)
    np.testing.assert_allclose(h["loglik"], d[0], rtol=1e-9)
    np.testing.assert_allclose(h["logdet"], d[1], rtol=1e-10)


@pytest.mark.parametrize("eps", [1e-4, 1e-6, 1e-8])
def test_theorem1_bound(case600, eps):
    P, theta, nug, C, Z = case600
    n = len(P)
    H = HLikelihood(P, 32, 2.0)
    res = H.loglik(theta, nug, Z, eps, 0)
    d = dense_loglik(P, Z, theta, nug)
    Lt = H.factor_to_dense()
    # undo the permutation: the factor lives in permuted order
    perm = H.perm
    Cp = C[np.ix_(perm, perm)]
    LLt = Lt @ Lt.T
    E = np.eye(n) - np.linalg.solve(LLt, Cp)
    e = np.linalg.norm(E, 2)
    assert e < 1
    c1 = max(1 / np.linalg.eigvalsh(Cp)[0], 1 / np.linalg.eigvalsh(LLt)[0])
    for j in range(Z.shape[1]):
        z2 = float(Z[:, j] @ Z[:, j])
        bound = 0.5 * n * (-math.log1p(-e)) + 0.5 * z2 * c1 * e
        assert abs(res["loglik"][j] - d[0][j]) <= bound
        assert abs(res["logdet"][j] - d[1][j]) <= -n * math.log1p(-e)


@pytest.mark.parametrize("eps", [1e-5, 1e-8])
def test_factor_residual(case600, eps):
    P, theta, nug, C, Z = case600
    H = HLikelihood(P, 32, 2.0)
    H.assemble(theta, nug, eps, 0)
    Ct = H.to_dense()
    H.factor()
    Lt = H.factor_to_dense()
    rel = np.linalg.norm(Ct - Lt @ Lt.T, 2) / np.linalg.norm(Ct, 2)
    assert rel < 50 * eps
    # the assembled matrix itself is eps-close to the exact covariance
    Cp = C[np.ix_(H.perm, H.perm)]
    assert np.linalg.norm(Cp - Ct, 2) / np.linalg.norm(Cp, 2) < 50 * eps


def test_fixed_rank_mode(case600):
    P, theta, nug, C, Z = case600
    H = HLikelihood(P, 32, 2.0)
    r = H.loglik(theta, nug, Z, 0.0, 6)
    assert r["status"] == "ok"
    assert max(H.stats.final_ranks) <= 6
    d = dense_loglik(P, Z, theta, nug)
    # rank 6 is coarse: only the order of magnitude is pinned
    assert abs(r["loglik"][0] - d[0][0]) < 0.05 * abs(d[0][0])


def test_not_spd_breakdown():
    P = wl.uniform_square(200, 3)
    P[150] = P[10]          # duplicate location, no nugget: singular covariance
    r = h_loglik(P, np.ones(200), (1.0, 0.2, 0.5), 0.0, n_min=16, eta=2.0, eps=1e-10)
    assert r["status"] == "not_spd"
    assert np.isnan(r["loglik"][0])
