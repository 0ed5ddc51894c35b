"""GPU tests of the accuracy diagnostics (Section 2.4; paper_1709_04419_amd/
diagnostics.py) against the oracle's dense matrices: the exact covariance
entries (eq. 2 plus the nugget), log|C| and the Kullback-Leibler divergence
between N(0, C) and N(0, C~) for a coarse C~, where D_KL is well above its
rounding floor, and the power-iteration estimate of ||I - C~^{-1} C||_2 against
the exact 2-norm.  C~ enters through its factor, C~ = L~ L~^T, and parity is
against the oracle's own L~ (HLikelihood.factor_to_dense), so a slip in the
trace, the log-determinants or the order of the exact entries fails."""
import numpy as np
import pytest

from oracle.dense import covariance_matrix
from oracle.hchol import HLikelihood
from oracle.matern import covariance_block
from paper_1709_04419_amd import workloads as wl

pytestmark = pytest.mark.gpu

THETA, NUGGET = (1.0, 0.1, 0.5), 1e-4


def test_exact_block_matches_oracle():
    from paper_1709_04419_amd import hmlik
    P = wl.basin_clusters(700, 91)
    ctx = hmlik.Context(0)
    try:
        ds = hmlik.Dataset(ctx, P, 32, 2.0)
        ds.set_z(wl.standard_normal(700, 1, 92))
        ds.loglik(THETA, NUGGET, 1e-8)
        rows, cols = np.arange(100, 430), np.arange(250, 700)
        got = ds.exact_block(100, 330, 250, 450)
        ref = covariance_block(P, rows, cols, THETA, NUGGET)
        np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-15)
        dev = ds.exact_block(0, 700, 0, 700, device=True).cpu().numpy()
        np.testing.assert_allclose(dev, covariance_matrix(P, THETA, NUGGET), rtol=1e-13, atol=1e-15)
        # the diagonal carries the nugget; an empty block is fine; a range past n is refused
        assert ds.exact_block(5, 0, 0, 3).shape == (0, 3)
        with pytest.raises(hmlik.HMError):
            ds.exact_block(690, 20, 0, 5)
    finally:
        ctx.close()


def test_kld_and_inverse_error_match_oracle():
    from paper_1709_04419_amd import diagnostics, hmlik
    n, eps = 900, 1e-3
    P = wl.uniform_square(n, 93)
    H = HLikelihood(P, n_min=32, eta=2.0)
    H.assemble(THETA, NUGGET, eps, 0)
    H.factor()
    Lt = H.factor_to_dense()                            # L~, tree order
    C = covariance_matrix(H.Pp, THETA, NUGGET)          # C, tree order
    # the diagnostics see C~ through its factor: log|L~ L~^T| and (L~ L~^T)^{-1} C
    ld_t = H.logdet()
    ld = np.linalg.slogdet(C)[1]
    M = np.linalg.solve(Lt.T, np.linalg.solve(Lt, C))
    kld_ref = 0.5 * (np.trace(M) - n + ld_t - ld)
    inv_ref = np.linalg.norm(np.eye(n) - M, 2)
    ctx = hmlik.Context(0)
    try:
        ds = hmlik.Dataset(ctx, P, 32, 2.0)
        ds.set_z(wl.standard_normal(n, 1, 94))
        d = diagnostics.accuracy(ds, THETA, NUGGET, eps=eps, power_iters=30)
    finally:
        ctx.close()
    assert d["status"] == 0
    assert abs(d["logdet_exact"] - ld) <= 1e-11 * abs(ld)
    assert abs(d["logdet_h"] - ld_t) <= 1e-10 * abs(ld_t)
    assert kld_ref > 1e-8                                # coarse enough to be measurable
    assert abs(d["kld"] - kld_ref) <= 1e-6 * kld_ref + 1e-9
    # power iteration approaches the 2-norm from below
    assert 0.5 * inv_ref <= d["inv_err"] <= inv_ref * (1 + 1e-6)
