"""GPU parity of the HIP H-likelihood path against the CPU oracle.

Every call goes through the C ABI (libhmlik.so via the ctypes binding).  The
oracle is the plain CPU implementation in oracle/ (independent code).  Bars:
  * cluster tree, permutation, boxes, block partition: bit-exact;
  * dense-leaf entries: 1e-14 relative; low-rank blocks U V^T: 1e-11 relative
    to the block's largest entry (the two sides take the same ACA pivots and
    truncation ranks; only rounding differs);
  * L~(theta), log|C~|, v^T v: 1e-10 relative;
  * breakdown: the same block and pivot as the oracle;
  * repeated evaluations: bitwise identical.
"""
import math

import numpy as np
import pytest

from oracle.dense import dense_loglik
from oracle.hchol import HLikelihood, NotSPD
from oracle.htree import DENSE, LOWRANK, NODE, BlockTree, ClusterTree
from paper_1709_04419_amd import workloads as wl

pytestmark = pytest.mark.gpu

REL = 1e-10


@pytest.fixture(scope="module")
def H():
    from paper_1709_04419_amd import hmlik
    return hmlik


@pytest.fixture(scope="module")
def ctx(H):
    c = H.Context(0)
    yield c
    c.close()


KINDS = {NODE: 0, DENSE: 1, LOWRANK: 2}


@pytest.mark.parametrize("kind,n,leaf,eta", [("uniform", 2000, 32, 2.0), ("basin", 6000, 64, 2.0),
                                              ("grid", 1024, 32, 2.0), ("uniform", 65, 32, 2.0),
                                              ("uniform", 1, 8, 2.0), ("basin", 3000, 17, 0.7)])
def test_trees_bit_exact(H, ctx, kind, n, leaf, eta):
    P = wl.make_points(kind, n, 5)
    ds = H.Dataset(ctx, P, leaf, eta)
    perm, ranges, boxes = ds.export_tree()
    rc, kinds = ds.export_blocks()
    T = ClusterTree(P, leaf)
    BT = BlockTree(T, eta)
    assert np.array_equal(perm, T.perm)
    assert np.array_equal(ranges, np.array([[c.begin, c.end] for c in T.clusters]))
    ob = np.array([[c.lo[0], c.lo[1], c.hi[0], c.hi[1]] for c in T.clusters])
    assert np.array_equal(boxes, ob)
    C = T.clusters
    orc = np.array([[C[b.row].begin, C[b.col].begin, C[b.row].size, C[b.col].size] for b in BT.blocks])
    assert np.array_equal(rc, orc)
    assert np.array_equal(kinds, np.array([KINDS[b.kind] for b in BT.blocks], dtype=np.int8))
    ds.close()


def _oracle_assembled(P, leaf, theta, nug, eps, k):
    Ho = HLikelihood(P, leaf, 2.0)
    Ho.assemble(theta, nug, eps, k)
    return Ho


@pytest.mark.parametrize("theta,eps,k", [((1.0, 0.1, 0.5), 1e-8, 0), ((1.3, 0.15, 0.325), 1e-7, 0),
                                         ((1.0, 0.2, 1.0), 0.0, 10), ((0.8, 0.05, 1.5), 1e-6, 0)])
def test_assembly_parity(H, ctx, theta, eps, k):
    n, leaf, nug = 1500, 32, 1e-6
    P = wl.uniform_square(n, 41)
    Ho = _oracle_assembled(P, leaf, theta, nug, eps, k)
    ds = H.Dataset(ctx, P, leaf, 2.0)
    ds.set_z(np.ones(n))
    ds.assemble(theta, nug, eps, k)
    rc, kinds = ds.export_blocks()
    for b, blk in enumerate(Ho.bt.blocks):
        if blk.kind == DENSE:
            g = ds.get_block(b, rc[b, 2], rc[b, 3])
            o = Ho.D[b]
            assert np.max(np.abs(g - o)) <= 1e-14 * np.max(np.abs(o)), b
        elif blk.kind == LOWRANK:
            U, V = ds.get_block(b, rc[b, 2], rc[b, 3])
            assert U.shape[1] == Ho.U[b].shape[1], b        # same truncated rank
            o = Ho.U[b] @ Ho.V[b].T
            assert np.max(np.abs(U @ V.T - o)) <= 1e-11 * np.max(np.abs(o)), b
    ds.close()


CASES = [
    # n, points, leaf, theta, nugget, eps, k
    (2000, ("uniform", 11), 32, (1.0, 0.1, 0.5), 1e-6, 1e-8, 0),       # uniform2k: the small configuration
    (300, ("uniform", 11), 16, (1.0, 0.1, 0.5), 1e-6, 1e-8, 0),
    (1200, ("basin", 31), 64, (1.0, 0.1, 0.325), 1e-6, 1e-7, 0),       # irregular domain, nu = 0.325
    (1000, ("uniform", 21), 32, (1.0, 0.05, 1.0), 1e-6, 0.0, 10),       # fixed rank, nu = 1 (mu = 0 in Temme)
    (1000, ("uniform", 22), 32, (1.0, 0.1, 1.5), 1e-6, 0.0, 12),        # fixed rank 12, nu = 3/2
    (784, ("grid", 7), 24, (2.0, 0.0334, 0.5), 1e-4, 1e-6, 0),          # perturbed grid of eq. (3)
    (777, ("uniform", 9), 20, (1.0, 0.05, 2.2), 1e-6, 1e-9, 0),         # ragged n, nu > 2 (two recurrences)
    (1000, ("uniform", 22), 32, (1.0, 0.2, 1.5), 1e-6, 0.0, 5),         # fixed rank 5: breaks down (not SPD)
    (6000, ("basin", 31), 64, (1.0, 0.1, 0.325), 1e-6, 1e-7, 0),       # low-rank blocks of 750 rows (tall panels)
]


@pytest.mark.parametrize("case", CASES, ids=[f"n{c[0]}_{c[1][0]}_nu{c[3][2]}_k{c[6]}" for c in CASES])
def test_loglik_parity(H, ctx, case):
    n, (kind, seed), leaf, theta, nug, eps, k = case
    P = wl.make_points(kind, n, seed)
    Z = wl.standard_normal(n, 2, seed + 1)
    o = HLikelihood(P, leaf, 2.0).loglik(theta, nug, Z, eps, k)
    ds = H.Dataset(ctx, P, leaf, 2.0)
    ds.set_z(Z)
    g = ds.loglik(theta, nug, eps, k)
    if o["status"] == "not_spd":
        # breakdown: the same block and pivot on both sides
        assert np.all(g["status"] == H.HM_ERR_NOT_SPD)
        assert g["fail_block"][0] == o["fail_block"] and g["fail_pivot"][0] == o["fail_pivot"]
        ds.close()
        return
    assert np.all(g["status"] == 0)
    for key in ("loglik", "logdet", "quadform"):
        np.testing.assert_allclose(g[key], o[key], rtol=REL, atol=0, err_msg=key)
    # repeat: bitwise identical
    g2 = ds.loglik(theta, nug, eps, k)
    for key in ("loglik", "logdet", "quadform"):
        assert np.array_equal(g[key], g2[key])
    ds.close()


def test_vs_dense_theorem1(H, ctx):
    """The H value is close to the exact dense likelihood (eq. 1) at eps = 1e-8."""
    n = 2000
    P = wl.uniform_square(n, 11)
    theta, nug = (1.0, 0.1, 0.5), 1e-6
    Z = wl.standard_normal(n, 1, 12)
    d = dense_loglik(P, Z, theta, nug)
    ds = H.Dataset(ctx, P, 32, 2.0)
    ds.set_z(Z)
    g = ds.loglik(theta, nug, 1e-8, 0)
    assert abs(g["loglik"][0] - d[0][0]) <= 1e-7 * abs(d[0][0])
    assert abs(g["logdet"][0] - d[1][0]) <= 1e-7 * abs(d[1][0])
    ds.close()


def test_multiple_rhs_equal_single(H, ctx):
    n = 900
    P = wl.uniform_square(n, 13)
    Z = wl.standard_normal(n, 3, 14)
    theta = (1.0, 0.1, 0.5)
    ds = H.Dataset(ctx, P, 32, 2.0)
    ds.set_z(Z)
    g = ds.loglik(theta, 1e-6, 1e-8, 0)
    for j in range(3):
        ds.set_z(Z[:, j])
        s = ds.loglik(theta, 1e-6, 1e-8, 0)
        np.testing.assert_allclose(s["loglik"][0], g["loglik"][j], rtol=1e-13)
    ds.close()


def test_breakdown_same_block_as_oracle(H, ctx):
    """Coarse rank-1 approximation of a smooth field without nugget is not
    positive definite: the paper's H-Cholesky 'crash' (Tables 6, 7) becomes a
    status with the failing block and pivot."""
    n, leaf = 400, 16
    P = wl.uniform_square(n, 3)
    theta = (1.0, 0.5, 1.5)
    with pytest.raises(NotSPD) as ei:
        Ho = HLikelihood(P, leaf, 2.0)
        Ho.assemble(theta, 0.0, 0.0, 1)
        Ho.factor()
    ds = H.Dataset(ctx, P, leaf, 2.0)
    ds.set_z(np.ones(n))
    g = ds.loglik(theta, 0.0, 0.0, 1)
    assert g["status"][0] == H.HM_ERR_NOT_SPD
    assert g["fail_block"][0] == ei.value.block
    assert g["fail_pivot"][0] == ei.value.pivot
    assert math.isnan(g["loglik"][0])
    ds.close()


def test_argument_errors(H, ctx):
    P = wl.uniform_square(100, 1)
    with pytest.raises(H.HMError):
        H.Dataset(ctx, P, 0, 2.0)
    with pytest.raises(H.HMError):
        H.Dataset(ctx, P, 65, 2.0)
    bad = P.copy()
    bad[3, 0] = np.nan
    with pytest.raises(H.HMError):
        H.Dataset(ctx, bad, 16, 2.0)
    ds = H.Dataset(ctx, P, 16, 2.0)
    ds.set_z(np.ones(100))
    for theta, nug, eps, k in [((0.0, 0.1, 0.5), 0.0, 1e-6, 0), ((1.0, -0.1, 0.5), 0.0, 1e-6, 0),
                               ((1.0, 0.1, 0.0), 0.0, 1e-6, 0), ((1.0, 0.1, 0.5), -1.0, 1e-6, 0),
                               ((1.0, 0.1, 0.5), 0.0, 0.0, 0), ((1.0, 0.1, 0.5), 0.0, 0.0, 65)]:
        with pytest.raises(H.HMError) as ei:
            ds.loglik(theta, nug, eps, k)
        assert ei.value.status == H.HM_ERR_ARG
    ds.close()


@pytest.mark.parametrize("m,n,r,eps,rk", [(64, 64, 20, 1e-8, 0), (250, 125, 64, 1e-7, 0), (31, 200, 40, 1e-6, 0),
                                          (128, 100, 90, 1e-8, 0), (64, 64, 64, 0.0, 7), (1, 50, 3, 1e-7, 0),
                                          (700, 650, 40, 1e-7, 0), (1500, 600, 64, 1e-7, 0), (300, 1400, 50, 1e-7, 0),
                                          (900, 800, 61, 0.0, 9), (3000, 2500, 64, 1e-7, 0), (2000, 530, 128, 1e-7, 0)])
def test_truncation_parity(H, ctx, m, n, r, eps, rk):
    """Device truncation of X Y^T vs numpy's SVD of the explicit product:
    same rank, Eckart-Young optimal error.  Panels of more than 512 rows take
    the blocked (compact WY) QR and Q application."""
    P = wl.uniform_square(16000 if m + n > 2000 else 4000, 2)
    ds = H.Dataset(ctx, P, 64, 2.0)
    rng = np.random.default_rng(m * 1000 + r)
    X = (rng.standard_normal((m, min(r, 25))) @ rng.standard_normal((min(r, 25), r))) * np.logspace(0, -13, r)
    Y = rng.standard_normal((n, r))
    M = X @ Y.T
    U, V, _ = H.test_truncate(ds, X, Y, eps, rk)
    sv = np.linalg.svd(M, compute_uv=False)
    k = min(rk, int(np.count_nonzero(sv > 0))) if rk else int(np.count_nonzero(sv > eps * sv[0]))
    assert U.shape[1] == k
    opt = sv[k] if k < len(sv) else 0.0
    assert np.linalg.norm(M - U @ V.T, 2) <= opt * (1 + 1e-6) + 1e-13 * sv[0]
    ds.close()


@pytest.mark.parametrize("m,n,eps,rk", [(62, 62, 1e-7, 0), (125, 125, 1e-7, 0), (250, 250, 1e-7, 0),
                                        (250, 180, 1e-8, 0), (200, 256, 0.0, 10), (1, 40, 1e-7, 0),
                                        (70, 1, 1e-7, 0), (256, 256, 1e-12, 0)])
def test_explicit_truncation_parity(H, ctx, m, n, eps, rk):
    """Truncation of an explicit matrix (the explicit flush of small low-rank
    blocks: pivoted QR, then Jacobi on R^T) vs numpy's SVD: same rank,
    Eckart-Young optimal error."""
    ds = H.Dataset(ctx, wl.uniform_square(4000, 2), 64, 2.0)
    rng = np.random.default_rng(m * 7 + n)
    q = min(m, n)
    A = rng.standard_normal((m, q)) * np.logspace(0, -15, q)
    B = rng.standard_normal((q, n))
    M = A @ B
    U, V, _ = H.test_truncate(ds, M, None, eps, rk)
    sv = np.linalg.svd(M, compute_uv=False)
    k = min(rk, int(np.count_nonzero(sv > 0))) if rk else min(int(np.count_nonzero(sv > eps * sv[0])), 64)
    assert U.shape[1] == k
    opt = sv[k] if k < len(sv) else 0.0
    assert np.linalg.norm(M - U @ V.T, 2) <= opt * (1 + 1e-6) + 1e-13 * sv[0]
    ds.close()


def test_loglik_batch_equals_single(H, ctx):
    """hm_loglik_batch: datasets of different sizes, shapes and theta (one of
    them breaking down) evaluated together give bitwise the results of
    separate hm_loglik calls."""
    specs = [(1500, ("uniform", 11), 32, (1.0, 0.1, 0.5), 1e-6, 1e-8, 0),
             (1200, ("basin", 31), 64, (1.0, 0.1, 0.325), 1e-6, 1e-7, 0),
             (784, ("grid", 7), 24, (2.0, 0.0334, 0.5), 1e-4, 1e-6, 0),
             (1000, ("uniform", 22), 32, (1.0, 0.2, 1.5), 1e-6, 0.0, 5)]
    single, dss = [], []
    for n, (kind, seed), leaf, theta, nug, eps, k in specs:
        P = wl.make_points(kind, n, seed)
        ds = H.Dataset(ctx, P, leaf, 2.0)
        ds.set_z(wl.standard_normal(n, 2, seed + 1))
        single.append(ds.loglik(theta, nug, eps, k))
        dss.append(ds)
    try:
        res = H.loglik_batch(ctx, dss, [s[3] for s in specs], [s[4] for s in specs], [s[5] for s in specs],
                             [s[6] for s in specs])
        assert single[3]["status"][0] == H.HM_ERR_NOT_SPD       # the fixed-rank case breaks down
        for i, r in enumerate(res):
            for key in ("loglik", "logdet", "quadform", "status", "fail_block", "fail_pivot", "max_rank"):
                assert np.array_equal(r[key], single[i][key], equal_nan=key in ("loglik", "logdet", "quadform")), \
                    (i, key)
    finally:
        for ds in dss:
            ds.close()


def test_tuned_schedule_same_results(H, ctx):
    """hm_tune_schedule re-balances the factorisation's levels; the results of
    later evaluations (other theta too, alone and batched) stay bitwise equal,
    and still match the oracle."""
    n = 3000
    P = wl.basin_clusters(n, 31)
    Z = wl.standard_normal(n, 1, 32)
    theta, nug, eps = (1.0, 0.1, 0.325), 1e-6, 1e-7
    ds = H.Dataset(ctx, P, 32, 2.0)
    ds2 = H.Dataset(ctx, wl.uniform_square(1500, 11), 32, 2.0)
    try:
        ds.set_z(Z)
        ds2.set_z(wl.standard_normal(1500, 1, 12))
        before = [ds.loglik(theta, nug, eps, 0), ds.loglik((1.2, 0.08, 0.5), nug, eps, 0)]
        assert ds.tune_schedule(theta, nug, eps, 0) == H.HM_OK
        after = [ds.loglik(theta, nug, eps, 0), ds.loglik((1.2, 0.08, 0.5), nug, eps, 0)]
        for b, a in zip(before, after):
            for key in ("loglik", "logdet", "quadform", "max_rank"):
                assert np.array_equal(a[key], b[key]), key
        o = HLikelihood(P, 32, 2.0).loglik(theta, nug, Z, eps, 0)
        np.testing.assert_allclose(after[0]["loglik"], o["loglik"], rtol=REL, atol=0)
        res = H.loglik_batch(ctx, [ds, ds2], [theta, (1.0, 0.1, 0.5)], [nug, nug], [eps, 1e-8], [0, 0])
        assert np.array_equal(res[0]["loglik"], after[0]["loglik"])
    finally:
        ds.close()
        ds2.close()
