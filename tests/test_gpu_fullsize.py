"""GPU parity at the full sizes of the benchmark workloads, on outputs the CPU
oracle can compute one at a time (its H-Cholesky cannot run at these sizes):

  * basin, n = 256,000, leaf 64, eta 2, eps = 1e-7 (the benchmark workload) and
    uniform, n = 64,000, fixed rank k = 10 (the fixed-rank configuration):
    cluster tree, permutation, boxes and block partition bit-exact; sampled
    dense leaves to 1e-14; sampled low-rank leaves (the largest ones included)
    against the oracle's ACA + truncation of the same block: same rank, and
    the two products equal to 1e-11 of their largest entry on 200 sampled
    rows and columns;
  * the fixed-rank configuration evaluated in full: bitwise repeatable, and
    either the H-Cholesky breaks down (status, block, pivot) or log|C~|
    respects Hadamard's bound n log(sigma^2 + tau^2), v^T v > 0 and L~ is finite.
"""
import math

import numpy as np
import pytest

from oracle.hchol import HLikelihood
from oracle.htree import DENSE, LOWRANK, NODE, BlockTree, ClusterTree
from paper_1709_04419_amd import workloads as wl

pytestmark = pytest.mark.gpu

KINDS = {NODE: 0, DENSE: 1, LOWRANK: 2}

FULL = [
    ("basin256k", lambda: wl.basin_clusters(256000, 31), 64, (1.0, 0.1, 0.325), 1e-6, 1e-7, 0),
    ("uniform64k_k10", lambda: wl.uniform_square(64000, 21), 64, (1.0, 0.05, 0.5), 1e-6, 0.0, 10),
]


@pytest.fixture(scope="module")
def H():
    from paper_1709_04419_amd import hmlik
    return hmlik


@pytest.fixture(scope="module")
def ctx(H):
    c = H.Context(0)
    yield c
    c.close()


def _sampled_diff(Ud, Vd, Uo, Vo, rng, s=200):
    """Largest entry of Ud Vd^T - Uo Vo^T and of Uo Vo^T over s sampled rows and
    columns (the full products of the largest blocks would not fit)."""
    rs = rng.choice(Ud.shape[0], min(s, Ud.shape[0]), replace=False)
    cs = rng.choice(Vd.shape[0], min(s, Vd.shape[0]), replace=False)
    d = Ud[rs] @ Vd[cs].T
    o = Uo[rs] @ Vo[cs].T
    return float(np.max(np.abs(d - o))), float(np.max(np.abs(o)))


@pytest.mark.parametrize("case", FULL, ids=[c[0] for c in FULL])
def test_fullsize_trees_and_sampled_blocks(H, ctx, case):
    name, gen, leaf, theta, nug, eps, k = case
    P = gen()
    n = len(P)
    ds = H.Dataset(ctx, P, leaf, 2.0)
    try:
        T = ClusterTree(P, leaf)
        BT = BlockTree(T, 2.0)
        perm, ranges, boxes = ds.export_tree()
        assert np.array_equal(perm, T.perm)
        assert np.array_equal(ranges, np.array([[c.begin, c.end] for c in T.clusters]))
        assert np.array_equal(boxes, np.array([[c.lo[0], c.lo[1], c.hi[0], c.hi[1]] for c in T.clusters]))
        rc, kinds = ds.export_blocks()
        C = T.clusters
        assert np.array_equal(rc, np.array([[C[b.row].begin, C[b.col].begin, C[b.row].size, C[b.col].size]
                                            for b in BT.blocks]))
        assert np.array_equal(kinds, np.array([KINDS[b.kind] for b in BT.blocks], dtype=np.int8))
        ds.set_z(np.ones(n))
        ds.assemble(theta, nug, eps, k)
        Ho = HLikelihood(P, leaf, 2.0)
        rng = np.random.default_rng(7)
        dense = [i for i, b in enumerate(BT.blocks) if b.kind == DENSE]
        lowr = [i for i, b in enumerate(BT.blocks) if b.kind == LOWRANK]
        sizes = np.array([rc[i, 2] * rc[i, 3] for i in lowr])
        largest = [lowr[j] for j in np.argsort(-sizes)[:2]]
        for i in rng.choice(dense, 10, replace=False):
            o = Ho.assemble_block(int(i), theta, nug, eps, k)
            g = ds.get_block(int(i), rc[i, 2], rc[i, 3])
            assert np.max(np.abs(g - o)) <= 1e-14 * np.max(np.abs(o)), i
        for i in list(rng.choice(lowr, 10, replace=False)) + largest:
            Uo, Vo = Ho.assemble_block(int(i), theta, nug, eps, k)
            Ud, Vd = ds.get_block(int(i), rc[i, 2], rc[i, 3])
            assert Ud.shape[1] == Uo.shape[1], i
            d, o = _sampled_diff(Ud, Vd, Uo, Vo, rng)
            assert d <= 1e-11 * o, (i, d / o)
    finally:
        ds.close()


def test_fullsize_fixed_rank_evaluation(H, ctx):
    name, gen, leaf, theta, nug, eps, k = FULL[1]
    P = gen()
    n = len(P)
    ds = H.Dataset(ctx, P, leaf, 2.0)
    try:
        ds.set_z(wl.standard_normal(n, 1, 22))
        r1 = ds.loglik(theta, nug, eps, k)
        r2 = ds.loglik(theta, nug, eps, k)
        for key in ("loglik", "logdet", "quadform", "status", "fail_block", "fail_pivot"):
            assert np.array_equal(r1[key], r2[key], equal_nan=key in ("loglik", "logdet", "quadform")), key
        if r1["status"][0] == H.HM_ERR_NOT_SPD:
            assert r1["fail_block"][0] >= 0 and r1["fail_pivot"][0] >= 0
            assert math.isnan(r1["loglik"][0])
        else:
            assert r1["status"][0] == 0
            assert r1["logdet"][0] <= n * math.log(theta[0] + nug)
            assert r1["quadform"][0] > 0 and math.isfinite(r1["loglik"][0])
    finally:
        ds.close()
