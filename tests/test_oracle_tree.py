"""Pins for the oracle's cluster tree and block cluster tree (Appendix B).

Checked against the defining properties of Definitions B.1-B.3 rather than
against the construction itself: leaves partition I with at most n_min
indices each; block leaves tile the lower triangle of I x I exactly once;
low-rank leaves satisfy Adm_eta (recomputed here by brute force from the
points, not from the stored boxes) and no other block does; dense leaves are
leaf x leaf; boxes are tight; each split halves the cluster along its longest
box side at the median.
"""
import numpy as np
import pytest

from oracle.htree import DENSE, LOWRANK, NODE, BlockTree, ClusterTree
from paper_1709_04419_amd import workloads as wl


def _points(kind, n, seed):
    return wl.make_points(kind, n, seed)


@pytest.mark.parametrize("kind,n,nmin", [("uniform", 2000, 32), ("basin", 3000, 64),
                                          ("uniform", 65, 32), ("grid", 1024, 32)])
def test_cluster_tree_properties(kind, n, nmin):
    P = _points(kind, n, 1)
    T = ClusterTree(P, nmin)
    assert sorted(T.perm.tolist()) == list(range(n))
    cover = np.zeros(n, dtype=int)
    for c in T.clusters:
        pts = P[T.perm[c.begin:c.end]]
        # tight boxes
        np.testing.assert_array_equal(c.lo, pts.min(axis=0))
        np.testing.assert_array_equal(c.hi, pts.max(axis=0))
        if c.is_leaf:
            assert 1 <= c.size <= nmin
            cover[c.begin:c.end] += 1
        else:
            assert c.size > nmin
            a, b = (T.clusters[s] for s in c.sons)
            assert a.begin == c.begin and a.end == b.begin and b.end == c.end
            assert a.size == c.size // 2
            ext = c.hi - c.lo
            ax = int(np.argmax(ext))
            # median split along the longest side: every left coordinate is <= every right one
            left = P[T.perm[a.begin:a.end], ax]
            right = P[T.perm[b.begin:b.end], ax]
            assert left.max() <= right.min()
    assert np.all(cover == 1)


def _brute_adm(P, T, t, s, eta):
    A = P[T.perm[T.clusters[t].begin:T.clusters[t].end]]
    B = P[T.perm[T.clusters[s].begin:T.clusters[s].end]]
    lo_a, hi_a = A.min(0), A.max(0)
    lo_b, hi_b = B.min(0), B.max(0)
    gap = np.maximum(0, np.maximum(lo_b - hi_a, lo_a - hi_b))
    dist = np.sqrt(np.sum(gap ** 2))
    diam = min(np.linalg.norm(hi_a - lo_a), np.linalg.norm(hi_b - lo_b))
    return dist > 0, diam, dist


@pytest.mark.parametrize("kind,n,nmin,eta", [("uniform", 2000, 32, 2.0), ("basin", 3000, 64, 2.0),
                                              ("uniform", 500, 16, 0.5), ("grid", 1024, 32, 2.0)])
def test_block_tree_properties(kind, n, nmin, eta):
    P = _points(kind, n, 2)
    T = ClusterTree(P, nmin)
    BT = BlockTree(T, eta)
    C = T.clusters
    cells = np.zeros((n, n), dtype=np.int32)
    for b in BT.blocks:
        t, s = C[b.row], C[b.col]
        assert t.begin >= s.begin
        if b.kind == NODE:
            assert b.sons
            pos, diam, dist = _brute_adm(P, T, b.row, b.col, eta)
            assert b.row == b.col or not (pos and diam <= eta * dist * (1 + 1e-12))
            continue
        cells[t.begin:t.end, s.begin:s.end] += 1
        if b.kind == DENSE:
            assert t.is_leaf and s.is_leaf
        else:
            assert b.row != b.col
            pos, diam, dist = _brute_adm(P, T, b.row, b.col, eta)
            assert pos and diam <= eta * dist * (1 + 1e-12)
    lower = np.tril(np.ones((n, n), dtype=bool))
    # leaves of the diagonal blocks cover their full square; off-diagonal ones the rest
    covered = cells > 0
    assert np.all(cells <= 1)
    assert np.all(covered[lower])
    assert not np.any(covered & ~lower & ~covered.T)


def test_no_admissible_blocks_when_eta_zero():
    P = _points("uniform", 400, 4)
    BT = BlockTree(ClusterTree(P, 16), 0.0)
    assert not any(b.kind == LOWRANK for b in BT.blocks)
