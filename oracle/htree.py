"""Cluster tree T_I and block cluster tree T_{IxI} for the oracle (Appendix B).

Cluster tree (Definition B.1).  The paper fixes only the defining properties:
the root is I, sons partition their father, leaves have at most n_min
indices.  It does not say how to split.  Reading used here (geometric
bisection):
  * a cluster with more than n_min indices is split;
  * take the tight axis-parallel bounding box of its points, split along the
    longest side (lowest axis on ties);
  * order the cluster's indices by (coordinate on that axis, original index),
    a total order, and give the first floor(|t|/2) to the first son;
  * the permutation of I is the left-to-right order of the leaves, so every
    cluster is a contiguous range of permuted positions.
Only comparisons are involved, so any correct implementation reproduces it
bit for bit.

Block cluster tree (Definition B.2) with the standard admissibility
condition Adm_eta (Definition B.3): for clusters tau, sigma with tight boxes
B_tau, B_sigma,
    min{diam(B_tau), diam(B_sigma)} <= eta * dist(B_tau, B_sigma),
evaluated on squares with a fixed operation order and no fused multiply-add:
    diam2 = dx*dx + dy*dy,  dist2 = sum over axes of gap^2,
    admissible  <=>  dist2 > 0  and  min(diam2_tau, diam2_sigma) <= (eta*eta)*dist2.
Boxes that touch (dist = 0) are never admissible.  Only the lower triangle
(tau.begin >= sigma.begin) is built, since the covariance is symmetric
(Remark 2.1).  Recursion from (I, I):
  * admissible, off-diagonal         -> low-rank leaf;
  * both clusters are leaves          -> dense leaf;
  * otherwise                         -> sons by the rule of Definition B.2
    (split only the non-leaf side, else both); sons in row-major order,
    upper-triangle sons of a diagonal block omitted.
Nodes are numbered in depth-first pre-order.

Parity pins (tests/test_oracle_tree.py): the leaves of T_I partition I and
are all <= n_min; the leaves of T_{IxI} partition the lower triangle of
I x I exactly once; every low-rank leaf satisfies Adm_eta and every
non-low-rank block fails it; dense leaves are leaf x leaf; boxes are tight.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Cluster:
    begin: int           # first permuted position
    end: int             # one past the last permuted position
    lo: np.ndarray       # tight box, shape (2,)
    hi: np.ndarray
    level: int
    sons: list = field(default_factory=list)   # indices into ClusterTree.clusters

    @property
    def size(self):
        return self.end - self.begin

    @property
    def is_leaf(self):
        return not self.sons


class ClusterTree:
    """Geometric bisection cluster tree over points P (n x 2)."""

    def __init__(self, P: np.ndarray, n_min: int):
        P = np.asarray(P, dtype=np.float64)
        self.P = P
        self.n_min = int(n_min)
        self.clusters: list[Cluster] = []
        self.perm = np.empty(len(P), dtype=np.int64)
        self._pos = 0
        self._build(np.arange(len(P), dtype=np.int64), 0)
        assert self._pos == len(P)

    def _build(self, idx: np.ndarray, level: int) -> int:
        pts = self.P[idx]
        lo = pts.min(axis=0)
        hi = pts.max(axis=0)
        cid = len(self.clusters)
        c = Cluster(begin=-1, end=-1, lo=lo, hi=hi, level=level)
        self.clusters.append(c)
        if len(idx) <= self.n_min:
            c.begin = self._pos
            self.perm[self._pos:self._pos + len(idx)] = idx
            self._pos += len(idx)
            c.end = self._pos
            return cid
        ext = hi - lo
        axis = int(np.argmax(ext))          # first maximum: lowest axis on ties
        # total order (coordinate, original index)
        order = np.lexsort((idx, pts[:, axis]))
        idx = idx[order]
        half = len(idx) // 2
        c.begin = self._pos
        s1 = self._build(idx[:half], level + 1)
        s2 = self._build(idx[half:], level + 1)
        c.end = self._pos
        c.sons = [s1, s2]
        return cid

    @property
    def root(self) -> int:
        return 0

    def leaves(self):
        return [i for i, c in enumerate(self.clusters) if c.is_leaf]


def diam2(c: Cluster) -> float:
    dx = c.hi[0] - c.lo[0]
    dy = c.hi[1] - c.lo[1]
    return dx * dx + dy * dy


def dist2(a: Cluster, b: Cluster) -> float:
    s = 0.0
    for ax in range(2):
        g = max(0.0, b.lo[ax] - a.hi[ax], a.lo[ax] - b.hi[ax])
        s = s + g * g
    return s


def admissible(a: Cluster, b: Cluster, eta: float) -> bool:
    d2 = dist2(a, b)
    return d2 > 0.0 and min(diam2(a), diam2(b)) <= (eta * eta) * d2


DENSE, LOWRANK, NODE = "dense", "lowrank", "node"


@dataclass
class Block:
    row: int            # cluster id (tau)
    col: int            # cluster id (sigma)
    kind: str           # DENSE, LOWRANK or NODE
    sons: list = field(default_factory=list)   # block ids, row-major order


class BlockTree:
    """Lower-triangular block cluster tree with standard admissibility."""

    def __init__(self, tree: ClusterTree, eta: float):
        self.tree = tree
        self.eta = float(eta)
        self.blocks: list[Block] = []
        self._build(tree.root, tree.root)

    def _build(self, t: int, s: int) -> int:
        T = self.tree.clusters
        bid = len(self.blocks)
        b = Block(row=t, col=s, kind=NODE)
        self.blocks.append(b)
        if t != s and admissible(T[t], T[s], self.eta):
            b.kind = LOWRANK
            return bid
        if T[t].is_leaf and T[s].is_leaf:
            b.kind = DENSE
            return bid
        rows = T[t].sons if not T[t].is_leaf else [t]
        cols = T[s].sons if not T[s].is_leaf else [s]
        sons = []
        for r in rows:
            for c in cols:
                if t == s and T[r].begin < T[c].begin:
                    continue        # upper triangle of a diagonal block
                sons.append(self._build(r, c))
        b.sons = sons
        return bid

    def leaves(self):
        return [i for i, b in enumerate(self.blocks) if b.kind != NODE]
