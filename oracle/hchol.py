"""H-matrix log-likelihood for the oracle: assembly, H-Cholesky, forward solve,
log-determinant and eq. (4) of Section 3.1.

    L~(theta) = -n/2 log(2 pi) - sum_i log L~_ii - 1/2 v^T v,   L~ v = Z,

where L~ is the H-Cholesky factor of the H-matrix approximation C~ of the
Matern covariance (eq. (2)) plus nugget.  Section 3.2 states that the factor
keeps the block structure of C~ and that log|C~| = 2 sum log L~_ii comes for
free; the paper does not print an H-Cholesky algorithm (it uses a closed
library).  The reading implemented here is the standard recursive formatted
Cholesky with deferred updates:

  HCHOL(tau):   leaf  -> FLUSH(tau,tau); dense Cholesky (pivot <= 0: not SPD)
                else  -> HCHOL(tau1); HTRSM((tau2,tau1), L_{tau1 tau1});
                         UPDATE((tau2,tau2), L_{tau2 tau1}, L_{tau2 tau1}); HCHOL(tau2)

  HTRSM(b=(rho,sigma)) solves X L_{sigma sigma}^T = A_b:
                dense   -> FLUSH(b); dense triangular solve
                lowrank -> FLUSH(b); V <- L_{sigma sigma}^{-1} V (exact H forward solve)
                node    -> per row son rho_i (in order):
                           X_i1 = HTRSM(b_i1); UPDATE(b_i2, X_i1, L_{sigma2 sigma1});
                           X_i2 = HTRSM(b_i2)
                           (only a row split if sigma is a leaf)

  UPDATE(c=(tau,sigma), A=(tau,rho), B=(sigma,rho)) records c -= A B^T:
                A low-rank U V^T   -> term (X, Y) = (U_A, B V_A)
                else B low-rank    -> term (X, Y) = (A V_B, U_B)
                both dense         -> term (X, Y) = (A, B)
                else               -> recurse over sons: tau' outer, sigma' middle,
                                      rho' inner; a diagonal target keeps tau' >= sigma'.
  A term aimed at a non-leaf block is split, by rows and columns, onto the
  leaves under it; a term aimed inside a leaf is zero-padded to the leaf.
  Every leaf keeps its terms in the order they were recorded.

  FLUSH(b) applies b's terms in order:
                dense   -> D -= X Y^T per term
                lowrank, both clusters of at most DENSE_FLUSH * n_min points
                        -> the updated block U V^T - sum X Y^T is formed exactly
                           and replaced by its best approximation at accuracy eps
                           (or rank k): one truncated SVD (lowrank.truncate_dense)
                lowrank, otherwise
                        -> the product [U, -X_1, ...][V, Y_1, ...]^T is truncated
                           (lowrank.truncate); the accumulation is truncated early
                           whenever its rank would exceed R_ACC.
  Every truncation reports whether the K_MAX rank cap bound (Stats.capped and
  the result's rank_capped count).

The forward solve uses the same recursion (dense triangular solves at the
diagonal leaves, z2 -= L21 v1 through the blocks of L21).  log|C~| sums the
diagonal leaves in permuted order.

Parity pins (tests/test_oracle_hchol.py): with no admissible blocks (eta = 0)
the method is an exact blocked Cholesky and must equal the dense oracle to
rounding (a full-rank block is represented exactly, Section 1); at tiny
eps it converges to the dense value; Theorem 1's bound holds against the
dense oracle at several eps; ||C~ - L~ L~^T|| / ||C~|| = O(eps).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg
from scipy.linalg import lapack

from .htree import DENSE, LOWRANK, NODE, BlockTree, ClusterTree
from .lowrank import K_MAX, aca, truncate, truncate_dense
from .matern import covariance_block

# The paper fixes what a flush must produce (the formatted sum, truncated to
# accuracy eps or rank k: Section 2.1, Remark 2.4) but not when the truncations
# happen; the two constants below are that choice.  Both only decide how often
# the sum is re-truncated, so every setting approximates the same matrix within
# the method's error (tests/test_oracle_hchol.py checks Theorem 1 for other
# settings too).
#
# Largest rank an accumulation of updates may reach before it is truncated: the
# same cap as a single block (K_MAX), so an accumulation never holds more than
# two blocks' worth of columns.
R_ACC = 64
# A low-rank block whose row and column clusters both hold at most
# DENSE_FLUSH * n_min points takes its pending updates on the explicit matrix
# (it is no larger than a 4 x 4 array of dense leaves) and is truncated once:
# the best approximation of the exact sum (Remark 2.4's truncation applied to
# the formatted sum as a whole).  Such a block receives terms of rank up to
# n_min (products of dense leaves), for which the factored form would hold more
# columns than the block has rows.
DENSE_FLUSH = 4


class NotSPD(Exception):
    def __init__(self, block, pivot):
        super().__init__(f"non-positive pivot {pivot} in block {block}")
        self.block = block
        self.pivot = pivot


@dataclass
class Stats:
    """Counters of one evaluation.  explicit_flushes / factored_flushes /
    early_truncations count the branches of FLUSH taken for low-rank leaves;
    capped collects, per truncation and ACA, whether the K_MAX cap bound in the
    accuracy mode (any True means some block misses eps)."""
    aca_ranks: list = field(default_factory=list)
    explicit_flushes: int = 0
    factored_flushes: int = 0
    early_truncations: int = 0
    capped: list = field(default_factory=list)
    flush_ranks: list = field(default_factory=list)     # accumulated rank per LR flush
    flush_terms: list = field(default_factory=list)
    final_ranks: list = field(default_factory=list)
    n_terms: int = 0
    term_kinds: dict = field(default_factory=lambda: {"lrA": 0, "lrB": 0, "dd": 0})


class HLikelihood:
    """One H-matrix log-likelihood evaluation on CPU, float64 throughout."""

    def __init__(self, P, n_min=32, eta=2.0, r_acc=R_ACC, dense_flush=DENSE_FLUSH):
        self.r_acc = int(r_acc)
        self.dense_flush = int(dense_flush)
        self.P = np.asarray(P, dtype=np.float64)
        self.n = len(self.P)
        self.n_min = n_min
        self.tree = ClusterTree(self.P, n_min)
        self.bt = BlockTree(self.tree, eta)
        self.perm = self.tree.perm
        self.Pp = self.P[self.perm]
        C = self.tree.clusters
        B = self.bt.blocks
        # (row cluster, col cluster) -> block id
        self.bid = {(b.row, b.col): i for i, b in enumerate(B)}
        self.rng_r = [(C[b.row].begin, C[b.row].end) for b in B]
        self.rng_c = [(C[b.col].begin, C[b.col].end) for b in B]

    # ------------------------------------------------------------ assembly
    def assemble(self, theta, nugget, eps, kfix):
        """Dense leaves entry by entry; low-rank leaves by ACA + TRUNCATE."""
        self.theta, self.nugget, self.eps, self.kfix = theta, nugget, eps, kfix
        self.stats = Stats()
        self.D, self.U, self.V = {}, {}, {}
        self.pending = {}
        for i, b in enumerate(self.bt.blocks):
            if b.kind == NODE:
                continue
            self.pending[i] = []
            if b.kind == DENSE:
                self.D[i] = self.assemble_block(i, theta, nugget, eps, kfix)
            else:
                self.U[i], self.V[i] = self.assemble_block(i, theta, nugget, eps, kfix)

    def assemble_block(self, i, theta, nugget, eps, kfix):
        """One leaf of C~: the dense block (entries of eq. 2 plus the nugget on
        the diagonal), or (U, V) of a low-rank block by ACA + TRUNCATE."""
        b = self.bt.blocks[i]
        r0, r1 = self.rng_r[i]
        c0, c1 = self.rng_c[i]
        rows = np.arange(r0, r1)
        cols = np.arange(c0, c1)
        Pp = self.Pp
        if b.kind == DENSE:
            return covariance_block(Pp, rows, cols, theta, nugget)
        row_fn = lambda li: covariance_block(Pp, rows[li:li + 1], cols, theta, 0.0)[0]
        col_fn = lambda lj: covariance_block(Pp, rows, cols[lj:lj + 1], theta, 0.0)[:, 0]
        st = getattr(self, "stats", None)
        capped = st.capped if st is not None else None
        U, V = aca(row_fn, col_fn, r1 - r0, c1 - c0, eps, kfix if kfix > 0 else K_MAX, capped)
        if st is not None:
            st.aca_ranks.append(U.shape[1])
        return truncate(U, V, eps, kfix, capped)

    def to_dense(self):
        """Explicit matrix of the current H representation (lower blocks
        mirrored), for checks only."""
        M = np.zeros((self.n, self.n))
        for i, b in enumerate(self.bt.blocks):
            if b.kind == NODE:
                continue
            r0, r1 = self.rng_r[i]
            c0, c1 = self.rng_c[i]
            blk = self.D[i] if b.kind == DENSE else self.U[i] @ self.V[i].T
            M[r0:r1, c0:c1] = blk
            if b.row != b.col:
                M[c0:c1, r0:r1] = blk.T
        return M

    def factor_to_dense(self):
        M = np.zeros((self.n, self.n))
        for i, b in enumerate(self.bt.blocks):
            if b.kind == NODE:
                continue
            r0, r1 = self.rng_r[i]
            c0, c1 = self.rng_c[i]
            M[r0:r1, c0:c1] = self.D[i] if b.kind == DENSE else self.U[i] @ self.V[i].T
        return M

    # ------------------------------------------------------------ helpers
    def _diag(self, c):
        return self.bid[(c, c)]

    def _son(self, bid, r, c):
        return self.bid[(r, c)]

    def hmatvec(self, bid, W):
        """Y = L_b W for a block b of the factor (any kind)."""
        b = self.bt.blocks[bid]
        if b.kind == DENSE:
            return self.D[bid] @ W
        if b.kind == LOWRANK:
            return self.U[bid] @ (self.V[bid].T @ W)
        r0 = self.rng_r[bid][0]
        c0 = self.rng_c[bid][0]
        Y = np.zeros((self.rng_r[bid][1] - r0, W.shape[1]))
        for s in b.sons:
            sr0, sr1 = self.rng_r[s]
            sc0, sc1 = self.rng_c[s]
            Y[sr0 - r0:sr1 - r0] += self.hmatvec(s, W[sc0 - c0:sc1 - c0])
        return Y

    def push(self, bid, R0, C0, X, Y):
        """Record X Y^T as a pending subtraction on the region whose top-left
        global position is (R0, C0), starting at block bid."""
        b = self.bt.blocks[bid]
        if b.kind != NODE:
            r0 = self.rng_r[bid][0]
            c0 = self.rng_c[bid][0]
            self.pending[bid].append((R0 - r0, C0 - c0, X, Y))
            return
        # a non-leaf target always covers the whole block: split onto sons
        for s in b.sons:
            sr0, sr1 = self.rng_r[s]
            sc0, sc1 = self.rng_c[s]
            self.push(s, sr0, sc0, X[sr0 - R0:sr1 - R0], Y[sc0 - C0:sc1 - C0])

    def _target(self, tgt, t, s):
        """Sub-target for clusters (t, s) inside target tgt = (bid, R0, C0)."""
        bid = tgt[0]
        C = self.tree.clusters
        if self.bt.blocks[bid].kind == NODE:
            bid = self._son(bid, t, s)
        return (bid, C[t].begin, C[s].begin)

    # ------------------------------------------------------------ arithmetic
    def update(self, tgt, A, B):
        """tgt -= L_A L_B^T (recorded as terms), A = (tau, rho), B = (sigma, rho)."""
        blocks = self.bt.blocks
        ka, kb = blocks[A].kind, blocks[B].kind
        if ka == LOWRANK:
            X, Y = self.U[A], self.hmatvec(B, self.V[A])
            self.stats.term_kinds["lrA"] += 1
        elif kb == LOWRANK:
            X, Y = self.hmatvec(A, self.V[B]), self.U[B]
            self.stats.term_kinds["lrB"] += 1
        elif ka == DENSE and kb == DENSE:
            X, Y = self.D[A], self.D[B]
            self.stats.term_kinds["dd"] += 1
        else:
            C = self.tree.clusters
            tau, rho = blocks[A].row, blocks[A].col
            sig = blocks[B].row
            tsons = C[tau].sons if (ka == NODE and not C[tau].is_leaf) else [tau]
            ssons = C[sig].sons if (kb == NODE and not C[sig].is_leaf) else [sig]
            rsons = C[rho].sons if not C[rho].is_leaf else [rho]
            diag = tau == sig
            for t in tsons:
                for s in ssons:
                    if diag and C[t].begin < C[s].begin:
                        continue
                    sub = self._target(tgt, t, s)
                    for r in rsons:
                        a = A if ka != NODE else self._son(A, t, r)
                        b = B if kb != NODE else self._son(B, s, r)
                        self.update(sub, a, b)
            return
        self.stats.n_terms += 1
        self.push(tgt[0], tgt[1], tgt[2], X, Y)

    def flush(self, bid):
        terms = self.pending[bid]
        self.pending[bid] = []
        if not terms:
            return
        kind = self.bt.blocks[bid].kind
        if kind == DENSE:
            D = self.D[bid]
            for (r0, c0, X, Y) in terms:
                D[r0:r0 + X.shape[0], c0:c0 + Y.shape[0]] -= X @ Y.T
            return
        m = self.rng_r[bid][1] - self.rng_r[bid][0]
        n = self.rng_c[bid][1] - self.rng_c[bid][0]
        C = self.tree.clusters
        b = self.bt.blocks[bid]
        st = self.stats
        if max(m, n) <= self.dense_flush * self.n_min:
            D = self.U[bid] @ self.V[bid].T
            for (r0, c0, X, Y) in terms:
                D[r0:r0 + X.shape[0], c0:c0 + Y.shape[0]] -= X @ Y.T
            st.flush_terms.append(len(terms))
            st.explicit_flushes += 1
            self.U[bid], self.V[bid] = truncate_dense(D, self.eps, self.kfix, st.capped)
            return
        st.factored_flushes += 1
        Xs, Ys = [self.U[bid]], [self.V[bid]]
        rank = self.U[bid].shape[1]
        peak = rank
        for (r0, c0, X, Y) in terms:
            r = X.shape[1]
            if rank > 0 and rank + r > self.r_acc:
                st.early_truncations += 1
                U, V = truncate(np.hstack(Xs), np.hstack(Ys), self.eps, self.kfix, st.capped)
                Xs, Ys, rank = [U], [V], U.shape[1]
            Xp = np.zeros((m, r))
            Yp = np.zeros((n, r))
            Xp[r0:r0 + X.shape[0]] = -X
            Yp[c0:c0 + Y.shape[0]] = Y
            Xs.append(Xp)
            Ys.append(Yp)
            rank += r
            peak = max(peak, rank)
        st.flush_ranks.append(peak)
        st.flush_terms.append(len(terms))
        self.U[bid], self.V[bid] = truncate(np.hstack(Xs), np.hstack(Ys), self.eps, self.kfix, st.capped)

    def potrf(self, bid):
        L, info = lapack.dpotrf(self.D[bid], lower=1, clean=1)
        if info != 0:
            raise NotSPD(bid, info - 1)
        self.D[bid] = L

    def hsolve(self, c, W):
        """W <- L_{cc}^{-1} W in place (H forward substitution)."""
        C = self.tree.clusters
        d = self._diag(c)
        if C[c].is_leaf:
            W[:] = scipy.linalg.solve_triangular(self.D[d], W, lower=True)
            return
        c1, c2 = C[c].sons
        o = C[c].begin
        s1 = slice(C[c1].begin - o, C[c1].end - o)
        s2 = slice(C[c2].begin - o, C[c2].end - o)
        self.hsolve(c1, W[s1])
        W[s2] -= self.hmatvec(self._son(d, c2, c1), W[s1])
        self.hsolve(c2, W[s2])

    def htrsm(self, bid):
        """Solve X L_{sigma sigma}^T = A_b for block b = (rho, sigma)."""
        C = self.tree.clusters
        b = self.bt.blocks[bid]
        sig = b.col
        if b.kind == DENSE:
            self.flush(bid)
            Ls = self.D[self._diag(sig)]
            self.D[bid] = scipy.linalg.solve_triangular(Ls, self.D[bid].T, lower=True).T
            return
        if b.kind == LOWRANK:
            self.flush(bid)
            self.hsolve(sig, self.V[bid])
            return
        rho = b.row
        rows = C[rho].sons if not C[rho].is_leaf else [rho]
        if C[sig].is_leaf:
            for r in rows:
                self.htrsm(self._son(bid, r, sig))
            return
        s1, s2 = C[sig].sons
        L21 = self._son(self._diag(sig), s2, s1)
        for r in rows:
            b1 = self._son(bid, r, s1)
            b2 = self._son(bid, r, s2)
            self.htrsm(b1)
            self.update((b2, C[r].begin, C[s2].begin), b1, L21)
            self.htrsm(b2)

    def hchol(self, c):
        C = self.tree.clusters
        d = self._diag(c)
        if C[c].is_leaf:
            self.flush(d)
            self.potrf(d)
            return
        c1, c2 = C[c].sons
        self.hchol(c1)
        b21 = self._son(d, c2, c1)
        self.htrsm(b21)
        self.update((self._diag(c2), C[c2].begin, C[c2].begin), b21, b21)
        self.hchol(c2)

    # ------------------------------------------------------------ outputs
    def factor(self):
        self.hchol(self.tree.root)
        self.stats.final_ranks = [self.U[i].shape[1] for i in self.U]

    def logdet(self):
        s = 0.0
        for c in self.tree.leaves():
            s += np.sum(np.log(np.diag(self.D[self._diag(c)])))
        return 2.0 * s

    def solve(self, Z):
        Z = np.asarray(Z, dtype=np.float64)
        if Z.ndim == 1:
            Z = Z[:, None]
        W = Z[self.perm].copy()
        self.hsolve(self.tree.root, W)
        return W

    def loglik(self, theta, nugget, Z, eps=0.0, kfix=0):
        """Eq. (4).  Returns dict(loglik, logdet, quadform, status, ...)."""
        self.assemble(theta, nugget, eps, kfix)
        Z = np.asarray(Z, dtype=np.float64)
        r = 1 if Z.ndim == 1 else Z.shape[1]
        try:
            self.factor()
        except NotSPD as e:
            nan = np.full(r, np.nan)
            return dict(loglik=nan, logdet=nan, quadform=nan, status="not_spd",
                        fail_block=e.block, fail_pivot=e.pivot, rank_capped=int(sum(self.stats.capped)))
        logdet = self.logdet()
        v = self.solve(Z)
        quad = np.sum(v * v, axis=0)
        ll = -0.5 * self.n * math.log(2.0 * math.pi) - 0.5 * logdet - 0.5 * quad
        return dict(loglik=ll, logdet=np.full(r, logdet), quadform=quad, status="ok",
                    fail_block=-1, fail_pivot=-1, rank_capped=int(sum(self.stats.capped)),
                    max_rank=max((u.shape[1] for u in self.U.values()), default=0))


def h_loglik(P, Z, theta, nugget, n_min=32, eta=2.0, eps=0.0, kfix=0, **kw):
    """Convenience wrapper: one evaluation of eq. (4) on the CPU."""
    H = HLikelihood(P, n_min, eta, **kw)
    return H.loglik(theta, nugget, Z, eps, kfix)
