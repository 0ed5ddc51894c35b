"""Low-rank approximation of admissible blocks for the oracle.

Section 2.1 names adaptive cross approximation (ACA) as the method that fills
admissible blocks in O(k n), and Remark 2.4 / Definition 2.1 define the two
accuracy strategies: a fixed maximal rank k, or a per-block relative accuracy
eps in the spectral norm.  The paper does not spell out the ACA variant.
Reading used here: ACA with partial pivoting (Bebendorf 2000), first pivot
row 0, stopping on the Frobenius-norm estimate, followed by an SVD
recompression:

  ACA  residual row r = M(i*,:) - sum_l U[i*,l] V[:,l];  j* = argmax |r|
       (lowest index on ties); if r[j*] == 0 move to the lowest unused row;
       v = r / r[j*];  u = M(:,j*) - sum_l V[j*,l] U[:,l];
       S2 += 2 sum_l (u_l.u)(v_l.v) + |u|^2 |v|^2;
       stop when |u| |v| <= eps sqrt(S2), or k = min(m, n), or k = k_max;
       next row i* = argmax over unused rows of |u_i| (lowest index on ties).

  TRUNCATE(X, Y) for the product X Y^T (m x r, n x r):
       Householder QR  X = Qx Rx,  Y = Qy Ry;  SVD  Rx Ry^T = W S Z^T;
       keep k' = #{s_i > eps s_1}   (relative spectral accuracy, Remark 2.4), or
            k' = min(k, #{s_i > 0}) in the fixed-rank mode (Definition 2.1);
       k' is also capped by K_MAX.  In the accuracy mode a binding cap means the
       block misses the requested accuracy; this is never silent: the caller
       passes a list `capped` and every truncation (and every ACA that stops at
       the cap before its accuracy test is met) appends whether the cap bound.
       U = Qx W[:, :k'] S[:k'],  V = Qy Z[:, :k'].

  TRUNCATE_DENSE(D) for an explicit (small) block: the same rank rule applied
       to the SVD D = W S Z^T;  U = W[:, :k'] S[:k'],  V = Z[:, :k'].

The same eps is used for assembly and for the truncations inside the
H-Cholesky (Tables 6 and 7 quote a single eps for both).

Parity pins (tests/test_oracle_lowrank.py): ACA recovers separable rank-r
matrices exactly in r steps; TRUNCATE matches the rank count and the
Eckart-Young error of numpy's SVD of the explicit product on small blocks;
the fixed-rank mode keeps at most k terms.
"""
from __future__ import annotations

import numpy as np

# Largest rank any low-rank block may carry (assembly, truncation, accumulation
# of updates).  The paper bounds ranks only through eps (Remark 2.4) or k
# (Definition 2.1); a finite cap is an implementation limit of storage.  64 is
# the leaf size n_min of the benchmark workloads, so a block at the cap is as
# expensive as a dense leaf row; the largest rank measured in the benchmark
# configurations is about half of it.  When the cap binds in the accuracy mode
# it is reported (see `capped` below), never applied silently.
K_MAX = 64


def aca(row_fn, col_fn, m: int, n: int, eps: float, kmax: int, capped=None):
    """Partial-pivoting ACA of an implicitly given m x n block.

    row_fn(i) -> M[i, :] (length n);  col_fn(j) -> M[:, j] (length m).
    Returns U (m x k), V (n x k) with M ~ U V^T.  If `capped` is a list, it
    receives True when the iteration stopped at kmax < min(m, n) with its
    accuracy test (eps > 0) not met, else False.
    """
    cap_binds = kmax < min(m, n)
    kmax = min(kmax, m, n)
    converged = False
    Us, Vs = [], []
    used = np.zeros(m, dtype=bool)
    i = 0
    S2 = 0.0
    while len(Us) < kmax:
        r = np.array(row_fn(i), dtype=np.float64)
        for l in range(len(Us)):
            r -= Us[l][i] * Vs[l]
        used[i] = True
        j = int(np.argmax(np.abs(r)))
        if r[j] == 0.0:
            if used.all():
                converged = True
                break
            i = int(np.argmin(used))     # lowest unused row
            continue
        v = r / r[j]
        u = np.array(col_fn(j), dtype=np.float64)
        for l in range(len(Us)):
            u -= Vs[l][j] * Us[l]
        cross = 0.0
        for l in range(len(Us)):
            cross += (Us[l] @ u) * (Vs[l] @ v)
        nu2 = u @ u
        nv2 = v @ v
        S2 = S2 + 2.0 * cross + nu2 * nv2
        Us.append(u)
        Vs.append(v)
        if np.sqrt(nu2) * np.sqrt(nv2) <= eps * np.sqrt(S2):
            converged = True
            break
        if used.all():
            converged = True
            break
        cand = np.where(used, -1.0, np.abs(u))
        i = int(np.argmax(cand))
    if capped is not None:
        capped.append(bool(eps > 0 and cap_binds and len(Us) == kmax and not converged))
    if not Us:
        return np.zeros((m, 0)), np.zeros((n, 0))
    return np.stack(Us, axis=1), np.stack(Vs, axis=1)


def _keep(s, eps, kfix, capped=None):
    """Rank kept from singular values s (descending); `capped` (a list, or
    None) receives whether the K_MAX cap lowered it in the accuracy mode."""
    k = 0
    if s.size and s[0] != 0.0:
        if kfix > 0:
            k = min(kfix, int(np.count_nonzero(s > 0.0)))
        else:
            k = int(np.count_nonzero(s > eps * s[0]))
    if capped is not None:
        capped.append(bool(kfix <= 0 and k > K_MAX))
    return min(k, K_MAX)


def truncate_dense(D: np.ndarray, eps: float, kfix: int, capped=None):
    """Best approximation of an explicit block D at relative accuracy eps
    (kfix == 0) or rank kfix, capped at K_MAX.  Returns (U, V)."""
    m, n = D.shape
    W, s, Zt = np.linalg.svd(D)
    k = _keep(s, eps, kfix, capped)
    return W[:, :k] * s[:k], Zt[:k, :].T.copy()


def truncate(X: np.ndarray, Y: np.ndarray, eps: float, kfix: int, capped=None):
    """Best approximation of X Y^T at relative accuracy eps (kfix == 0) or
    rank kfix (kfix > 0), capped at K_MAX.  Returns (U, V)."""
    m, r = X.shape
    n = Y.shape[0]
    if r == 0:
        if capped is not None:
            capped.append(False)
        return np.zeros((m, 0)), np.zeros((n, 0))
    Qx, Rx = np.linalg.qr(X, mode="reduced")
    Qy, Ry = np.linalg.qr(Y, mode="reduced")
    W, s, Zt = np.linalg.svd(Rx @ Ry.T)
    k = _keep(s, eps, kfix, capped)
    if k == 0:
        return np.zeros((m, 0)), np.zeros((n, 0))
    U = Qx @ (W[:, :k] * s[:k])
    V = Qy @ Zt[:k, :].T
    return U, V
