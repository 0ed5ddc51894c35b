"""GPU checks of the mixed-precision form (HM_MIXED, include/hmlik.h): low-rank
factors of C~ and L~ FP32-valued, their update products on FP32 matrix
instructions with FP32 accumulation, dense leaves / log-determinant /
recompressions in FP64, and C~^{-1} Z refined iteratively in FP64.

  * the refinement converges: the relative residual ||Z - C~ x|| / ||Z|| of
    every column reaches refine_tol (or the FP64 rounding floor of the
    residual, u ||C|| ||x|| / ||Z||, where that is larger) within
    refine_max_iter corrections;
  * the error against the FP64 oracle (the dense likelihood, eq. 1) respects
    Theorem 1 (Section 3.2) with eps_inv = ||I - (L~ L~^T)^{-1} C||_2 of the
    mixed factor, computed densely here;
  * log|C~| and L~ of the mixed form stay within stated relative distances
    of the FP64 form (measured values printed);
  * mixed results are bitwise repeatable.
"""
import math

import numpy as np
import pytest

from oracle.dense import covariance_matrix, dense_loglik
from oracle.hchol import HLikelihood
from paper_1709_04419_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    from paper_1709_04419_amd import hmlik
    return hmlik


@pytest.fixture(scope="module")
def ctx(H):
    c = H.Context(0)
    yield c
    c.close()


CASES = [("uniform", 2000, 32, (1.0, 0.1, 0.5), 1e-8), ("basin", 3000, 64, (1.0, 0.1, 0.325), 1e-7),
         ("uniform", 4000, 64, (1.0, 0.2, 1.0), 1e-7)]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}{c[1]}" for c in CASES])
def test_mixed_against_fp64_and_theorem1(H, ctx, case):
    cloud, n, leaf, theta, eps = case
    nug = 1e-6
    P = wl.basin_clusters(n, 500 + n) if cloud == "basin" else wl.uniform_square(n, 500 + n)
    C = covariance_matrix(P, theta, nug)
    # data drawn through the dense Cholesky factor (Section 4's simulation)
    Z = np.linalg.cholesky(C) @ wl.standard_normal(n, 1, 501 + n)
    ds = H.Dataset(ctx, P, leaf, 2.0)
    ds.set_z(Z)
    f = ds.loglik(theta, nug, eps)
    m = ds.loglik(theta, nug, eps, prec=H.HM_MIXED, refine_max_iter=20, refine_tol=1e-13)
    m2 = ds.loglik(theta, nug, eps, prec=H.HM_MIXED, refine_max_iter=20, refine_tol=1e-13)
    assert int(f["status"][0]) == 0 and int(m["status"][0]) == 0
    for k in ("loglik", "logdet", "quadform", "refine_quad", "refine_resid"):
        assert np.array_equal(m[k], m2[k])
    # the residual Z - C~ x is formed in FP64: below u ||C|| ||x|| / ||Z|| it is
    # rounding (a dense LAPACK solve of the smooth uniform4000 case leaves
    # 7.8e-13), so the target is refine_tol or that floor, whichever is larger
    x = np.linalg.solve(C, Z)
    floor = np.finfo(np.float64).eps * np.linalg.norm(C, 2) * np.linalg.norm(x) / np.linalg.norm(Z)
    assert m["refine_resid"][0] <= max(1e-13, floor) and 1 <= int(m["refine_iters"][0]) <= 20
    d_logdet = abs(m["logdet"][0] - f["logdet"][0]) / abs(f["logdet"][0])
    d_ll = abs(m["loglik"][0] - f["loglik"][0]) / abs(f["loglik"][0])
    d_quad = abs(m["refine_quad"][0] - f["quadform"][0]) / abs(f["quadform"][0])
    print(f"{cloud}{n}: mixed vs FP64: logdet {d_logdet:.2e}, refined quad {d_quad:.2e}, L {d_ll:.2e}; "
          f"iters {int(m['refine_iters'][0])}, resid {m['refine_resid'][0]:.1e}")
    assert d_logdet <= 1e-5 and d_ll <= 1e-5 and d_quad <= 1e-5
    if n > 2000:
        ds.close()
        return
    # Theorem 1 against the exact likelihood: the log-determinant comes from
    # L~ (eps_LL = ||I - (L~ L~^T)^{-1} C||), the refined quadratic form from
    # the assembled C~ (eps_q = ||I - C~^{-1} C||)
    def cols(op, M):
        return np.hstack([ds.apply(op, M[:, j:j + 64]) for j in range(0, M.shape[1], 64)])
    Ct = cols(H.HM_OP_C, np.eye(n))
    e_ll = np.linalg.norm(np.eye(n) - cols(H.HM_OP_SOLVE, C), 2)
    e_q = np.linalg.norm(np.eye(n) - np.linalg.solve(Ct, C), 2)
    dl, dlogdet, dquad = dense_loglik(P, Z, theta, nug)
    cinv = max(np.linalg.norm(np.linalg.inv(C), 2), np.linalg.norm(np.linalg.inv(Ct), 2))
    bound = 0.5 * n * (-math.log(1.0 - e_ll)) + 0.5 * float(Z[:, 0] @ Z[:, 0]) * cinv * e_q
    err = abs(float(m["loglik"][0]) - float(dl))
    print(f"{cloud}{n}: |L_mixed - L| = {err:.3e}, Theorem 1 bound {bound:.3e} (eps_LL {e_ll:.2e}, eps_q {e_q:.2e})")
    assert e_ll < 1 and e_q < 1 and err <= bound
    ds.close()
