"""CPU oracle for the H-matrix Gaussian log-likelihood (Litvinenko, Sun, Genton,
Keyes, "Likelihood Approximation With Hierarchical Matrices For Large Spatial
Datasets", arXiv:1709.04419).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
anything in this package: only the test-suite, the smoke check and the
benchmark's CPU-baseline leg do.  The device path and this oracle share no
code; the only shared module is the seeded input generator
(`paper_1709_04419_amd.workloads`), which holds none of the method's
arithmetic.

Everything here is plain float64 numpy, written for readability rather than
speed:

  besselk   K_nu by the integral representation (trapezoidal rule)
  matern    the Matern covariance, eq. (2), plus the nugget (Section 2.4)
  dense     the exact Gaussian log-likelihood, eq. (1)
  htree     cluster tree and block cluster tree, Appendix B (Defs. B.1-B.3)
  lowrank   adaptive cross approximation and SVD truncation (Section 2.1,
            Remark 2.4, Definition 2.1)
  hchol     H-Cholesky, log-determinant, forward solve and eq. (4)

Parity status of each function is stated in its module header.
"""
