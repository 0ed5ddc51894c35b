"""Accuracy diagnostics of the H-matrix approximation (Section 2.4, Tables 2-3).

For a dataset assembled and factored at theta (any Dataset.loglik call):

- the relative error of the log-determinant, |log|C~| - log|C|| / |log|C||;
- the Kullback-Leibler divergence between N(0, C) and N(0, C~),
  D_KL = 1/2 { tr(C~^{-1} C) - n + log|C~| - log|C| };
- ||I - (L~ L~^T)^{-1} C||_2 by power iteration (hm_inverse_accuracy);
- the storage of C~ and L~ (bytes at the actual ranks).

The H-side quantities (log|C~| and the columns of (L~ L~^T)^{-1} C, by the
library's forward and backward substitution) come from the library.  The
reference side needs the exact covariance: its entries come from the library
(hm_exact_block, eq. 2 plus the nugget), and log|C| from a dense Cholesky
factorisation of those entries by the vendor dense solver (torch.linalg on
the GPU) -- a reference value, as the dense matrix is exactly what the method
avoids forming.  n is limited by the n x n dense matrix (16,641 points, the
size of the paper's tables, take 2.2 GB).
"""
from __future__ import annotations

import math
from typing import Dict, Sequence

import numpy as np

from . import hmlik as H


def _quiet(msg: str) -> None:
    pass


def exact_logdet(ds, chunk: int = 4096, log=_quiet) -> float:
    """log|C| of the exact covariance at the dataset's last assembled theta."""
    import torch
    n = ds.n
    C = torch.empty((n, n), dtype=torch.float64, device=f"cuda:{ds.ctx.device}")
    for j0 in range(0, n, chunk):
        nj = min(chunk, n - j0)
        C[:, j0:j0 + nj] = ds.exact_block(0, n, j0, nj, device=True)
    log(f"diagnostics: exact covariance formed ({n} x {n}), dense Cholesky")
    L = torch.linalg.cholesky(C)
    del C
    v = float(2.0 * torch.sum(torch.log(torch.diagonal(L))).item())
    log(f"diagnostics: log|C| = {v:.10g}")
    return v


def trace_inv_exact(ds, chunk: int = 64, log=_quiet) -> float:
    """tr(C~^{-1} C) = tr((L~ L~^T)^{-1} C), column chunk by column chunk."""
    import torch
    n = ds.n
    tr = 0.0
    for j0 in range(0, n, chunk):
        nj = min(chunk, n - j0)
        Cj = ds.exact_block(0, n, j0, nj, device=True)          # C(:, j0:j0+nj)
        Y = ds.apply(H.HM_OP_SOLVE, Cj)                          # (L~ L~^T)^{-1} C(:, j0:j0+nj)
        tr += float(torch.sum(torch.diagonal(Y[j0:j0 + nj, :])).item())
        if (j0 // chunk) % 64 == 63:
            log(f"diagnostics: trace, {j0 + nj} of {n} columns")
    return tr


def accuracy(ds, theta, nugget: float, eps: float = 0.0, rank: int = 0, power_iters: int = 10,
             seed: int = 7, logdet_exact: float = None, log=_quiet) -> Dict[str, float]:
    """Evaluates the H-likelihood at theta (eps or rank), then the diagnostics
    of the module docstring.  logdet_exact may be passed in when several
    accuracies are compared at one theta (it does not depend on eps)."""
    res = ds.loglik(theta, nugget, eps, rank)
    if int(res["status"][0]) != 0:
        return dict(status=int(res["status"][0]), eps=eps, rank=rank)
    logdet_h = float(res["logdet"][0])
    if logdet_exact is None:
        logdet_exact = exact_logdet(ds, log=log)
    tr = trace_inv_exact(ds, log=log)
    n = ds.n
    kld = 0.5 * (tr - n + logdet_h - logdet_exact)
    x0 = np.random.default_rng(seed).standard_normal(n)
    inv_err = ds.inverse_accuracy(x0, power_iters)
    return dict(status=0, eps=eps, rank=rank, n=n, logdet_h=logdet_h, logdet_exact=logdet_exact,
                logdet_rel_err=abs(logdet_h - logdet_exact) / abs(logdet_exact), trace=tr, kld=kld,
                inv_err=inv_err, max_rank=int(res["max_rank"][0]), bytes_C=int(res["bytes_C"][0]),
                bytes_L=int(res["bytes_L"][0]))


def sweep(ds, theta, nugget: float, eps_list: Sequence[float] = (), ranks: Sequence[int] = (),
          power_iters: int = 10, log=_quiet) -> list:
    """Table 2 (accuracy eps) / Table 3 (fixed rank k) style sweep at one theta."""
    ds.loglik(theta, nugget, eps_list[0] if eps_list else 0.0, ranks[0] if ranks and not eps_list else 0)
    ld = exact_logdet(ds, log=log)
    rows = [accuracy(ds, theta, nugget, eps=e, power_iters=power_iters, logdet_exact=ld, log=log) for e in eps_list]
    rows += [accuracy(ds, theta, nugget, rank=k, power_iters=power_iters, logdet_exact=ld, log=log) for k in ranks]
    return rows
