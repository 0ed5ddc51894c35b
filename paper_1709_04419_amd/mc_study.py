"""Monte-Carlo study of the maximum-likelihood estimates (Section 4, Fig. 3).

One set of locations; R replicates Z_j = L~(theta*, 1e-10) W_j with W_j
standard normal, simulated on the device (hm_simulate, Section 4); for each
replicate theta-hat by the Nelder-Mead driver (mle.py) over the H-likelihood
of eq. (4) at accuracy eps, in FP64 (all replicates advanced together through
a request server) and, optionally, in the mixed-precision form (one replicate
after another: the server runs FP64 only).  Reported per precision: the
quartiles of nu-hat, ell-hat, sigma2-hat and of sigma2-hat / ell-hat^(2 nu-hat)
(the combination Fig. 3 shows alongside the three parameters), and per
replicate the FP64-versus-mixed differences of the four quantities.

Every likelihood evaluation runs in the library's kernels; this module only
draws the seeded inputs and steers the searches.
"""
from __future__ import annotations

import math
import time
from typing import Dict, List, Sequence

import numpy as np

from . import hmlik as H
from . import mle
from . import workloads as wl

QUANTITIES = ("nu", "ell", "sigma2", "sigma2/ell^(2nu)")


def _quantities(theta) -> Dict[str, float]:
    s2, ell, nu = theta
    return {"nu": nu, "ell": ell, "sigma2": s2, "sigma2/ell^(2nu)": s2 / ell ** (2.0 * nu)}


def _quartiles(vals: Sequence[float]) -> Dict[str, float]:
    v = np.asarray(vals, dtype=np.float64)
    q = np.quantile(v, [0.0, 0.25, 0.5, 0.75, 1.0])
    return dict(min=float(q[0]), q1=float(q[1]), median=float(q[2]), q3=float(q[3]), max=float(q[4]),
                mean=float(v.mean()), std=float(v.std(ddof=1)) if v.size > 1 else 0.0)


def simulate_replicates(ctx, points, replicates: int, theta_true, nugget: float, seed: int,
                        leaf_size: int = 64, eta: float = 2.0, sim_eps: float = 1e-10) -> np.ndarray:
    """Z (n x replicates) = L~(theta*, sim_eps) W, W seeded standard normal."""
    ds = H.Dataset(ctx, points, leaf_size, eta)
    try:
        W = wl.standard_normal(points.shape[0], replicates, seed)
        return ds.simulate(theta_true, nugget, W, eps=sim_eps)
    finally:
        ds.close()


class _Progress:
    """A Dataset seen through its loglik calls, reporting every `every` calls
    (a search of hundreds of evaluations prints while it runs)."""

    def __init__(self, ds, label: str, log, every: int = 25):
        self._ds, self._label, self._log, self._every = ds, label, log, every
        self.calls = self.breakdowns = 0

    def loglik(self, *a, **k):
        r = self._ds.loglik(*a, **k)
        self.calls += 1
        if int(r["status"][0]) != 0:
            self.breakdowns += 1
        if self.calls % self._every == 0:
            self._log(f"{self._label}: {self.calls} evaluations, {self.breakdowns} not SPD")
        return r


def run(ctx, n: int, replicates: int, theta_true=(1.0, 0.7, 0.9), nugget: float = 1e-6,
        eps: float = 1e-7, theta0=None, points: str = "uniform", seed: int = 101, leaf_size: int = 64,
        eta: float = 2.0, mixed: bool = True, mixed_replicates: int = 0, slots: int = 16,
        max_evals: int = 300, ftol: float = 1e-9, xtol: float = 1e-4, step: float = 0.1,
        refine_max_iter: int = 10, refine_tol: float = 1e-12, log=print) -> dict:
    """Runs the study; returns a dict with the per-replicate estimates, their
    quartiles per precision and the FP64-vs-mixed differences.  theta = (sigma2,
    ell, nu); theta_true defaults to the study's (ell, nu, sigma) = (0.7, 0.9, 1.0).
    mixed_replicates > 0 limits the mixed-precision fits to the first replicates."""
    P = wl.make_points(points, n, seed)
    t0 = time.perf_counter()
    Z = simulate_replicates(ctx, P, replicates, theta_true, nugget, seed + 1, leaf_size, eta)
    t_sim = time.perf_counter() - t0
    log(f"mc: n={n}: {replicates} replicates simulated on the device in {t_sim:.2f} s")
    th0 = tuple(theta0) if theta0 is not None else tuple(1.3 * np.asarray(theta_true))
    kw = dict(step=step, ftol=ftol, xtol=xtol, max_evals=max_evals)
    dss: List = []
    try:
        for j in range(replicates):
            ds = H.Dataset(ctx, P, leaf_size, eta)
            dss.append(ds)
            ds.set_z(Z[:, j])
        t0 = time.perf_counter()
        with H.Server(ctx, max_active=min(slots, replicates)) as sv:
            fp64 = mle.fit_many(sv, dss, [th0] * replicates, nugget, eps=eps, log=log, **kw)
        t_fp64 = time.perf_counter() - t0
        log(f"mc: FP64 fits of {replicates} replicates in {t_fp64:.1f} s "
            f"({sum(r['evals'] for r in fp64)} evaluations)")
        mix = []
        t_mixed = 0.0
        if mixed:
            nm = replicates if mixed_replicates <= 0 else min(mixed_replicates, replicates)
            lk = dict(prec=H.HM_MIXED, refine_max_iter=refine_max_iter, refine_tol=refine_tol)
            t0 = time.perf_counter()
            for j in range(nm):
                pr = _Progress(dss[j], f"mc: mixed fit {j + 1}/{nm}", log)
                mix.append(mle.fit(pr, th0, nugget, eps=eps, loglik_kw=lk, **kw))
                mix[-1]["breakdowns"] = pr.breakdowns
                log(f"mc: mixed fit {j + 1}/{nm}: theta {tuple(round(v, 5) for v in mix[-1]['theta'])}")
            t_mixed = time.perf_counter() - t0
    finally:
        for ds in dss:
            ds.close()
    out = dict(n=n, replicates=replicates, theta_true=tuple(theta_true), nugget=nugget, eps=eps,
               points=points, seed=seed, theta0=th0, seconds=dict(simulate=t_sim, fp64=t_fp64, mixed=t_mixed),
               fp64=[dict(theta=r["theta"], loglik=r["loglik"], evals=r["evals"], converged=r["converged"])
                     for r in fp64],
               mixed=[dict(theta=r["theta"], loglik=r["loglik"], evals=r["evals"], converged=r["converged"],
                           breakdowns=r["breakdowns"]) for r in mix])
    # mixed searches that never left a breakdown (every evaluation not SPD) have
    # no estimate; the FP64-vs-mixed comparison is over the others
    mix_ok = [(a, b) for a, b in zip(fp64, mix) if math.isfinite(b["loglik"])]
    out["mixed_without_estimate"] = len(mix) - len(mix_ok)
    mix = [b for _, b in mix_ok]
    fp64_paired = [a for a, _ in mix_ok]
    out["summary"] = {}
    for name, fits in (("fp64", fp64), ("mixed", mix)):
        if fits:
            qs = [_quantities(r["theta"]) for r in fits]
            out["summary"][name] = {q: _quartiles([x[q] for x in qs]) for q in QUANTITIES}
    if mix:
        diffs = {q: [] for q in QUANTITIES}
        for a, b in zip(fp64_paired, mix):
            qa, qb = _quantities(a["theta"]), _quantities(b["theta"])
            for q in QUANTITIES:
                diffs[q].append(abs(qb[q] - qa[q]) / abs(qa[q]))
        out["fp64_vs_mixed_rel"] = {q: dict(max=float(np.max(v)), median=float(np.median(v)))
                                    for q, v in diffs.items()}
    return out
