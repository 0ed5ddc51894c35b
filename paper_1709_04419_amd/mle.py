"""Maximum-likelihood estimation of theta = (sigma^2, ell, nu) on top of the
H-matrix likelihood of eq. (4) (Section 3.1).

The paper maximises L~(theta) with the derivative-free Brent-Dekker method
(Section 3.1), a one-dimensional search.  For the three Matern parameters
together this module uses the Nelder-Mead simplex search (Nelder and Mead,
Computer Journal 7, 1965), also derivative-free, on x = log(theta), which
keeps every parameter positive.  Coefficients: reflection 1, expansion 2,
contraction 1/2, shrink 1/2.

The search is written as a generator that yields the point to evaluate and
receives -L~ there, so that one driver can advance many independent searches
together: `fit` runs one search with hm_loglik, `fit_many` runs one search
per dataset (e.g. Monte-Carlo replicates) through a request server, with one
evaluation of every unfinished search on the device at once.  Every step of
each evaluation runs in the library's kernels; this module only steers.
"""
from __future__ import annotations

import math
from typing import Callable, Generator, List, Sequence

import numpy as np

ALPHA, GAMMA, RHO, SIGMA = 1.0, 2.0, 0.5, 0.5


def nelder_mead(x0: Sequence[float], step: float = 0.1, ftol: float = 1e-7, xtol: float = 1e-5,
                max_evals: int = 400) -> Generator[np.ndarray, float, dict]:
    """Minimises f from x0.  Yields points, receives f there; returns
    dict(x, f, evals, converged).  Stops when the spread of f over the
    simplex is at most ftol * (1 + |f_best|) and every vertex is within xtol
    (max norm) of the best one, or after max_evals evaluations.  A
    non-finite f counts as +infinity (the point is never kept as best)."""
    x0 = np.asarray(x0, dtype=np.float64)
    d = x0.size
    evals = 0

    def value(v):
        return v if math.isfinite(v) else math.inf

    pts = [x0.copy()]
    for i in range(d):
        p = x0.copy()
        p[i] += step
        pts.append(p)
    fs = []
    for p in pts:
        fs.append(value((yield p.copy())))
        evals += 1
    while True:
        order = np.argsort(fs, kind="stable")
        pts = [pts[i] for i in order]
        fs = [fs[i] for i in order]
        spread = fs[-1] - fs[0] if math.isfinite(fs[-1]) else math.inf
        size = max(float(np.max(np.abs(p - pts[0]))) for p in pts[1:])
        if (spread <= ftol * (1.0 + abs(fs[0])) and size <= xtol) or evals >= max_evals:
            return dict(x=pts[0], f=fs[0], evals=evals, converged=evals < max_evals)
        centroid = np.mean(pts[:-1], axis=0)
        xr = centroid + ALPHA * (centroid - pts[-1])
        fr = value((yield xr.copy()))
        evals += 1
        if fr < fs[0]:
            xe = centroid + GAMMA * (xr - centroid)
            fe = value((yield xe.copy()))
            evals += 1
            pts[-1], fs[-1] = (xe, fe) if fe < fr else (xr, fr)
            continue
        if fr < fs[-2]:
            pts[-1], fs[-1] = xr, fr
            continue
        # contraction: outside if the reflected point beats the worst, else inside
        if fr < fs[-1]:
            xc = centroid + RHO * (xr - centroid)
        else:
            xc = centroid + RHO * (pts[-1] - centroid)
        fc = value((yield xc.copy()))
        evals += 1
        if fc < min(fr, fs[-1]):
            pts[-1], fs[-1] = xc, fc
            continue
        # shrink towards the best vertex
        for i in range(1, d + 1):
            pts[i] = pts[0] + SIGMA * (pts[i] - pts[0])
            fs[i] = value((yield pts[i].copy()))
            evals += 1


def minimise(f: Callable[[np.ndarray], float], x0, **kw) -> dict:
    """Runs nelder_mead on a plain function (host objective)."""
    gen = nelder_mead(x0, **kw)
    x = next(gen)
    try:
        while True:
            x = gen.send(f(x))
    except StopIteration as stop:
        return stop.value


def _objective(res) -> float:
    """-L~ summed over the columns of Z; +inf after a breakdown (not SPD)."""
    if int(res["status"][0]) != 0:
        return math.inf
    return -float(np.sum(res["loglik"]))


def _theta(x) -> tuple:
    """theta = exp(x), or None where the library would reject it (overflow to
    inf or 0, or nu above the largest order the K_nu routine accepts, 50)."""
    th = np.exp(np.asarray(x, dtype=np.float64))
    if not (np.all(np.isfinite(th)) and np.all(th > 0.0) and th[2] <= 50.0):
        return None
    return tuple(float(v) for v in th)


def _point(x, nugget, fit_nugget):
    """(theta, nugget) at the search point x: x = log(theta), or with a fitted
    nugget x = (log theta, log tau^2); None where the library would reject it."""
    th = _theta(x[:3])
    if th is None:
        return None
    if not fit_nugget:
        return th, nugget
    tau2 = float(np.exp(x[3]))
    if not (math.isfinite(tau2) and tau2 > 0.0):
        return None
    return th, tau2


def _start(theta0, nugget, fit_nugget):
    x0 = list(np.log(np.asarray(theta0, dtype=np.float64)))
    if fit_nugget:
        x0.append(math.log(nugget))
    return np.asarray(x0)


def _estimate(r, nugget, fit_nugget) -> dict:
    x = np.asarray(r["x"])
    return dict(theta=tuple(float(v) for v in np.exp(x[:3])),
                nugget=float(np.exp(x[3])) if fit_nugget else nugget,
                loglik=-r["f"], evals=r["evals"], converged=r["converged"])


def fit(ds, theta0, nugget: float, eps: float = 1e-7, rank: int = 0, fit_nugget: bool = False,
        loglik_kw: dict = None, **kw) -> dict:
    """Maximum-likelihood estimate of theta for one hmlik.Dataset (with Z set);
    returns dict(theta, nugget, loglik, evals, converged).  With fit_nugget the
    nugget tau^2 is a fourth parameter, searched on log tau^2 from `nugget`
    (the paper treats it as fixed; its Section 6 names the extension).
    loglik_kw goes to Dataset.loglik (e.g. prec, refine_max_iter, refine_tol)."""
    lk = loglik_kw or {}
    gen = nelder_mead(_start(theta0, nugget, fit_nugget), **kw)
    x = next(gen)
    try:
        while True:
            pt = _point(x, nugget, fit_nugget)
            x = gen.send(math.inf if pt is None else _objective(ds.loglik(pt[0], pt[1], eps, rank, **lk)))
    except StopIteration as stop:
        r = stop.value
    return _estimate(r, nugget, fit_nugget)


def fit_many(server, datasets: List, theta0s, nugget: float,
             eps: float = 1e-7, rank: int = 0, fit_nugget: bool = False, log=None, **kw) -> List[dict]:
    """One search per hmlik.Dataset, advanced together through an
    hmlik.Server (give it a slot per dataset): each round submits the
    pending point of every unfinished search to the server and feeds back the
    results.  Each search sees exactly the values `fit` would, so the
    estimates equal those of separate `fit` calls."""
    gens, pending, out = [], [], [None] * len(datasets)
    for th in theta0s:
        g = nelder_mead(_start(th, nugget, fit_nugget), **kw)
        gens.append(g)
        pending.append(next(g))
    live = list(range(len(datasets)))
    rounds = 0
    while live:
        rounds += 1
        if log is not None and rounds % 25 == 0:
            log(f"fit_many: round {rounds}, {len(live)} searches running")
        tickets = {}
        for i in live:
            pt = _point(pending[i], nugget, fit_nugget)
            if pt is not None:
                tickets[i] = server.submit(datasets[i], pt[0], pt[1], eps, rank)
        still = []
        for i in live:
            f = _objective(server.poll(tickets[i], wait=True)) if i in tickets else math.inf
            try:
                pending[i] = gens[i].send(f)
                still.append(i)
            except StopIteration as stop:
                out[i] = _estimate(stop.value, nugget, fit_nugget)
        live = still
    return out


def gradient(ds, theta, nugget: float, eps: float = 1e-7, rank: int = 0, h: float = 1e-4,
             fit_nugget: bool = False, loglik_kw: dict = None) -> np.ndarray:
    """Gradient of L~ (summed over the columns of Z) with respect to log theta
    (and log tau^2 with fit_nugget), by central differences of step h in the
    log parameters: 2 d evaluations of the device likelihood.  The paper names
    the gradient as an extension (Section 6) without giving a method; this is
    the plain numerical one (truncation error O(h^2), rounding error about
    |L~| u / h, and the H-approximation error of L~ divided by h)."""
    lk = loglik_kw or {}
    x0 = _start(theta, nugget, fit_nugget)
    g = np.empty_like(x0)
    for i in range(x0.size):
        vals = []
        for sgn in (1.0, -1.0):
            x = x0.copy()
            x[i] += sgn * h
            pt = _point(x, nugget, fit_nugget)
            if pt is None:
                raise ValueError("gradient: a difference point is outside the parameter domain")
            r = ds.loglik(pt[0], pt[1], eps, rank, **lk)
            if int(r["status"][0]) != 0:
                raise ValueError("gradient: the factorisation broke down at a difference point")
            vals.append(float(np.sum(r["loglik"])))
        g[i] = (vals[0] - vals[1]) / (2.0 * h)
    return g
