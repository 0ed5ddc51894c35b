"""Modified Bessel function of the second kind, K_nu(x), for the oracle.

The Matern covariance of eq. (2) (Section 2.2) needs K_nu for real nu > 0.
This module evaluates the standard integral representation

    K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt,      x > 0,

in the exponentially scaled form

    exp(x) K_nu(x) = int_0^inf exp(-2 x sinh^2(t/2)) cosh(nu t) dt,

with the trapezoidal rule.  The integrand is entire and decays
double-exponentially, so the trapezoidal rule converges geometrically in the
step.  To keep the step resolution uniform for large x, where the integrand is
a narrow Gaussian of width ~ 1/sqrt(x), the variable is rescaled t = u / s with
s = max(1, sqrt(x)) and the rule is applied in u with a fixed step H.

This is deliberately a different method from the series / continued-fraction
evaluation used by the device kernels, so that the two cannot share a mistake.

Parity pins (tests/test_oracle_besselk.py): closed forms at nu = 1/2, 3/2, 5/2;
mpmath.besselk at 40 digits over x in [1e-8, 700]; the three-term recurrence;
the small-x limit x^nu K_nu(x) -> 2^(nu-1) Gamma(nu).
"""
from __future__ import annotations

import numpy as np

H_STEP = 0.1          # trapezoid step in the rescaled variable u
TAIL_EXPONENT = 60.0  # stop once 2 x sinh^2(t/2) - nu t exceeds this
_CHUNK = 1 << 14


def _nodes_needed(x_min: float, nu: float, s: float) -> int:
    # smallest u_max with 2 x_min sinh^2(u/(2s)) - nu u/s >= TAIL_EXPONENT
    lo, hi = 0.0, 1.0
    f = lambda u: 2.0 * x_min * np.sinh(u / (2 * s)) ** 2 - nu * u / s
    while f(hi) < TAIL_EXPONENT:
        hi *= 2.0
        if hi > 1e6:
            break
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if f(mid) < TAIL_EXPONENT:
            lo = mid
        else:
            hi = mid
    return int(np.ceil(hi / H_STEP)) + 2


def kve(nu: float, x) -> np.ndarray:
    """exp(x) * K_nu(x) for x > 0 (array), real nu (K_{-nu} = K_nu)."""
    nu = abs(float(nu))
    x = np.asarray(x, dtype=np.float64)
    flat = x.reshape(-1)
    out = np.empty_like(flat)
    if np.any(flat <= 0):
        raise ValueError("kve requires x > 0")
    # group by scale so that one node count serves a chunk
    order = np.argsort(flat, kind="stable")
    xs = flat[order]
    res = np.empty_like(xs)
    start = 0
    while start < len(xs):
        # chunk with x within a factor 4 of each other so s is comparable
        stop = min(start + _CHUNK, len(xs))
        hi_lim = xs[start] * 4.0
        stop = start + int(np.searchsorted(xs[start:stop], hi_lim, side="right"))
        stop = max(stop, start + 1)
        xc = xs[start:stop]
        s = np.maximum(1.0, np.sqrt(xc))
        # node count: the largest requirement over the chunk (checked at both
        # ends and the geometric middle; the requirement is monotone in x
        # within a factor-4 chunk)
        xm = float(np.sqrt(xc[0] * xc[-1]))
        nn = max(_nodes_needed(float(v), nu, max(1.0, float(np.sqrt(v))))
                 for v in (float(xc[0]), xm, float(xc[-1])))
        u = H_STEP * np.arange(nn, dtype=np.float64)
        t = u[None, :] / s[:, None]
        w = np.full(nn, H_STEP)
        w[0] = 0.5 * H_STEP
        sh = np.sinh(0.5 * t)
        f = np.exp(-2.0 * xc[:, None] * sh * sh) * np.cosh(nu * t)
        res[start:stop] = (f @ w) / s
        start = stop
    out[order] = res
    return out.reshape(x.shape)


def kv(nu: float, x) -> np.ndarray:
    """K_nu(x) for x > 0 (underflows to 0 for x beyond ~745)."""
    x = np.asarray(x, dtype=np.float64)
    return kve(nu, x) * np.exp(-x)
