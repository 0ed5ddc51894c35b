"""CPU checks of the Nelder-Mead search behind the maximum-likelihood driver
(paper_1709_04419_amd/mle.py) against minima that the mathematics fixes:
a weighted quadratic bowl, the Rosenbrock function (minimum at (1, 1)), and
a function that is +inf outside a box.  The device likelihood is exercised
by tests/test_gpu_mle.py."""
import math

import numpy as np

from paper_1709_04419_amd.mle import minimise, nelder_mead


def test_quadratic_bowl():
    c = np.array([0.3, -1.2, 2.0])
    w = np.array([1.0, 10.0, 0.5])
    r = minimise(lambda x: float(np.sum(w * (x - c) ** 2)), np.zeros(3), ftol=1e-14, xtol=1e-7, max_evals=2000)
    assert r["converged"]
    np.testing.assert_allclose(r["x"], c, atol=1e-5)
    assert r["f"] < 1e-9


def test_rosenbrock():
    f = lambda x: float(100.0 * (x[1] - x[0] ** 2) ** 2 + (1.0 - x[0]) ** 2)
    r = minimise(f, [-1.2, 1.0], step=0.5, ftol=1e-14, xtol=1e-8, max_evals=3000)
    assert r["converged"]
    np.testing.assert_allclose(r["x"], [1.0, 1.0], atol=1e-5)


def test_infinite_outside_box():
    # minimum of (x - 0.5)^2 + (y + 0.25)^2 inside |x|, |y| < 1; +inf (or NaN) outside
    def f(x):
        if np.max(np.abs(x)) >= 1.0:
            return math.nan if x[0] > 0 else math.inf
        return float((x[0] - 0.5) ** 2 + (x[1] + 0.25) ** 2)
    r = minimise(f, [0.9, 0.9], step=0.05, ftol=1e-14, xtol=1e-7, max_evals=3000)
    np.testing.assert_allclose(r["x"], [0.5, -0.25], atol=1e-5)


def test_generator_counts_evaluations():
    gen = nelder_mead([1.0, 2.0], max_evals=25)
    n = 0
    x = next(gen)
    try:
        while True:
            n += 1
            x = gen.send(float(np.sum(x ** 2)))
    except StopIteration as stop:
        r = stop.value
    assert r["evals"] == n
    assert n <= 25 + 2          # a shrink may overrun the budget by at most d - 1 points


def test_fitted_nugget_point_mapping():
    from paper_1709_04419_amd.mle import _point, _start
    x = _start((1.0, 0.1, 0.5), 0.05, True)
    assert x.shape == (4,)
    th, tau2 = _point(x, 0.05, True)
    np.testing.assert_allclose(th, (1.0, 0.1, 0.5), rtol=1e-15)
    assert abs(tau2 - 0.05) <= 1e-16
    # a fixed nugget passes through; nu above 50 or an overflowing nugget is rejected
    assert _point(_start((1.0, 0.1, 0.5), 0.05, False), 0.05, False)[1] == 0.05
    assert _point(np.array([0.0, 0.0, math.log(60.0), 0.0]), 0.0, True) is None
    assert _point(np.array([0.0, 0.0, 0.0, 1e4]), 0.0, True) is None
