"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds random number generation and geometry only: point clouds,
standard-normal draws, parameter tuples.  It contains none of the likelihood
method's arithmetic (no covariance entries, no factorisations), so that both
the device path and the CPU oracle can take identical inputs from it without
sharing any of the computation they are compared on.

Point-cloud shapes follow the workloads the paper measures on:
  * uniform points in the unit square (Sections 2.3 and 4 use [0,1]^2),
  * the perturbed grid of eq. (3) (Section 2.3, used for Tables 2 and 3),
  * an irregular, non-convex region with gaps and dense clusters, standing in
    for the soil-moisture locations of Section 5.1 (a 1830 x 1329 grid with
    missing cells over a river basin), which are not available here.

All generators use numpy's PCG64 (`numpy.random.default_rng(seed)`).
"""
from __future__ import annotations

import numpy as np

# Vertices of the simple, non-convex polygon used as the irregular domain.
# It is a fixed stand-in for a river basin outline (Section 5.1); area 0.522.
BASIN_POLYGON = np.array(
    [
        (0.05, 0.10), (0.45, 0.02), (0.60, 0.25), (0.95, 0.15), (0.90, 0.55),
        (0.70, 0.60), (0.85, 0.95), (0.40, 0.85), (0.30, 0.55), (0.10, 0.70),
    ],
    dtype=np.float64,
)


def uniform_square(n: int, seed: int) -> np.ndarray:
    """n points i.i.d. uniform on [0,1]^2, shape (n, 2), row-major float64."""
    rng = np.random.default_rng(seed)
    return rng.random((n, 2))


def perturbed_grid(m: int, seed: int) -> np.ndarray:
    """The irregular grid of eq. (3): n = m*m points
    ((i - 0.5 + X_ij)/m, (j - 0.5 + Y_ij)/m), X, Y i.i.d. U(-0.4, 0.4),
    ordered lexicographically by (i, j)."""
    rng = np.random.default_rng(seed)
    i, j = np.meshgrid(np.arange(1, m + 1), np.arange(1, m + 1), indexing="ij")
    x = rng.uniform(-0.4, 0.4, size=(m, m))
    y = rng.uniform(-0.4, 0.4, size=(m, m))
    pts = np.stack([(i - 0.5 + x) / m, (j - 0.5 + y) / m], axis=-1)
    return pts.reshape(-1, 2).astype(np.float64)


def _inside_polygon(p: np.ndarray, poly: np.ndarray) -> np.ndarray:
    """Even-odd ray casting point-in-polygon test (geometry, not the method)."""
    x, y = p[:, 0], p[:, 1]
    inside = np.zeros(len(p), dtype=bool)
    k = len(poly)
    for a in range(k):
        x1, y1 = poly[a]
        x2, y2 = poly[(a + 1) % k]
        cond = (y1 > y) != (y2 > y)
        with np.errstate(divide="ignore", invalid="ignore"):
            xc = x1 + (y - y1) * (x2 - x1) / (y2 - y1)
        inside ^= cond & (x < xc)
    return inside


def basin_clusters(n: int, seed: int, cluster_frac: float = 0.2,
                   n_clusters: int = 10, cluster_sigma: float = 0.02) -> np.ndarray:
    """Irregular non-convex cloud: (1 - cluster_frac) of the points uniform in
    BASIN_POLYGON (rejection sampling), the rest in `n_clusters` isotropic
    Gaussian clusters (std `cluster_sigma`) whose centres are uniform in the
    polygon; cluster points falling outside the polygon are redrawn."""
    rng = np.random.default_rng(seed)
    n_cl = int(round(n * cluster_frac))
    n_un = n - n_cl
    out = []
    need = n_un
    while need > 0:
        cand = rng.random((max(2 * need, 1024), 2))
        cand = cand[_inside_polygon(cand, BASIN_POLYGON)]
        out.append(cand[:need])
        need -= len(out[-1])
    centres = []
    while len(centres) < n_clusters:
        c = rng.random((1, 2))
        if _inside_polygon(c, BASIN_POLYGON)[0]:
            centres.append(c[0])
    per = [n_cl // n_clusters + (1 if c < n_cl % n_clusters else 0) for c in range(n_clusters)]
    for c, cnt in zip(centres, per):
        need = cnt
        while need > 0:
            cand = c + cluster_sigma * rng.standard_normal((max(2 * need, 64), 2))
            cand = cand[_inside_polygon(cand, BASIN_POLYGON)]
            out.append(cand[:need])
            need -= len(out[-1])
    pts = np.concatenate(out, axis=0)
    return np.ascontiguousarray(pts[:n], dtype=np.float64)


def standard_normal(n: int, r: int, seed: int) -> np.ndarray:
    """W ~ N(0, I), shape (n, r) (column j is right-hand side j)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, r))


# Named workloads (sizes and parameters of the configurations the method is
# measured on).  theta = (sigma2, ell, nu), nugget tau^2.
WORKLOADS = {
    # n=2000 uniform points, exponential Matern (nu = 1/2), H with leaf 32, eta 2, eps 1e-8.
    "uniform2k": dict(n=2000, points=("uniform", 11), w_seed=12, theta=(1.0, 0.1, 0.5),
                      nugget=1e-6, leaf=32, eta=2.0, eps=1e-8, rank=0),
    # n=64,000 uniform points, fixed rank k in {5,10,20}; ell in {0.05,0.2}, nu in {0.5,1,1.5}.
    "uniform64k": dict(n=64000, points=("uniform", 21), w_seed=22, theta=(1.0, 0.05, 0.5),
                       nugget=1e-6, leaf=64, eta=2.0, eps=0.0, rank=10),
    # n=256,000 points on the irregular basin with clusters, nu = 0.325, ell = 0.1, eps 1e-7.
    "basin256k": dict(n=256000, points=("basin", 31), w_seed=32, theta=(1.0, 0.1, 0.325),
                      nugget=1e-6, leaf=64, eta=2.0, eps=1e-7, rank=0),
}


def make_points(kind: str, n: int, seed: int) -> np.ndarray:
    if kind == "uniform":
        return uniform_square(n, seed)
    if kind == "basin":
        return basin_clusters(n, seed)
    if kind == "grid":
        m = int(round(np.sqrt(n)))
        assert m * m == n
        return perturbed_grid(m, seed)
    raise ValueError(kind)
