"""Writes tests/golden/fullsize.json: the oracle's H-matrix log-likelihood at the
full sizes of the benchmark workloads, for the GPU parity test
tests/test_gpu_fullsize_golden.py.

Only `oracle/` and the seeded input generators are used.  Cases:

  * basin, n = 256,000 (80% uniform in a non-convex basin, 20% in ten Gaussian
    clusters, seed 31), theta = (1, 0.1, 0.325), nugget 1e-6, leaf 64, eta 2,
    accuracy eps = 1e-7 (Remark 2.4); the same at n = 64,000 (seed 33);
  * uniform on [0,1]^2, n = 64,000 (seed 21), nugget 1e-6, leaf 64, eta 2, fixed
    rank (Definition 2.1): ell in {0.05, 0.2} x nu in {0.5, 1.0, 1.5} at k = 10,
    and k = 5, 20 at ell = 0.05, nu = 0.5.

Z is one seeded standard-normal column (seed 32 / 34 for the basin clouds, 22
for the uniform cloud).  Each case records L~, log|C~|, v^T v (eq. (4), Section 3.1),
the status with the failing block and pivot on a breakdown, the largest rank,
whether the rank cap bound, and the storage of C~ and L~ in bytes at the actual
ranks (dense entries plus (m + n) k per low-rank block, 8 bytes each).

    python tests/golden/make_fullsize.py [--jobs J] [--only NAME ...]

Cases run in parallel processes with one BLAS thread each; a case's result is
merged into the JSON file as soon as it finishes.  The basin case takes the
longest (tens of minutes on one core).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "fullsize.json")

CASES = [("basin256k_eps1e-7", "basin", 256000, 31, 32, (1.0, 0.1, 0.325), 1e-7, 0),
         ("basin64k_eps1e-7", "basin", 64000, 33, 34, (1.0, 0.1, 0.325), 1e-7, 0)]
for _ell in (0.05, 0.2):
    for _nu in (0.5, 1.0, 1.5):
        CASES.append((f"uniform64k_l{_ell}_nu{_nu}_k10", "uniform", 64000, 21, 22, (1.0, _ell, _nu), 0.0, 10))
CASES += [("uniform64k_l0.05_nu0.5_k5", "uniform", 64000, 21, 22, (1.0, 0.05, 0.5), 0.0, 5),
          ("uniform64k_l0.05_nu0.5_k20", "uniform", 64000, 21, 22, (1.0, 0.05, 0.5), 0.0, 20)]
NUGGET, LEAF, ETA = 1e-6, 64, 2.0


def storage_bytes(H):
    """Bytes of the current H representation at the actual ranks."""
    b = 0
    for i in H.D:
        b += H.D[i].size
    for i in H.U:
        b += H.U[i].size + H.V[i].size
    return 8 * b


def run_case(case):
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    sys.path.insert(0, ROOT)
    import numpy as np

    from oracle.hchol import HLikelihood, NotSPD
    from paper_1709_04419_amd import workloads as wl

    name, cloud, n, pseed, zseed, theta, eps, kfix = case
    P = wl.basin_clusters(n, pseed) if cloud == "basin" else wl.uniform_square(n, pseed)
    Z = wl.standard_normal(n, 1, zseed)
    t0 = time.perf_counter()
    H = HLikelihood(P, LEAF, ETA)
    H.assemble(theta, NUGGET, eps, kfix)
    bytes_C = storage_bytes(H)
    rec = dict(name=name, cloud=cloud, n=n, points_seed=pseed, z_seed=zseed, theta=list(theta),
               nugget=NUGGET, leaf=LEAF, eta=ETA, eps=eps, fixed_rank=kfix, bytes_C=bytes_C)
    try:
        H.factor()
    except NotSPD as e:
        rec.update(status="not_spd", fail_block=int(e.block), fail_pivot=int(e.pivot),
                   loglik=None, logdet=None, quadform=None, max_rank=None, bytes_L=None,
                   rank_capped=int(sum(H.stats.capped)))
    else:
        logdet = H.logdet()
        v = H.solve(Z)
        quad = float(np.sum(v * v))
        ll = -0.5 * n * np.log(2.0 * np.pi) - 0.5 * logdet - 0.5 * quad
        rec.update(status="ok", fail_block=-1, fail_pivot=-1, loglik=float(ll), logdet=float(logdet),
                   quadform=quad, max_rank=int(max((u.shape[1] for u in H.U.values()), default=0)),
                   bytes_L=storage_bytes(H), rank_capped=int(sum(H.stats.capped)))
    rec["oracle_seconds"] = time.perf_counter() - t0
    return rec


def merge(rec):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    data[rec["name"]] = rec
    with open(OUT + ".tmp", "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(OUT + ".tmp", OUT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    ap.add_argument("--only", nargs="*")
    args = ap.parse_args()
    todo = [c for c in CASES if not args.only or c[0] in args.only]
    from concurrent.futures import ProcessPoolExecutor, as_completed
    with ProcessPoolExecutor(max_workers=args.jobs) as ex:
        futs = {ex.submit(run_case, c): c[0] for c in todo}
        for f in as_completed(futs):
            rec = f.result()
            merge(rec)
            print(f"{rec['name']}: {rec['status']} L={rec['loglik']} ({rec['oracle_seconds']:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
