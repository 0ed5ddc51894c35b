"""GPU parity of the whole evaluation at the full sizes of the benchmark
workloads, against values the CPU oracle computed once
(tests/golden/fullsize.json, written by tests/golden/make_fullsize.py from
`oracle/` and the seeded generators only):

  * basin clouds, n = 256,000 and 64,000, eps = 1e-7 (Remark 2.4);
  * uniform cloud, n = 64,000, fixed rank (Definition 2.1): ell in {0.05, 0.2}
    x nu in {0.5, 1.0, 1.5} at k = 10, and k = 5, 20 at ell = 0.05, nu = 0.5.

L~, log|C~| and v^T v (eq. 4, Section 3.1) agree to 1e-10 relative; a
breakdown (the paper's "crash", Tables 6 and 7) happens at the same block and
pivot; the largest rank and the storage of C~ and L~ at the actual ranks
(Table 5's columns) are equal.
"""
import json
import os

import numpy as np
import pytest

from paper_1709_04419_amd import workloads as wl

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullsize.json")
CASES = json.load(open(GOLDEN)) if os.path.exists(GOLDEN) else {}
TOL = 1e-10


@pytest.fixture(scope="module")
def H():
    from paper_1709_04419_amd import hmlik
    return hmlik


@pytest.fixture(scope="module")
def ctx(H):
    c = H.Context(0)
    yield c
    c.close()


_datasets = {}


def _dataset(H, ctx, rec):
    key = (rec["cloud"], rec["n"], rec["points_seed"], rec["z_seed"])
    if key not in _datasets:
        _datasets.clear()
        gen = wl.basin_clusters if rec["cloud"] == "basin" else wl.uniform_square
        ds = H.Dataset(ctx, gen(rec["n"], rec["points_seed"]), rec["leaf"], rec["eta"])
        ds.set_z(wl.standard_normal(rec["n"], 1, rec["z_seed"]))
        _datasets[key] = ds
    return _datasets[key]


@pytest.mark.parametrize("name", sorted(CASES))
def test_fullsize_against_oracle(H, ctx, name):
    rec = CASES[name]
    ds = _dataset(H, ctx, rec)
    print(f"case {name}", flush=True)
    g = ds.loglik(tuple(rec["theta"]), rec["nugget"], rec["eps"], rec["fixed_rank"])
    assert int(g["bytes_C"][0]) == rec["bytes_C"]
    if rec["status"] == "not_spd":
        assert int(g["status"][0]) == H.HM_ERR_NOT_SPD
        assert int(g["fail_block"][0]) == rec["fail_block"]
        assert int(g["fail_pivot"][0]) == rec["fail_pivot"]
        return
    assert int(g["status"][0]) == H.HM_OK
    for k in ("loglik", "logdet", "quadform"):
        d, o = float(g[k][0]), rec[k]
        assert abs(d - o) <= TOL * abs(o), (k, d, o, abs(d - o) / abs(o))
    assert int(g["max_rank"][0]) == rec["max_rank"]
    assert int(g["bytes_L"][0]) == rec["bytes_L"]
    assert int(g["rank_capped"][0]) == rec["rank_capped"]


def teardown_module(module):
    _datasets.clear()
