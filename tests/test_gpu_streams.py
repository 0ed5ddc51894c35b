"""GPU test of the factorisation on several streams (hm_tune_schedule builds a
stream program: the big blocks' flush steps, the long low-rank flushes and the
rest on their own streams, cross-stream dependencies as events).  Every task
runs on the same inputs as in the level schedule, so the evaluation is
bitwise equal before and after tuning, with and without the extra streams,
and over repeated evaluations; and it still agrees with the oracle."""
import os

import numpy as np
import pytest

from oracle.hchol import h_loglik
from paper_1709_04419_amd import workloads as wl

pytestmark = pytest.mark.gpu

THETA, NUGGET, EPS = (1.0, 0.1, 0.325), 1e-6, 1e-7


def _vals(r):
    return (float(r["loglik"][0]), float(r["logdet"][0]), float(r["quadform"][0]), int(r["status"][0]))


@pytest.mark.parametrize("n,leaf", [(3000, 32), (24000, 64)])
def test_stream_program_is_bitwise_equal(n, leaf):
    from paper_1709_04419_amd import hmlik
    P = wl.basin_clusters(n, 41)
    Z = wl.standard_normal(n, 1, 42)
    ctx = hmlik.Context(0)
    try:
        ds = hmlik.Dataset(ctx, P, leaf, 2.0)
        ds.set_z(Z)
        base = _vals(ds.loglik(THETA, NUGGET, EPS))
        os.environ["HMLIK_SINGLE_STREAM"] = "1"
        try:
            ds.tune_schedule(THETA, NUGGET, EPS)
        finally:
            del os.environ["HMLIK_SINGLE_STREAM"]
        single = _vals(ds.loglik(THETA, NUGGET, EPS))
        ds.tune_schedule(THETA, NUGGET, EPS)
        multi = [_vals(ds.loglik(THETA, NUGGET, EPS)) for _ in range(3)]
    finally:
        ctx.close()
    assert base[3] == 0
    assert single == base
    for v in multi:
        assert v == base
    if n <= 3000:
        ref = h_loglik(P, Z, THETA, NUGGET, n_min=leaf, eta=2.0, eps=EPS)
        assert abs(base[0] - float(ref["loglik"][0])) <= 1e-10 * abs(float(ref["loglik"][0]))
