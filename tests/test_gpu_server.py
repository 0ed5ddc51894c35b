"""GPU tests of the request server (hm_server_*): continuous batching of
likelihood evaluations (eq. 4) over resident datasets.

Every served result is compared bit for bit with hm_loglik of the same
request alone (the server runs the same tasks on the same inputs in the same
per-dataset order), and one served result with the oracle.  Also covered:
admission while other requests are on the device, the HBM budget with
release of idle datasets' factor storage, cancellation, the busy state of
the context's direct calls, and destroying a dataset with queued requests.
"""
import time

import numpy as np
import pytest

from oracle.hchol import HLikelihood
from paper_1709_04419_amd import workloads as wl

pytestmark = pytest.mark.gpu

KEYS = ("loglik", "logdet", "quadform", "status", "fail_block", "fail_pivot", "max_rank")

# (n, (points, seed), leaf size, theta, nugget, eps, fixed rank)
SPECS = [(1500, ("uniform", 11), 32),
         (1200, ("basin", 31), 64),
         (1000, ("uniform", 22), 32)]
REQUESTS = [(0, (1.0, 0.1, 0.5), 1e-6, 1e-8, 0),
            (1, (1.0, 0.1, 0.325), 1e-6, 1e-7, 0),
            (2, (1.0, 0.2, 1.5), 1e-6, 0.0, 5),        # breaks down (not SPD)
            (0, (1.3, 0.15, 0.7), 1e-6, 1e-6, 0),
            (1, (0.9, 0.08, 0.5), 1e-6, 0.0, 12),
            (2, (1.0, 0.1, 0.5), 1e-6, 1e-7, 0),
            (0, (1.0, 0.05, 1.0), 0.0, 1e-7, 0)]


@pytest.fixture(scope="module")
def H():
    from paper_1709_04419_amd import hmlik
    return hmlik


def _datasets(H, ctx, specs=SPECS, r=2):
    dss = []
    for n, (kind, seed), leaf in specs:
        ds = H.Dataset(ctx, wl.make_points(kind, n, seed), leaf, 2.0)
        ds.set_z(wl.standard_normal(n, r, seed + 1))
        dss.append(ds)
    return dss


def _singles(dss, requests):
    return [dss[d].loglik(th, nug, eps, k) for d, th, nug, eps, k in requests]


def _same(a, b):
    return all(np.array_equal(a[k], b[k], equal_nan=k in ("loglik", "logdet", "quadform")) for k in KEYS)


def test_served_results_equal_single(H):
    ctx = H.Context(0)
    try:
        dss = _datasets(H, ctx)
        ref = _singles(dss, REQUESTS)
        assert ref[2]["status"][0] == H.HM_ERR_NOT_SPD
        with H.Server(ctx, max_active=4) as sv:
            tickets = [sv.submit(dss[d], th, nug, eps, k) for d, th, nug, eps, k in REQUESTS]
            out = [sv.poll(t, wait=True) for t in tickets]
        for i, (o, r) in enumerate(zip(out, ref)):
            assert _same(o, r), i
            assert o["request_status"] == int(r["status"][0])
            assert o["steps"] >= 1 and 1 <= o["peak_batch"] <= 4
        assert max(o["peak_batch"] for o in out) >= 2          # requests shared level launches
        # one served result against the oracle (basin points, eps = 1e-7)
        n, (kind, seed), leaf = SPECS[1]
        d, th, nug, eps, k = REQUESTS[1]
        o = HLikelihood(wl.make_points(kind, n, seed), leaf, 2.0).loglik(
            th, nug, wl.standard_normal(n, 2, seed + 1), eps, k)
        np.testing.assert_allclose(out[1]["loglik"], o["loglik"], rtol=1e-10, atol=0)
    finally:
        ctx.close()


def test_admission_while_others_run(H):
    """A long request is on the device; requests submitted meanwhile are
    admitted beside it (continuous batching), finish first, and still give
    bitwise their single results."""
    ctx = H.Context(0)
    try:
        specs = [(6000, ("basin", 31), 64), (900, ("uniform", 5), 32), (784, ("grid", 7), 24)]
        dss = _datasets(H, ctx, specs, r=1)
        reqs = [(0, (1.0, 0.1, 0.325), 1e-6, 1e-7, 0), (1, (1.0, 0.1, 0.5), 1e-6, 1e-8, 0),
                (2, (2.0, 0.0334, 0.5), 1e-4, 1e-6, 0)]
        ref = _singles(dss, reqs)
        with H.Server(ctx, max_active=4) as sv:
            t_big = sv.submit(dss[0], *reqs[0][1:])
            time.sleep(0.05)
            small = [sv.submit(dss[d], th, nug, eps, k) for d, th, nug, eps, k in reqs[1:]]
            out_small = [sv.poll(t, wait=True) for t in small]
            big_done_early = sv.poll(t_big) is not None
            out_big = sv.poll(t_big, wait=True) if not big_done_early else None
        assert _same(out_small[0], ref[1]) and _same(out_small[1], ref[2])
        if out_big is not None:
            assert _same(out_big, ref[0])
            assert out_big["t_latency"] > max(o["t_latency"] for o in out_small)
            assert max(o["peak_batch"] for o in out_small) >= 2
    finally:
        ctx.close()


def test_hbm_budget_and_release(H):
    ctx = H.Context(0)
    try:
        dss = _datasets(H, ctx)
        ref = _singles(dss, REQUESTS)
        fb = [ds.footprint()["factor_bytes"] for ds in dss]
        order = np.argsort(fb)
        # room for the two smaller datasets' factor storage, not for the largest
        budget = fb[order[0]] + fb[order[1]]
        assert sum(fb) > budget                   # the three cannot be attached together
        for ds in dss:
            ds.release()
            assert not ds.footprint()["attached"]
        with H.Server(ctx, max_active=3, hbm_budget=budget) as sv:
            ok = [i for i, q in enumerate(REQUESTS) if fb[q[0]] <= budget]
            tickets = {i: sv.submit(dss[REQUESTS[i][0]], *REQUESTS[i][1:]) for i in ok}
            for i in ok:
                o = sv.poll(tickets[i], wait=True)
                assert _same(o, ref[i]), i
                att = sum(f for f, ds in zip(fb, dss) if ds.footprint()["attached"])
                assert att <= budget
        big = H.Server(ctx, max_active=2, hbm_budget=fb[order[2]] - 1)
        try:
            with pytest.raises(H.HMError) as ei:
                big.submit(dss[order[2]], (1.0, 0.1, 0.5), 1e-6, 1e-7)
            assert ei.value.status == H.HM_ERR_OOM
        finally:
            big.close()
        # after the server: storage is attached again on demand
        r = dss[0].loglik(*REQUESTS[0][1:])
        assert _same(r, ref[0])
    finally:
        ctx.close()


def test_cancel_busy_and_destroy(H):
    ctx = H.Context(0)
    try:
        dss = _datasets(H, ctx)
        ref = _singles(dss, REQUESTS[:3])
        sv = H.Server(ctx, max_active=1)
        try:
            with pytest.raises(H.HMError) as ei:
                dss[0].loglik(*REQUESTS[0][1:])
            assert ei.value.status == H.HM_ERR_BUSY
            with pytest.raises(H.HMError) as ei:
                H.Server(ctx)
            assert ei.value.status == H.HM_ERR_BUSY
            t = [sv.submit(dss[d], th, nug, eps, k) for d, th, nug, eps, k in REQUESTS[:3]]
            t_cancel = sv.submit(dss[1], (1.0, 0.1, 0.5), 1e-6, 1e-7)
            t_gone = sv.submit(dss[2], (1.0, 0.1, 0.5), 1e-6, 1e-7)
            sv.cancel(t_cancel)
            dss[2].close()             # its queued request is cancelled; the admitted one finishes first
            c = sv.poll(t_cancel, wait=True)
            assert c["request_status"] == H.HM_ERR_CANCELLED and np.isnan(c["loglik"]).all()
            g = sv.poll(t_gone, wait=True)
            assert g["request_status"] == H.HM_ERR_CANCELLED
            out = [sv.poll(x, wait=True) for x in t]
            for i in range(2):
                assert _same(out[i], ref[i]), i
            assert out[2]["request_status"] in (H.HM_ERR_NOT_SPD, H.HM_ERR_CANCELLED)
            with pytest.raises(H.HMError):
                sv.poll(t[0])          # retired
            with pytest.raises(H.HMError):
                sv.cancel(123456789)
        finally:
            sv.close()
        r = dss[0].loglik(*REQUESTS[0][1:])
        assert _same(r, ref[0])
    finally:
        ctx.close()


def test_batch_more_datasets_than_slots(H):
    """hm_loglik_batch with 18 datasets: at most 16 are on the device at once,
    the rest wait for a slot; every result is bitwise its hm_loglik alone."""
    ctx = H.Context(0)
    try:
        specs = [(300 + 37 * i, ("uniform", 700 + i), 32) for i in range(18)]
        dss = _datasets(H, ctx, specs, r=1)
        thetas = [(1.0, 0.05 + 0.01 * i, 0.5 + 0.05 * (i % 5)) for i in range(18)]
        ref = [ds.loglik(th, 1e-6, 1e-7) for ds, th in zip(dss, thetas)]
        res = H.loglik_batch(ctx, dss, thetas, [1e-6] * 18, 1e-7)
        for i, (a, b) in enumerate(zip(res, ref)):
            assert _same(a, b), i
    finally:
        ctx.close()
