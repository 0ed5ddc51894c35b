#!/usr/bin/env python3
"""Throughput benchmark: H-matrix Gaussian log-likelihood evaluations per second.

Workload (the configuration the metric is quoted on): n = 256,000 locations,
80% uniform on an irregular non-convex basin plus 20% in ten Gaussian
clusters (sigma = 0.02), Matern theta = (sigma^2, ell, nu) = (1, 0.1, 0.325),
nugget 1e-6, leaf size 64, eta = 2, accuracy eps = 1e-7, FP64.  One step =
one evaluation of eq. (4): Matern/ACA assembly of C~(theta), H-Cholesky,
forward solve, log-determinant.  The data Z is a seeded standard-normal
vector (the cost of an evaluation does not depend on Z).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n N] [--no-cpu-baseline]
                    [--no-tune] [--calib-copy-gib G]
    python bench.py --form served [--datasets D] [--requests R] [--max-active A] [--n N]
    python bench.py --form batched [--replicates M]
    python bench.py --form stream [--datasets D] [--requests R] [--rate L] [--budget-gib B]

Prints one JSON line on stdout (progress goes to stderr).  `value` is evals/s
with the dataset (locations, trees, task schedule, Z) resident on the device
before timing starts.  Warm-up is at most one evaluation: by default it is the
evaluation of hm_tune_schedule, which times every task and builds from those
times the stream program the timed steps run (eight streams: the bench gives
the HIP runtime 10 hardware queues; results are unchanged;
--no-tune skips it and runs a plain warm-up evaluation instead, and the steps
keep the longest-path levels on one stream).  Up to --steps evaluations are then
timed, fewer if the next one would overrun the run's wall budget
(--deadline-s, counted from the start of the process); `steps` is the number
actually timed, `steps_requested` the number asked for.

roofline: the dominant kernel is the H-Cholesky executor k_level, launched once
per level of the schedule (with the tuned schedule: the launches of the
stream program, which overlap in time).  achieved = (algorithmic flops of
one factorisation, counted by the device from the actual ranks) / (number of
launches) / (wall time per launch), where the wall time per launch is the
factorisation time measured with HIP events on the library's stream (which
joins the others) divided by the number of launches -- that is, the
factorisation's flop rate; peak = MI355X FP64 rate.  traffic comes from the
committed rocprofv3 counter summary for k_level (HBM bytes per factorisation
over the launches) when the kernel source is unchanged since the counters
were taken, else null.

cpu_baseline times the oracle (oracle/, one thread) at two sample sizes of the
same workload (n = 3000 and 6000) and extrapolates to n with the growth
exponent measured between them; the measured rates are reported beside it.

--calib-copy-gib G adds one plain device copy of G GiB after the timed steps
(outside the timed region), the reference kernel for HBM counter calibration.

--form served measures the request server instead: D resident datasets of the
same generator (seeds 31, 41, ...), each with its schedule tuned (untimed), and
R requests submitted at once, round-robin over the datasets, at theta values
perturbed around the workload's theta as a Nelder-Mead simplex would be (seeded).
The server keeps up to A requests on the device (default: one per dataset), each on a
stream of its own; GPU_MAX_HW_QUEUES is raised to A + 1 (at least 4) for this form.
value = completed evaluations / wall time from the first submission to the last
result; latency percentiles are per request (submission to result).

--form batched measures one hm_loglik_batch call over M Monte-Carlo replicates
of uneven size: replicate r has n_r ~ U{4000..64000} points uniform on [0,1]^2
(seed 4000 + r), theta = (1, 0.1, 0.5), nugget 1e-6, eps 1e-7, leaf 64, and its
own Z (seeded).  value = replicates / wall time of the call (min(M, 16) on the
device at once).

--form stream serves an open-loop request stream: D resident datasets of the
basin generator with n_i = 16000 * 16^(i / (D - 1)) (16k to 256k, seeds
5000 + i, schedules not tuned); R requests arriving as a Poisson process of
rate L per second (seed 5100), each for a dataset drawn uniformly (seed 5101)
at the next theta of that dataset's simulated Nelder-Mead trace (the search of
the MLE driver run on a quadratic surrogate in log theta around (1, 0.1, 0.5),
seed 5200 + i); the server holds at most B GiB of factor storage (releasing
idle datasets' storage to admit others) and one slot per dataset.
value = completed requests / (last completion - first arrival); latency is
per request, from arrival to result.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import subprocess
import sys
import time

T_START = time.perf_counter()
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "likelihood evals/sec at n=256k, ε=1e-7 (FP64 vs mixed); p50/p99 latency"
FP64_VECTOR_PEAK_TFLOPS = 78.6     # MI355X: 256 CUs x 2.4 GHz x 128 FP64 flop/clk/CU
KERNEL_SRC = os.path.join(ROOT, "paper_1709_04419_amd", "csrc", "hm_device.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_level_basin256k_traffic.json")
THETA, NUGGET, LEAF, ETA = (1.0, 0.1, 0.325), 1e-6, 64, 2.0


def log(msg: str) -> None:
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def cpu_baseline(n_full: int, eps: float, sizes=(3000, 6000)) -> dict:
    """Time one oracle evaluation (assembly, H-Cholesky, solve; the trees are
    built before the clock starts, as on the device) at two sample sizes of the
    same generator, theta, eps, leaf size and eta, on one thread in a child
    process.  The value at n_full is extrapolated with the growth exponent
    measured between the two sizes (t ~ n^alpha) and is labelled as such; the
    measured rates are reported beside it."""
    code = f"""
import sys, time, json
sys.path.insert(0, {ROOT!r})
from oracle.hchol import HLikelihood
from paper_1709_04419_amd import workloads as wl
out = []
for n in {tuple(sizes)!r}:
    P = wl.basin_clusters(n, 31)
    Z = wl.standard_normal(n, 1, 32)
    H = HLikelihood(P, {LEAF}, {ETA})
    t = time.perf_counter()
    r = H.loglik({THETA!r}, {NUGGET}, Z, {eps}, 0)
    out.append(dict(n=n, seconds=time.perf_counter() - t, status=r['status']))
print(json.dumps(out))
"""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    res = json.loads(out.stdout.strip().splitlines()[-1])
    (n1, t1), (n2, t2) = [(r["n"], r["seconds"]) for r in res]
    alpha = math.log(t2 / t1) / math.log(n2 / n1)
    t_full = t2 * (n_full / n2) ** alpha
    return {"value": 1.0 / t_full, "unit": "evals/s", "cores": 1, "kind": "oracle", "extrapolated": True,
            "measured": [{"n": r["n"], "seconds": r["seconds"], "evals_per_s": 1.0 / r["seconds"]} for r in res],
            "growth_exponent": alpha,
            "sample": f"one oracle evaluation (assembly + H-Cholesky + solve, numpy/scipy on 1 thread) of the "
                      f"same generator, theta, eps, leaf size and eta at n={n1} ({t1:.2f} s) and n={n2} "
                      f"({t2:.2f} s); value at n={n_full} extrapolated by the measured growth t ~ n^{alpha:.2f}"}


def full_size_oracle_seconds(n: int, eps: float) -> dict | None:
    """The oracle's own time for one full-size evaluation, recorded when the
    stored full-size values were written (tests/golden/make_fullsize.py, on the
    machine that ran it, one process): a measured check of the extrapolation."""
    try:
        with open(os.path.join(ROOT, "tests", "golden", "fullsize.json")) as f:
            rec = json.load(f).get(f"basin{n // 1000}k_eps{eps:g}".replace("e-0", "e-"))
    except (OSError, ValueError):
        return None
    if not rec or rec.get("n") != n or "oracle_seconds" not in rec:
        return None
    return {"n": n, "seconds": rec["oracle_seconds"], "evals_per_s": 1.0 / rec["oracle_seconds"],
            "measured_by": "tests/golden/make_fullsize.py (build host, one process)"}


def oracle_error(n: int, eps: float, r) -> dict | None:
    """Relative differences to the oracle's FP64 values for this workload,
    stored by tests/golden/make_fullsize.py (None when there are none)."""
    path = os.path.join(ROOT, "tests", "golden", "fullsize.json")
    try:
        with open(path) as f:
            rec = json.load(f).get(f"basin{n // 1000}k_eps" + f"{eps:g}".replace("e-0", "e-"))
    except (OSError, ValueError):
        return None
    if not rec or rec.get("n") != n or rec.get("points_seed") != 31 or rec.get("status") != "ok":
        return None
    out = {k: abs(float(r[k][0]) - rec[k]) / abs(rec[k]) for k in ("loglik", "logdet", "quadform")}
    out["source"] = "oracle (tests/golden/fullsize.json)"
    return out


def traffic_per_launch(n: int, launches: int):
    """HBM bytes per k_level launch: the committed counter summary's bytes per
    factorisation (calibrated FETCH_SIZE + WRITE_SIZE summed over its
    dispatches) over this schedule's launches; None when there is no summary
    for this workload or the kernel source has changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        with open(KERNEL_SRC, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != sha or rec.get("n") != n or "hbm_bytes_per_factorisation" not in rec:
        return None
    return rec["hbm_bytes_per_factorisation"] / launches


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1, help="at most 1 is run")
    ap.add_argument("--deadline-s", type=float, default=480.0,
                    help="wall budget of the whole run; timed steps stop early to keep it")
    ap.add_argument("--no-tune", action="store_true", help="keep the longest-path level schedule")
    ap.add_argument("--n", type=int, default=256000)
    ap.add_argument("--eps", type=float, default=1e-7)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy-gib", type=float, default=0.0)
    ap.add_argument("--form", choices=("plain", "served", "batched", "stream", "mc", "accuracy"), default="plain")
    ap.add_argument("--acc-m", type=int, default=129, help="accuracy form: grid side (n = m^2, eq. 3)")
    ap.add_argument("--mc-n", type=int, default=4000, help="mc form: locations")
    ap.add_argument("--mc-mixed-replicates", type=int, default=0,
                    help="mc form: mixed-precision fits for the first replicates only (0: all)")
    ap.add_argument("--mc-max-evals", type=int, default=300)
    ap.add_argument("--mc-theta", type=str, default="1.0,0.7,0.9",
                    help="mc form: true theta sigma2,ell,nu (default: Section 4's (ell, nu, sigma) = (0.7, 0.9, 1))")
    ap.add_argument("--mc-nugget", type=float, default=1e-6)
    ap.add_argument("--prec", choices=("fp64", "mixed"), default="fp64",
                    help="plain form: FP64, or the mixed-precision form with refinement of C~^-1 Z")
    ap.add_argument("--refine-max-iter", type=int, default=10)
    ap.add_argument("--refine-tol", type=float, default=1e-12)
    ap.add_argument("--rate", type=float, default=0.25)
    ap.add_argument("--budget-gib", type=float, default=96.0)
    ap.add_argument("--replicates", type=int, default=16)
    ap.add_argument("--compare-sequential", action="store_true",
                    help="batched form: also time the replicates one after another (before the batch)")
    ap.add_argument("--datasets", type=int, default=2)
    ap.add_argument("--requests", type=int, default=4)
    ap.add_argument("--max-active", type=int, default=0, help="batch slots (default: one per dataset)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the evaluation is not sharded across GPUs.", file=sys.stderr)
        sys.exit(2)

    if args.form == "served":
        return served(args)
    if args.form == "batched":
        return batched(args)
    if args.form == "stream":
        return stream(args)
    if args.form == "mc":
        return mc(args)
    if args.form == "accuracy":
        return accuracy(args)

    # the tuned factorisation runs on eight streams (hm_tune_schedule): one
    # hardware queue each, plus the default stream's
    hwq = raise_hw_queues(9)
    nstreams = 1 if args.no_tune else (8 if hwq >= 9 else 6 if hwq >= 7 else 4)   # as hm_tune_schedule chooses
    import numpy as np
    import torch

    from paper_1709_04419_amd import hmlik
    from paper_1709_04419_amd import workloads as wl

    n, eps = args.n, args.eps
    mixed = args.prec == "mixed"
    pk = dict(prec=hmlik.HM_MIXED, refine_max_iter=args.refine_max_iter, refine_tol=args.refine_tol) if mixed else {}
    P = wl.basin_clusters(n, 31)
    Z = wl.standard_normal(n, 1, 32)
    ctx = hmlik.Context(0)
    t0 = time.perf_counter()
    ds = hmlik.Dataset(ctx, P, LEAF, ETA)
    t_setup = time.perf_counter() - t0
    ds.set_z(Z)
    info = ds.info()
    log(f"dataset n={n}: {info['nblocks']} blocks, {info['ntasks']} tasks, {info['nlevels']} levels, "
        f"set-up {t_setup:.2f} s")
    # warm-up: at most one evaluation; with schedule tuning (the default) the
    # tuning evaluation is that warm-up
    t_tune = 0.0
    warm = min(args.warmup, 1)
    if not args.no_tune:
        s = time.perf_counter()
        ds.tune_schedule(THETA, NUGGET, eps, 0, prec=pk.get("prec", hmlik.HM_FP64))
        t_tune = time.perf_counter() - s
        warm = 1
        log(f"warm-up: schedule tuned from one timed evaluation, {t_tune:.2f} s")
    elif warm:
        s = time.perf_counter()
        ds.loglik(THETA, NUGGET, eps, 0, **pk)
        log(f"warm-up evaluation: {time.perf_counter() - s:.2f} s")
    torch.cuda.synchronize()
    # timed steps: up to --steps, within the wall budget (at least one)
    reserve = 0.0 if args.no_cpu_baseline else 60.0
    deadline = T_START + args.deadline_s - reserve
    lat, fac, asm, sol = [], [], [], []
    t0 = time.perf_counter()
    for k in range(args.steps):
        if lat and time.perf_counter() + max(lat) > deadline:
            log(f"wall budget reached after {k} of {args.steps} steps")
            break
        s = time.perf_counter()
        r = ds.loglik(THETA, NUGGET, eps, 0, **pk)
        lat.append(time.perf_counter() - s)
        fac.append(r["t_factor"][0])
        asm.append(r["t_assemble"][0])
        sol.append(r["t_solve"][0])
        log(f"step {k + 1}/{args.steps}: {lat[-1]:.2f} s (factor {fac[-1]:.2f} s)")
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    steps = len(lat)
    if int(r["status"][0]) != 0:
        raise SystemExit(f"bench: evaluation failed with status {int(r['status'][0])}")
    if args.calib_copy_gib > 0:
        m = int(args.calib_copy_gib * (1 << 30)) // 8
        src = torch.ones(m, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {m * 8} bytes done")
        del src, dst

    flops = ds.factor_flops()
    launches = ds.info()["nlevels"]      # after tuning: the schedule the steps ran
    t_fac = float(np.mean(fac))
    avg_launch = t_fac / launches
    achieved = flops / launches / avg_launch / 1e12
    lat_ms = np.array(lat) * 1e3
    out = {
        "metric": METRIC,
        "value": steps / total,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": steps,
        "steps_requested": args.steps,
        "warmup": warm,
        "ms_per_step": total / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": "basin256k" if n == 256000 else f"basin{n}", "n": n,
                   "points": "basin_clusters(seed 31): 80% uniform in a non-convex basin, 20% in 10 clusters",
                   "theta": {"sigma2": THETA[0], "ell": THETA[1], "nu": THETA[2]}, "nugget": NUGGET,
                   "eps": eps, "leaf_size": LEAF, "eta": ETA,
                   "precision": (f"mixed: FP32 low-rank factors and update products, FP64 leaves/log-det/"
                                 f"recompression, refinement of C~^-1 Z (at most {args.refine_max_iter} steps, "
                                 f"tol {args.refine_tol:g})") if mixed else "fp64",
                   "blocks": info["nblocks"], "tasks": info["ntasks"], "levels": launches,
                   "levels_longest_path": info["nlevels"],
                   "schedule": "longest-path levels" if args.no_tune else
                               f"{nstreams}-stream program built from one timed evaluation (untimed, before "
                               "the steps; the data's forward solve runs inside it)"},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))},
        "phases_ms": {"assemble": float(np.mean(asm)) * 1e3, "factor": t_fac * 1e3,
                      "solve": float(np.mean(sol)) * 1e3, "dataset_setup_host": t_setup * 1e3,
                      "schedule_tuning": t_tune * 1e3},
        "loglik": float(r["loglik"][0]),
        "logdet": float(r["logdet"][0]),
        "quadform": float(r["quadform"][0]),
        "refine": ({"quad": float(r["refine_quad"][0]), "resid": float(r["refine_resid"][0]),
                    "iters": int(r["refine_iters"][0])} if mixed else None),
        "bytes_C": int(r["bytes_C"][0]), "bytes_L": int(r["bytes_L"][0]), "max_rank": int(r["max_rank"][0]),
        "vs_oracle": oracle_error(n, eps, r),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": traffic_per_launch(n, launches),
                     "kernel": "k_level (H-Cholesky task executor, one launch per level of the schedule)",
                     "streams": nstreams, "hw_queues": hwq,
                     "launches": launches, "avg_launch_ms": avg_launch * 1e3,
                     "flops_per_launch": flops / launches},
    }
    if not args.no_cpu_baseline:
        log("timing the oracle sample on the host")
        cb = cpu_baseline(n, eps)
        # the device on the largest sample (same points, Z, theta, eps): a
        # like-for-like ratio beside the extrapolated full-size value
        n_s = cb["measured"][-1]["n"]
        ds_s = hmlik.Dataset(ctx, wl.basin_clusters(n_s, 31), LEAF, ETA)
        ds_s.set_z(wl.standard_normal(n_s, 1, 32))
        ds_s.loglik(THETA, NUGGET, eps, 0, **pk)
        s = time.perf_counter()
        ds_s.loglik(THETA, NUGGET, eps, 0, **pk)
        t_dev = time.perf_counter() - s
        ds_s.close()
        cb["device_same_n"] = {"n": n_s, "seconds": t_dev,
                               "oracle_over_device": cb["measured"][-1]["seconds"] / t_dev}
        ref = full_size_oracle_seconds(n, eps)
        if ref is not None:
            cb["full_size_reference"] = ref
        out["cpu_baseline"] = cb
    ds.close()
    ctx.close()
    print(json.dumps(out), flush=True)


def raise_hw_queues(slots: int) -> int:
    """Every batch slot's stream needs a hardware queue of its own, plus one for
    the default stream.  The HIP runtime reads GPU_MAX_HW_QUEUES when it
    initialises (at the first library call); a larger setting is kept."""
    need = max(4, slots + 1)
    try:
        have = int(os.environ.get("GPU_MAX_HW_QUEUES", "0"))
    except ValueError:
        have = 0
    if have < need:
        os.environ["GPU_MAX_HW_QUEUES"] = str(need)
    return int(os.environ["GPU_MAX_HW_QUEUES"])


def batched(args):
    """The batched form: uneven Monte-Carlo replicates in one hm_loglik_batch call."""
    m = args.replicates
    raise_hw_queues(min(16, m))
    import numpy as np

    from paper_1709_04419_amd import hmlik
    from paper_1709_04419_amd import workloads as wl

    theta, nug, eps = (1.0, 0.1, 0.5), 1e-6, args.eps
    ctx = hmlik.Context(0)
    dss, ns = [], []
    for r in range(m):
        n_r = int(np.random.default_rng(4000 + r).integers(4000, 64001))
        ds = hmlik.Dataset(ctx, wl.uniform_square(n_r, 4000 + r), LEAF, ETA)
        ds.set_z(wl.standard_normal(n_r, 1, 4200 + r))
        ds.release()                      # factor storage is attached on admission
        dss.append(ds)
        ns.append(n_r)
    log(f"{m} replicates, n from {min(ns)} to {max(ns)} (sum {sum(ns)})")
    seq = None
    if args.compare_sequential:
        seq_res = []
        t0 = time.perf_counter()
        for r, ds in enumerate(dss):
            seq_res.append(ds.loglik(theta, nug, eps))
            log(f"replicate {r + 1}/{m} alone: n={ns[r]}, {seq_res[-1]['t_factor'][0]:.2f} s factor")
        seq = time.perf_counter() - t0
    # one batched call per group of at most 16 replicates (all on the device at
    # once); a group's factor storage is released before the next group, so
    # any number of replicates fits in HBM
    group = 16
    t0 = time.perf_counter()
    res = []
    flops = 0.0
    for g0 in range(0, m, group):
        part = dss[g0:g0 + group]
        res += hmlik.loglik_batch(ctx, part, [theta] * len(part), [nug] * len(part), eps)
        # flop counts are read while the factors are attached (released
        # factors report none)
        flops += sum(ds.factor_flops() for ds in part)
        for ds in part:
            ds.release()
        log(f"replicates {g0 + 1}..{g0 + len(part)} done, {time.perf_counter() - t0:.1f} s")
    wall = time.perf_counter() - t0
    fac = [float(r["t_factor"][0]) for r in res]
    achieved = flops / wall / 1e12
    out = {
        "metric": METRIC,
        "value": m / wall,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": m,
        "warmup": 0,
        "ms_per_step": wall / m * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "form": "batched",
        "config": {"workload": f"mc_replicates{m}", "replicates": m, "n_min": min(ns), "n_max": max(ns),
                   "n_sum": sum(ns), "points": "uniform [0,1]^2, replicate r: n_r ~ U{4000..64000} and points "
                   "from seed 4000 + r", "theta": {"sigma2": 1.0, "ell": 0.1, "nu": 0.5}, "nugget": nug,
                   "eps": eps, "leaf_size": LEAF, "eta": ETA, "slots": min(16, m),
                   "hw_queues": int(os.environ["GPU_MAX_HW_QUEUES"]), "schedule": "longest-path levels"},
        "batch_wall_s": wall,
        "batch_calls": (m + group - 1) // group,
        "sequential_wall_s": seq,
        "bitwise_equal_to_sequential": (None if seq is None else
                                        all(np.array_equal(a["loglik"], b["loglik"]) for a, b in zip(res, seq_res))),
        "replicate_factor_s": {"min": min(fac), "max": max(fac)},
        "status": [int(r["status"][0]) for r in res],
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": None,
                     "kernel": "k_level on one stream per replicate (whole-call average: algorithmic flops of "
                               "all factorisations / wall time)"},
    }
    for ds in dss:
        ds.close()
    ctx.close()
    print(json.dumps(out), flush=True)


def nm_trace(seed: int, length: int):
    """theta values a Nelder-Mead search proposes on a quadratic surrogate in
    log theta (centre and scales drawn from `seed`), in proposal order."""
    import numpy as np

    from paper_1709_04419_amd.mle import nelder_mead
    rng = np.random.default_rng(seed)
    centre = np.log([1.0, 0.1, 0.5]) + rng.uniform(-0.1, 0.1, 3)
    scale = rng.uniform(0.3, 1.0, 3)
    gen = nelder_mead(centre + rng.uniform(-0.2, 0.2, 3), step=0.1, ftol=0.0, xtol=0.0, max_evals=10 ** 6)
    out, x = [], next(gen)
    while len(out) < length:
        out.append(tuple(float(v) for v in np.exp(x)))
        x = gen.send(float(np.sum(((x - centre) / scale) ** 2)))
    return out


def accuracy(args):
    """Accuracy diagnostics in the style of Table 2 (Section 2.4): the perturbed
    grid of eq. 3 (n = m^2), exponential covariance (nu = 0.5) at two length
    scales, a list of eps: log-det error, KLD, ||I - C~^{-1} C||_2 (10 power
    steps) and storage, per (ell, eps)."""
    from paper_1709_04419_amd import diagnostics, hmlik
    from paper_1709_04419_amd import workloads as wl

    m = args.acc_m
    n = m * m
    P = wl.perturbed_grid(m, 7)
    ctx = hmlik.Context(0)
    rows = []
    try:
        ds = hmlik.Dataset(ctx, P, LEAF, ETA)
        ds.set_z(wl.standard_normal(n, 1, 8))
        for ell in (0.0334, 0.2337):
            theta = (1.0, ell, 0.5)
            t0 = time.perf_counter()
            for r in diagnostics.sweep(ds, theta, 0.0, eps_list=(1e-3, 1e-5, 1e-7, 1e-9), log=log):
                r["ell"] = ell
                rows.append(r)
                log(f"accuracy: ell {ell} eps {r['eps']:g}: " + (
                    f"logdet rel err {r['logdet_rel_err']:.2e}, KLD {r['kld']:.3e}, inverse error {r['inv_err']:.2e}, "
                    f"max rank {r['max_rank']}" if r["status"] == 0 else f"status {r['status']}"))
            log(f"accuracy: ell {ell} done in {time.perf_counter() - t0:.1f} s")
        ds.close()
    finally:
        ctx.close()
    print(json.dumps({"metric": "H-matrix accuracy diagnostics (Section 2.4, Table 2 style)", "form": "accuracy",
                      "data": "synthetic", "n": n, "points": f"perturbed grid (eq. 3), {m} x {m}, seed 7",
                      "nugget": 0.0, "leaf_size": LEAF, "eta": ETA, "rows": rows}), flush=True)


def mc(args):
    """Monte-Carlo study of theta-hat (Section 4, Fig. 3): replicates simulated
    on the device, FP64 fits through the request server, mixed fits one by one."""
    raise_hw_queues(min(16, args.replicates))   # one hardware queue per server slot
    from paper_1709_04419_amd import hmlik
    from paper_1709_04419_amd import mc_study

    ctx = hmlik.Context(0)
    try:
        th = tuple(float(v) for v in args.mc_theta.split(","))
        out = mc_study.run(ctx, args.mc_n, args.replicates, theta_true=th, nugget=args.mc_nugget, eps=args.eps,
                           mixed=(args.prec == "mixed"),
                           mixed_replicates=args.mc_mixed_replicates, max_evals=args.mc_max_evals,
                           refine_max_iter=args.refine_max_iter, refine_tol=args.refine_tol, log=log)
    finally:
        ctx.close()
    out.update(metric="Monte-Carlo theta-hat study (Section 4, Fig. 3)", form="mc", data="synthetic",
               n_gpus=1)
    print(json.dumps(out), flush=True)


def stream(args):
    """Open-loop Poisson request stream over resident datasets of different n."""
    D = max(2, args.datasets)
    raise_hw_queues(D)
    import numpy as np

    from paper_1709_04419_amd import hmlik
    from paper_1709_04419_amd import workloads as wl

    sizes = [int(round(16000 * 16 ** (i / (D - 1)))) for i in range(D)]
    ctx = hmlik.Context(0)
    dss = []
    for i, n_i in enumerate(sizes):
        ds = hmlik.Dataset(ctx, wl.basin_clusters(n_i, 5000 + i), LEAF, ETA)
        ds.set_z(wl.standard_normal(n_i, 1, 5050 + i))
        ds.release()                      # factor storage is attached on admission
        dss.append(ds)
    fb = [ds.footprint()["factor_bytes"] for ds in dss]
    log(f"{D} datasets, n = {sizes}; factor storage {sum(fb) / 2**30:.1f} GiB in all")
    traces = [nm_trace(5200 + i, args.requests) for i in range(D)]
    arrivals = np.cumsum(np.random.default_rng(5100).exponential(1.0 / args.rate, args.requests))
    which = np.random.default_rng(5101).integers(0, D, args.requests)
    sv = hmlik.Server(ctx, max_active=D, hbm_budget=int(args.budget_gib * 2 ** 30))
    nxt = [0] * D
    t0 = time.perf_counter()
    tickets, res, done_at = [], {}, {}
    last, j = t0, 0
    while len(res) < args.requests:
        now = time.perf_counter() - t0
        while j < args.requests and arrivals[j] <= now:
            d = int(which[j])
            th = traces[d][nxt[d]]
            nxt[d] += 1
            tickets.append((j, d, sv.submit(dss[d], th, NUGGET, args.eps, 0)))
            j += 1
        for (q, d, t) in tickets:
            if q not in res:
                r = sv.poll(t)
                if r is not None:
                    res[q] = (d, r)
                    done_at[q] = time.perf_counter() - t0
        if time.perf_counter() - last > 30:
            last = time.perf_counter()
            log(f"{j} arrived, {len(res)} done, {last - t0:.0f} s")
        time.sleep(0.005)
    sv.close()
    lat = np.array([res[q][1]["t_latency"] for q in range(args.requests)]) * 1e3
    span = max(done_at.values()) - arrivals[0]
    ok = sum(1 for q in res if res[q][1]["request_status"] in (hmlik.HM_OK, hmlik.HM_ERR_NOT_SPD))
    by_n = {}
    for d in range(D):
        v = [res[q][1]["t_latency"] * 1e3 for q in res if res[q][0] == d]
        if v:
            by_n[str(sizes[d])] = {"requests": len(v), "latency_ms_p50": float(np.median(v))}
    out = {
        "metric": METRIC,
        "value": ok / span,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.requests,
        "warmup": 0,
        "ms_per_step": span / args.requests * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "form": "stream",
        "config": {"workload": f"basin16k-256k_stream{D}", "sizes": sizes, "requests": args.requests,
                   "rate_per_s": args.rate, "hbm_budget_gib": args.budget_gib,
                   "factor_storage_gib": [round(b / 2 ** 30, 2) for b in fb], "slots": D,
                   "hw_queues": int(os.environ["GPU_MAX_HW_QUEUES"]), "eps": args.eps, "leaf_size": LEAF,
                   "eta": ETA, "nugget": NUGGET, "schedule": "longest-path levels",
                   "theta": "Nelder-Mead proposals on a quadratic surrogate around (1, 0.1, 0.5), seeds 5200+i"},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "by_n": by_n,
        "queue_ms_p50": float(np.percentile([res[q][1]["t_queue"] * 1e3 for q in res], 50)),
        "peak_batch": int(max(res[q][1]["peak_batch"] for q in res)),
        "status": sorted({int(res[q][1]["request_status"]) for q in res}),
        "attached_at_end": [bool(ds.footprint()["attached"]) for ds in dss],
    }
    for ds in dss:
        ds.close()
    ctx.close()
    print(json.dumps(out), flush=True)


def served(args):
    """The served form: continuous batching of evaluations over resident datasets."""
    if args.max_active <= 0:
        args.max_active = min(16, args.datasets)
    raise_hw_queues(args.max_active)
    import numpy as np

    from paper_1709_04419_amd import hmlik
    from paper_1709_04419_amd import workloads as wl

    n, eps = args.n, args.eps
    ctx = hmlik.Context(0)
    dss = []
    for i in range(args.datasets):
        ds = hmlik.Dataset(ctx, wl.basin_clusters(n, 31 + 10 * i), LEAF, ETA)
        ds.set_z(wl.standard_normal(n, 1, 32 + 10 * i))
        if not args.no_tune:
            s = time.perf_counter()
            ds.tune_schedule(THETA, NUGGET, eps, 0)
            log(f"dataset {i}: schedule tuned ({time.perf_counter() - s:.1f} s)")
        dss.append(ds)
    info = dss[0].info()
    rng = np.random.default_rng(5200)
    base = np.log(np.array(THETA))
    thetas = [tuple(np.exp(base + rng.uniform(-0.1, 0.1, 3))) for _ in range(args.requests)]
    sv = hmlik.Server(ctx, max_active=args.max_active)
    t0 = time.perf_counter()
    tickets = [sv.submit(dss[j % args.datasets], thetas[j], NUGGET, eps, 0) for j in range(args.requests)]
    res = [None] * len(tickets)
    last = time.perf_counter()
    while any(r is None for r in res):
        for j, t in enumerate(tickets):
            if res[j] is None:
                r = sv.poll(t)
                if r is not None:
                    res[j] = r
                    log(f"request {j + 1}/{args.requests}: status {r['request_status']}, latency "
                        f"{r['t_latency']:.1f} s, peak batch {r['peak_batch']}")
        if time.perf_counter() - last > 30:
            last = time.perf_counter()
            log(f"{sum(r is not None for r in res)} of {len(res)} requests done, {last - t0:.0f} s")
        time.sleep(0.01)
    wall = time.perf_counter() - t0
    sv.close()
    flops = sum(ds.factor_flops() for ds in dss) * args.requests / args.datasets
    done = sum(1 for r in res if r["request_status"] in (hmlik.HM_OK, hmlik.HM_ERR_NOT_SPD))
    lat = np.array([r["t_latency"] for r in res]) * 1e3
    achieved = flops / wall / 1e12
    out = {
        "metric": METRIC,
        "value": done / wall,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.requests,
        "warmup": 0,
        "ms_per_step": wall / args.requests * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "form": "served",
        "config": {"workload": ("basin256k" if n == 256000 else f"basin{n}") + "_served", "n": n,
                   "datasets": args.datasets, "requests": args.requests, "max_active": args.max_active,
                   "hw_queues": int(os.environ["GPU_MAX_HW_QUEUES"]),
                   "points": "basin_clusters(seeds 31, 41, ...)", "eps": eps, "leaf_size": LEAF, "eta": ETA,
                   "theta": "exp(log(1, 0.1, 0.325) + U(-0.1, 0.1)^3), seed 5200", "nugget": NUGGET,
                   "blocks": info["nblocks"], "tasks": info["ntasks"],
                   "schedule": "longest-path levels" if args.no_tune else "levels tuned per dataset (untimed)"},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "requests": [{"latency_s": r["t_latency"], "queue_s": r["t_queue"], "steps": r["steps"],
                      "peak_batch": r["peak_batch"], "status": r["request_status"],
                      "loglik": float(r["loglik"][0])} for r in res],
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": None,
                     "kernel": "k_level on one stream per request (whole-run average: algorithmic flops of "
                               "all factorisations / wall time)"},
    }
    for ds in dss:
        ds.close()
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
