"""Benchmark: online-DMD rank-1 updates/s and HBM GB/s at n = 160,000.

Workload: a cylinder-wake-shaped synthetic stream on a 400 x 200 (u, v)
grid (n = 160,000), 2000 snapshots, relative noise 1e-6, r_max = 40,
tol = 1e-8, FP64 basis and snapshots.  All snapshots are resident in HBM
before timing starts.

One step = the whole hot path over the stream: 1999 chained rank-1
updates (projection, CGS2, core SVD, basis rotation, A~), the
eigendecomposition of A~, and a 500-state rollout, on a fresh model.
value = updates per second over the timed steps.

Printed beside it (one JSON line): the streaming pass's roofline (its
algorithmic bytes n (r + r') 8 + 2 n 8 per update divided by its average
HIP-event duration, against 8 TB/s), p50/p99 device latency of one update,
and the CPU oracle timed on a bounded sample on this host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "online-DMD rank-1 updates/s + HBM GB/s at n=160k; p50/p99 update latency"
NX, NY, SNAPS, R_MAX, TOL, NOISE = 400, 200, 2000, 40, 1e-8, 1e-6
ROLLOUT = 500
PEAK_HBM_GBPS = 8000.0
STEADY_FROM = 100          # updates after which the rank has saturated at r_max


def make_stream():
    from paper_2311_18715_amd import synth
    s = synth.wake(nx=NX, ny=NY, noise=NOISE)
    return s, s.snapshots(0, SNAPS)


PROFILE = os.path.join(ROOT, "profiles", "k_pass_f64_r40_wake_n160k.md")
PASS_SOURCES = ("pass.hip", "pass.h", "odmd_internal.h")


def measured_traffic():
    """HBM bytes per pass launch from the committed rocprofv3 counter summary,
    or None when the pass sources changed since the counters were taken."""
    import hashlib
    import re
    try:
        text = open(PROFILE).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for f in PASS_SOURCES:
        with open(os.path.join(ROOT, "paper_2311_18715_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    m_sha = re.search(r"kernel_source_sha256: ([0-9a-f]+)", text)
    m_bytes = re.search(r"traffic_bytes_per_launch: (\d+)", text)
    if not m_sha or not m_bytes or m_sha.group(1) != h.hexdigest():
        return None
    return int(m_bytes.group(1))


def cpu_baseline(X, seconds: float = 15.0):
    """The FP64 oracle on this host: warm up to the saturated rank, then time
    as many updates as fit in about `seconds` (at least 5)."""
    from oracle import odmd_oracle as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    o = O.OnlineDMD(X.shape[0], R_MAX, TOL)
    k = 0
    while o.r < R_MAX and k < 200:
        o.update(X[:, k], X[:, k + 1])
        k += 1
    k0, t0 = k, time.perf_counter()
    while k < X.shape[1] - 1:
        o.update(X[:, k], X[:, k + 1])
        k += 1
        if time.perf_counter() - t0 > seconds and k - k0 >= 5:
            break
    dt = time.perf_counter() - t0
    return {"value": (k - k0) / dt, "unit": "updates/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{k - k0} consecutive updates of the same n={X.shape[0]} stream at the "
                      f"saturated rank {R_MAX} (after {k0} warm-up updates), FP64 NumPy/LAPACK"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after timing, copy MIB MiB once on the device (a reference "
                         "kernel of known traffic for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2311_18715_amd.odmd import ODMD

    torch.cuda.set_device(0)
    _, X = make_stream()
    n = X.shape[0]
    Xd = torch.from_numpy(np.ascontiguousarray(X.T)).to("cuda")
    out = torch.empty((ROLLOUT, n), dtype=torch.float64, device="cuda")
    m = SNAPS - 1
    models = [ODMD(n, R_MAX, TOL) for _ in range(args.warmup + args.steps)]
    torch.cuda.synchronize()

    cap = m - STEADY_FROM
    for g in models:                    # create the timing events up front
        g.profile(cap)
        g.profile(0)

    def one_step(g, profile):
        for k in range(m):
            if profile and k == STEADY_FROM:
                g.profile(cap)
            g.update(Xd[k], Xd[k + 1])
        g.profile(0)
        g.eigs(vectors=False)           # synchronising
        g.predict(ROLLOUT, out=out)

    for i in range(args.warmup):
        one_step(models[i], False)
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    for i in range(args.steps):
        one_step(models[args.warmup + i], True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    pass_ms, core_ms = [], []
    for i in range(args.steps):
        a, b = models[args.warmup + i].profile_samples()
        pass_ms.append(a)
        core_ms.append(b)
    pass_ms, core_ms = np.concatenate(pass_ms), np.concatenate(core_ms)
    for g in models:
        g.sync()
    infos = [g.info() for g in models]
    assert all(i.r == R_MAX for i in infos), [i.r for i in infos]

    updates = args.steps * m
    value = updates / elapsed
    bytes_upd = n * (R_MAX + R_MAX) * 8 + 2 * n * 8      # read U, write U', read x, y
    pass_avg_s = float(np.mean(pass_ms)) * 1e-3
    achieved = bytes_upd / pass_avg_s / 1e9
    lat = (pass_ms + core_ms) * 1e3
    result = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"cylinder-wake-shaped stream, n={n} (u,v on {NX}x{NY}), {SNAPS} snapshots, "
                        f"noise {NOISE:g}, r_max={R_MAX}, tol={TOL:g}, FP64; step = {m} updates + "
                        f"eigs + {ROLLOUT}-state rollout",
            "n": n, "r_max": R_MAX, "snapshots": SNAPS, "rollout": ROLLOUT,
        },
        "hbm_gbps_whole_step": round(value * bytes_upd / 1e9, 1),
        "latency_us": {"p50": round(float(np.percentile(lat, 50)), 2),
                       "p99": round(float(np.percentile(lat, 99)), 2),
                       "samples": int(lat.size)},
        "phase_us": {"pass_mean": round(float(np.mean(pass_ms)) * 1e3, 2),
                     "core_mean": round(float(np.mean(core_ms)) * 1e3, 2)},
        "roofline": {
            "bound": "hbm",
            "kernel": "k_pass<double,double,40> (streaming pass)",
            "achieved": round(achieved, 1),
            "peak": PEAK_HBM_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBPS, 4),
            "bytes_per_launch": bytes_upd,
            "launches_timed": int(pass_ms.size),
            "traffic": measured_traffic(),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        },
    }
    if args.calibrate_copy > 0:
        a = torch.ones(args.calibrate_copy << 17, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        result["calibration_copy_bytes"] = 2 * a.numel() * 8
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(X)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
