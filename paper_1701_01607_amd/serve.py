"""Serving loop: a seeded Poisson stream of non-LTE solves of different sizes and atoms,
submitted through the C-ABI as they arrive and continuously batched by the library
(FIFO admission by device footprint, concurrent solves on separate HIP streams).

Reports p50/p99 time-to-convergence (arrival to result ready), atmospheres/hr over the
stream and the admission statistics.  Usage:

    python -m paper_1701_01607_amd.serve --requests 24 --max-running 4
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import nlte, synth

SIZES = [(32, 32, 33), (64, 64, 129), (128, 128, 129), (256, 256, 257)]
SIZE_P = [0.4, 0.3, 0.2, 0.1]


def draw_request(j, rng, sizes, probs):
    """(seed, size, two-level?) of request j: size drawn from `sizes`, two-level or
    six-level with equal odds, atmosphere seed 10000 + j."""
    size = sizes[rng.choice(len(sizes), p=probs)]
    two = rng.random() < 0.5
    return 10000 + j, size, two


def make_request(j, rng, sizes, probs):
    """(atom, atmosphere, params, tag) of request j (see draw_request)."""
    return build_request(*draw_request(j, rng, sizes, probs))


def build_request(seed, size, two):
    """(atom, atmosphere, params, tag) of one solve of the given size and atom kind."""
    nx, ny, nz = size
    atm = synth.atmos_stratified(nx=nx, ny=ny, nz=nz, dx=48 * synth.KM, seed=seed)
    if two:
        atom = synth.two_level_atom(1e-3)
        atm["chi_c"] = None
        atm["ntot"] = atm["ntot"] * 0.5
        p = nlte.SolveParams(method=nlte.FAS, precision=nlte.MIXED, nlev=3, nu0=0, nu1=2, nu2=2, nu3=32,
                             E_target=1e-3, max_iter=40)
    else:
        atom = synth.caii_like_atom(101)
        p = nlte.SolveParams(method=nlte.FAS, precision=nlte.MIXED, nlev=3, nu0=20, nu1=4, nu2=8, nu3=32,
                             E_target=1e-3, max_iter=40)
    return atom, atm, p, ("two-level" if two else "six-level", (nx, ny, nz))


def run_stream(ctx, requests, rate_hz, seed=1607005, max_running=4, log=None, batch_max=1):
    """Submit requests at Poisson arrival times while a collector thread releases each
    solve as soon as it is done (freeing its memory for queued ones); returns records.
    A request is an (atom, atmosphere, params, tag) tuple or a callable that builds one
    (called while waiting for its arrival time, so the host's input generation overlaps
    the stream)."""
    import threading
    ctx.serve_config(max_running)
    ctx.serve_batching(batch_max)
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=len(requests))
    arrivals = np.cumsum(gaps) - gaps[0]
    pending, recs = [], []
    lock = threading.Lock()
    done_submitting = threading.Event()

    def collect():
        while True:
            with lock:
                items = list(pending)
            if not items and done_submitting.is_set():
                return
            for item in items:
                job, tag = item
                if job.poll() >= nlte.JOB_DONE:
                    inf = job.info()
                    rec = {"kind": tag[0], "grid": tag[1], "status": inf.status,
                           "latency_s": inf.t_done - inf.t_submit, "queue_s": inf.t_admit - inf.t_submit,
                           "run_s": inf.t_done - inf.t_admit, "footprint_mb": inf.footprint / 2 ** 20,
                           "cycles": inf.result.cycles, "t_submit": inf.t_submit, "t_done": inf.t_done,
                           "batch": inf.batch, "fallback": inf.result.fallback}
                    job.close()
                    with lock:
                        pending.remove(item)
                        recs.append(rec)
                    if log:
                        log(rec)
            time.sleep(0.002)

    th = threading.Thread(target=collect)
    th.start()
    t0 = time.monotonic()
    for req, ta in zip(requests, arrivals):
        atom, atm, p, tag = req() if callable(req) else req
        while time.monotonic() - t0 < ta:
            time.sleep(min(0.005, ta - (time.monotonic() - t0)))
        A, M = ctx.atom(atom), ctx.atmos(atm)
        job = ctx.submit(M, A, p)
        with lock:
            pending.append((job, tag))
    done_submitting.set()
    th.join()
    return recs


def expected_run_time(times, probs):
    """Mean single-stream run time of a request of the mix: times[i] = (two-level, six-level)
    run times of size i, probs[i] the size's odds, the two atoms equally likely."""
    return float(sum(p * 0.5 * (t2 + t6) for p, (t2, t6) in zip(probs, times)))


def busy_fraction(recs, t0, t1):
    """Fraction of [t0, t1] during which at least one solve was running on the device."""
    iv = sorted((r["t_submit"] + r["queue_s"], r["t_done"]) for r in recs)
    busy, cur_a, cur_b = 0.0, None, None
    for a, b in iv:
        if cur_b is None or a > cur_b:
            if cur_b is not None:
                busy += cur_b - cur_a
            cur_a, cur_b = a, b
        else:
            cur_b = max(cur_b, b)
    if cur_b is not None:
        busy += cur_b - cur_a
    return busy / (t1 - t0) if t1 > t0 else 0.0


def summarize(recs):
    lat = np.array([r["latency_s"] for r in recs])
    t0 = min(r["t_submit"] for r in recs)
    t1 = max(r["t_done"] for r in recs)
    span = t1 - t0
    return {"requests": len(recs), "converged": int(sum(r["status"] == 0 for r in recs)),
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "atmospheres_per_hr": 3600.0 * len(recs) / span, "makespan_s": span,
            "mean_queue_s": float(np.mean([r["queue_s"] for r in recs])),
            "device_busy_fraction": busy_fraction(recs, t0, t1)}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--requests", type=int, default=24)
    ap.add_argument("--rate", type=float, default=0.0, help="arrivals per second (0: 80%% of measured capacity)")
    ap.add_argument("--max-running", type=int, default=4)
    ap.add_argument("--max-size", type=int, default=3, help="use the first N sizes of the mix")
    ap.add_argument("--batch", type=int, default=1,
                    help="continuous batching: compatible requests share batches of up to this many")
    args = ap.parse_args()
    import torch
    torch.cuda.init()
    ctx = nlte.Context(0, torch.cuda.current_stream().cuda_stream)
    sizes = SIZES[: args.max_size]
    probs = np.array(SIZE_P[: args.max_size])
    probs = probs / probs.sum()
    rng = np.random.default_rng(1607005)
    draws = [draw_request(j, rng, sizes, probs) for j in range(args.requests)]
    reqs = [lambda d=d: build_request(*d) for d in draws]
    rate = args.rate
    if rate <= 0:
        # capacity: one solve of each size and atom alone (seeds outside the stream's), the
        # mean run time of a request of the mix from the size odds, and 80 % of its inverse
        times = []
        for i, size in enumerate(sizes):
            cal = run_stream(ctx, [build_request(90000 + 2 * i + k, size, k == 0) for k in (0, 1)],
                             rate_hz=1e6, max_running=1)
            by = {r["kind"]: r["run_s"] for r in cal}
            times.append((by["two-level"], by["six-level"]))
            print(json.dumps({"calibration": list(size), "run_s": by}), flush=True)
        rate = 0.8 / expected_run_time(times, probs)
    recs = run_stream(ctx, reqs, rate_hz=rate, max_running=args.max_running,
                      log=lambda r: print(json.dumps(r), flush=True), batch_max=args.batch)
    out = summarize(recs)
    out.update({"rate_hz": rate, "max_running": args.max_running, "batch_max": args.batch, "sizes": sizes})
    print(json.dumps(out))


if __name__ == "__main__":
    main()
