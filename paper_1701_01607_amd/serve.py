"""Serving loop: a seeded Poisson stream of non-LTE solves of different sizes and atoms,
submitted through the C-ABI as they arrive and continuously batched by the library
(FIFO admission by device footprint, concurrent solves on separate HIP streams).

Reports p50/p99 time-to-convergence (arrival to result ready), atmospheres/hr over the
stream and the admission statistics.  Usage:

    python -m paper_1701_01607_amd.serve --requests 24 --max-running 4
    python -m paper_1701_01607_amd.serve --requests 100 --first 100 --rate 0.2 --max-size 4 > part2.log
    python -m paper_1701_01607_amd.serve --combine part1.log part2.log
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


def draw_stream(n, sizes, probs, seed=1607005):
    """The first n requests of the seeded stream: [(seed, size, two-level?), ...] and their
    inter-arrival gaps at unit rate (exponential, mean 1).  One generator gives request j's
    size, atom and gap in turn, so any contiguous part of the stream is the same whatever
    its length."""
    rng = np.random.default_rng(seed)
    draws, gaps = [], []
    for j in range(n):
        draws.append(draw_request(j, rng, sizes, probs))
        gaps.append(rng.exponential(1.0))
    return draws, np.array(gaps)


def arrival_times(gaps, rate_hz):
    """Arrival times of a part of the stream at the given rate, the first at 0."""
    t = np.cumsum(np.asarray(gaps, dtype=float) / rate_hz)
    return t - t[0] if len(t) else t


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


def run_stream(ctx, requests, arrivals, max_running=4, log=None, batch_max=1, prefetch=4):
    """Submit requests at the given arrival times (seconds from the start) while a
    collector thread releases each solve as soon as it is done (freeing its memory for
    queued ones); returns records.  A request is an (atom, atmosphere, params, tag) tuple
    or a callable that builds one; callables run on a producer thread up to `prefetch`
    requests ahead, so the host's input generation overlaps the stream."""
    import queue
    import threading
    ctx.serve_config(max_running)
    ctx.serve_batching(batch_max)
    pending, recs = [], []
    lock = threading.Lock()
    done_submitting = threading.Event()
    built = queue.Queue(maxsize=max(1, prefetch))

    def produce():
        for req in requests:
            try:
                built.put(req() if callable(req) else req)
            except BaseException as e:     # handed to the submitting thread, which raises it
                built.put(e)
                return

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

    producer = threading.Thread(target=produce, daemon=True)
    producer.start()
    th = threading.Thread(target=collect)
    th.start()
    t0 = time.monotonic()
    try:
        for ta in arrivals:
            item = built.get()
            if isinstance(item, BaseException):
                raise item
            atom, atm, p, tag = item
            while time.monotonic() - t0 < ta:
                time.sleep(min(0.005, ta - (time.monotonic() - t0)))
            A, M = ctx.atom(atom), ctx.atmos(atm)
            job = ctx.submit(M, A, p)
            with lock:
                pending.append((job, tag))
    finally:
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


def combine(parts):
    """Summary of a stream served in consecutive parts (each a list of records from its
    own run and clock): latencies pooled, makespans and busy time added."""
    parts = [p for p in parts if p]
    sums = [summarize(p) for p in parts]
    lat = np.array([r["latency_s"] for p in parts for r in p])
    span = sum(s["makespan_s"] for s in sums)
    n = sum(s["requests"] for s in sums)
    return {"requests": n, "converged": sum(s["converged"] for s in sums),
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "atmospheres_per_hr": 3600.0 * n / span, "makespan_s": span,
            "mean_queue_s": float(np.mean([r["queue_s"] for p in parts for r in p])),
            "device_busy_fraction": sum(s["device_busy_fraction"] * s["makespan_s"] for s in sums) / span,
            "parts": len(parts)}


def calibrate(ctx, sizes, probs):
    """Single-stream capacity of the mix: one solve of each size and atom alone (seeds
    outside the stream's); returns the mean run time of a request of the mix."""
    times = []
    for i, size in enumerate(sizes):
        cal = run_stream(ctx, [build_request(90000 + 2 * i + k, size, k == 0) for k in (0, 1)],
                         arrivals=[0.0, 0.0], max_running=1)
        by = {r["kind"]: r["run_s"] for r in cal}
        times.append((by["two-level"], by["six-level"]))
        print(json.dumps({"calibration": list(size), "run_s": by}), flush=True)
    return expected_run_time(times, probs)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--requests", type=int, default=24)
    ap.add_argument("--first", type=int, default=0,
                    help="serve requests first .. first+requests-1 of the seeded stream")
    ap.add_argument("--rate", type=float, default=0.0, help="arrivals per second (0: 80%% of measured capacity)")
    ap.add_argument("--max-running", type=int, default=4)
    ap.add_argument("--max-size", type=int, default=3, help="use the first N sizes of the mix")
    ap.add_argument("--batch", type=int, default=1,
                    help="continuous batching: compatible requests share batches of up to this many")
    ap.add_argument("--calibrate", type=int, default=0,
                    help="N > 0: only measure capacity: one solve of each size and atom alone (single-stream "
                         "capacity of the mix) and a burst of N requests of the mix submitted at once")
    ap.add_argument("--combine", nargs="+", default=None, metavar="LOG",
                    help="no GPU: summarise the records printed by runs of consecutive parts of a stream")
    args = ap.parse_args()
    if args.combine:
        parts = []
        for path in args.combine:
            with open(path) as f:
                parts.append([r for r in (json.loads(x) for x in f if x.startswith("{")) if "latency_s" in r])
        print(json.dumps(combine(parts)))
        return
    import torch
    torch.cuda.init()
    ctx = nlte.Context(0, torch.cuda.current_stream().cuda_stream)
    sizes = SIZES[: args.max_size]
    probs = np.array(SIZE_P[: args.max_size])
    probs = probs / probs.sum()
    draws, gaps = draw_stream(args.first + args.requests, sizes, probs)
    draws, gaps = draws[args.first:], gaps[args.first:]
    reqs = [lambda d=d: build_request(*d) for d in draws]
    rate = args.rate
    if args.calibrate > 0:
        single = calibrate(ctx, sizes, probs)
        bd, _ = draw_stream(args.calibrate, sizes, probs, seed=50000)
        burst = [lambda d=(50000 + j, size, two): build_request(*d) for j, (_, size, two) in enumerate(bd)]
        recs = run_stream(ctx, burst, arrivals=np.zeros(len(burst)), max_running=args.max_running,
                          batch_max=args.batch)
        out = summarize(recs)
        print(json.dumps({"single_stream_s_per_request": single, "single_stream_rate_80pct_hz": 0.8 / single,
                          "burst": out, "burst_rate_80pct_hz": 0.8 * len(recs) / out["makespan_s"],
                          "max_running": args.max_running, "batch_max": args.batch}))
        return
    if rate <= 0:
        rate = 0.8 / calibrate(ctx, sizes, probs)
    print(json.dumps({"stream": {"first": args.first, "requests": args.requests, "rate_hz": rate}}), flush=True)
    recs = run_stream(ctx, reqs, arrival_times(gaps, rate), max_running=args.max_running,
                      log=lambda r: print(json.dumps(r), flush=True), batch_max=args.batch)
    out = summarize(recs)
    out.update({"rate_hz": rate, "first": args.first, "max_running": args.max_running, "batch_max": args.batch,
                "sizes": sizes})
    print(json.dumps(out))


if __name__ == "__main__":
    main()
