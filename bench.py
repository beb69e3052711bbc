#!/usr/bin/env python
"""Benchmark: voxel-angle-frequency updates/s and converged atmospheres/hr, FAS/FMG with
an FP32 sweep against plain FP64 MALI, on one MI355X.

Default workload, caii6_504x504x497: the six-level atom (5 lines x 101 frequencies, 24
directions) on the 504x504x497 radiation-MHD-like atmosphere with 20 km spacing (126M
voxels), the largest configuration one GPU holds.  Its full-multigrid job (4 grids, FP32
sweep, FP64 rates and populations) is built before the timed region: atmosphere,
hierarchy, level constants and zero-radiation populations resident in HBM.  A step is
one finest-grid MALI iteration of that job - the FP32 formal solution over every voxel,
direction and frequency, then the FP64 rate solve at every voxel - the paper's unit of
cost (Sect. 4.9).  value = updates of one finest-grid formal solution / step time.  The
line also carries the projected atmospheres/hr of the whole solve at this size (the
step time times the solve's measured work in finest-grid formal solutions), the
64x64x129 workload's whole FAS solve timed end to end (atmospheres/hr), its plain
MALI-FP64 comparison and the FP32 path's error per result against the FP64 path there.

--workload caii6_64x64x129 makes a step one whole solve of that workload instead
(setup, zero-radiation start, 3-level FAS V-cycles to rho/(1-rho) C <= 1e-3, emergent
intensity).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3        # MI355X vector FP32 (published)
PEAK_HBM_GBS = 8000.0           # MI355X HBM3E (published)
PEAK_FP64_TFLOPS = 78.6         # MI355X vector FP64 (published)
# FP32 FMAs without the packed (two per lane) form, which this code does not use:
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz.
PEAK_FP32_UNPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12

# Algorithmic HBM bytes per voxel-direction-frequency update of the sweep.  The plane
# state (one cell per direction, frequency and plane point: I and phi, 8 B, in FP32;
# I, S and chi, 24 B, in FP64) lives in HBM between plane steps: each cell is written
# once and read back once by the next step (its four upwind readers share it through
# L2).  Per (voxel, line, direction group) the block also reads 11 per-voxel constants
# and writes 2 partial sums.
STATE_BYTES_PER_UPDATE = {False: 16.0, True: 48.0}   # keyed by "FP64 sweep"
# HBM bytes per update of the finest-grid sweep launches from FETCH_SIZE + WRITE_SIZE
# counter runs of `bench.py --kernel-probe` (each scaled by the counter's reading for a
# plain device copy of known size), keyed by (workload, directions per block).  Only for
# the kernel as it was when the counters were taken: FETCH 9.35 B + WRITE 8.03 B on the
# 504x504x497 grid with three-direction blocks and non-temporal cell stores (each upwind
# cell reaches HBM about 1.17 times for its four readers).
MEASURED_BYTES_PER_UPDATE = {("caii6_504x504x497", 3): 17.38}
VOXEL_BYTES_PER_GROUP = (11 + 2) * 4.0   # FP32; twice that in FP64

# Algorithmic flops per update (FMA = 2; a reciprocal, exponential or cosine = 1) of the
# linear short-characteristics update: profile argument 2, opacity and source function 7,
# three bilinear interpolations 21, optical depth 3, segment coefficients 7, intensity 5,
# quadrature weight 2, accumulations 10 (57, the ~60 of the scope table's count); plus
# the line profile as evaluated: the Weideman N=32 series (run in FP64) 154, the FP32
# small-damping series (a < 0.04, |u| < 5) 35, the FP32 asymptotic wing with its Gaussian
# term 64, a pure Gaussian 3.  The FP32 cells' rebuild of the upwind corners' opacity and
# source function from phi is storage-format work, not the method's, and is not counted.
FLOPS_PER_UPDATE_BASE = 57
FLOPS_VOIGT_CORE, FLOPS_VOIGT_SMALL, FLOPS_VOIGT_WING, FLOPS_GAUSS = 154, 35, 64, 3
VOIGT_SMALL_A = 0.04

# Work of the whole FMG solve of caii6_504x504x497 in finest-grid formal-solution
# equivalents (4 cycles to rho/(1-rho) C <= 1e-3), measured by one full solve on the
# GPU (nlte_result.fine_fs_equiv); the projected atmospheres/hr uses it.
M4_FINE_FS_EQUIV = 61.8

WORKLOADS = {
    "caii6_64x64x129": dict(nlev=3, nu0=20, nu1=4, nu2=8, nu3=32, nu_fmg=16, method="FAS", fp64=False,
                            E_target=1e-3, tol_C=0.0),
    "caii6_256x256x257": dict(nlev=4, nu0=20, nu1=4, nu2=8, nu3=32, nu_fmg=16, method="FMG", fp64=False,
                              E_target=1e-3, tol_C=0.0),
    "caii6_504x504x497": dict(nlev=4, nu0=20, nu1=4, nu2=8, nu3=32, nu_fmg=16, method="FMG", fp64=False,
                              E_target=1e-3, tol_C=0.0),
    # plain FP64 MALI to a maximum relative correction of 1e-4
    "two_level_16x16x32": dict(nlev=1, nu0=0, nu1=2, nu2=2, nu3=32, nu_fmg=16, method="MALI", fp64=True,
                               E_target=0.0, tol_C=1e-4),
}
STEP_IS_FINE_ITERATION = {"caii6_504x504x497"}
METRIC = "converged atmospheres/hr + voxel-angle-freq updates/s, FAS-FP32 vs MALI-FP64"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def flops_per_update(atom, atm, fp64, nsample=6000):
    """Mean algorithmic flops per update on the finest grid: in FP32 sweeps the profile
    costs the small-damping series where |u| < 5 and the damping a < 0.04, the Weideman
    series where |u| < 5 otherwise (everywhere in FP64 sweeps) and the asymptotic wing
    elsewhere, so the fractions are counted on a sample of voxels over all directions and
    frequencies.  Returns (flops per update, fraction of Weideman series evaluations)."""
    import numpy as np
    kb, amu, c_light = 1.380649e-16, 1.66053906660e-24, 2.99792458e10
    nvox = np.asarray(atm["T"]).size
    sl = slice(None, None, max(1, nvox // nsample))
    T = np.asarray(atm["T"], dtype=np.float64).ravel()[sl]
    nH = np.asarray(atm["nH"], dtype=np.float64).ravel()[sl]
    vD = np.sqrt(2.0 * kb * T / (atom["mass_amu"] * amu) + atom["xi"] ** 2)
    v = np.stack([np.asarray(atm[c], dtype=np.float64).ravel()[sl] for c in ("vx", "vy", "vz")])
    m1, m2 = 1.0 / 3.0, np.sqrt(7.0) / 3.0
    up = [(sx * a, sy * b, c) for sx, sy in ((1, 1), (1, -1), (-1, 1), (-1, -1))
          for a, b, c in ((m1, m1, m2), (m1, m2, m1), (m2, m1, m1))]
    mus = np.array(up + [(-a, -b, -c) for a, b, c in up])
    vn = mus @ v                                                   # [24][sample]
    total = core = 0.0
    flops = 0.0
    base = FLOPS_PER_UPDATE_BASE
    for ln in atom["lines"]:
        q = np.asarray(ln["q"], dtype=np.float64)
        n = q.size * vn.size
        total += n
        if not (ln["gamma_rad"] or ln["gamma_vdw"]):
            flops += n * (base + FLOPS_GAUSS)
            continue
        u = (q[:, None, None] - vn[None]) / vD[None, None]
        if fp64:
            core += n
            flops += n * (base + FLOPS_VOIGT_CORE)
            continue
        lv = atom["levels"]
        nu0 = c_light * (lv[ln["upper"]]["E"] - lv[ln["lower"]]["E"])
        gam = ln["gamma_rad"] + ln["gamma_vdw"] * nH * (T / 5000.0) ** 0.3
        small = (gam / (4.0 * np.pi * nu0 * vD / c_light) < VOIGT_SMALL_A)[None, None]
        inside = np.abs(u) < 5.0
        cs = float(np.count_nonzero(inside & small))
        c = float(np.count_nonzero(inside)) - cs
        core += c
        flops += n * base + cs * FLOPS_VOIGT_SMALL + c * FLOPS_VOIGT_CORE + (n - c - cs) * FLOPS_VOIGT_WING
    return flops / total, core / total


# ------------------------------------------------------------------ oracle beside it
_CPU = {}   # the oracle level and populations shared with forked workers


def _oracle_fs_part(dirs):
    from oracle.formal import formal_solution
    return formal_solution(_CPU["lev"], _CPU["n"], dirs=dirs)


def _oracle_norm_part(dirs):
    return _CPU["lev"].norm_sum(dirs)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_sample(nx=32, nfreq=7, workers=None):
    """The FP64 oracle's MALI iteration (formal solution over all 24 directions, then the
    rate solve) timed on a bounded sample of the default workload: the same generator and
    seed at 20 km spacing, all 497 planes, a 32x32 horizontal patch and 7 frequencies per
    line.  The 24 directions are dealt to forked workers (min(24, cores, 16)); the profile
    normalisation (set-up) is computed the same way beforehand and not timed.  Runs before
    the GPU is initialised."""
    import multiprocessing as mp

    import numpy as np

    from oracle.levels import Level
    from oracle.rates import fine_rhs, solve, zero_radiation
    from paper_1701_01607_amd import synth
    atom = synth.caii_like_atom(nfreq)
    atm = synth.atmos_rmhd_like(nx=nx, ny=nx, nz=497, dx=20.0 * synth.KM, seed=1607004)
    lev = Level(atom, atm)
    n0 = zero_radiation(lev)
    cores = os.cpu_count() or 1
    w = workers or max(1, min(24, cores, 16))
    chunks = [tuple(range(24))[i::w] for i in range(w)]
    _CPU["lev"], _CPU["n"] = lev, n0
    ctx = mp.get_context("fork")
    with ctx.Pool(w) as pool:
        lev._norm = 1.0 / np.sum(pool.map(_oracle_norm_part, chunks), axis=0)
    with ctx.Pool(w) as pool:
        t0 = time.perf_counter()
        parts = pool.map(_oracle_fs_part, chunks)
        Jeff = np.sum([p[0] for p in parts], axis=0)
        omL = np.sum([p[1] for p in parts], axis=0)
        t1 = time.perf_counter()
    solve(lev, Jeff, omL, fine_rhs(lev))
    t2 = time.perf_counter()
    updates = lev.nx * lev.ny * lev.nz * 24 * lev.nf
    return {"updates": updates, "t_fs": t1 - t0, "t_rates": t2 - t1, "workers": w, "cores": cores,
            "shape": (lev.nx, lev.ny, lev.nz), "nf": lev.nf}


def cpu_baseline(sample, fine_updates, fine_fs_equiv):
    """The oracle's updates/s on the sample (formal solution + rate solve of one MALI
    iteration), and the atmospheres/hr it would reach at the same work per solve as the
    GPU's (projected linearly from the sample)."""
    ups = sample["updates"] / (sample["t_fs"] + sample["t_rates"])
    nx, ny, nz = sample["shape"]
    return {
        "value": ups, "unit": "voxel-angle-freq updates/s", "cores": sample["workers"], "kind": "oracle",
        "sample": f"one FP64 MALI iteration of the oracle (formal solution, 24 A4 directions over "
                  f"{sample['workers']} forked workers, {sample['t_fs']:.1f} s; rate solve in the parent, "
                  f"{sample['t_rates']:.1f} s) on the default workload's generator at {nx}x{ny}x{nz}, "
                  f"{sample['nf']} frequencies (7 per line); profile normalisation precomputed",
        "projected_atmospheres_per_hr": 3600.0 / (fine_fs_equiv * fine_updates / ups),
        "host": {"nproc": sample["cores"], "cpu_model": cpu_model()},
    }


# ------------------------------------------------------------------ helpers
def roofline(atom, atm, fp64, upd, ms_sweep, launches, dirs_per_block, workload):
    fl, core_frac = flops_per_update(atom, atm, fp64)
    nf = sum(len(l["q"]) for l in atom["lines"])
    nslot = 24 // dirs_per_block if dirs_per_block else 8
    nfl = nf / len(atom["lines"])
    wbytes = 2.0 if fp64 else 1.0
    bytes_upd = STATE_BYTES_PER_UPDATE[fp64] + wbytes * VOXEL_BYTES_PER_GROUP * nslot / (24.0 * nfl)
    peak_alu = PEAK_FP64_TFLOPS if fp64 else PEAK_FP32_TFLOPS
    if not ms_sweep or not launches:
        return None
    avg_launch_us = 1e3 * ms_sweep / launches
    per_launch = upd / launches
    achieved_alu = per_launch * fl / (avg_launch_us * 1e-6) / 1e12
    achieved_hbm = per_launch * bytes_upd / (avg_launch_us * 1e-6) / 1e9
    measured = MEASURED_BYTES_PER_UPDATE.get((workload, dirs_per_block))
    traffic = per_launch * measured / (avg_launch_us * 1e-6) / 1e9 if measured else None
    return {"bound": "alu", "achieved": achieved_alu, "peak": peak_alu, "unit": "TFLOP/s",
            "frac": achieved_alu / peak_alu, "traffic": traffic,
            "traffic_unit": "GB/s (measured HBM bytes per launch / average launch time)",
            "traffic_bytes_per_update": measured,
            "kernel": f"sweep_step_kernel<{'double' if fp64 else 'float'},{dirs_per_block}>",
            "avg_launch_us": avg_launch_us, "launches": launches, "updates_per_launch": per_launch,
            "flops_per_update": fl, "voigt_core_fraction": core_frac,
            "unpacked_fp32": None if fp64 else
            {"peak": PEAK_FP32_UNPACKED_TFLOPS, "frac": achieved_alu / PEAK_FP32_UNPACKED_TFLOPS},
            "hbm": {"achieved": achieved_hbm, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": achieved_hbm / PEAK_HBM_GBS, "bytes_per_update": bytes_upd}}


def hbm_copy_gbs(torch):
    """This box's achievable HBM bandwidth for context: a 2 GiB device-to-device copy."""
    src = torch.empty(2 ** 29, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    out = 5 * 2 * src.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return out


def solve_params(nlte, wl, **kw):
    method = {"FAS": nlte.FAS, "FMG": nlte.FMG, "MALI": nlte.MALI}[wl["method"]]
    p = dict(method=method, precision=nlte.FP64 if wl["fp64"] else nlte.MIXED, nlev=wl["nlev"],
             nu0=wl["nu0"], nu1=wl["nu1"], nu2=wl["nu2"], nu3=wl["nu3"], nu_fmg=wl["nu_fmg"],
             E_target=wl["E_target"], tol_C=wl["tol_C"], max_iter=60 if method != nlte.MALI else 2000, timing=1)
    p.update(kw)
    return nlte.SolveParams(**p)


def solve_extras(nlte, ctx, torch, np, name="caii6_64x64x129", solves=2, mali_max_iter=800, fp32_error=True):
    """A workload solved end to end with the FP32 sweep (atmospheres/hr over `solves`
    timed solves after a warm-up one), the plain MALI-FP64 solve of the same atmosphere
    beside it, and (fp32_error) the FP32 error per result (populations, line source
    functions, emergent intensity) against the FP64 path run with the same cycles."""
    from paper_1701_01607_amd import synth
    wl = WORKLOADS[name]
    atom, atm = synth.workload(name)
    A, M = ctx.atom(atom), ctx.atmos(atm)
    N, L = len(atom["levels"]), len(atom["lines"])
    nf = sum(len(l["q"]) for l in atom["lines"])
    sh = (N, atm["nz"], atm["ny"], atm["nx"])
    mu = np.array([[0.0, 0.0, 1.0]])

    def solve(prec, **kw):
        job = ctx.job(M, A, solve_params(nlte, wl, precision=prec, **kw))
        rc, r = job.run()
        n = job.populations(wl["nlev"] - 1, sh)
        S = job.source_function((L,) + sh[1:])
        I = job.emergent(mu, nf, atm["ny"], atm["nx"])
        job.close()
        return rc, r, n, S, I

    solve(nlte.MIXED)                       # warm-up (autotune of the three level shapes)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(solves):
        rc, r, n32, S32, I32 = solve(nlte.MIXED)
    torch.cuda.synchronize()
    t_solve = (time.perf_counter() - t0) / solves
    log(f"{name} {wl['method']}-FP32: rc={rc} cycles={r.cycles} E_est={r.E_est:.3e} {t_solve:.2f} s per solve")
    err = None
    if fp32_error:
        _, r64, n64, S64, I64 = solve(nlte.FP64, E_target=0.0, max_iter=r.cycles)
        ok = np.isfinite(S64) & np.isfinite(S32)
        err = {"n": float(np.max(np.abs(n32 / n64 - 1))),
               "S_l": float(np.max(np.abs(S32[ok] / S64[ok] - 1))),
               "I_top": float(np.max(np.abs(I32.astype(np.float64) / I64.astype(np.float64) - 1))),
               "reference": f"{wl['method']} with the FP64 sweep, the same {r.cycles} cycles",
               "n_tiny_excluded": False}
    mp = nlte.SolveParams(method=nlte.MALI, precision=nlte.FP64, nlev=1, E_target=1e-3, max_iter=mali_max_iter,
                          timing=1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    job = ctx.job(M, A, mp)
    rcm, rm = job.run()
    torch.cuda.synchronize()
    tm = time.perf_counter() - t1
    nm = job.populations(0, sh)
    job.close()
    log(f"{name} MALI-FP64: rc={rcm} iterations={rm.iterations} E_est={rm.E_est:.3e} {tm:.1f} s")
    return {"workload": name, "atmospheres_per_hr": 3600.0 / t_solve, "seconds_per_solve": t_solve,
            "converged": rc == 0, "cycles": r.cycles, "E_est": r.E_est, "fine_fs_equiv": r.fine_fs_equiv,
            "fp32_error_vs_fp64": err,
            "mali_fp64": {"seconds": tm, "iterations": rm.iterations, "converged": rcm == 0, "E_est": rm.E_est,
                          "atmospheres_per_hr": 3600.0 / tm, "speedup_fp32_multigrid": tm / t_solve,
                          "max_rel_diff_vs_fas": float(np.max(np.abs(n32 / nm - 1)))}}


def batch_bench(args):
    """--batch N: N small solves of one kind, run one after another (each alone) and then as
    one batch (nlte_batch_run: shared work-list sweep launches).  Kinds: the two-level
    16x16x32 workload (plain FP64 MALI to C <= 1e-4; the N atmospheres differ in density)
    or six-level 16x16x33 stratified atmospheres (FAS, FP32 sweep, 3 grids; N seeds)."""
    import numpy as np
    import torch

    from paper_1701_01607_amd import nlte, synth
    n = args.batch
    inputs = []
    if args.workload == "two_level_16x16x32":
        wl = WORKLOADS[args.workload]
        for j in range(n):
            atom, atm = synth.workload(args.workload)
            atm["ntot"] = atm["ntot"] * (0.5 + j / max(1, n - 1))
            inputs.append((atom, atm))
        params = solve_params(nlte, wl, graph=int(args.graph), timing=0 if args.graph else 1)
        kind = "two_level_16x16x32 x %d (MALI FP64, tol_C 1e-4)" % n
    else:
        for j in range(n):
            atm = synth.atmos_stratified(nx=16, ny=16, nz=33, dx=150 * synth.KM, seed=1607100 + j)
            inputs.append((synth.caii_like_atom(101), atm))
        params = nlte.SolveParams(method=nlte.FAS, precision=nlte.MIXED, nlev=3, nu0=20, nu1=4, nu2=8, nu3=32,
                                  E_target=1e-3, max_iter=60, timing=0 if args.graph else 1, graph=int(args.graph))
        kind = "caii6_16x16x33 x %d (FAS FP32, 3 grids, E <= 1e-3)" % n
    torch.cuda.init()
    ctx = nlte.Context(0, torch.cuda.current_stream().cuda_stream)
    handles = [(ctx.atmos(atm), ctx.atom(atom)) for atom, atm in inputs]

    def alone():
        out = []
        for M, A in handles:
            j = ctx.job(M, A, params)
            rc, r = j.run()
            out.append((r, j.history()))
            j.close()
        return out

    def batched():
        jobs = [ctx.job(M, A, params) for M, A in handles]
        rc, res = ctx.batch_run(jobs)
        hist = [j.history() for j in jobs]
        for j in jobs:
            j.close()
        return list(zip(res, hist))

    for fn in (alone, batched):      # warm-up: autotuning and first launches
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ra = alone()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rb = batched()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    same = all(np.array_equal(ha, hb) for (_, ha), (_, hb) in zip(ra, rb))
    la = sum(r.sweep_launches for r, _ in ra)
    sa = sum(r.ms_sweep for r, _ in ra)
    # replayed graphs are not timed: launch times only for eager runs
    per_launch = (lambda ms, n_: 1e3 * ms / n_ if n_ and not args.graph else None)
    out = {"metric": "batched small solves", "kind": kind, "n": n, "graph": bool(args.graph),
           "alone": {"seconds": t1 - t0, "atmospheres_per_hr": 3600.0 * n / (t1 - t0),
                     "sweep_launches": la, "sweep_ms": sa, "us_per_launch": per_launch(sa, la)},
           "batched": {"seconds": t2 - t1, "atmospheres_per_hr": 3600.0 * n / (t2 - t1),
                       "sweep_ms": rb[0][0].ms_sweep,
                       # one launch per plane step and chunk class: the longest job's count
                       "sweep_launches": max(r.sweep_launches for r, _ in rb),
                       "us_per_launch": per_launch(rb[0][0].ms_sweep, max(r.sweep_launches for r, _ in rb))},
           "speedup": (t1 - t0) / (t2 - t1), "histories_equal": same,
           "iterations_or_cycles": [max(r.iterations, r.cycles) for r, _ in ra]}
    print(json.dumps(out))


# ------------------------------------------------------------------ main
def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="caii6_504x504x497", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mali", action="store_true", help="skip the whole solves reported beside the steps")
    ap.add_argument("--no-fp32-error", action="store_true",
                    help="other workloads: skip the FP64 solve with the same cycles that measures the FP32 error")
    ap.add_argument("--mali-max-iter", type=int, default=800)
    ap.add_argument("--dirs-per-block", type=int, default=0, help="sweep block shape (0: autotune)")
    ap.add_argument("--graph", type=int, default=0, help="1: replay V-cycles from a captured HIP graph")
    ap.add_argument("--active-continua", action="store_true",
                    help="sweep the atom's continua as active transitions (41 continuum frequencies); the "
                         "line-sweep roofline is then not reported")
    ap.add_argument("--seven-level", action="store_true",
                    help="the workload's atmosphere with the seven-level atom, whose continua end on two upper "
                         "levels (with --active-continua: continuum sweeps with two upper levels); no "
                         "roofline or CPU baseline")
    ap.add_argument("--batch", type=int, default=0,
                    help="N > 0: time N small solves (two_level_16x16x32 with that workload, else six-level "
                         "16x16x33) one after another and as one batch; prints its own JSON line")
    ap.add_argument("--kernel-probe", action="store_true",
                    help="only one MALI iteration (one formal solution + rate solve) and a 512 MiB "
                         "device copy, for hardware-counter runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU (one process per GPU); nothing here uses a "
                                   "second one, so --gpus must be 1"}))
        sys.exit(2)

    if args.batch > 0:
        batch_bench(args)
        return

    import numpy as np

    wl = WORKLOADS[args.workload]
    fine_step = args.workload in STEP_IS_FINE_ITERATION
    from paper_1701_01607_amd import synth
    log(f"generating {args.workload} ...")
    t_gen = time.perf_counter()
    atom, atm = synth.workload(args.workload)
    log(f"generated in {time.perf_counter() - t_gen:.1f} s")
    if args.seven_level:
        atom = synth.two_ion_level_atom(len(atom["lines"][0]["q"]))
    if args.active_continua:
        atom = synth.with_active_continua(atom)
    sample = None
    if not args.no_cpu_baseline and not args.kernel_probe and not args.seven_level:
        log("cpu baseline (oracle sample, before the GPU is initialised) ...")
        sample = cpu_baseline_sample()
        log(f"oracle: {sample['updates'] / (sample['t_fs'] + sample['t_rates']):.3e} updates/s on "
            f"{sample['workers']} workers")

    import torch

    from paper_1701_01607_amd import nlte
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    torch.cuda.init()
    log("uploading the atmosphere ...")
    stream = torch.cuda.current_stream()
    ctx = nlte.Context(0, stream.cuda_stream)
    A = ctx.atom(atom)
    torch.cuda.synchronize()
    t_up = time.perf_counter()
    M = ctx.atmos(atm)              # resident on the device before the timed region
    torch.cuda.synchronize()
    upload_s = time.perf_counter() - t_up
    log(f"atmosphere uploaded from host memory in {upload_s:.2f} s")
    params = solve_params(nlte, wl, timing=0 if args.graph else 1, dirs_per_block=args.dirs_per_block,
                          graph=args.graph)
    nf = sum(len(l["q"]) for l in atom["lines"])
    N = len(atom["levels"])
    nvox = atm["nx"] * atm["ny"] * atm["nz"]
    fine_updates = float(nvox) * 24 * nf
    footprint = ctx.footprint(M, A, params)
    log(f"device footprint of one solve: {footprint / 1e9:.2f} GB")
    mu_out = np.array([[0.0, 0.0, 1.0]])

    if args.kernel_probe:
        probe = nlte.SolveParams(method=nlte.MALI, precision=nlte.MIXED, nlev=1, E_target=0.0, max_iter=1,
                                 dirs_per_block=args.dirs_per_block)
        job = ctx.job(M, A, probe)
        rc, r = job.run()
        job.close()
        src = torch.empty(512 * 2 ** 20 // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"probe": args.workload, "updates": r.updates, "sweep_launches": r.sweep_launches,
                          "dirs_per_block": r.dirs_per_block, "copy_bytes": src.numel() * 4}))
        return

    top = wl["nlev"] - 1
    if fine_step:
        # the steps iterate the finest grid, so it starts from its own zero-radiation
        # populations (made by a one-grid job that is released before the FMG job is built)
        zr = ctx.job(M, A, nlte.SolveParams(method=nlte.MALI, precision=nlte.MIXED, nlev=1, max_iter=0))
        n0 = zr.populations(0, (N, atm["nz"], atm["ny"], atm["nx"]))
        zr.close()
        t_build = time.perf_counter()
        job = ctx.job(M, A, params)
        torch.cuda.synchronize()
        log(f"{wl['method']} job built in {time.perf_counter() - t_build:.1f} s (hierarchy of {wl['nlev']} grids)")
        job.set_populations(top, n0)
        del n0

        def step():
            c = job.mali(top, 1)
            return c
    else:
        def step():
            j = ctx.job(M, A, params)
            rc, r = j.run()
            Itop = torch.empty((1, nf, atm["ny"], atm["nx"]), dtype=torch.float32, device="cuda")
            ctx.check(ctx.lib.nlte_emergent_intensity(ctx.h, j.id, 1, mu_out.ctypes.data_as(nlte.ct.c_void_p),
                                                      nlte.ct.c_void_p(Itop.data_ptr()), nlte.MEM_DEVICE))
            j.close()
            return (rc, r)

    for i in range(args.warmup):
        t = time.perf_counter()
        res = step()
        torch.cuda.synchronize()
        log(f"warmup {i}: {time.perf_counter() - t:.2f} s" + (f" C={res:.3e}" if fine_step else
                                                               f" rc={res[0]} cycles={res[1].cycles}"))
    s0 = job.stats() if fine_step else None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for i in range(args.steps):
        t = time.perf_counter()
        results.append(step())
        if fine_step:
            torch.cuda.synchronize()
            log(f"step {i}: C={results[-1]:.3e} {time.perf_counter() - t:.2f} s")
        else:
            rc, r = results[-1]
            log(f"step {i}: rc={rc} cycles={r.cycles} E_est={r.E_est:.3e} ms={r.ms_total:.0f}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps

    if fine_step:
        s1 = job.stats()
        upd = s1.updates - s0.updates
        sweep_ms = s1.ms_sweep - s0.ms_sweep
        launches = s1.sweep_launches - s0.sweep_launches
        dpb = s1.dirs_per_block
        value = fine_updates * args.steps / elapsed
        job.close()
        extra = {"step": "one finest-grid MALI iteration of the resident FMG job (FP32 formal solution + FP64 "
                         "rate solve)",
                 "updates_per_step": fine_updates,
                 "rates_ms_per_step": (s1.ms_rates - s0.ms_rates) / args.steps,
                 "sweep_ms_per_step": sweep_ms / args.steps,
                 "footprint_gb": footprint / 1e9,
                 "projected": {"atmospheres_per_hr": 3600.0 / (M4_FINE_FS_EQUIV * elapsed / args.steps),
                               "basis": f"step time x {M4_FINE_FS_EQUIV} finest-grid formal-solution equivalents "
                                        f"of the whole FMG solve (measured by one full solve)"}}
    else:
        upd = sum(r.updates for _, r in results)
        sweep_ms = sum(r.ms_sweep for _, r in results)
        launches = sum(r.sweep_launches for _, r in results)
        r = results[-1][1]
        dpb = r.dirs_per_block
        value = 3600.0 / (elapsed / args.steps)
        extra = {"converged": all(rc == 0 for rc, _ in results), "cycles": r.cycles,
                 "fine_fs_equiv": r.fine_fs_equiv, "E_est": r.E_est,
                 "updates_per_s_wall": upd / elapsed,
                 "phase_ms": {"setup": r.ms_setup, "sweep": r.ms_sweep, "rates": r.ms_rates,
                              "transfer": r.ms_transfer, "total": r.ms_total}}
    updates_per_s_sweep = upd / (sweep_ms * 1e-3) if sweep_ms else None

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "voxel-angle-freq updates/s" if fine_step else "atmospheres/hr",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if wl["fp64"] else "f32 sweep / f64 rates",
        "data": "synthetic (seeded)",
        "config": {"workload": args.workload, "grid": [atm["nx"], atm["ny"], atm["nz"]],
                   "lines": len(atom["lines"]), "frequencies": nf, "directions": 24, "method": wl["method"],
                   "levels": wl["nlev"], "nu": [wl["nu_fmg"], wl["nu0"], wl["nu1"], wl["nu2"], wl["nu3"]],
                   "E_target": wl["E_target"] or None, "tol_C": wl["tol_C"] or None,
                   "continua": "active" if args.active_continua else "fixed", "atom": atom["name"]},
        "updates_per_s_sweep": updates_per_s_sweep,
        "roofline": None if args.active_continua or args.graph or args.seven_level else
        roofline(atom, atm, wl["fp64"], upd, sweep_ms, launches, dpb, args.workload),
    }
    out.update(extra)
    out["atmosphere_upload_s"] = upload_s   # host to device, once per atmosphere, outside every figure
    out["hbm_copy_gbs"] = hbm_copy_gbs(torch)
    del M
    if not args.no_mali and not wl["fp64"]:
        if fine_step:
            out["solve_64x64x129"] = solve_extras(nlte, ctx, torch, np, mali_max_iter=args.mali_max_iter)
        else:
            ex = solve_extras(nlte, ctx, torch, np, name=args.workload, solves=1, mali_max_iter=args.mali_max_iter,
                              fp32_error=not args.no_fp32_error)
            out["mali_fp64"] = ex["mali_fp64"]
            out["fp32_error_vs_fp64"] = ex["fp32_error_vs_fp64"]
    if sample is not None:
        feq = M4_FINE_FS_EQUIV if fine_step else out.get("fine_fs_equiv", 60.0)
        out["cpu_baseline"] = cpu_baseline(sample, fine_updates, feq)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
