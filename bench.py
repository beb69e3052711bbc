#!/usr/bin/env python
"""Benchmark: converged atmospheres/hr and voxel-angle-frequency updates/s,
FAS with an FP32 sweep against plain FP64 MALI, on one MI355X.

A step is one whole solve of the six-level 64x64x129 workload (seeded synthetic
stratified atmosphere, 5 lines x 101 frequencies, 24 directions): per-level setup
and zero-radiation initialisation, 3-level FAS V-cycles with (nu0, nu1, nu2, nu3) =
(20, 4, 8, 32) until the error estimate rho/(1-rho) C <= 1e-3, then the emergent
intensity at mu = (0, 0, 1).  The atmosphere and atom are resident on the device
before the timed region.  Prints one JSON line.
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
# the kernel as it was when the counters were taken.
MEASURED_BYTES_PER_UPDATE = {("caii6_64x64x129", 6): 16.37}
VOXEL_BYTES_PER_GROUP = (11 + 2) * 4.0   # FP32; twice that in FP64

# Flops per update (FMA = 2, a reciprocal, exponential or cosine = 1) for the ALU side
# of the roofline: profile argument 2, opacity/source function 7, three bilinear
# interpolations 21, optical depth 3, segment coefficients 7, intensity 5, quadrature
# weight 2, accumulations 10 (57); FP32 cells add the opacity and source function of
# the four upwind corners rebuilt from phi (4 x 6); plus the profile: the Weideman N=32
# series (evaluated in FP64) 154, the FP32 small-damping series (a < 0.04, |u| < 5) 35,
# the FP32 asymptotic wing with its Gaussian term 64, a pure Gaussian 3.
FLOPS_PER_UPDATE_BASE = {False: 57 + 24, True: 57}
FLOPS_VOIGT_CORE, FLOPS_VOIGT_SMALL, FLOPS_VOIGT_WING, FLOPS_GAUSS = 154, 35, 64, 3
VOIGT_SMALL_A = 0.04

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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def flops_per_update(atom, atm, fp64, stride=61):
    """Mean flops per update on the finest grid: in FP32 sweeps the profile costs the
    small-damping series where |u| < 5 and the damping a < 0.04, the Weideman series where
    |u| < 5 otherwise (everywhere in FP64 sweeps) and the asymptotic wing elsewhere, so the
    fractions are counted on a sample of voxels over all directions and frequencies.
    Returns (flops per update, fraction of Weideman series evaluations)."""
    import numpy as np
    kb, amu, c_light = 1.380649e-16, 1.66053906660e-24, 2.99792458e10
    sl = slice(None, None, stride)
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
    base = FLOPS_PER_UPDATE_BASE[fp64]
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


_CPU_SAMPLE = None   # (one-line oracle level, k+, e) shared with forked workers


def _oracle_sweeps(dirs):
    """Time the FP64 oracle's sweep over `dirs` for the prepared one-line level."""
    import numpy as np
    from oracle.formal import source_function, sweep
    lev, kk, ee = _CPU_SAMPLE
    lo = lev.line_of
    t0 = time.perf_counter()
    for d in dirs:
        mu = lev.mu[d]

        def local(k, mu=mu):
            phi = lev.profile(k, mu)
            chi = lev.chi_c[lo, k] + kk[lo, k] * phi
            S = source_function(chi, lev.chi_c[lo, k], lev.eta_c[lo, k], kk[lo, k], ee[lo, k], phi)
            return chi, S, None

        if mu[2] > 0:
            bc = lambda k: np.broadcast_to(lev.B[lo, k], (lev.nf, lev.ny, lev.nx)).copy()
        else:
            bc = lambda k: np.zeros((lev.nf, lev.ny, lev.nx))
        sweep(lev, mu, local, bc, None)
    return time.perf_counter() - t0, len(dirs) * lev.nx * lev.ny * lev.nz * lev.nf


def cpu_baseline_sample(atom, atm, line=0, single_dirs=(0, 5, 14, 19), workers=16):
    """Time the FP64 oracle on a bounded sample of the workload: one line, every plane and
    frequency of it on the full grid, (a) four directions of the A4 set in this process
    (one core) and (b) all 24 directions over a pool of forked workers (one core each).
    Runs before the GPU is initialised."""
    import multiprocessing as mp
    global _CPU_SAMPLE
    from oracle.levels import Level
    from oracle.rates import zero_radiation
    full = Level(atom, atm)
    n = zero_radiation(full)
    sub_atom = dict(atom, lines=[atom["lines"][line]])
    sub_atm = dict(atm, chi_c=None if atm.get("chi_c") is None else atm["chi_c"][line:line + 1])
    lev = Level(sub_atom, sub_atm)
    kk, ee = lev.line_coefficients(n)
    _CPU_SAMPLE = (lev, kk, ee)
    t1, u1 = _oracle_sweeps(single_dirs)
    workers = max(1, min(workers, os.cpu_count() or 1, 24))
    chunks = [tuple(range(24))[i::workers] for i in range(workers)]
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(_oracle_sweeps, chunks)
    tp = max(t for t, _ in res)
    up = sum(u for _, u in res)
    return {"nf_full": full.nf, "nvox": lev.nx * lev.ny * lev.nz, "nf_line": lev.nf, "shape": (lev.nx, lev.ny, lev.nz),
            "single": (t1, u1, len(single_dirs)), "pool": (tp, up, workers)}


def cpu_baseline(sample, fine_fs_equiv):
    """Project the oracle's sampled updates/s to atmospheres/hr with the GPU solve's work
    count (finest-grid formal-solution equivalents); rate solves are not included."""
    nx, ny, nz = sample["shape"]
    fs_updates = sample["nvox"] * 24 * sample["nf_full"]
    t1, u1, nd = sample["single"]
    tp, up, w = sample["pool"]
    ups1, upsp = u1 / t1, up / tp
    return {
        "value": 3600.0 / (fine_fs_equiv * fs_updates / upsp), "unit": "atmospheres/hr", "cores": w,
        "kind": "oracle",
        "sample": f"one line ({sample['nf_line']} frequencies) x all {nz} planes of {nx}x{ny}x{nz}: all 24 A4 "
                  f"directions over {w} forked workers ({tp:.1f} s wall), projected to {fine_fs_equiv:.1f} "
                  f"finest-grid formal solutions per solve (the GPU solve's count); rate solves not included",
        "updates_per_s": upsp,
        "single_core": {"value": 3600.0 / (fine_fs_equiv * fs_updates / ups1), "updates_per_s": ups1,
                        "sample": f"{nd} directions in one process ({t1:.1f} s)"},
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="caii6_64x64x129", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mali", action="store_true", help="skip the FP64 MALI comparison solve")
    ap.add_argument("--mali-max-iter", type=int, default=800)
    ap.add_argument("--dirs-per-block", type=int, default=0, help="sweep block shape (0: autotune)")
    ap.add_argument("--graph", type=int, default=0, help="1: replay V-cycles from a captured HIP graph")
    ap.add_argument("--active-continua", action="store_true",
                    help="sweep the atom's continua as active transitions (41 continuum frequencies); the "
                         "line-sweep roofline is then not reported")
    ap.add_argument("--kernel-probe", action="store_true",
                    help="only one MALI iteration (one formal solution + rate solve) and a 512 MiB "
                         "device copy, for hardware-counter runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU per process; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1701_01607_amd import nlte, synth

    wl = WORKLOADS[args.workload]
    log(f"generating {args.workload} ...")
    atom, atm = synth.workload(args.workload)
    if args.active_continua:
        atom = synth.with_active_continua(atom)
    sample = None
    if not args.no_cpu_baseline and not args.kernel_probe:
        log("cpu baseline (oracle sample, before the GPU is initialised) ...")
        sample = cpu_baseline_sample(atom, atm)

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    torch.cuda.init()
    log("uploading the atmosphere ...")
    stream = torch.cuda.current_stream()
    ctx = nlte.Context(0, stream.cuda_stream)
    A = ctx.atom(atom)
    M = ctx.atmos(atm)              # resident on the device before the timed region
    method = {"FAS": nlte.FAS, "FMG": nlte.FMG, "MALI": nlte.MALI}[wl["method"]]
    params = nlte.SolveParams(method=method, precision=nlte.FP64 if wl["fp64"] else nlte.MIXED, nlev=wl["nlev"],
                              nu0=wl["nu0"], nu1=wl["nu1"], nu2=wl["nu2"], nu3=wl["nu3"], nu_fmg=wl["nu_fmg"],
                              E_target=wl["E_target"], tol_C=wl["tol_C"], max_iter=60 if method != nlte.MALI else 2000,
                              timing=0 if args.graph else 1,
                              dirs_per_block=args.dirs_per_block,
                              graph=args.graph)
    nf = sum(len(l["q"]) for l in atom["lines"])
    log(f"device footprint of one solve: {ctx.footprint(M, A, params) / 1e9:.2f} GB")
    mu_out = np.array([[0.0, 0.0, 1.0]])
    N = len(atom["levels"])

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
                          "copy_bytes": src.numel() * 4}))
        return

    def step():
        job = ctx.job(M, A, params)
        rc, r = job.run()
        Itop = torch.empty((1, nf, atm["ny"], atm["nx"]), dtype=torch.float32, device="cuda")
        ctx.check(ctx.lib.nlte_emergent_intensity(ctx.h, job.id, 1, mu_out.ctypes.data_as(nlte.ct.c_void_p),
                                                  nlte.ct.c_void_p(Itop.data_ptr()), nlte.MEM_DEVICE))
        job.close()
        return rc, r

    for i in range(args.warmup):
        rc, r = step()
        log(f"warmup {i}: rc={rc} cycles={r.cycles} C={r.C:.3e} E_est={r.E_est:.3e} ms={r.ms_total:.0f}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for i in range(args.steps):
        rc, r = step()
        results.append((rc, r))
        log(f"step {i}: rc={rc} cycles={r.cycles} C={r.C:.3e} E_est={r.E_est:.3e} ms={r.ms_total:.0f} "
            f"sweep_ms={r.ms_sweep:.0f}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    converged = all(rc == 0 for rc, _ in results)
    r = results[-1][1]
    upd = sum(x.updates for _, x in results)
    sweep_ms = sum(x.ms_sweep for _, x in results)
    launches = sum(x.sweep_launches for _, x in results)
    fl, core_frac = flops_per_update(atom, atm, wl["fp64"])
    nslot = 24 // r.dirs_per_block if r.dirs_per_block else 8
    nfl = nf / len(atom["lines"])
    wbytes = 2.0 if wl["fp64"] else 1.0
    bytes_upd = STATE_BYTES_PER_UPDATE[wl["fp64"]] + wbytes * VOXEL_BYTES_PER_GROUP * nslot / (24.0 * nfl)
    peak_alu = PEAK_FP64_TFLOPS if wl["fp64"] else PEAK_FP32_TFLOPS
    measured = MEASURED_BYTES_PER_UPDATE.get((args.workload, r.dirs_per_block))
    traffic = None
    if sweep_ms > 0:
        avg_launch_us = 1e3 * sweep_ms / launches
        if measured:
            traffic = upd * measured / launches / (avg_launch_us * 1e-6) / 1e9
        achieved = upd * bytes_upd / launches / (avg_launch_us * 1e-6) / 1e9
        achieved_alu = upd * fl / launches / (avg_launch_us * 1e-6) / 1e12
        ups_sweep = upd / (sweep_ms * 1e-3)
    else:   # graph replay: no per-phase events
        avg_launch_us = achieved = achieved_alu = ups_sweep = None

    out = {
        "metric": "converged atmospheres/hr + voxel-angle-freq updates/s, FAS-FP32 vs MALI-FP64",
        "value": 3600.0 / (elapsed / args.steps),
        "unit": "atmospheres/hr",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if wl["fp64"] else "f32 sweep / f64 rates",
        "data": "synthetic (seeded)",
        "config": {"workload": args.workload, "grid": [atm["nx"], atm["ny"], atm["nz"]], "lines": len(atom["lines"]),
                   "frequencies": nf, "directions": 24, "method": wl["method"], "levels": wl["nlev"],
                   "nu": [wl["nu_fmg"], wl["nu0"], wl["nu1"], wl["nu2"], wl["nu3"]],
                   "E_target": wl["E_target"] or None, "tol_C": wl["tol_C"] or None,
                   "continua": "active" if args.active_continua else "fixed"},
        "converged": converged,
        "updates_per_s": ups_sweep,
        "updates_per_s_wall": upd / elapsed,
        "cycles": r.cycles, "fine_fs_equiv": r.fine_fs_equiv, "E_est": r.E_est,
        "phase_ms": {"setup": r.ms_setup, "sweep": r.ms_sweep, "rates": r.ms_rates, "transfer": r.ms_transfer,
                     "total": r.ms_total},
        # The sweep issues VALU instructions on ~76-81 % of the cycles and moves HBM at ~69 %
        # of the device-copy rate (counter runs): vector ALU issue is its largest resource.
        # traffic is the measured HBM rate (GB/s); the hbm block gives the algorithmic one;
        # unpacked_fp32 relates the flops to the ceiling without packed FP32 instructions.
        "roofline": {"bound": "alu", "achieved": achieved_alu, "peak": peak_alu, "unit": "TFLOP/s",
                     "frac": achieved_alu / peak_alu if achieved_alu else None, "traffic": traffic,
                     "kernel": f"sweep_step_kernel<{'double' if wl['fp64'] else 'float'},{r.dirs_per_block}>",
                     "avg_launch_us": avg_launch_us, "launches": launches,
                     "flops_per_update": fl, "voigt_core_fraction": core_frac,
                     "unpacked_fp32": None if wl["fp64"] or not achieved_alu else
                     {"peak": PEAK_FP32_UNPACKED_TFLOPS, "frac": achieved_alu / PEAK_FP32_UNPACKED_TFLOPS},
                     "hbm": {"achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                             "frac": achieved / PEAK_HBM_GBS if achieved else None,
                             "bytes_per_update": bytes_upd}},
    }
    if args.active_continua:
        # the sweep phase then also holds the continuum sweep, which the line-sweep
        # models above do not describe
        out["roofline"] = None

    # this box's achievable HBM bandwidth for context: a 2 GiB device-to-device copy
    src = torch.empty(2 ** 29, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    out["hbm_copy_gbs"] = 5 * 2 * src.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst

    if not args.no_mali and not wl["fp64"]:
        mp = nlte.SolveParams(method=nlte.MALI, precision=nlte.FP64, nlev=1, E_target=1e-3,
                              max_iter=args.mali_max_iter, timing=1,
                              dirs_per_block=args.dirs_per_block)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        job = ctx.job(M, A, mp)
        rc, rm = job.run()
        torch.cuda.synchronize()
        tm = time.perf_counter() - t1
        nm = job.populations(0, (N, atm["nz"], atm["ny"], atm["nx"]))
        job.close()
        # the FAS result of the last timed step, for the agreement of the two solutions
        jf = ctx.job(M, A, params)
        jf.run()
        nfas = jf.populations(wl["nlev"] - 1, (N, atm["nz"], atm["ny"], atm["nx"]))
        jf.close()
        log(f"MALI-FP64: rc={rc} iterations={rm.iterations} C={rm.C:.3e} E_est={rm.E_est:.3e} s={tm:.1f}")
        out["mali_fp64"] = {"seconds": tm, "iterations": rm.iterations, "converged": rc == 0, "E_est": rm.E_est,
                            "updates_per_s": rm.updates / (rm.ms_sweep * 1e-3) if rm.ms_sweep else None,
                            "atmospheres_per_hr": 3600.0 / tm,
                            "speedup_fas_fp32": tm / (elapsed / args.steps),
                            "max_rel_diff_vs_fas": float(np.max(np.abs(nfas / nm - 1)))}
    if sample is not None:
        out["cpu_baseline"] = cpu_baseline(sample, r.fine_fs_equiv)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
