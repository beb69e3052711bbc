"""Multigrid operator and strategy study on synthetic atmospheres.

Runs the design comparisons of the paper's Sect. 4 on seeded synthetic stand-ins for its
atmospheres, through the library (every solve on the GPU):

* restriction of populations and residuals: full weighting, half weighting, injection
  (Sect. 4.4, Fig. 4);
* coarse model atmospheres by full weighting or injection (Sect. 4.7);
* three against four grids (Sect. 4.3, Fig. 3);
* zero-radiation against LTE initial populations (Sect. 4.11), with the smoothing
  number rho_L(i) = max |D2[n_i - n_inf]| after i MALI iterations (Fig. 7);
* post-smoothing counts nu_2 with the number of negative-population repairs
  (Sect. 4.10, Fig. 6);
* trilinear against monotone cubic Hermite prolongation (Sect. 4.5);
* plain MALI as the reference curve.

The true error E_i = max |n_i - n_ref| / n_ref (Sect. 3.3) is measured against a tightly
converged FP64 FAS solution.  A solve is deterministic, so the populations after i cycles
are those of a solve capped at i cycles; each point of a curve is such a solve.  Work is
counted in finest-grid formal solutions (the paper's unit; coarse formal solutions count
1/8 per level).  Reading of D2: the second difference along z in index space of the
relative error (n_i - n_inf)/n_inf, the paper's figure being for 1D columns.

    python -m paper_1701_01607_amd.study --atmos stratified --out study.jsonl
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import nlte, synth

ATMOSPHERES = {
    # smooth stratification with random-field perturbations (stand-in for FAL-C-like cases)
    "stratified": lambda: synth.workload("caii6_64x64x129"),
    # granulation-scale fields and chromospheric shock fronts (stand-in for Model 1)
    "rmhd_like": lambda: synth.workload("caii6_256x256x257", nx=64, ny=64, nz=129),
}

MG = dict(method=nlte.FAS, precision=nlte.MIXED, nlev=3, nu0=0, nu1=2, nu2=2, nu3=32)

VARIANTS = {
    "fas3_full": {},
    "fas3_half": dict(restriction=nlte.RESTRICT_HALF),
    "fas3_inject": dict(restriction=nlte.RESTRICT_INJECT),
    "fas3_atmos_inject": dict(coarse_atmos=nlte.RESTRICT_INJECT),
    "fas4_full": dict(nlev=4),
    "fas3_lte_init": dict(init=nlte.INIT_LTE),
    "fas3_nu2_8": dict(nu2=8),
    "fas3_hermite": dict(interpolation=nlte.INTERP_HERMITE),
}


def rel_error(n, ref):
    return float(np.max(np.abs(n / ref - 1.0)))


def smoothing_number(n, ref):
    e = n / ref - 1.0                                  # [N][nz][ny][nx]
    d2 = e[:, 2:] - 2.0 * e[:, 1:-1] + e[:, :-2]
    return float(np.max(np.abs(d2)))


def solve(ctx, M, A, shape, **kw):
    """One solve from scratch; stopping rules off unless kw sets them."""
    p = nlte.SolveParams(**dict(dict(E_target=0.0, tol_C=0.0, timing=1), **kw))
    job = ctx.job(M, A, p)
    t0 = time.perf_counter()
    rc, r = job.run()
    dt = time.perf_counter() - t0
    lev = (p.nlev if p.method != nlte.MALI else 1) - 1
    n = job.populations(lev, shape)
    job.close()
    return rc, r, n, dt


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--atmos", default="stratified", choices=sorted(ATMOSPHERES))
    ap.add_argument("--cycles", type=int, default=6, help="V-cycles on the longest curve")
    ap.add_argument("--mali", default="4,8,16,32,64,128,192", help="MALI iteration counts on its curve")
    ap.add_argument("--variants", default=",".join(VARIANTS))
    ap.add_argument("--smoothing", default="1,2,4,8,16", help="MALI iterations for the smoothing number")
    ap.add_argument("--out", default="-")
    args = ap.parse_args(argv)
    out = sys.stdout if args.out == "-" else open(args.out, "w")

    def emit(rec):
        out.write(json.dumps(rec) + "\n")
        out.flush()
        if out is not sys.stdout:
            print(json.dumps(rec), flush=True)

    import torch
    nlte.load()
    atom, atm = ATMOSPHERES[args.atmos]()
    ctx = nlte.Context(0, torch.cuda.current_stream().cuda_stream)
    A, M = ctx.atom(atom), ctx.atmos(atm)
    shape = (len(atom["levels"]), atm["nz"], atm["ny"], atm["nx"])

    # reference: FP64 FAS to an estimated error of 1e-8
    rc, r, ref, dt = solve(ctx, M, A, shape, **dict(MG, precision=nlte.FP64, max_iter=60, E_target=1e-8))
    emit(dict(kind="reference", atmos=args.atmos, status=rc, cycles=r.cycles, C=r.C, E_est=r.E_est, seconds=dt))

    for it in (int(x) for x in args.mali.split(",") if x):
        rc, r, n, dt = solve(ctx, M, A, shape, method=nlte.MALI, precision=nlte.MIXED, nlev=1, max_iter=it)
        emit(dict(kind="mali", atmos=args.atmos, iterations=it, E=rel_error(n, ref), C=r.C,
                  work=r.fine_fs_equiv, seconds=dt))

    for name in (v for v in args.variants.split(",") if v):
        kw = dict(MG)
        kw.update(VARIANTS[name])
        for c in range(1, args.cycles + 1):
            rc, r, n, dt = solve(ctx, M, A, shape, **dict(kw, max_iter=c))
            bad = rc < 0 or not np.all(np.isfinite(n))
            emit(dict(kind="mg", variant=name, atmos=args.atmos, cycles=c, status=rc,
                      E=None if bad else rel_error(n, ref), C=r.C, E_est=r.E_est, work=r.fine_fs_equiv,
                      repairs=r.repairs, seconds=dt))
            if bad:
                break

    for init, tag in ((nlte.INIT_ZERO_RAD, "zero_radiation"), (nlte.INIT_LTE, "lte")):
        for it in (int(x) for x in args.smoothing.split(",") if x):
            rc, r, n, dt = solve(ctx, M, A, shape, method=nlte.MALI, precision=nlte.MIXED, nlev=1,
                                 max_iter=it, init=init)
            emit(dict(kind="smoothing", init=tag, atmos=args.atmos, iterations=it,
                      rho_L=smoothing_number(n, ref), E=rel_error(n, ref)))
    if out is not sys.stdout:
        out.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
