"""Checks at the benchmark's full grid sizes, in the launch configuration bench.py times
(autotuned block shapes, one frequency chunk per wave on the finest grid).

* 64x64x129, six-level atom, horizontally homogeneous stratification with a height-
  dependent velocity: every column of the GPU result must equal the oracle's 1x1x129
  column, element by element (formal solution, then three MALI iterations).
* The bench workload itself (64x64x129, random 3D fields): the FP32-sweep FAS solve
  against the FP64 FAS solve, the labelled proxy reference, to 1e-5 (measured 1.0e-6); particle
  conservation and positivity.
* Twins of the 256x256x257 and 504x504x497 workloads (same generator, horizontal size /8,
  25 frequencies per line, 4-level FMG): FP32 sweep against FP64 to 1e-5 (measured 4.6e-7
  and 9.4e-7).
"""
import numpy as np
import pytest

from oracle.formal import formal_solution
from oracle.levels import Level
from oracle.rates import fine_rhs, zero_radiation
from oracle.solver import mali
from paper_1701_01607_amd import synth

pytestmark = pytest.mark.gpu


def relerr(a, b):
    return float(np.max(np.abs(np.asarray(a, dtype=np.float64) / np.asarray(b, dtype=np.float64) - 1.0)))


@pytest.fixture(scope="module")
def nl():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a HIP device"
    from paper_1701_01607_amd import nlte
    return nlte


@pytest.fixture(scope="module")
def ctx(nl):
    import torch
    c = nl.Context(0, torch.cuda.current_stream().cuda_stream)
    yield c
    c.close()


def homogeneous(nx, ny):
    """The bench's mean stratification without perturbations, plus v(z)."""
    atm = synth.atmos_stratified(nx=nx, ny=ny, dT=0.0, drho=0.0, vmax=0.0)
    z = atm["z"]
    prof = lambda amp, ph: np.broadcast_to((amp * synth.KM * np.sin(2 * np.pi * z / synth.MM + ph))[:, None, None],
                                           (atm["nz"], ny, nx)).copy()
    atm["vx"], atm["vy"], atm["vz"] = prof(3.0, 0.0), prof(2.0, 1.0), prof(4.0, 2.0)
    return atm


@pytest.mark.parametrize("prec,tol_fs,tol_n", [(0, 1e-9, 1e-9), (1, 1e-5, 1e-5)], ids=["fp64", "fp32"])
def test_full_size_homogeneous_equals_1d_oracle(nl, ctx, prec, tol_fs, tol_n):
    atom = synth.caii_like_atom(101)
    atm3, atm1 = homogeneous(64, 64), homogeneous(1, 1)
    lev = Level(atom, atm1)
    n0 = zero_radiation(lev)
    jo, oo = formal_solution(lev, n0)
    N, L = len(atom["levels"]), len(atom["lines"])
    shp_n, shp_l = (N, 129, 64, 64), (L, 129, 64, 64)
    job = ctx.job(ctx.atmos(atm3), ctx.atom(atom), nl.SolveParams(method=nl.MALI, precision=prec, nlev=1))
    jg, og = job.formal_solution(0, shp_l)
    ej = relerr(jg, np.broadcast_to(jo, shp_l))
    eo = relerr(og, np.broadcast_to(oo, shp_l))
    job.mali(0, 3)
    n3, _ = mali(lev, 1, n0, fine_rhs(lev), 3)
    en = relerr(job.populations(0, shp_n), np.broadcast_to(n3, shp_n))
    print(f"prec={prec} 64x64x129 vs 1D oracle: Jeff {ej:.2e} 1-L* {eo:.2e} populations after 3 MALI {en:.2e}")
    assert ej < tol_fs and eo < tol_fs and en < tol_n


def solve(nl, ctx, atom, atm, prec, method, nlev, cycles):
    p = nl.SolveParams(method=method, precision=prec, nlev=nlev, nu0=20, nu1=4, nu2=8, nu3=32, nu_fmg=16,
                       E_target=0.0, tol_C=0.0, max_iter=cycles)
    job = ctx.job(ctx.atmos(atm), ctx.atom(atom), p)
    rc, r = job.run()
    assert rc >= 0
    n = job.populations(nlev - 1, (len(atom["levels"]), atm["nz"], atm["ny"], atm["nx"]))
    job.close()
    return n, r


def test_bench_workload_fp32_against_fp64(nl, ctx):
    atom, atm = synth.workload("caii6_64x64x129")
    n32, r32 = solve(nl, ctx, atom, atm, nl.MIXED, nl.FAS, 3, 3)
    n64, r64 = solve(nl, ctx, atom, atm, nl.FP64, nl.FAS, 3, 3)
    e = relerr(n32, n64)
    cons = relerr(n32.sum(axis=0), atm["ntot"])
    print(f"64x64x129 FAS 3 cycles: FP32 vs FP64 {e:.2e}; conservation {cons:.1e}; "
          f"C {r32.C:.2e} / {r64.C:.2e}")
    assert np.isfinite(n32).all() and (n32 > 0).all()
    assert cons < 1e-12
    assert e < 1e-5


@pytest.mark.parametrize("name,nx,ny", [("caii6_256x256x257", 32, 32), ("caii6_504x504x497", 64, 64)])
def test_fmg_twins_fp32_against_fp64(nl, ctx, name, nx, ny):
    atom, atm = synth.workload(name, nx=nx, ny=ny, nfreq=25)
    n32, r32 = solve(nl, ctx, atom, atm, nl.MIXED, nl.FMG, 4, 3)
    n64, r64 = solve(nl, ctx, atom, atm, nl.FP64, nl.FMG, 4, 3)
    e = relerr(n32, n64)
    cons = relerr(n32.sum(axis=0), atm["ntot"])
    print(f"{name} twin {nx}x{ny}x{atm['nz']} FMG 3 cycles: FP32 vs FP64 {e:.2e}; conservation {cons:.1e}; "
          f"C {r32.C:.2e} / {r64.C:.2e}")
    assert np.isfinite(n32).all() and (n32 > 0).all()
    assert cons < 1e-12
    assert e < 1e-5
