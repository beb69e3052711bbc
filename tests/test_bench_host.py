"""Host logic of bench.py: the algorithmic flop count behind the ALU roofline (the linear
short-characteristics update plus the line profile as evaluated; the FP32 cells' corner
rebuild is not method work and is not counted), and the one-GPU guard of the command line."""
import os
import subprocess
import sys

import numpy as np

import bench
from paper_1701_01607_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_flops_fp64_sweep_counts_the_series_everywhere():
    atom, atm = synth.workload("caii6_64x64x129")
    fl, core = bench.flops_per_update(atom, atm, True)
    assert core == 1.0
    assert fl == bench.FLOPS_PER_UPDATE_BASE + bench.FLOPS_VOIGT_CORE


def test_flops_undamped_line_is_a_gaussian():
    atom = synth.two_level_atom()
    atm = synth.atmos_stratified(nx=8, ny=8, nz=5, dx=100 * synth.KM, seed=3)
    for fp64 in (False, True):
        fl, core = bench.flops_per_update(atom, atm, fp64)
        assert core == 0.0
        assert fl == bench.FLOPS_PER_UPDATE_BASE + bench.FLOPS_GAUSS


def test_flops_fp32_split_between_the_three_profile_evaluations():
    atom, atm = synth.workload("caii6_64x64x129")
    fl, core = bench.flops_per_update(atom, atm, False)
    base = bench.FLOPS_PER_UPDATE_BASE
    # every damped update costs one of: small-damping series, Weideman series, wing
    assert base + bench.FLOPS_VOIGT_SMALL < fl < base + bench.FLOPS_VOIGT_CORE
    assert 0.0 < core < 0.5
    # the damping threshold decides: with no small-damping path the Weideman fraction grows
    saved = bench.VOIGT_SMALL_A
    try:
        bench.VOIGT_SMALL_A = 0.0
        fl0, core0 = bench.flops_per_update(atom, atm, False)
    finally:
        bench.VOIGT_SMALL_A = saved
    assert core0 > core and fl0 > fl
    assert np.isclose(core0, 0.308, atol=0.02)   # |u| < 5 fraction of the bench workload


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=ROOT, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stdout


def test_flop_base_is_the_scope_tables_update_without_the_corner_rebuild():
    # profile argument 2, opacity/source function 7, three bilinear interpolations 21,
    # optical depth 3, segment coefficients 7, intensity 5, weight 2, accumulations 10
    assert bench.FLOPS_PER_UPDATE_BASE == 2 + 7 + 21 + 3 + 7 + 5 + 2 + 10
