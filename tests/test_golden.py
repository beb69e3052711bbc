"""Values the paper prints, kept as cited fixtures under tests/golden/: the iteration
counts of Table 1 that the bench workloads use, and the model grid sizes of Sect. 3 with
the grid-size rules of Sect. 4 that the coarsening and the largest workload follow."""
import json
import os

import numpy as np

import bench
from oracle.transfer import coarsen_atmosphere
from paper_1701_01607_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_bench_iteration_counts_are_table1_rows():
    runs = load("table1_runs.json")["runs"]
    m2 = [r for r in runs if r["atmosphere"] == "Model 2" and r["atom"] == "6-level Ca II"][0]["nu"]
    fmg = [r for r in runs if r["method"] == "3-grid full-MG"][0]["nu"]
    for name in ("caii6_64x64x129", "caii6_256x256x257", "caii6_504x504x497"):
        w = bench.WORKLOADS[name]
        # nu_0..nu_3 of the six-level Ca II run; nu_FMG of the full-multigrid run
        assert [w["nu0"], w["nu1"], w["nu2"], w["nu3"]] == m2[1:]
        assert w["nu_fmg"] == fmg[0]
    assert bench.WORKLOADS["caii6_256x256x257"]["method"] == "FMG"


def test_model_grids_obey_the_grid_size_rules():
    g = load("model_grids.json")
    l = g["grids"]
    for m in g["models"]:
        nx, ny, nz = m["used"]
        assert (nz - 1) % 2 ** l == 0 and nz % 2 == 1
        assert nx % 2 ** l == 0 and ny % 2 ** l == 0
    m1 = g["models"][0]
    assert m1["used"][2] == m1["snapshot"][2] + 1   # one extrapolated layer


def test_largest_workload_has_model1_grid_and_coarsens_to_it():
    m1 = load("model_grids.json")["models"][0]
    assert list(synth.GRIDS["caii6_504x504x497"]) == m1["used"]
    assert bench.WORKLOADS["caii6_504x504x497"]["nlev"] == 4
    atom, atm = synth.workload("caii6_504x504x497", nx=8, ny=8, nz=9)   # the recipe at a small size
    # coarsening a grid of the paper's form halves nx, ny and maps nz -> (nz - 1) / 2 + 1
    c = coarsen_atmosphere(atm)
    assert (c["nx"], c["ny"], c["nz"]) == (4, 4, 5)
    sizes = [tuple(m1["used"])]
    for _ in range(3):
        nx, ny, nz = sizes[-1]
        sizes.append((nx // 2, ny // 2, (nz - 1) // 2 + 1))
    assert sizes[-1] == (63, 63, 63)
    assert np.all([s[2] % 2 == 1 for s in sizes])
