"""The rate solve alone (nlte_rate_solve): given J-bar^eff and 1 - Lambda* per line and voxel,
the library's batched FP64 LU solve of the preconditioned rate equations against the
oracle's (LAPACK per voxel, then rescaled to the conservation row), on a ragged grid of
the six-level atom.  Both sides solve in FP64; in the mixed-precision job the inputs are
FP32 accumulators, so the oracle gets the same FP32-rounded values."""
import numpy as np
import pytest

from oracle.levels import Level
from oracle.rates import fine_rhs, max_rel_change, solve, zero_radiation
from paper_1701_01607_amd import synth

pytestmark = pytest.mark.gpu


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


def radiation(lev, seed):
    """Seeded J-bar^eff in [0.02, 1.2] B and 1 - Lambda* in [0.02, 1] per line and voxel."""
    rng = np.random.default_rng(seed)
    shape = lev.B.shape
    return lev.B * rng.uniform(0.02, 1.2, shape), rng.uniform(0.02, 1.0, shape)


@pytest.mark.parametrize("prec", [0, 1])
def test_rate_solve_parity(nl, ctx, prec):
    atom = synth.caii_like_atom(9)
    atm = synth.atmos_stratified(nx=13, ny=10, nz=9, dx=120 * synth.KM, seed=71)
    lev = Level(atom, atm)
    N = len(atom["levels"])
    npop = (N, atm["nz"], atm["ny"], atm["nx"])
    job = ctx.job(ctx.atmos(atm), ctx.atom(atom), nl.SolveParams(method=nl.MALI, precision=prec, nlev=1))
    n_before = job.populations(0, npop)
    assert np.max(np.abs(n_before / zero_radiation(lev) - 1.0)) < 1e-11
    dt = np.float64 if prec == 0 else np.float32
    f = fine_rhs(lev)
    for seed in (5, 6):
        Jeff, omL = radiation(lev, seed)
        Jeff, omL = Jeff.astype(dt).astype(np.float64), omL.astype(dt).astype(np.float64)
        C = job.rate_solve(0, Jeff, omL)
        n_gpu = job.populations(0, npop)
        n_ref = solve(lev, Jeff, omL, f)
        err = float(np.max(np.abs(n_gpu / n_ref - 1.0)))
        C_ref = max_rel_change(n_ref, n_before)
        print(f"prec={prec} seed={seed}: populations max rel err {err:.2e}, C gpu {C:.6e} oracle {C_ref:.6e}")
        assert err < 1e-11
        assert abs(C / C_ref - 1.0) < 1e-6
        assert np.allclose(n_gpu.sum(axis=0), atm["ntot"], rtol=1e-13)
        n_before = n_gpu
    job.close()


def test_rate_solve_rejects_active_continua(nl, ctx):
    atom = synth.with_active_continua(synth.caii_like_atom(9))
    atm = synth.atmos_stratified(nx=8, ny=8, nz=5, dx=120 * synth.KM, seed=72)
    job = ctx.job(ctx.atmos(atm), ctx.atom(atom), nl.SolveParams(method=nl.MALI, precision=0, nlev=1))
    shape = (len(atom["lines"]), atm["nz"], atm["ny"], atm["nx"])
    with pytest.raises(nl.NlteError):
        job.rate_solve(0, np.zeros(shape), np.ones(shape))
    job.close()
