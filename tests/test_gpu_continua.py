"""Active overlapping continua on the GPU against the oracle (FP64 and mixed precision):
zero-radiation start, MALI iterations and FAS cycles."""
import numpy as np
import pytest

from oracle.levels import Level
from oracle.rates import fine_rhs, zero_radiation
from oracle.solver import Params as OParams
from oracle.solver import mali, solve_fas
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


def case(nx=12, ny=10, nz=9, seed=21):
    atom = synth.with_active_continua(synth.caii_like_atom(9))
    atm = synth.atmos_stratified(nx=nx, ny=ny, nz=nz, dx=120 * synth.KM, seed=seed)
    return atom, atm


@pytest.fixture(scope="module")
def ragged():
    atom, atm = case()
    lev = Level(atom, atm)
    n0 = zero_radiation(lev)
    return atom, atm, lev, n0


@pytest.mark.parametrize("prec,tol", [(0, 1e-9), (1, 1e-5)])
def test_active_continua_mali_parity(nl, ctx, ragged, prec, tol):
    atom, atm, lev, n0 = ragged
    N = len(atom["levels"])
    shape = (N, atm["nz"], atm["ny"], atm["nx"])
    job = ctx.job(ctx.atmos(atm), ctx.atom(atom), nl.SolveParams(method=nl.MALI, precision=prec, nlev=1))
    e0 = relerr(job.populations(0, shape), n0)
    job.mali(0, 3)
    n3, _ = mali(lev, 1, n0, fine_rhs(lev), 3)
    e3 = relerr(job.populations(0, shape), n3)
    # the fixed-continuum solution differs by far more than the tolerance
    lev_fixed = Level(synth.caii_like_atom(9), atm)
    d = relerr(zero_radiation(lev_fixed), n0)
    print(f"prec={prec} active continua: zero-radiation err {e0:.2e}, MALI x3 err {e3:.2e}; "
          f"fixed continua differ by {d:.2e}")
    assert e0 < 1e-11
    assert e3 < tol
    if prec == 0:
        assert d > 1e3 * tol
    assert np.allclose(job.populations(0, shape).sum(axis=0), atm["ntot"], rtol=1e-13)


@pytest.mark.parametrize("prec,tol", [(0, 1e-7), (1, 1e-5)])
@pytest.mark.parametrize("fmg", [False, True])
def test_active_continua_fas_parity(nl, ctx, prec, tol, fmg):
    atom, atm = case(nx=8, ny=8, nz=17, seed=31)
    atm["ntot"] = atm["ntot"] * 0.1
    n_or, st, _ = solve_fas(atom, atm, OParams(nlev=3, nu1=2, nu2=2, nu3=6, nu_fmg=4), fmg=fmg, cycles=2)
    job = ctx.job(ctx.atmos(atm), ctx.atom(atom),
                  nl.SolveParams(method=nl.FMG if fmg else nl.FAS, precision=prec, nlev=3, nu1=2, nu2=2, nu3=6,
                                 nu_fmg=4, E_target=0.0, tol_C=0.0, max_iter=2))
    rc, r = job.run()
    N = len(atom["levels"])
    e = relerr(job.populations(2, (N, atm["nz"], atm["ny"], atm["nx"])), n_or)
    print(f"prec={prec} fmg={fmg} active continua FAS 2 cycles err {e:.2e}")
    assert r.cycles == 2 and e < tol
    assert abs(r.C / st.C[-1] - 1) < 0.05
