"""What the C-ABI promises beyond the default path, on the GPU and against the oracle:
a capped run's warning with a readable result, LTE and user initial populations (a run
resumed from its own populations), a prescribed upper boundary (Sect. 4.2), the
negative-population repair of Sect. 4.10 inside a V-cycle, and the fallback from
diverging cycles to plain MALI."""
import numpy as np
import pytest

from oracle.formal import formal_solution
from oracle.levels import Level, build_hierarchy
from oracle.rates import fine_rhs, zero_radiation
from oracle.solver import Params as OParams
from oracle.solver import Stats, mali, vcycle
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


def ragged_case():
    atom = synth.caii_like_atom(9)
    atm = synth.atmos_stratified(nx=12, ny=10, nz=9, dx=120 * synth.KM, seed=21)
    return atom, atm


def mg_case():
    atom = synth.caii_like_atom(7)
    atm = synth.atmos_stratified(nx=8, ny=8, nz=17, dx=150 * synth.KM, seed=31)
    atm["ntot"] = atm["ntot"] * 0.1
    return atom, atm


def shape(atom, atm):
    return (len(atom["levels"]), atm["nz"], atm["ny"], atm["nx"])


@pytest.mark.parametrize("prec,tol", [(0, 1e-9), (1, 1e-5)])
def test_iteration_cap_warns_and_keeps_a_readable_result(nl, ctx, prec, tol):
    atom, atm = ragged_case()
    lev = Level(atom, atm)
    job = ctx.job(ctx.atmos(atm), ctx.atom(atom),
                  nl.SolveParams(method=nl.MALI, precision=prec, nlev=1, E_target=1e-12, max_iter=2))
    rc, r = job.run()
    assert rc == nl.W_NOT_CONVERGED and r.status == nl.W_NOT_CONVERGED
    assert r.iterations == 2 and len(job.history()) == 2
    n2, _ = mali(lev, 1, zero_radiation(lev), fine_rhs(lev), 2)
    e = relerr(job.populations(0, shape(atom, atm)), n2)
    print(f"prec={prec} capped MALI: population err {e:.2e}")
    assert e < tol
    # cycles too: FAS capped at one cycle
    atom2, atm2 = mg_case()
    job2 = ctx.job(ctx.atmos(atm2), ctx.atom(atom2),
                   nl.SolveParams(method=nl.FAS, precision=prec, nlev=3, nu3=6, E_target=1e-12, max_iter=1))
    rc2, r2 = job2.run()
    assert rc2 == nl.W_NOT_CONVERGED and r2.cycles == 1
    assert np.all(np.isfinite(job2.populations(2, shape(atom2, atm2))))


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("method", ["MALI", "FAS"])
def test_lte_initial_populations_are_the_oracles_saha_boltzmann(nl, ctx, prec, method):
    atom, atm = mg_case()
    m = nl.MALI if method == "MALI" else nl.FAS
    job = ctx.job(ctx.atmos(atm), ctx.atom(atom),
                  nl.SolveParams(method=m, precision=prec, nlev=1 if m == nl.MALI else 3, init=nl.INIT_LTE))
    top = 0 if m == nl.MALI else 2
    e = relerr(job.populations(top, shape(atom, atm)), Level(atom, atm).nstar)
    print(f"prec={prec} {method} LTE start err {e:.2e}")
    assert e < 1e-12


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("method", ["MALI", "FAS"])
def test_a_run_resumed_from_its_populations_repeats_it_bitwise(nl, ctx, prec, method):
    # nu0 = 0: the resumed run's first cycle is an ordinary cycle, as in the long run
    atom, atm = mg_case()
    m = nl.MALI if method == "MALI" else nl.FAS
    nlev, top = (1, 0) if m == nl.MALI else (3, 2)
    base = dict(method=m, precision=prec, nlev=nlev, nu0=0, nu1=2, nu2=2, nu3=6, E_target=0.0, tol_C=0.0)
    total, first = (5, 3) if m == nl.MALI else (3, 2)
    longrun = ctx.job(ctx.atmos(atm), ctx.atom(atom), nl.SolveParams(max_iter=total, **base))
    longrun.run()
    part = ctx.job(ctx.atmos(atm), ctx.atom(atom), nl.SolveParams(max_iter=first, **base))
    part.run()
    mid = part.populations(top, shape(atom, atm))
    resumed = ctx.job(ctx.atmos(atm), ctx.atom(atom),
                      nl.SolveParams(max_iter=total - first, init=nl.INIT_USER, init_pops=mid, **base))
    resumed.run()
    assert np.array_equal(resumed.populations(top, shape(atom, atm)), longrun.populations(top, shape(atom, atm)))
    assert np.array_equal(resumed.history(), longrun.history()[first:])


@pytest.mark.parametrize("prec,tol_fs,tol_n", [(0, 1e-9, 1e-8), (1, 1e-5, 1e-5)])
def test_prescribed_upper_boundary_parity(nl, ctx, prec, tol_fs, tol_n):
    atom, atm = ragged_case()
    lev0 = Level(atom, atm)
    rng = np.random.default_rng(8)
    # incoming intensity at the top plane: a fraction of the local Planck function per line
    top_I = lev0.B[lev0.line_of, -1] * rng.uniform(0.2, 1.5, (lev0.nf, atm["ny"], atm["nx"]))
    lev = Level(atom, atm, top_I=top_I)
    n0 = zero_radiation(lev)
    job = ctx.job(ctx.atmos(atm), ctx.atom(atom), nl.SolveParams(method=nl.MALI, precision=prec, nlev=1, top_I=top_I))
    L = len(atom["lines"])
    jg, og = job.formal_solution(0, (L, atm["nz"], atm["ny"], atm["nx"]))
    jo, oo = formal_solution(lev, n0)
    jfree, _ = formal_solution(lev0, n0)
    ej, eo = relerr(jg, jo), relerr(og, oo)
    print(f"prec={prec} prescribed top: Jeff err {ej:.2e}  1-L* err {eo:.2e}")
    assert ej < tol_fs and eo < tol_fs
    assert relerr(jo, jfree) > 1e-3          # the boundary matters in this case
    job.mali(0, 2)
    n2, _ = mali(lev, 1, n0, fine_rhs(lev), 2)
    en = relerr(job.populations(0, shape(atom, atm)), n2)
    print(f"prec={prec} prescribed top: populations after 2 MALI err {en:.2e}")
    assert en < tol_n


def rough_case():
    """Two grids; fine populations far from equilibrium (log-normal, unit spread), for
    which the coarse solve of a V-cycle without pre-smoothing goes negative (Sect. 4.10).
    Every oracle decision n_old (1 + I e) <= 0 lies at least 1.6e-3 n_old from the
    boundary, so both precisions take the same ones."""
    atom = synth.caii_like_atom(7)
    atm = synth.atmos_stratified(nx=8, ny=8, nz=17, dx=150 * synth.KM, seed=31)
    levels = build_hierarchy(atom, atm, 2)
    fine = levels[-1]
    n0 = zero_radiation(fine)
    n = n0 * np.exp(np.random.default_rng(1).standard_normal(n0.shape))
    n *= (fine.ntot / n.sum(axis=0))[None]
    return atom, atm, levels, n


@pytest.mark.parametrize("prec,tol", [(0, 1e-8), (1, 2e-5)])
def test_vcycle_negative_population_repair_parity(nl, ctx, prec, tol):
    atom, atm, levels, n = rough_case()
    st = Stats()
    p = OParams(nlev=2, nu0=0, nu1=0, nu2=0, nu3=8)
    n_or = vcycle(levels, 2, n, fine_rhs(levels[-1]), p, stats=st)
    job = ctx.job(ctx.atmos(atm), ctx.atom(atom),
                  nl.SolveParams(method=nl.FAS, precision=prec, nlev=2, nu0=0, nu1=0, nu2=0, nu3=8))
    job.set_populations(1, n)
    rep = job.vcycle(1, first=False)
    got = job.populations(1, n.shape)
    # errors of the coarse relative correction e reach a population as n_old * d(Ie):
    # compare against n_old (1 + |I e|) element by element
    scale = n + np.abs(n_or - n)
    err = float(np.max(np.abs(got - n_or) / scale))
    print(f"prec={prec} repairs gpu {rep} oracle {st.repairs}; population err {err:.2e}")
    assert st.repairs == 78 and rep == st.repairs
    repaired = np.isclose(n_or, 0.1 * n, rtol=1e-15, atol=0)
    assert np.array_equal(got[repaired], 0.1 * n[repaired])
    assert err < tol
    assert np.all(got > 0)


@pytest.mark.parametrize("prec", [0, 1])
def test_diverging_cycles_fall_back_to_mali(nl, ctx, prec):
    # The guard is forced from the host: a growth factor of 1e-300 counts every cycle
    # after the first as growing, so the second cycle is declared divergent.
    atom, atm = mg_case()
    cyc = dict(method=nl.FAS, precision=prec, nlev=3, nu0=0, nu1=2, nu2=2, nu3=6)
    forced = dict(diverge_cycles=1, diverge_growth=1e-300)
    with pytest.raises(nl.NlteError) as ei:
        ctx.job(ctx.atmos(atm), ctx.atom(atom), nl.SolveParams(E_target=1e-3, max_iter=50, **cyc, **forced)).run()
    assert ei.value.code == nl.E_DIVERGED
    fb = ctx.job(ctx.atmos(atm), ctx.atom(atom),
                 nl.SolveParams(E_target=1e-3, max_iter=300, fallback_mali=1, **cyc, **forced))
    rc, r = fb.run()
    assert rc == nl.OK and r.fallback == 1 and r.cycles == 2
    # the same as one cycle, then MALI from its populations under the same stop rule
    one = ctx.job(ctx.atmos(atm), ctx.atom(atom), nl.SolveParams(E_target=0.0, max_iter=1, **cyc))
    one.run()
    n1 = one.populations(2, shape(atom, atm))
    ml = ctx.job(ctx.atmos(atm), ctx.atom(atom),
                 nl.SolveParams(method=nl.MALI, precision=prec, nlev=1, E_target=1e-3, max_iter=300,
                                init=nl.INIT_USER, init_pops=n1))
    rcm, rm = ml.run()
    print(f"prec={prec} fallback after 2 cycles: {r.iterations} MALI iterations (MALI alone {rm.iterations})")
    assert rcm == nl.OK and r.iterations == rm.iterations
    assert np.array_equal(fb.populations(2, shape(atom, atm)), ml.populations(0, shape(atom, atm)))
    h = fb.history()
    assert len(h) == 2 + r.iterations and np.array_equal(h[2:], ml.history())
    # the default guard leaves a converging run alone
    ok = ctx.job(ctx.atmos(atm), ctx.atom(atom), nl.SolveParams(E_target=1e-3, max_iter=50, fallback_mali=1, **cyc))
    rc2, r2 = ok.run()
    assert rc2 == nl.OK and r2.fallback == 0


def test_naturally_diverging_cycles_match_the_oracle_and_fall_back(nl, ctx):
    # An 8x8x9 atmosphere whose 4x4x5 coarse grid makes the FAS cycles diverge (Sect. 4.10):
    # the oracle's corrections C grow in cycles 8, 9 and 10 (above 1e-3), where the default
    # guard stops the run; with the fallback the run ends as plain MALI.
    from oracle.solver import solve_fas
    atom = synth.caii_like_atom(9)
    atm = synth.atmos_stratified(nx=8, ny=8, nz=9, dx=150 * synth.KM, seed=801)
    atm["ntot"] = atm["ntot"] * 0.1
    _, st, _ = solve_fas(atom, atm, OParams(nlev=2, nu1=2, nu2=2, nu3=8, E_target=None, tol_C=None), cycles=10)
    C = np.array(st.C)
    grew = [c > p and c > 1e-3 for p, c in zip(C[:-1], C[1:])]
    assert grew[-3:] == [True, True, True] and not all(grew[-4:])   # fires at cycle 10, not before
    cyc = dict(method=nl.FAS, precision=nl.FP64, nlev=2, nu1=2, nu2=2, nu3=8, E_target=1e-3, max_iter=300)
    with pytest.raises(nl.NlteError) as ei:
        ctx.job(ctx.atmos(atm), ctx.atom(atom), nl.SolveParams(**cyc)).run()
    assert ei.value.code == nl.E_DIVERGED
    job = ctx.job(ctx.atmos(atm), ctx.atom(atom), nl.SolveParams(fallback_mali=1, **cyc))
    rc, r = job.run()
    h = job.history()
    e = float(np.max(np.abs(h[:10] / C - 1)))
    print(f"diverging cycles: gpu C {h[:10]}; oracle err {e:.2e}; then {r.iterations} MALI iterations")
    assert r.cycles == 10 and r.fallback == 1 and rc == nl.OK
    assert e < 1e-6
