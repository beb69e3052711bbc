"""Active overlapping continua on the GPU against the oracle (FP64 and mixed precision):
zero-radiation start, MALI iterations and FAS cycles, for continua ending on one upper
level and on two (the seven-level atom), the residual with the cross terms of two upper
levels, the emergent intensity at the continuum frequencies, and the atoms and settings
the library refuses."""
import numpy as np
import pytest

from oracle.formal import continuum_emergent_intensity, continuum_formal_solution, formal_solution
from oracle.levels import Level
from oracle.rates import apply_W, cross_terms, fine_rhs, rate_matrix, system_matrix, zero_radiation
from oracle.solver import Params as OParams
from oracle.solver import mali, solve_fas
from paper_1701_01607_amd import synth

ATOMS = {"one_upper": synth.caii_like_atom, "two_upper": synth.two_ion_level_atom}

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


def case(nx=12, ny=10, nz=9, seed=21, kind="one_upper"):
    atom = synth.with_active_continua(ATOMS[kind](9))
    atm = synth.atmos_stratified(nx=nx, ny=ny, nz=nz, dx=120 * synth.KM, seed=seed)
    return atom, atm


@pytest.fixture(scope="module", params=list(ATOMS))
def ragged(request):
    atom, atm = case(kind=request.param)
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
    lev_fixed = Level({k: v for k, v in atom.items() if k != "continuum_nu"}, atm)
    d = relerr(zero_radiation(lev_fixed), n0)
    print(f"prec={prec} active continua: zero-radiation err {e0:.2e}, MALI x3 err {e3:.2e}; "
          f"fixed continua differ by {d:.2e}")
    assert e0 < 1e-11
    assert e3 < tol
    if prec == 0:
        assert d > 1e3 * tol
    assert np.allclose(job.populations(0, shape).sum(axis=0), atm["ntot"], rtol=1e-13)


@pytest.mark.parametrize("prec,tol", [(0, 1e-7), (1, 1e-5)])
@pytest.mark.parametrize("fmg,kind", [(False, "one_upper"), (True, "one_upper"), (False, "two_upper")])
def test_active_continua_fas_parity(nl, ctx, prec, tol, fmg, kind):
    atom, atm = case(nx=8, ny=8, nz=17, seed=31, kind=kind)
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


def test_two_upper_level_residual_parity_with_cross_terms(nl, ctx):
    # W(n) after an extra formal solution, element by element against the oracle's, with
    # the error measured against the terms each entry sums; leaving out the terms in the
    # other upper level's population moves the oracle's W by far more than the tolerance
    atom, atm = case(kind="two_upper")
    lev = Level(atom, atm)
    n0 = zero_radiation(lev)
    N = len(atom["levels"])
    npop = (N, atm["nz"], atm["ny"], atm["nx"])
    job = ctx.job(ctx.atmos(atm), ctx.atom(atom), nl.SolveParams(method=nl.MALI, precision=0, nlev=1))
    job.mali(0, 2)
    n2, _ = mali(lev, 1, n0, fine_rhs(lev), 2)
    rg = job.residual(0, npop)
    Jeff, omL = formal_solution(lev, n2)
    cont = continuum_formal_solution(lev, n2)
    ro = fine_rhs(lev) - apply_W(lev, n2, Jeff, omL, cont)
    A = system_matrix(rate_matrix(lev, Jeff, omL, cont), cross_terms(lev, cont))
    nv = n2.reshape(N, -1).T
    scale = np.einsum("vij,vj->vi", np.abs(A), np.abs(nv)).T.reshape(n2.shape)
    err = float(np.max(np.abs(rg - ro) / scale))
    A0 = system_matrix(rate_matrix(lev, Jeff, omL, cont))
    r0 = fine_rhs(lev) - np.einsum("vij,vj->vi", A0, nv).T.reshape(n2.shape)
    d = float(np.max(np.abs(r0 - ro) / scale))
    print(f"two upper levels: residual err relative to its terms {err:.2e}; without cross terms {d:.2e}")
    assert err < 1e-10
    assert d > 100 * 1e-10


def test_atoms_the_active_continua_cannot_represent_are_refused(nl, ctx):
    # a line reaching above a continuum edge (no bound-free opacity in the line sweeps)
    low = synth.caii_like_atom(9)
    low["levels"] = [dict(lv) for lv in low["levels"]]
    low["levels"][5]["E"] = 40000.0
    ctx.atom(low)                               # fine as fixed continua
    with pytest.raises(nl.NlteError) as ei:
        ctx.atom(synth.with_active_continua(low))
    assert ei.value.code == nl.E_INVALID
    # continua ending on five upper levels
    q = synth.caii_like_atom(9)["lines"][0]["q"]
    wide = {"name": "five-uppers", "mass_amu": 40.0, "xi": 2.0 * synth.KM, "epsilon": None,
            "levels": [{"E": 0.0, "g": 2.0, "stage": 1}, {"E": 13700.0, "g": 4.0, "stage": 1}]
            + [{"E": 90000.0 + 1000.0 * i, "g": 1.0, "stage": 2} for i in range(5)],
            "lines": [{"lower": 0, "upper": 1, "A": 1.0e7, "gamma_rad": 1.5e8, "gamma_vdw": 2.0e-8, "q": q}],
            "continua": [{"lower": 0, "upper": 2 + i, "alpha0": 1.0e-18} for i in range(5)],
            "collisions": [{"lower": 0, "upper": 1, "c_ul": 1.0e-7, "T_ref": 5000.0, "beta": -0.5}]}
    ctx.atom(wide)
    with pytest.raises(nl.NlteError) as ei:
        ctx.atom(synth.with_active_continua(wide))
    assert ei.value.code == nl.E_INVALID


@pytest.mark.parametrize("prec", [0, 1])
def test_continuum_emergent_intensity_parity(nl, ctx, ragged, prec):
    # the kernel works in FP64 from the job's populations in both precisions: against the
    # oracle at the same populations only the FP32 output rounding is left
    atom, atm, lev, n0 = ragged
    N = len(atom["levels"])
    job = ctx.job(ctx.atmos(atm), ctx.atom(atom), nl.SolveParams(method=nl.MALI, precision=prec, nlev=1))
    job.mali(0, 2)
    n = job.populations(0, (N, atm["nz"], atm["ny"], atm["nx"]))
    mus = np.array([[0.0, 0.0, 1.0], [0.3, -0.2, 0.93], [-1.0, 2.0, 3.0]])
    nfc = len(atom["continuum_nu"])
    Ig = job.emergent_continuum(mus, nfc, atm["ny"], atm["nx"])
    Io = continuum_emergent_intensity(lev, n, mus)
    e = relerr(Ig, Io)
    print(f"prec={prec} {len(lev.cont_uppers)} upper level(s): continuum emergent intensity err {e:.2e}")
    assert Ig.shape == Io.shape and np.all(Io > 0)
    assert e < 2e-7


@pytest.mark.parametrize("method", ["FAS", "MALI"])
def test_graph_replay_with_active_continua_equals_eager(nl, ctx, method):
    # under capture the continuum sweep follows the line sweep on the job's stream instead
    # of running beside it: histories and populations must stay bitwise the same
    atom, atm = case(nx=8, ny=8, nz=17, seed=31, kind="two_upper")
    atm["ntot"] = atm["ntot"] * 0.1
    m = nl.FAS if method == "FAS" else nl.MALI
    nlev = 3 if m == nl.FAS else 1
    N = len(atom["levels"])
    outs = []
    for graph in (0, 1):
        job = ctx.job(ctx.atmos(atm), ctx.atom(atom),
                      nl.SolveParams(method=m, precision=nl.MIXED, nlev=nlev, nu0=3, nu1=2, nu2=2, nu3=6,
                                     E_target=0.0, max_iter=4, graph=graph))
        rc, r = job.run()
        assert rc >= 0
        outs.append((job.history(), job.populations(nlev - 1, (N, atm["nz"], atm["ny"], atm["nx"]))))
        job.close()
    assert len(outs[0][0]) > 0
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


def test_continuum_emergent_intensity_into_device_memory_equals_the_host_copy(nl, ctx):
    import ctypes as ct
    import torch
    atom, atm = case(kind="two_upper")
    job = ctx.job(ctx.atmos(atm), ctx.atom(atom), nl.SolveParams(method=nl.MALI, precision=1, nlev=1))
    job.mali(0, 1)
    mus = np.ascontiguousarray([[0.0, 0.0, 1.0], [0.5, 0.1, 0.8]], dtype=np.float64)
    nfc = len(atom["continuum_nu"])
    host = job.emergent_continuum(mus, nfc, atm["ny"], atm["nx"])
    dev = torch.full((2, nfc, atm["ny"], atm["nx"]), float("nan"), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    ctx.check(ctx.lib.nlte_emergent_continuum_intensity(ctx.h, job.id, 2, mus.ctypes.data_as(ct.c_void_p),
                                                        ct.c_void_p(dev.data_ptr()), nl.MEM_DEVICE))
    assert np.array_equal(dev.cpu().numpy(), host)


def test_continuum_emergent_intensity_is_refused_where_it_does_not_apply(nl, ctx):
    atom, atm = case()
    # no active continua
    plain = {k: v for k, v in atom.items() if k != "continuum_nu"}
    job = ctx.job(ctx.atmos(atm), ctx.atom(plain), nl.SolveParams(method=nl.MALI, precision=0, nlev=1))
    with pytest.raises(nl.NlteError) as ei:
        job.emergent_continuum([[0.0, 0.0, 1.0]], 41, atm["ny"], atm["nx"])
    assert ei.value.code == nl.E_INVALID
    # the continuum sweeps have no bicubic upwind interpolation
    with pytest.raises(nl.NlteError) as ei:
        ctx.job(ctx.atmos(atm), ctx.atom(atom), nl.SolveParams(method=nl.MALI, precision=0, nlev=1, sc_interp=1))
    assert ei.value.code == nl.E_INVALID
