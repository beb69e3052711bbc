"""Batches (nlte_batch_run): several jobs solved together with shared work-list sweep
launches give each job exactly what it gets alone (GPU)."""
import numpy as np
import pytest

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


def mixed_inputs():
    """Grids of uneven size (plane counts 9..33, planes of 8x8 to 64x64, so two classes of
    frequency chunks) with the six-level and the two-level atom."""
    out = []
    for j, (n, nz, two) in enumerate([(16, 17, False), (8, 9, True), (16, 33, True), (64, 17, False),
                                      (8, 17, False), (32, 9, True)]):
        atm = synth.atmos_stratified(nx=n, ny=n, nz=nz, dx=150 * synth.KM, seed=900 + j)
        if two:
            atom = synth.two_level_atom(1e-2)
            atm["chi_c"] = None
        else:
            atom = synth.caii_like_atom(9)
            atm["ntot"] = atm["ntot"] * 0.1
        out.append((atom, atm))
    return out


def pops(job, atom, atm, level):
    return job.populations(level, (len(atom["levels"]), atm["nz"], atm["ny"], atm["nx"]))


def alone_and_batched(nl, ctx, inputs, params_for, level):
    alone = []
    for i, (atom, atm) in enumerate(inputs):
        job = ctx.job(ctx.atmos(atm), ctx.atom(atom), params_for(i))
        rc, r = job.run()
        alone.append((rc, r.iterations, r.cycles, job.history(), pops(job, atom, atm, level), r.fallback))
        job.close()
    jobs = [ctx.job(ctx.atmos(atm), ctx.atom(atom), params_for(i)) for i, (atom, atm) in enumerate(inputs)]
    rc, res = ctx.batch_run(jobs)
    batched = [(r.status, r.iterations, r.cycles, j.history(), pops(j, atom, atm, level), r.fallback)
               for j, r, (atom, atm) in zip(jobs, res, inputs)]
    for j in jobs:
        j.close()
    return alone, batched


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("method", ["FAS", "FMG"])
def test_batched_multigrid_solves_equal_alone_solves(nl, ctx, prec, method):
    inputs = mixed_inputs()
    m = nl.FAS if method == "FAS" else nl.FMG

    def params_for(i):
        # stop rules differ per job, so jobs leave the batch at different cycles
        return nl.SolveParams(method=m, precision=prec, nlev=2, nu0=3, nu1=2, nu2=2, nu3=8, nu_fmg=6,
                              E_target=(1e-3, 1e-5, 1e-4)[i % 3], max_iter=20)

    alone, batched = alone_and_batched(nl, ctx, inputs, params_for, 1)
    cycles = [a[2] for a in alone]
    print(f"prec={prec} {method}: cycles alone {cycles}")
    assert len(set(cycles)) > 1
    for i, (a, b) in enumerate(zip(alone, batched)):
        assert a[0] == b[0] and a[2] == b[2], i
        assert np.array_equal(a[3], b[3]), f"job {i}: history differs"
        assert np.array_equal(a[4], b[4]), f"job {i}: populations differ"


@pytest.mark.parametrize("prec", [0, 1])
def test_batched_mali_solves_equal_alone_solves(nl, ctx, prec):
    # the two-level workload's kind of problem: plain MALI to C <= tol on several grids
    inputs = []
    for j, scale in enumerate((1.0, 0.3, 3.0, 1.0)):
        atom = synth.two_level_atom()
        atm = synth.atmos_isothermal(nx=16 if j != 3 else 8, ny=16 if j != 3 else 8, nz=32 if j < 2 else 24)
        atm["ntot"] = atm["ntot"] * scale
        inputs.append((atom, atm))

    def params_for(i):
        return nl.SolveParams(method=nl.MALI, precision=prec, nlev=1, tol_C=(1e-4, 1e-3)[i % 2], E_target=0.0,
                              max_iter=400)

    alone, batched = alone_and_batched(nl, ctx, inputs, params_for, 0)
    print(f"prec={prec} MALI iterations alone {[a[1] for a in alone]}")
    for i, (a, b) in enumerate(zip(alone, batched)):
        assert a[0] == b[0] == nl.OK and a[1] == b[1], i
        assert np.array_equal(a[3], b[3]) and np.array_equal(a[4], b[4]), i


def test_a_job_falling_back_to_mali_inside_a_batch(nl, ctx):
    inputs = mixed_inputs()[:3]

    def params_for(i):
        forced = dict(fallback_mali=1, diverge_cycles=1, diverge_growth=1e-300) if i == 1 else {}
        return nl.SolveParams(method=nl.FAS, precision=nl.MIXED, nlev=2, nu1=2, nu2=2, nu3=8, E_target=1e-3,
                              max_iter=200, **forced)

    alone, batched = alone_and_batched(nl, ctx, inputs, params_for, 1)
    assert alone[1][5] == 1 and batched[1][5] == 1
    for i, (a, b) in enumerate(zip(alone, batched)):
        assert a[:3] == b[:3] and np.array_equal(a[3], b[3]) and np.array_equal(a[4], b[4]), i


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("method", ["FAS", "MALI"])
def test_graph_replayed_batches_equal_alone_solves(nl, ctx, prec, method):
    """Jobs asking for HIP-graph replay batch together: each repeated step of the job set
    is captured once and replayed; populations, histories and the counters the host keeps
    for replayed work (formal solutions, updates, launches) equal the alone runs'."""
    inputs = mixed_inputs()[:4] if method == "FAS" else [
        (synth.two_level_atom(), synth.atmos_isothermal(nx=16, ny=16, nz=32 - 8 * (j % 2))) for j in range(3)]

    def params_for(i):
        if method == "FAS":
            return nl.SolveParams(method=nl.FAS, precision=prec, nlev=2, nu0=3, nu1=2, nu2=2, nu3=8,
                                  E_target=(1e-3, 1e-5, 1e-4)[i % 3], max_iter=20, graph=1)
        return nl.SolveParams(method=nl.MALI, precision=prec, nlev=1, tol_C=(1e-4, 1e-3)[i % 2], E_target=0.0,
                              max_iter=400, graph=1)

    level = 1 if method == "FAS" else 0
    alone = []
    for i, (atom, atm) in enumerate(inputs):
        job = ctx.job(ctx.atmos(atm), ctx.atom(atom), params_for(i))
        rc, r = job.run()
        alone.append((rc, r.iterations, r.cycles, job.history(), pops(job, atom, atm, level), r.updates,
                      r.fine_fs_equiv))
        job.close()
    jobs = [ctx.job(ctx.atmos(atm), ctx.atom(atom), params_for(i)) for i, (atom, atm) in enumerate(inputs)]
    rc, res = ctx.batch_run(jobs)
    for i, (j, r, (atom, atm)) in enumerate(zip(jobs, res, inputs)):
        a = alone[i]
        assert (r.status, r.iterations, r.cycles) == a[:3], i
        assert np.array_equal(j.history(), a[3]), f"job {i}: history differs"
        assert np.array_equal(pops(j, atom, atm, level), a[4]), f"job {i}: populations differ"
        assert r.updates == a[5] and abs(r.fine_fs_equiv - a[6]) < 1e-9, f"job {i}: bookkeeping differs"
    print(f"prec={prec} {method}: steps alone {[a[1] if method == 'MALI' else a[2] for a in alone]}")
    for j in jobs:
        j.close()


def test_incompatible_jobs_are_rejected_before_any_work(nl, ctx):
    (atom, atm), (atom2, atm2) = mixed_inputs()[:2]
    base = dict(method=nl.FAS, nlev=2, nu1=2, nu2=2, nu3=8)
    for other in (dict(precision=nl.FP64), dict(nu3=4), dict(sc_interp=nl.SC_HERMITE), dict(nlev=1), dict(graph=1)):
        p2 = dict(base, precision=nl.MIXED)
        p2.update(other)
        a = ctx.job(ctx.atmos(atm), ctx.atom(atom), nl.SolveParams(precision=nl.MIXED, **base))
        b = ctx.job(ctx.atmos(atm2), ctx.atom(atom2), nl.SolveParams(**p2))
        before = a.populations(1, (6, atm["nz"], atm["ny"], atm["nx"]))
        with pytest.raises(nl.NlteError) as ei:
            ctx.batch_run([a, b])
        assert ei.value.code == nl.E_INVALID, other
        assert np.array_equal(a.populations(1, before.shape), before)
        a.close()
        b.close()
