"""Pins of the oracle's active continua (no GPU): the frequency quadrature against the
analytic photo-ionisation rate, detailed balance in a Planck field, the fixed point of
the preconditioned rates, and convergence of MALI and FAS with active continua."""
import numpy as np
import pytest

from oracle import physics as ph
from oracle.formal import continuum_formal_solution, formal_solution
from oracle.levels import Level
from oracle.rates import apply_W, fine_rhs, zero_radiation
from oracle.solver import Params, mali, solve_fas, solve_mali
from paper_1701_01607_amd import synth


def small_case(nx=4, ny=4, nz=9, seed=7, **grid):
    atom = synth.with_active_continua(synth.caii_like_atom(9), **grid)
    atm = synth.atmos_stratified(nx=nx, ny=ny, nz=nz, dx=150 * synth.KM, seed=seed)
    atm["ntot"] = atm["ntot"] * 0.1
    return atom, atm


@pytest.mark.parametrize("T", [5000.0, 8000.0, 12000.0])
def test_planck_photo_rates_converge_to_the_analytic_integral(T):
    # 4 pi int alpha B / (h nu) dnu on the continuum grid against the exact E1 series of
    # the fixed bound-free rates; the error falls at second order as the grid is refined
    atom = synth.caii_like_atom(9)
    Ta = np.array([T])
    nstar = np.ones((6, 1))
    exact = ph.fixed_bf_rates(atom, Ta, nstar)
    errs = []
    for n_seg, n_top in ((12, 32), (24, 64), (48, 128)):
        nu = synth.continuum_grid(atom, n_seg=n_seg, n_top=n_top, top=4.0)
        alpha, w = ph.continuum_quadrature(atom, nu)
        B = ph.planck_nu(nu, T)
        e = []
        for t, ct in enumerate(atom["continua"]):
            r = 4.0 * np.pi * np.sum(w[t] * alpha[t] * B / (ph.H * nu))
            e.append(abs(r / exact[ct["lower"], ct["upper"], 0] - 1.0))
        errs.append(max(e))
    # a wrong factor or exponent would leave an error that does not shrink
    assert errs[2] < 1e-2
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


def test_detailed_balance_in_a_planck_field():
    # J = B at every frequency: n_l* U_t = n_c* (G_t + F_t) for every continuum, any grid
    atom, atm = small_case()
    lev = Level(atom, atm)
    f = 4.0 * np.pi / (ph.H * lev.cont_nu)
    for t in range(lev.ncont):
        l, c = lev.cont_lower[t], lev.cont_upper[t]
        wa = (lev.cont_w[t] * lev.cont_alpha[t] * f)[:, None, None, None]
        U = np.sum(wa * lev.cont_B, axis=0)
        G = np.sum(wa * lev.cont_g[t] * lev.cont_B, axis=0)
        assert np.allclose(lev.nstar[l] * U, lev.nstar[c] * (G + lev.cont_F[t]), rtol=1e-12)


def test_preconditioned_rates_equal_the_plain_rates_at_the_populations_they_came_from():
    # Built from a formal solution at n, the preconditioned matrix applied to n gives the
    # statistical equilibrium with the actual mean intensities, lines and continua
    atom, atm = small_case()
    lev = Level(atom, atm)
    n = zero_radiation(lev)
    n, _ = mali(lev, 1, n, fine_rhs(lev), 2)
    Jeff, omL, Jbar = formal_solution(lev, n, want_jbar=True)
    cont, J = continuum_formal_solution(lev, n, want_j=True)
    W = apply_W(lev, n, Jeff, omL, cont)
    P = lev.fixed.copy()
    for l in range(lev.nline):
        A, Bij, Bji = lev.einstein[l]
        i, j = lev.lower[l], lev.upper[l]
        P[i, j] += Bij * Jbar[l]
        P[j, i] += A + Bji * Jbar[l]
    f = (4.0 * np.pi / (ph.H * lev.cont_nu))[:, None, None, None]
    for t in range(lev.ncont):
        l, c = lev.cont_lower[t], lev.cont_upper[t]
        wa = lev.cont_w[t][:, None, None, None] * lev.cont_alpha[t][:, None, None, None] * f
        P[l, c] += np.sum(wa * J, axis=0)
        P[c, l] += np.sum(wa * lev.cont_g[t] * (lev.cont_e + J), axis=0)
    out = np.einsum("i...,ij...->i...", n, P) - np.einsum("j...,ji...->i...", n, P)
    out[0] = n.sum(axis=0)
    scale = np.einsum("i...,ij...->i...", n, P).max(axis=0)
    assert np.max(np.abs(W[1:] - out[1:]) / scale) < 1e-9
    # the continua carry real radiative rates here (not a vacuous check)
    assert np.max(np.abs(cont[2])) > 0 and np.max(cont[0]) > 0


def test_mali_and_fas_converge_to_the_same_solution_with_active_continua():
    atom, atm = small_case(nz=9)
    p = Params(nlev=2, nu1=2, nu2=2, nu3=12, E_target=1e-8, max_iter=400)
    nm, stm, lev = solve_mali(atom, atm, p)
    nf, stf, _ = solve_fas(atom, atm, p)
    tol = 4 * (stm.E_est[-1] + stf.E_est[-1]) + 1e-12
    assert np.max(np.abs(nf / nm - 1)) < max(tol, 1e-8)
    assert np.all(nm > 0) and np.allclose(nm.sum(axis=0), lev.ntot, rtol=1e-13)
    # the active continua change the solution against the fixed ones
    atom0 = synth.caii_like_atom(9)
    n0, _, _ = solve_mali(atom0, atm, p)
    assert np.max(np.abs(n0 / nm - 1)) > 1e-3
