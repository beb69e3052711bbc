"""Pins of the oracle's active continua (no GPU): the frequency quadrature against the
analytic photo-ionisation rate, detailed balance in a Planck field, the fixed point of
the preconditioned rates (continua ending on one upper level and on two, where the
cross terms must be there), convergence of MALI and FAS with active continua, the
refusal of lines that reach a continuum edge, and the emergent intensity at the
continuum frequencies (isothermal LTE gives B, empty upper levels give Beer's law)."""
import numpy as np
import pytest

from oracle import physics as ph
from oracle.formal import continuum_emergent_intensity, continuum_formal_solution, formal_solution
from oracle.levels import Level
from oracle.rates import apply_W, fine_rhs, rate_matrix, system_matrix, zero_radiation
from oracle.solver import Params, mali, solve_fas, solve_mali
from paper_1701_01607_amd import synth


ATOMS = {"one_upper": synth.caii_like_atom, "two_upper": synth.two_ion_level_atom}


def small_case(nx=4, ny=4, nz=9, seed=7, kind="one_upper", **grid):
    atom = synth.with_active_continua(ATOMS[kind](9), **grid)
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


@pytest.mark.parametrize("kind", list(ATOMS))
def test_detailed_balance_in_a_planck_field(kind):
    # J = B at every frequency: n_l* U_t = n_c* (G_t + F_t) for every continuum, any grid
    atom, atm = small_case(kind=kind)
    lev = Level(atom, atm)
    f = 4.0 * np.pi / (ph.H * lev.cont_nu)
    for t in range(lev.ncont):
        l, c = lev.cont_lower[t], lev.cont_upper[t]
        wa = (lev.cont_w[t] * lev.cont_alpha[t] * f)[:, None, None, None]
        U = np.sum(wa * lev.cont_B, axis=0)
        G = np.sum(wa * lev.cont_g[t] * lev.cont_B, axis=0)
        assert np.allclose(lev.nstar[l] * U, lev.nstar[c] * (G + lev.cont_F[t]), rtol=1e-12)


@pytest.mark.parametrize("kind", list(ATOMS))
def test_preconditioned_rates_equal_the_plain_rates_at_the_populations_they_came_from(kind):
    # Built from a formal solution at n, the preconditioned matrix applied to n gives the
    # statistical equilibrium with the actual mean intensities, lines and continua.  With
    # two upper levels the local part of J holds both levels' emissivities, so the identity
    # needs the cross terms in the other upper level's population as well.
    atom, atm = small_case(kind=kind)
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
    assert cont.shape[0] == 2 + len(lev.cont_uppers)
    if kind == "two_upper":
        assert lev.cont_uppers == [5, 6]
        # every continuum has a non-zero sum for the other upper level, and leaving the
        # cross terms out breaks the identity
        for t in range(lev.ncont):
            assert np.max(np.abs(cont[2 + (1 - lev.cont_uidx[t]), t])) > 0
        # per level, against the level's own outflow: the identity holds to rounding
        # (measured 6e-14), and without the cross terms it fails by 3e-8
        own = np.einsum("i...,ij...->i...", n, P)
        A0 = system_matrix(rate_matrix(lev, Jeff, omL, cont))
        N = lev.N
        W0 = np.einsum("vij,vj->vi", A0, n.reshape(N, -1).T).T.reshape(n.shape)
        assert np.max(np.abs(W[1:] - out[1:]) / own[1:]) < 1e-12
        assert np.max(np.abs(W0[1:] - out[1:]) / own[1:]) > 1e-8


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


def test_mali_and_fas_converge_to_the_same_solution_with_two_upper_levels():
    atom, atm = small_case(nz=9, kind="two_upper")
    p = Params(nlev=2, nu1=2, nu2=2, nu3=12, E_target=1e-8, max_iter=400)
    nm, stm, lev = solve_mali(atom, atm, p)
    nf, stf, _ = solve_fas(atom, atm, p)
    tol = 4 * (stm.E_est[-1] + stf.E_est[-1]) + 1e-12
    assert np.max(np.abs(nf / nm - 1)) < max(tol, 1e-8)
    assert np.all(nm > 0) and np.allclose(nm.sum(axis=0), lev.ntot, rtol=1e-13)


def test_lines_reaching_a_continuum_edge_are_refused():
    # the line sweeps carry no bound-free opacity: a continuum whose edge lies below a
    # line's frequencies is refused when continua are active, accepted as fixed rates
    atom, atm = small_case()
    low = synth.caii_like_atom(9)
    low["levels"] = [dict(lv) for lv in low["levels"]]
    low["levels"][5]["E"] = 40000.0          # edge from level 4 at 14600 cm^-1, below the lines
    Level(low, atm)
    with pytest.raises(ValueError, match="continuum edge"):
        Level(synth.with_active_continua(low), atm)


# ---------------------------------------------------------------- emergent intensity

def _planck(nu, T):
    # B_nu(T) from its definition, not the oracle's
    return 2.0 * ph.H * nu ** 3 / ph.C ** 2 / np.expm1(ph.H * nu / (ph.KB * T))


@pytest.mark.parametrize("kind", list(ATOMS))
def test_continuum_emergent_intensity_of_an_isothermal_lte_atmosphere_is_planck(kind):
    # LTE populations: chi_t = alpha n_l* (1 - e^{-h nu/kT}) and eta = e^{-h nu/kT} 2 h nu^3/c^2
    # sum alpha n_l*, so S = B at every continuum frequency, and I = B along every ray
    atom, atm = small_case(kind=kind, nx=6, ny=5)
    T = 6400.0
    atm["T"] = np.full_like(atm["T"], T)
    lev = Level(atom, atm)
    mus = np.array([[0.0, 0.0, 1.0], [0.3, -0.2, 0.93], [1.0, 2.0, 3.0], [-0.7, 0.1, 0.2]])
    I = continuum_emergent_intensity(lev, lev.nstar, mus)
    assert I.shape == (4, lev.cont_nu.size, 5, 6)
    assert np.allclose(I, _planck(lev.cont_nu, T)[None, :, None, None], rtol=1e-11, atol=0)


def test_continuum_emergent_intensity_with_empty_upper_levels_follows_beers_law():
    # n_c = 0: no emission, so B(T) from below is attenuated by exp(-chi L / mu_z) with
    # chi = sum_t alpha0_t (nu_edge/nu)^3 n_l over the continua open at nu (hydrogenic)
    atom = synth.with_active_continua(synth.two_ion_level_atom(9))
    z = np.array([0.0, 1.0, 3.0, 4.0, 7.0, 11.0]) * synth.KM
    shape = (z.size, 2, 3)
    T = 5500.0
    atm = {"nx": 3, "ny": 2, "nz": z.size, "dx": 50 * synth.KM, "dy": 70 * synth.KM, "z": z,
           "T": np.full(shape, T), "ne": np.full(shape, 1e12), "nH": np.full(shape, 1e16),
           "ntot": np.full(shape, 1e8), "vx": np.zeros(shape), "vy": np.zeros(shape), "vz": np.zeros(shape),
           "chi_c": None}
    lev = Level(atom, atm)
    n = np.zeros((7,) + shape)
    for i, v in enumerate((9.0e11, 6.0e11, 4.5e11, 1.2e12, 7.5e11)):
        n[i] = v
    mus = np.array([[0.6, -0.3, 1.5], [0.0, 0.0, 2.0], [-1.0, 1.0, 1.0]])
    I = continuum_emergent_intensity(lev, n, mus)
    nu = lev.cont_nu
    lv = atom["levels"]
    chi = np.zeros_like(nu)
    for ct in atom["continua"]:
        nue = ph.C * (lv[ct["upper"]]["E"] - lv[ct["lower"]]["E"])
        on = nu >= nue * (1 - 1e-12)
        chi[on] += ct["alpha0"] * (nue / nu[on]) ** 3 * n[ct["lower"], 0, 0, 0]
    assert chi.min() * (z[-1] - z[0]) > 1.0   # optically thick at every continuum frequency
    for d, mu in enumerate(mus):
        muz = mu[2] / np.linalg.norm(mu)
        expect = _planck(nu, T) * np.exp(-chi * (z[-1] - z[0]) / muz)
        assert np.allclose(I[d], expect[:, None, None], rtol=1e-10, atol=0)


def test_continuum_sweeps_refuse_bicubic_upwind_interpolation():
    atom, atm = small_case()
    lev = Level(atom, atm, sc_interp="hermite")
    with pytest.raises(ValueError, match="bilinear"):
        continuum_emergent_intensity(lev, lev.nstar, [[0.0, 0.0, 1.0]])
    with pytest.raises(ValueError, match="bilinear"):
        continuum_formal_solution(lev, lev.nstar)


def test_cross_terms_by_hand():
    # Two continua, 0 -> 2 and 1 -> 3, so two upper levels.  The net upward rate of
    # continuum 0 holds n_3 L_0,3: a flux out of level 0 (X[0, 3] = +L) into level 2
    # (X[2, 3] = -L); likewise continuum 1 with n_2 L_1,2 (X[1, 2] = +L, X[3, 2] = -L).  The
    # terms in each continuum's own upper level stay out of X (they are in P).
    from types import SimpleNamespace
    from oracle.rates import cross_terms
    lev = SimpleNamespace(active_continua=True, N=4, ncont=2, cont_lower=[0, 1], cont_upper=[2, 3],
                          cont_uppers=[2, 3])
    cont = np.zeros((4, 2, 1, 1, 1))
    cont[2, 0] = 5.0      # L_0,2 (own)
    cont[3, 0] = 3.0      # L_0,3
    cont[2, 1] = 7.0      # L_1,2
    cont[3, 1] = 11.0     # L_1,3 (own)
    X = cross_terms(lev, cont)[..., 0, 0, 0]
    expect = np.zeros((4, 4))
    expect[0, 3], expect[2, 3] = 3.0, -3.0
    expect[1, 2], expect[3, 2] = 7.0, -7.0
    assert np.array_equal(X, expect)
    # one upper level: nothing to add
    lev1 = SimpleNamespace(active_continua=True, N=4, ncont=2, cont_lower=[0, 1], cont_upper=[2, 2],
                           cont_uppers=[2])
    assert cross_terms(lev1, np.zeros((3, 2, 1, 1, 1))) is None
