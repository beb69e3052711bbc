"""Pins of the oracle's line physics and of its coarse-grid correction (no GPU).

Each test fixes one part of the oracle against something other than its own formulas:
textbook line-broadening and oscillator-strength relations, the Doppler formula, Beer's
law for a purely absorbing slab, and hand-computed values of the repair rule of
Sect. 4.10.
"""
import numpy as np
import pytest

from oracle.formal import emergent_intensity
from oracle.levels import Level, build_hierarchy
from oracle.rates import fine_rhs, zero_radiation
from oracle.solver import Params, Stats, apply_correction, vcycle
from paper_1701_01607_amd import synth

# CGS constants (CODATA 2018), restated here so the pins do not reuse the oracle's
H = 6.62607015e-27
C = 2.99792458e10
KB = 1.380649e-16
ME = 9.1093837015e-28
AMU = 1.66053906660e-24
E_CHARGE = 4.803204712570263e-10   # statcoulomb
KM = 1.0e5


def planck(nu, T):
    return 2.0 * H * nu ** 3 / C ** 2 / np.expm1(H * nu / (KB * T))


def one_line_atom(q, gamma_rad=0.0, gamma_vdw=0.0, mass=40.0, xi=0.0, E=20000.0, gl=2.0, gu=4.0, A=2.0e8):
    return {"name": "one-line", "mass_amu": mass, "xi": xi,
            "levels": [{"E": 0.0, "g": gl, "stage": 1}, {"E": E, "g": gu, "stage": 1}],
            "lines": [{"lower": 0, "upper": 1, "A": A, "gamma_rad": gamma_rad, "gamma_vdw": gamma_vdw,
                       "q": np.asarray(q, dtype=np.float64)}],
            "continua": [], "collisions": [{"lower": 0, "upper": 1, "c_ul": 1e-7, "T_ref": 5000.0, "beta": 0.0}],
            "epsilon": None}


def uniform_atmos(nx=1, ny=1, z=(0.0, 1.0e6), T=6000.0, nH=1.0e16, ne=1.0e12, ntot=1.0e8, v=(0.0, 0.0, 0.0)):
    z = np.asarray(z, dtype=np.float64)
    shape = (z.size, ny, nx)
    return {"nx": nx, "ny": ny, "nz": z.size, "dx": 50 * KM, "dy": 70 * KM, "z": z,
            "T": np.full(shape, T), "ne": np.full(shape, ne), "nH": np.full(shape, nH),
            "ntot": np.full(shape, ntot), "vx": np.full(shape, v[0]), "vy": np.full(shape, v[1]),
            "vz": np.full(shape, v[2]), "chi_c": None}


# ---------------------------------------------------------------- the repair rule (Sect. 4.10)

def test_correction_repairs_exactly_the_non_positive_entries():
    # hand-computed: n_old (1 + Ie) and, where that is <= 0, 10 % of n_old
    n_old = np.array([2.0, 3.0, 1.0, 4.0, 5.0, 8.0])
    Ie = np.array([-1.5, -1.0, -0.5, 0.25, -1.0000001, -0.999])
    n_new, rep = apply_correction(n_old, Ie, 0.1)
    expect = np.array([0.2, 0.3, 0.5, 5.0, 0.5, 8.0 * (1.0 - 0.999)])
    assert rep == 3
    assert np.array_equal(n_new[[0, 1, 4]], 0.1 * n_old[[0, 1, 4]])   # repaired, equality included
    assert np.allclose(n_new, expect, rtol=1e-12, atol=0)
    assert np.array_equal(n_new[[2, 3, 5]], n_old[[2, 3, 5]] * (1.0 + Ie[[2, 3, 5]]))   # untouched
    assert np.all(n_new > 0)
    # the fraction is the argument's, and the input array is not modified
    n2, rep2 = apply_correction(n_old, Ie, 0.25)
    assert rep2 == 3 and n2[0] == 0.5 and n_old[0] == 2.0


def test_vcycle_from_rough_populations_repairs_and_stays_positive():
    # Without pre-smoothing the coarse solve of rough populations goes negative
    # (Sect. 4.10); the repair keeps every corrected population positive.
    atom = synth.caii_like_atom(7)
    atm = synth.atmos_stratified(nx=8, ny=8, nz=17, dx=150 * synth.KM, seed=31)
    levels = build_hierarchy(atom, atm, 2)
    fine = levels[-1]
    n0 = zero_radiation(fine)
    n = n0 * np.exp(np.random.default_rng(1).standard_normal(n0.shape))
    n *= (fine.ntot / n.sum(axis=0))[None]
    st = Stats()
    out = vcycle(levels, 2, n, fine_rhs(fine), Params(nlev=2, nu0=0, nu1=0, nu2=0, nu3=8), stats=st)
    assert st.repairs > 0
    assert np.all(out > 0)


# ---------------------------------------------------------------- line profile and opacity

def test_damping_far_wing_is_the_lorentzian_of_the_damping_constant():
    # Far from the core the Voigt profile becomes the Lorentzian of the damping constant
    # Gamma = gamma_rad + gamma_vdw n_H (T/5000)^0.3: phi -> Gamma / (4 pi^2 dnu^2).
    T, nH = 6000.0, 3.0e16
    g_rad, g_vdw = 1.0e9, 3.0e-8
    vD = np.sqrt(2 * KB * T / (40.0 * AMU))
    q = np.array([-600.0, -300.0, 0.0, 300.0, 600.0]) * vD
    lev = Level(one_line_atom(q, g_rad, g_vdw), uniform_atmos(T=T, nH=nH))
    phi = lev.profile(0, np.array([0.0, 0.0, 1.0]))[:, 0, 0]
    gam = g_rad + g_vdw * nH * (T / 5000.0) ** 0.3
    nu0 = C * 20000.0
    dnu = nu0 * q / C
    wing = np.abs(q) > 0
    lor = gam / (4 * np.pi ** 2 * dnu[wing] ** 2)
    assert np.allclose(phi[wing], lor, rtol=5e-5, atol=0)


@pytest.mark.parametrize("d", range(24))
def test_profile_peak_sits_at_plus_v_dot_n(d):
    # Doppler formula: an absorber moving with v sees a photon of direction n at
    # nu (1 - v.n/c), so the lab-frame profile is centred at q = +v.n.
    v = np.array([3.0, -2.0, 5.0]) * KM
    q = np.linspace(-20.0, 20.0, 4001) * KM
    lev = Level(one_line_atom(q, mass=83.14), uniform_atmos(T=5000.0, v=v))
    mu = lev.mu[d]
    phi = lev.profile(0, mu)[:, 0, 0]
    centroid = np.trapezoid(q * phi, q) / np.trapezoid(phi, q)
    vn = float(v @ mu)
    assert abs(vn) > 0.1 * KM   # far above the tolerance below: a flipped sign fails
    assert centroid == pytest.approx(vn, abs=1e-6 * KM)
    assert q[np.argmax(phi)] == pytest.approx(vn, abs=0.01 * KM)


def test_frequency_integrated_line_opacity_matches_the_oscillator_strength():
    # int k phi dnu = (pi e^2 / m_e c) f_ij n_i (1 - g_i n_j / (g_j n_i)), with
    # f_ij = (m_e c^3 / (8 pi^2 e^2 nu0^2)) (g_j / g_i) A_ji.
    gl, gu, A, E = 2.0, 4.0, 1.3e8, 25000.0
    q = np.linspace(-12.0, 12.0, 2401) * KM
    lev = Level(one_line_atom(q, mass=83.14, gl=gl, gu=gu, A=A, E=E), uniform_atmos(T=5000.0))
    n = np.array([3.0e6, 2.0e4]).reshape(2, 1, 1, 1) * np.ones((2, 2, 1, 1))
    kk, _ = lev.line_coefficients(n)
    phi = lev.profile(0, np.array([0.0, 0.0, 1.0]))[:, 0, 0]
    nu0 = C * E
    nu = nu0 * (1.0 + q / C)
    integral = kk[0, 0, 0, 0] * np.trapezoid(phi, nu)
    f = ME * C ** 3 / (8 * np.pi ** 2 * E_CHARGE ** 2 * nu0 ** 2) * (gu / gl) * A
    expect = np.pi * E_CHARGE ** 2 / (ME * C) * f * n[0, 0, 0, 0] * (1.0 - gl * n[1, 0, 0, 0] / (gu * n[0, 0, 0, 0]))
    assert integral == pytest.approx(expect, rel=1e-9)


# ---------------------------------------------------------------- emergent intensity

def test_emergent_intensity_of_an_isothermal_lte_atmosphere_is_planck_in_every_upward_direction():
    # S = B everywhere and I = B at the lower boundary, so I = B along every ray.
    atom = synth.caii_like_atom(9)
    T = 5800.0
    atm = synth.atmos_stratified(nx=6, ny=5, nz=9, dx=80 * synth.KM, seed=3)
    atm["T"] = np.full_like(atm["T"], T)
    # the background (thermal, at the same T) is kept
    lev = Level(atom, atm)
    mus = np.array([[0.0, 0.0, 1.0], [0.3, -0.2, 0.93], [1.0, 2.0, 3.0], [-0.7, 0.1, 0.2]])
    I = emergent_intensity(lev, lev.nstar, mus)
    for l, ln in enumerate(atom["lines"]):
        nu0 = C * (atom["levels"][ln["upper"]]["E"] - atom["levels"][ln["lower"]]["E"])
        sl = slice(int(lev.fstart[l]), int(lev.fstart[l] + lev.nfreq[l]))
        assert np.allclose(I[:, sl], planck(nu0, T), rtol=1e-11, atol=0)


def test_emergent_intensity_of_a_purely_absorbing_slab_follows_beers_law():
    # Empty upper level and no background: S = 0, so the lower-boundary intensity B(T)
    # is attenuated by exp(-chi L / mu_z), chi = (pi e^2/m_e c) f n_i phi, mu normalised.
    T, E, A, gl, gu = 5000.0, 20000.0, 1.0e7, 1.0, 3.0
    q = np.linspace(-4.0, 4.0, 17) * KM
    z = np.array([0.0, 1.0, 3.0, 4.0, 7.0, 11.0]) * KM
    atom = one_line_atom(q, mass=83.14, gl=gl, gu=gu, A=A, E=E)
    lev = Level(atom, uniform_atmos(nx=3, ny=2, z=z, T=T))
    n_i = 4.0e6
    n = np.zeros((2,) + lev.T.shape)
    n[0] = n_i
    mus = np.array([[0.6, -0.3, 1.5], [0.0, 0.0, 2.0], [-1.0, 1.0, 1.0]])
    I = emergent_intensity(lev, n, mus)
    nu0 = C * E
    vD = np.sqrt(2 * KB * T / (83.14 * AMU))
    phi = np.exp(-(q / vD) ** 2) / (np.sqrt(np.pi) * nu0 * vD / C)
    f = ME * C ** 3 / (8 * np.pi ** 2 * E_CHARGE ** 2 * nu0 ** 2) * (gu / gl) * A
    chi = np.pi * E_CHARGE ** 2 / (ME * C) * f * n_i * phi
    assert chi.max() * (z[-1] - z[0]) > 1.0   # the line core is optically thick
    for d, mu in enumerate(mus):
        muz = mu[2] / np.linalg.norm(mu)
        expect = planck(nu0, T) * np.exp(-chi * (z[-1] - z[0]) / muz)
        assert np.allclose(I[d], expect[:, None, None], rtol=1e-10, atol=0)
