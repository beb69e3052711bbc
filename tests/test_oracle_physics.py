"""Pins of the oracle's local physics against closed forms, published constants,
library routines and limits (no GPU)."""
import numpy as np
import pytest
from scipy import integrate
from scipy.special import wofz

from oracle import physics as ph
from paper_1701_01607_amd import synth

SIGMA_SB = 5.670374419e-5   # Stefan-Boltzmann constant, erg cm^-2 s^-1 K^-4 (CODATA 2018)


def test_planck_integral_is_stefan_boltzmann():
    # pi * integral of B_nu over nu equals sigma T^4
    for T in (3000.0, 5000.0, 20000.0):
        val, _ = integrate.quad(lambda lnnu: ph.planck_nu(np.exp(lnnu), T) * np.exp(lnnu),
                                np.log(1e10), np.log(1e17), limit=400, epsabs=0, epsrel=1e-12)
        assert np.pi * val == pytest.approx(SIGMA_SB * T ** 4, rel=1e-9)


def test_planck_rayleigh_jeans_and_wien_limits():
    T = 6000.0
    nu = 1e9   # h nu / kT ~ 8e-6
    rj = 2.0 * nu ** 2 * ph.KB * T / ph.C ** 2
    assert ph.planck_nu(nu, T) == pytest.approx(rj, rel=1e-5)
    nu = 3e16  # h nu / kT ~ 240
    wien = 2.0 * ph.H * nu ** 3 / ph.C ** 2 * np.exp(-ph.H * nu / (ph.KB * T))
    assert ph.planck_nu(nu, T) == pytest.approx(wien, rel=1e-12)


def test_saha_factor_textbook_constant():
    # (2 pi m_e k T / h^2)^{3/2} = 2.4147e15 T^{3/2} cm^-3 (standard value)
    T = np.array([4000.0, 10000.0])
    val = ph.saha_phi(T, 1.0) / 2.0 / T ** 1.5
    assert np.allclose(val, 2.4147e15, rtol=2e-4)


def test_hydrogen_like_ionisation_balance():
    # One bound level (g=2) and a bare continuum (g=1) 13.598 eV above: the ionised
    # fraction x obeys x^2/(1-x) n_H = (2.4147e15 T^1.5) exp(-157807/T) with n_e = x n_H.
    atom = {"levels": [{"E": 109678.77, "g": 2.0, "stage": 1}, {"E": 109678.77 * 2, "g": 1.0, "stage": 2}]}
    atom["levels"][0]["E"] = 0.0
    atom["levels"][1]["E"] = 109678.77   # 13.598 eV in cm^-1
    T = 10000.0
    nH = 1e15
    x = 0.5
    for _ in range(200):   # fixed point on the electron density
        ne = x * nH
        n = ph.lte_populations(atom, T, ne, nH)
        x = n[1] / nH
    lhs = x * x / (1 - x) * nH
    rhs = 2.4147e15 * T ** 1.5 * np.exp(-157807.0 / T)
    assert lhs == pytest.approx(rhs, rel=2e-3)


def test_boltzmann_ratio_and_line_source_function_in_lte():
    # In LTE the line source function n_j A_ji / (n_i B_ij - n_j B_ji) equals B_nu0(T).
    atom = synth.caii_like_atom(11)
    T = np.array([4000.0, 6000.0, 9000.0])
    ne = np.array([1e11, 1e12, 1e13])
    nst = ph.lte_populations(atom, T, ne, np.ones(3))
    assert np.allclose(nst.sum(axis=0), 1.0, rtol=1e-15)
    for l, ln in enumerate(atom["lines"]):
        A, Bij, Bji = ph.einstein(atom, l)
        i, j = ln["lower"], ln["upper"]
        S = nst[j] * A / (nst[i] * Bij - nst[j] * Bji)
        assert np.allclose(S, ph.planck_nu(ph.line_nu0(atom, l), T), rtol=1e-12)


def test_collisions_detailed_balance():
    atom = synth.caii_like_atom(11)
    T = np.array([4500.0, 7000.0])
    ne = np.array([3e11, 2e13])
    nst = ph.lte_populations(atom, T, ne, np.ones(2))
    C = ph.collision_matrix(atom, T, ne, nst)
    R = ph.fixed_bf_rates(atom, T, nst)
    for M in (C, R):
        flux = nst[:, None] * M            # n_i* P_ij
        assert np.allclose(flux, np.swapaxes(flux, 0, 1), rtol=1e-12, atol=0)


def test_epsilon_mode_two_level_source_function():
    # S = (1-eps) J + eps B for the statistical equilibrium of a two-level atom with the
    # eps-mode collision rate, for arbitrary J.
    eps = 1e-3
    atom = synth.two_level_atom(eps)
    T = np.array([5000.0])
    nst = ph.lte_populations(atom, T, np.zeros(1), np.ones(1))
    C = ph.collision_matrix(atom, T, np.zeros(1), nst)
    A, B12, B21 = ph.einstein(atom, 0)
    B = ph.planck_nu(ph.line_nu0(atom, 0), T)
    for J in (0.0, 0.3 * B, 2.0 * B):
        r = (B12 * J + C[0, 1]) / (A + B21 * J + C[1, 0])      # n2 / n1
        S = r * A / (B12 - r * B21)
        assert S == pytest.approx((1 - eps) * J + eps * B, rel=1e-12)


def test_bf_planck_integral_matches_quadrature():
    for x in (0.5, 3.0, 12.0, 35.0):
        val, _ = integrate.quad(lambda t: 1.0 / (t * np.expm1(t)), x, np.inf, epsabs=0, epsrel=1e-12)
        assert ph.bf_planck_integral(x) == pytest.approx(val, rel=1e-10)


def test_voigt_gaussian_limit_integral_and_wings():
    u = np.linspace(-8, 8, 161)
    assert np.allclose(ph.voigt_H(0.0, u), np.exp(-u * u), rtol=1e-13, atol=1e-300)
    for a in (1e-3, 0.05, 0.5):
        val, _ = integrate.quad(lambda t: ph.voigt_H(a, t), -np.inf, np.inf, limit=500, epsrel=1e-10)
        assert val == pytest.approx(np.sqrt(np.pi), rel=1e-7)
        uw = 300.0
        assert ph.voigt_H(a, uw) == pytest.approx(a / (np.sqrt(np.pi) * uw * uw), rel=1e-4)
    assert ph.voigt_H(0.3, 1.7) == pytest.approx(wofz(1.7 + 0.3j).real, rel=1e-15)


def test_doppler_width_two_level_atom_is_one_km_s():
    atom = synth.two_level_atom()
    assert ph.doppler_velocity(atom, 5000.0) == pytest.approx(1.0e5, rel=1e-4)


def test_trapezoid_weights():
    x = np.array([0.0, 1.0, 3.0, 3.5])
    w = ph.trapezoid_weights(x)
    assert w.sum() == pytest.approx(3.5)
    assert np.dot(w, 2 * x + 1) == pytest.approx(3.5 ** 2 + 3.5)   # exact for linear
