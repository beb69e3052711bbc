"""Local physics per voxel, FP64 (oracle; test infrastructure only).

Sect. 2.1 states that collisional terms and background opacity/emissivity are
constant and fixed by the input atmosphere.  The paper does not give their form;
the readings used here are:

* Planck function at line centre for the whole line and for the thermal
  background source function (background = thermal only, no scattering).
* LTE populations by Saha-Boltzmann.
* Collisional rates: downward C_ul = n_e c_ul (T/T_ref)^beta, upward by detailed
  balance with the LTE ratio.  Two-level atoms may instead give a constant
  destruction probability eps, for which C_21 = eps A_21 / ((1-eps)(1-exp(-h nu/kT))),
  which makes S = (1-eps) Jbar + eps B exactly.
* Fixed bound-free transitions with a hydrogenic cross-section
  alpha0 (nu_edge/nu)^3 in a Planck radiation field at the local temperature:
  R_ic = (8 pi alpha0 nu_e^3 / c^2) sum_k E1(k h nu_e / kT), R_ci = R_ic (n_i/n_c)*.
  Or, when the atom carries a continuum frequency grid, active continua swept by the
  formal solution (formal.continuum_formal_solution), with the same cross-section and
  no background at continuum frequencies.
* Doppler width v_D = sqrt(2kT/m + xi^2); damping a = Gamma / (4 pi dnu_D) with
  Gamma = gamma_rad + gamma_vdw n_H (T/5000)^0.3.
* Voigt function H(a,u) = Re w(u + i a), w the Faddeeva function.
"""
from __future__ import annotations

import numpy as np
from scipy.special import exp1, wofz

# CGS constants (exact SI definitions and CODATA 2018)
H = 6.62607015e-27        # erg s
C = 2.99792458e10         # cm / s
KB = 1.380649e-16         # erg / K
ME = 9.1093837015e-28     # g
AMU = 1.66053906660e-24   # g
HC_K = H * C / KB         # cm K  (second radiation constant)


def planck_nu(nu, T):
    """B_nu(T) = (2 h nu^3 / c^2) / (exp(h nu / kT) - 1), erg cm^-2 s^-1 Hz^-1 sr^-1."""
    return (2.0 * H * nu ** 3 / C ** 2) / np.expm1(H * nu / (KB * T))


def line_nu0(atom, l):
    ln = atom["lines"][l]
    lv = atom["levels"]
    return C * (lv[ln["upper"]]["E"] - lv[ln["lower"]]["E"])


def einstein(atom, l):
    """(A_ji, B_ij, B_ji) for line l: B_ji = A_ji c^2 / (2 h nu0^3), g_i B_ij = g_j B_ji."""
    ln = atom["lines"][l]
    nu0 = line_nu0(atom, l)
    gi = atom["levels"][ln["lower"]]["g"]
    gj = atom["levels"][ln["upper"]]["g"]
    Aji = ln["A"]
    Bji = Aji * C ** 2 / (2.0 * H * nu0 ** 3)
    Bij = gj / gi * Bji
    return Aji, Bij, Bji


def saha_phi(T, ne):
    """Phi(T, n_e) = 2 (2 pi m_e k T / h^2)^{3/2} / n_e, so that n_{s+1,0} / n_{s,i} = (g_{s+1,0}/g_{s,i}) Phi exp(-dE/kT)."""
    return 2.0 * (2.0 * np.pi * ME * KB * T / H ** 2) ** 1.5 / ne


def lte_populations(atom, T, ne, ntot):
    """Saha-Boltzmann populations, shape (N, ...), summing to ntot.

    n_i* is proportional to g_i exp(-h c E_i / kT) Phi^(s_i - s_min), with energies
    E_i (cm^-1) measured from the atom's ground level and s_i the ionisation stage.
    """
    lv = atom["levels"]
    smin = min(l["stage"] for l in lv)
    T = np.asarray(T, dtype=np.float64)
    logw = []
    for l in lv:
        lw = np.log(l["g"]) - HC_K * l["E"] / T
        if l["stage"] != smin:
            lw = lw + (l["stage"] - smin) * np.log(saha_phi(T, ne))
        logw.append(lw)
    logw = np.stack(logw)
    logw = logw - logw.max(axis=0, keepdims=True)
    w = np.exp(logw)
    return ntot * w / w.sum(axis=0)


def collision_matrix(atom, T, ne, nstar):
    """Collisional rates C[i, j] (s^-1, rate from level i to level j), shape (N, N, ...)."""
    N = len(atom["levels"])
    Cm = np.zeros((N, N) + np.shape(T))
    if atom.get("epsilon") is not None:
        eps = atom["epsilon"]
        for l, ln in enumerate(atom["lines"]):
            i, j = ln["lower"], ln["upper"]
            nu0 = line_nu0(atom, l)
            c21 = eps * ln["A"] / ((1.0 - eps) * (-np.expm1(-H * nu0 / (KB * T))))
            Cm[j, i] += c21
            Cm[i, j] += c21 * nstar[j] / nstar[i]
        return Cm
    for cl in atom["collisions"]:
        l, u = cl["lower"], cl["upper"]
        cul = ne * cl["c_ul"] * (T / cl["T_ref"]) ** cl["beta"]
        Cm[u, l] += cul
        Cm[l, u] += cul * nstar[u] / nstar[l]
    return Cm


def bf_planck_integral(x_edge, tol=1e-17, kmax=100000):
    """sum_{k>=1} E1(k x): the integral of dx / (x (e^x - 1)) from x_edge to infinity."""
    x = np.asarray(x_edge, dtype=np.float64)
    total = exp1(x)
    k = 2
    while k < kmax:
        term = exp1(k * x)
        total = total + term
        if np.all(term <= tol * total):
            break
        k += 1
    return total


def fixed_bf_rates(atom, T, nstar):
    """Fixed bound-free rates R[i, c] and R[c, i] (s^-1), shape (N, N, ...).

    Photo-ionisation in a Planck field at the local temperature with cross-section
    alpha0 (nu_edge / nu)^3 above the edge; recombination by detailed balance.
    """
    N = len(atom["levels"])
    R = np.zeros((N, N) + np.shape(T))
    lv = atom["levels"]
    for ct in atom["continua"]:
        i, c = ct["lower"], ct["upper"]
        nue = C * (lv[c]["E"] - lv[i]["E"])
        x = H * nue / (KB * T)
        ric = 8.0 * np.pi * ct["alpha0"] * nue ** 3 / C ** 2 * bf_planck_integral(x)
        R[i, c] += ric
        R[c, i] += ric * nstar[i] / nstar[c]
    return R


def continuum_quadrature(atom, nu):
    """Active continua: alpha_t(nu_k) = alpha0 (nu_edge/nu_k)^3 at or above the edge, else 0,
    and the trapezoid weights w_tk of the integral over [nu_edge, nu_max] on the grid points
    at or above the edge (the grid contains every edge).  Shapes (ncont, nfc)."""
    nu = np.asarray(nu, dtype=np.float64)
    lv = atom["levels"]
    nc = len(atom["continua"])
    alpha = np.zeros((nc, nu.size))
    w = np.zeros((nc, nu.size))
    for t, ct in enumerate(atom["continua"]):
        nue = C * (lv[ct["upper"]]["E"] - lv[ct["lower"]]["E"])
        on = nu >= nue * (1.0 - 1e-12)
        idx = np.nonzero(on)[0]
        alpha[t, idx] = ct["alpha0"] * (nue / nu[idx]) ** 3
        d = np.diff(nu[idx])
        w[t, idx[:-1]] += 0.5 * d
        w[t, idx[1:]] += 0.5 * d
    return alpha, w


def doppler_velocity(atom, T):
    """v_D = sqrt(2 k T / m + xi^2) (cm/s)."""
    m = atom["mass_amu"] * AMU
    return np.sqrt(2.0 * KB * T / m + atom["xi"] ** 2)


def damping(atom, l, T, nH, vD):
    """Voigt damping parameter a = Gamma / (4 pi dnu_D) for line l."""
    ln = atom["lines"][l]
    gam = ln["gamma_rad"] + ln["gamma_vdw"] * nH * (T / 5000.0) ** 0.3
    dnuD = line_nu0(atom, l) * vD / C
    return gam / (4.0 * np.pi * dnuD)


def voigt_H(a, u):
    """H(a, u) = Re w(u + i a), normalised so that its integral over u is sqrt(pi)."""
    return wofz(u + 1j * a).real


def trapezoid_weights(x):
    """Trapezoid quadrature weights for nodes x (any spacing)."""
    x = np.asarray(x, dtype=np.float64)
    w = np.zeros_like(x)
    if len(x) == 1:
        w[0] = 1.0
        return w
    d = np.diff(x)
    w[:-1] += 0.5 * d
    w[1:] += 0.5 * d
    return w
