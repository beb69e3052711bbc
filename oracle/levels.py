"""Per-grid-level problem data and the grid hierarchy (oracle; test infrastructure only).

A ``Level`` holds one grid level's atmosphere and everything derived from it that
does not depend on the populations: Planck functions, Doppler widths, damping,
background opacity/emissivity, the frequency quadrature, LTE populations and the fixed
(collisional + bound-free) rates, and the profile normalisation.

Readings:
* Frequencies: each line has velocity offsets q_m; nu_m = nu0 (1 + q_m / c) and the
  weights are trapezoid weights in Hz.
* Profile: phi = H(a, u) / (sqrt(pi) dnu_D) with u = (q_m - v.n) / v_D, n the
  propagation direction (the lab-frame profile moves to +v.n).
* Normalisation: phi~ = phi / sum_d sum_m w_d w_m phi per (voxel, line), so that an
  isotropic I = B gives Jbar = B exactly.  Used only inside the Jbar and Lambda*
  quadratures.
* Active continua: every line frequency must lie below every continuum edge (the line
  sweeps carry no bound-free opacity); an atom whose lines reach an edge is refused.
* Grid hierarchy (Sect. 4.1, 4.2, 4.7): the coarse level keeps every second point;
  its atmosphere is the restriction of the finer one (full weighting unless another
  operator is asked for).  Level index
  k = 1 is the coarsest, k = nlev the finest (Sect. 2.2).
"""
from __future__ import annotations

import numpy as np

from . import physics as ph
from .angles import a4_directions
from .transfer import coarsen_atmosphere


class Level:
    def __init__(self, atom, atmos, top_I=None, sc_interp="bilinear"):
        self.atom = atom
        self.atmos = atmos
        self.nx, self.ny, self.nz = atmos["nx"], atmos["ny"], atmos["nz"]
        self.dx, self.dy = atmos["dx"], atmos["dy"]
        self.z = np.asarray(atmos["z"], dtype=np.float64)
        self.N = len(atom["levels"])
        self.nline = len(atom["lines"])
        T = atmos["T"]
        self.T = T
        self.ntot = atmos["ntot"]
        self.v = np.stack([atmos["vx"], atmos["vy"], atmos["vz"]])
        self.vD = ph.doppler_velocity(atom, T)

        self.nu0 = np.array([ph.line_nu0(atom, l) for l in range(self.nline)])
        self.lower = [ln["lower"] for ln in atom["lines"]]
        self.upper = [ln["upper"] for ln in atom["lines"]]
        self.einstein = [ph.einstein(atom, l) for l in range(self.nline)]
        self.B = np.stack([ph.planck_nu(self.nu0[l], T) for l in range(self.nline)])
        self.a = np.stack([ph.damping(atom, l, T, atmos["nH"], self.vD) for l in range(self.nline)])
        if atmos.get("chi_c") is not None:
            self.chi_c = np.asarray(atmos["chi_c"], dtype=np.float64)[: self.nline]
        else:
            self.chi_c = np.zeros((self.nline,) + T.shape)
        self.eta_c = self.chi_c * self.B

        # flat frequency list over all lines
        qs = [np.asarray(ln["q"], dtype=np.float64) for ln in atom["lines"]]
        self.nfreq = np.array([len(q) for q in qs])
        self.fstart = np.concatenate([[0], np.cumsum(self.nfreq)[:-1]])
        self.q = np.concatenate(qs)
        self.line_of = np.concatenate([np.full(len(q), l) for l, q in enumerate(qs)])
        self.wnu = np.concatenate(
            [ph.trapezoid_weights(self.nu0[l] * (1.0 + qs[l] / ph.C)) for l in range(self.nline)])
        self.nf = len(self.q)

        self.mu, self.wmu = a4_directions()
        self.nstar = ph.lte_populations(atom, T, atmos["ne"], self.ntot)
        self.active_continua = atom.get("continuum_nu") is not None
        self.fixed = ph.collision_matrix(atom, T, atmos["ne"], self.nstar)
        if self.active_continua:
            self._continuum_setup(atom, T)
        else:
            self.fixed = self.fixed + ph.fixed_bf_rates(atom, T, self.nstar)
        self.top_I = top_I
        self.sc_interp = sc_interp   # upwind interpolation of the formal solution
        self._norm = None

    # ---- active continua ---------------------------------------------------
    def _continuum_setup(self, atom, T):
        """Frequencies, cross-sections and weights of the active continua, the LTE ratio
        g_t(nu) = (n_l*/n_c*) exp(-h nu/kT) per voxel, and the spontaneous part of the
        downward rate F_t = 4 pi sum_k w_tk alpha_tk g_tk (2 h nu^3/c^2) / (h nu)."""
        self.cont_nu = np.asarray(atom["continuum_nu"], dtype=np.float64)
        self.cont_alpha, self.cont_w = ph.continuum_quadrature(atom, self.cont_nu)
        self.cont_lower = [ct["lower"] for ct in atom["continua"]]
        self.cont_upper = [ct["upper"] for ct in atom["continua"]]
        self.ncont = len(self.cont_lower)
        # the distinct upper levels, in order of first appearance, and each continuum's
        # index among them
        self.cont_uppers = list(dict.fromkeys(self.cont_upper))
        self.cont_uidx = [self.cont_uppers.index(c) for c in self.cont_upper]
        # the line sweeps carry no bound-free opacity, so every line must lie below every
        # edge, where the continua's cross-sections vanish
        edge = min(ph.C * (atom["levels"][c]["E"] - atom["levels"][l]["E"])
                   for l, c in zip(self.cont_lower, self.cont_upper))
        for l in range(self.nline):
            top = self.nu0[l] * (1.0 + np.max(atom["lines"][l]["q"]) / ph.C)
            if top >= edge:
                raise ValueError("line %d reaches %.6e Hz, at or above the continuum edge %.6e Hz" % (l, top, edge))
        nu = self.cont_nu[:, None, None, None]
        x = np.exp(-ph.H * nu / (ph.KB * T[None]))                  # (nfc, nz, ny, nx)
        self.cont_g = np.stack([(self.nstar[l] / self.nstar[c])[None] * x
                                for l, c in zip(self.cont_lower, self.cont_upper)])   # (ncont, nfc, ...)
        self.cont_e = 2.0 * ph.H * nu ** 3 / ph.C ** 2                  # 2 h nu^3 / c^2
        self.cont_B = ph.planck_nu(nu, T[None])                          # (nfc, nz, ny, nx)
        f = 4.0 * np.pi / (ph.H * self.cont_nu)                          # 4 pi / (h nu)
        self.cont_F = np.stack([np.tensordot(self.cont_w[t] * self.cont_alpha[t] * f, self.cont_g[t] * self.cont_e,
                                             axes=(0, 0)) for t in range(self.ncont)])

    # ---- profile -----------------------------------------------------------
    def profile(self, k, mu):
        """phi (Hz^-1) at plane k for propagation direction mu, shape (nf, ny, nx)."""
        lo = self.line_of
        vD = self.vD[k][None]
        vn = (mu[0] * self.v[0, k] + mu[1] * self.v[1, k] + mu[2] * self.v[2, k])[None]
        u = (self.q[:, None, None] - vn) / vD
        a = self.a[lo, k]
        dnuD = self.nu0[lo][:, None, None] * vD / ph.C
        return ph.voigt_H(a, u) / (np.sqrt(np.pi) * dnuD)

    def norm_sum(self, dirs=None):
        """sum_d sum_m w_d w_m phi per (line, voxel) over the directions ``dirs`` (all by
        default)."""
        acc = np.zeros((self.nline, self.nz, self.ny, self.nx))
        for d in (range(len(self.wmu)) if dirs is None else dirs):
            for k in range(self.nz):
                phi = self.profile(k, self.mu[d])
                wp = self.wmu[d] * self.wnu[:, None, None] * phi
                acc[:, k] += np.add.reduceat(wp, self.fstart, axis=0)
        return acc

    def norm(self):
        """Profile normalisation N_l per (line, voxel): 1 / sum_d sum_m w_d w_m phi."""
        if self._norm is None:
            self._norm = 1.0 / self.norm_sum()
        return self._norm

    # ---- population-dependent line quantities --------------------------------
    def line_coefficients(self, n):
        """(k_l^+, e_l) per (line, voxel): k = (h nu0/4pi)(n_i B_ij - n_j B_ji) clipped at 0
        and e = (h nu0/4pi) n_j A_ji, from n^+ = max(n, 0)."""
        npos = np.maximum(n, 0.0)
        kk = np.empty((self.nline,) + n.shape[1:])
        ee = np.empty_like(kk)
        for l in range(self.nline):
            Aji, Bij, Bji = self.einstein[l]
            i, j = self.lower[l], self.upper[l]
            hnu = ph.H * self.nu0[l] / (4.0 * np.pi)
            kk[l] = np.maximum(hnu * (npos[i] * Bij - npos[j] * Bji), 0.0)
            ee[l] = hnu * npos[j] * Aji
        return kk, ee


def build_hierarchy(atom, atmos, nlev, top_I=None, coarse_op="full", sc_interp="bilinear"):
    """Levels [k=1 (coarsest), ..., k=nlev (finest)] as a list indexed k-1; each coarser
    atmosphere is the restriction (`coarse_op`) of the next finer one."""
    nx, ny, nz = atmos["nx"], atmos["ny"], atmos["nz"]
    step = 2 ** (nlev - 1)
    if nx % step or ny % step or (nz - 1) % step:
        raise ValueError("grid %dx%dx%d does not admit %d levels" % (nx, ny, nz, nlev))
    atms = [atmos]
    for _ in range(nlev - 1):
        atms.append(coarsen_atmosphere(atms[-1], coarse_op))
    levels = [Level(atom, a, sc_interp=sc_interp) for a in reversed(atms)]
    if top_I is not None:
        levels[-1].top_I = top_I
    return levels
