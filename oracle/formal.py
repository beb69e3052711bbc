"""Short-characteristics formal solution with MALI accumulations (oracle; test only).

Solves the transfer equation dI/dtau = S - I (Eq. 1) for every direction of the A4
set and every frequency, plane by plane (Sect. 3: short characteristics of Kunasz &
Auer 1988 with linear interpolation, complete redistribution), and accumulates per
(line, voxel) the two quantities the preconditioned rate equations need (Rybicki &
Hummer 1991 with a diagonal operator, Sect. 2.1 and 3):

    Jeff  = sum_d sum_m w_d w_m phi~ (I_u e + Psi_u S_u + Psi_o eta_c / chi_o)
    1-L*  = sum_d sum_m w_d w_m phi~ ((1 - Psi_o) + Psi_o chi_c / chi_o)

so that Jbar = Jeff + L* S_l, with S_l the line source function.  Both sums have
only non-negative terms.  Where the intensity is fixed by a boundary, I itself goes
into Jeff and 1 into 1-L*.

Readings of the geometry and boundaries:
* The upwind point of a voxel lies on the adjacent z-plane at horizontal offset
  -ds (mu_x, mu_y), ds = dz / |mu_z|.  I, S and chi there come from bilinear
  interpolation with periodic wrap, or (the paper's alternative, Sect. 3) from monotone
  bicubic Hermite interpolation on the 4x4 surrounding points: along x on the four
  rows, then along y, each 1D step the cubic Hermite interpolant between the two middle
  points with the Fritsch-Butland derivatives (zero where the adjacent slopes differ in
  sign, else their harmonic mean), so every value stays within the range of its 2x2
  cell.  S varies linearly along the segment and dtau = (chi_u + chi_o) ds / 2.
* Lower boundary (upward rays): I = B_nu0(T) at the local gas temperature.  Upper
  boundary (downward rays): I = 0, or a prescribed array (Sect. 4.2).
* Where the total opacity vanishes (the profile underflows far out in a wing, or a
  clipped line opacity without background), S is the limit of (eta_c + e phi) /
  (chi_c + k phi) as phi -> 0: eta_c/chi_c with a background, else the line source
  function e/k, else 0.  A segment from an opaque upwind point still sees this S.
* Segment update: e = exp(-dtau), e0 = 1 - e, Psi_o = 1 - e0/dtau, Psi_u = e0/dtau - e,
  I_o = I_u e + Psi_u S_u + Psi_o S_o; for dtau < 1e-2 the exact series of Psi_o and
  Psi_u (6 terms) replaces the direct formula.
"""
from __future__ import annotations

import numpy as np

from . import physics as ph

SERIES_DTAU = 1.0e-2


def psi_coefficients(dtau):
    """(e, Psi_u, Psi_o) of the linear short-characteristics segment, FP64."""
    dtau = np.asarray(dtau, dtype=np.float64)
    ex = np.exp(-dtau)
    e0 = -np.expm1(-dtau)
    small = dtau < SERIES_DTAU
    with np.errstate(divide="ignore", invalid="ignore"):
        r = e0 / dtau
        psi_o = 1.0 - r
        psi_u = r - ex
    if np.any(small):
        x = dtau[small]
        # Psi_o = sum_{n>=1} (-1)^{n+1} x^n/(n+1)!, Psi_u = sum_{n>=1} (-1)^{n+1} n x^n/(n+1)!
        po = np.zeros_like(x)
        pu = np.zeros_like(x)
        fact = 1.0
        xn = np.ones_like(x)
        for nn in range(1, 7):
            xn = xn * x
            fact *= (nn + 1)
            sgn = 1.0 if nn % 2 == 1 else -1.0
            po += sgn * xn / fact
            pu += sgn * nn * xn / fact
        psi_o[small] = po
        psi_u[small] = pu
    return ex, psi_u, psi_o


def _hermite_between(v0, v1, v2, v3, t):
    """Monotone cubic Hermite interpolant between v1 and v2 (unit spacing) at fraction t."""
    def slope(sl, sr):
        same = sl * sr > 0.0
        return np.where(same, sl * sr / np.where(same, 0.5 * sr + 0.5 * sl, 1.0), 0.0)
    d1 = slope(v1 - v0, v2 - v1)
    d2 = slope(v2 - v1, v3 - v2)
    t2, t3 = t * t, t * t * t
    return (2 * t3 - 3 * t2 + 1) * v1 + (t3 - 2 * t2 + t) * d1 + (-2 * t3 + 3 * t2) * v2 + (t3 - t2) * d2


def upwind_interp(Q, sx, sy, op="bilinear"):
    """Periodic interpolation of Q[..., ny, nx] at (i + sx, j + sy), bilinear or monotone
    bicubic Hermite."""
    ix = int(np.floor(sx))
    iy = int(np.floor(sy))
    fx = sx - ix
    fy = sy - iy
    if op == "hermite":
        def at(dr, dc):
            return np.roll(Q, (-iy - dr, -ix - dc), axis=(-2, -1))
        rows = [_hermite_between(at(r, -1), at(r, 0), at(r, 1), at(r, 2), fx) for r in (-1, 0, 1, 2)]
        return _hermite_between(rows[0], rows[1], rows[2], rows[3], fy)
    if op != "bilinear":
        raise ValueError("unknown upwind interpolation %r" % (op,))
    q00 = np.roll(Q, (-iy, -ix), axis=(-2, -1))
    q01 = np.roll(Q, (-iy, -ix - 1), axis=(-2, -1))
    q10 = np.roll(Q, (-iy - 1, -ix), axis=(-2, -1))
    q11 = np.roll(Q, (-iy - 1, -ix - 1), axis=(-2, -1))
    return (1.0 - fy) * ((1.0 - fx) * q00 + fx * q01) + fy * ((1.0 - fx) * q10 + fx * q11)


def safe_div(num, chi):
    """num / chi where chi > 0, else 0."""
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(chi > 0.0, num / chi, 0.0)


def source_function(chi, chi_c, eta_c, k, e, phi):
    """(eta_c + e phi) / chi, or its limit as phi -> 0 where chi vanishes."""
    with np.errstate(divide="ignore", invalid="ignore"):
        lim = np.where(chi_c > 0.0, eta_c / chi_c, np.where(k > 0.0, e / k, 0.0))
        return np.where(chi > 0.0, (eta_c + e * phi) / chi, lim)


def plane_order(nz, mu_z):
    return range(nz) if mu_z > 0 else range(nz - 1, -1, -1)


def sweep(geom, mu, local, boundary, accumulate=None, keep_top=False):
    """Sweep one direction through all z-planes.

    geom: object with nz, dx, dy, z and optionally sc_interp ("bilinear" by default).  local(k) -> (chi, S, extra) at plane k,
    arrays (nf, ny, nx).  boundary(k) -> I at the boundary plane k.
    accumulate(k, kind, data) is called per plane with kind 'bc' (data = (I, extra))
    or 'seg' (data = (I_u, S_u, ex, psi_u, psi_o, I_o, chi, S, extra)).
    Returns I at the last plane of the sweep if keep_top.
    """
    order = list(plane_order(geom.nz, mu[2]))
    k0 = order[0]
    chi_p, S_p, extra = local(k0)
    I_p = boundary(k0)
    if accumulate is not None:
        accumulate(k0, "bc", (I_p, extra))
    for kp, k in zip(order[:-1], order[1:]):
        dz = abs(geom.z[k] - geom.z[kp])
        ds = dz / abs(mu[2])
        sx = -ds * mu[0] / geom.dx
        sy = -ds * mu[1] / geom.dy
        op = getattr(geom, "sc_interp", "bilinear")
        I_u = upwind_interp(I_p, sx, sy, op)
        S_u = upwind_interp(S_p, sx, sy, op)
        chi_u = upwind_interp(chi_p, sx, sy, op)
        chi_o, S_o, extra = local(k)
        dtau = 0.5 * (chi_u + chi_o) * ds
        ex, psi_u, psi_o = psi_coefficients(dtau)
        I_o = I_u * ex + psi_u * S_u + psi_o * S_o
        if accumulate is not None:
            accumulate(k, "seg", (I_u, S_u, ex, psi_u, psi_o, I_o, chi_o, S_o, extra))
        I_p, S_p, chi_p = I_o, S_o, chi_o
    return I_p if keep_top else None


def formal_solution(lev, n, want_jbar=False, dirs=None):
    """Formal solution at populations n on level ``lev``.

    Returns (Jeff, one_minus_Lstar) with shape (nline, nz, ny, nx), plus the plain
    Jbar = sum w phi~ I if want_jbar.  ``dirs`` restricts the direction sums to a subset
    of the A4 directions (their partial sums; the default is all of them).
    """
    kk, ee = lev.line_coefficients(n)
    norm = lev.norm()
    lo = lev.line_of
    nline = lev.nline
    shape = (nline, lev.nz, lev.ny, lev.nx)
    Jeff = np.zeros(shape)
    omL = np.zeros(shape)
    Jbar = np.zeros(shape) if want_jbar else None
    fs = lev.fstart

    for d in (range(len(lev.wmu)) if dirs is None else dirs):
        mu = lev.mu[d]

        def local(k, mu=mu):
            phi = lev.profile(k, mu)
            chi_c = lev.chi_c[lo, k]
            eta_c = lev.eta_c[lo, k]
            chi = chi_c + kk[lo, k] * phi
            S = source_function(chi, chi_c, eta_c, kk[lo, k], ee[lo, k], phi)
            wphi = lev.wmu[d] * lev.wnu[:, None, None] * phi * norm[lo, k]
            return chi, S, (wphi, chi_c, eta_c)

        def boundary(k, mu=mu):
            if mu[2] > 0:
                return np.broadcast_to(lev.B[lo, k], (lev.nf, lev.ny, lev.nx)).copy()
            if lev.top_I is not None:
                return np.array(lev.top_I, dtype=np.float64)
            return np.zeros((lev.nf, lev.ny, lev.nx))

        def accumulate(k, kind, data):
            if kind == "bc":
                I, (wphi, _, _) = data
                Jeff[:, k] += np.add.reduceat(wphi * I, fs, axis=0)
                omL[:, k] += np.add.reduceat(wphi, fs, axis=0)
                if want_jbar:
                    Jbar[:, k] += np.add.reduceat(wphi * I, fs, axis=0)
                return
            I_u, S_u, ex, psi_u, psi_o, I_o, chi, S, (wphi, chi_c, eta_c) = data
            Jeff[:, k] += np.add.reduceat(wphi * (I_u * ex + psi_u * S_u + psi_o * safe_div(eta_c, chi)), fs, axis=0)
            omL[:, k] += np.add.reduceat(wphi * ((1.0 - psi_o) + psi_o * safe_div(chi_c, chi)), fs, axis=0)
            if want_jbar:
                Jbar[:, k] += np.add.reduceat(wphi * I_o, fs, axis=0)

        sweep(lev, mu, local, boundary, accumulate)
    if want_jbar:
        return Jeff, omL, Jbar
    return Jeff, omL


def _continuum_bilinear_only(lev):
    if getattr(lev, "sc_interp", "bilinear") != "bilinear":
        raise ValueError("the continuum frequencies are swept with bilinear upwind interpolation only")


def continuum_opacity_source(lev, n, k):
    """At plane k and every continuum frequency, from populations n: the opacities chi_t of
    the continua, chi = sum_t chi_t, E_u per upper level u (both in the continuum_formal_
    solution notation) and S = sum_u n_u E_u / chi (0 where chi = 0).  Arrays (nfc, ny, nx)."""
    nup = len(lev.cont_uppers)
    e2 = lev.cont_e[:, :, :, 0]                                     # (nfc, 1, 1)
    chis = [lev.cont_alpha[t][:, None, None]
            * np.maximum(n[lev.cont_lower[t]][k] - n[lev.cont_upper[t]][k] * lev.cont_g[t][:, k], 0.0)
            for t in range(lev.ncont)]
    E = [sum(lev.cont_alpha[t][:, None, None] * lev.cont_g[t][:, k]
             for t in range(lev.ncont) if lev.cont_uidx[t] == u) * e2 for u in range(nup)]
    chi = sum(chis)
    eta = sum(n[lev.cont_uppers[u]][k] * E[u] for u in range(nup))
    return chis, chi, E, safe_div(eta, chi)


def continuum_formal_solution(lev, n, want_j=False):
    """Formal solution at the frequencies of the active continua, with the accumulations
    of the preconditioned continuum rates.

    At a continuum frequency nu every continuum t open there (nu >= its edge) adds
    opacity chi_t = alpha_t (n_l - n_c g_t)^+ and emissivity eta_t = n_c g_t alpha_t 2 h nu^3/c^2
    (g_t = (n_l*/n_c*) exp(-h nu/kT), n_l and n_c the populations of t's lower and upper
    level); there is no background; S = sum eta / sum chi.  Boundaries as for the lines:
    I = B_nu(T) below, I = 0 above.  The net radiative rate of continuum t,
    4 pi int dnu/(h nu) (chi_t J - eta_t), with J = Jeff + L* S at the point, is made linear
    in the new populations the way Rybicki & Hummer (1991, 1992) precondition overlapping
    transitions: the local part L* S uses the new emissivity, sum_u n_u E_u with
    E_u = sum_s g_s alpha_s 2 h nu^3/c^2 over the continua s open at nu whose upper level
    is u, and the opacity ratio chi_t / chi of the current populations.  Per voxel and
    continuum this gives the sums over directions and frequencies

        U_t   = 4 pi sum w_d w_tk alpha_t Jeff_d / (h nu)            (times n_l: upward)
        G_t   = 4 pi sum w_d w_tk alpha_t g_t Jeff_d / (h nu)        (times n_c: downward)
        L_t,u = 4 pi sum w_d w_tk (chi_t / chi) Psi_o E_u / (h nu)   (times n_u: upward)

    with Jeff_d = I_u e + Psi_u S_u on a segment and the fixed I at a boundary.  The net
    upward rate of continuum t is n_l U_t - n_c (G_t + F_t) + sum_u n_u L_t,u (F_t, the
    spontaneous part, is the level's cont_F); the term of t's own upper level joins the
    downward rate coefficient, G_t + F_t - L_t,c.  The upper levels u are lev.cont_uppers.
    Returns an array (2 + nup, ncont, nz, ny, nx) of (U, G, L_.,0, ..., L_.,nup-1), and the
    mean intensity J (nfc, nz, ny, nx) too if want_j.
    """
    _continuum_bilinear_only(lev)
    nfc = lev.cont_nu.size
    shape = (lev.nz, lev.ny, lev.nx)
    nup = len(lev.cont_uppers)
    acc = np.zeros((2 + nup, lev.ncont) + shape)
    Jm = np.zeros((nfc,) + shape) if want_j else None
    f = 4.0 * np.pi / (ph.H * lev.cont_nu)                         # (nfc,)
    wa = lev.cont_w * lev.cont_alpha * f[None, :]                   # (ncont, nfc)

    def plane(k):
        return continuum_opacity_source(lev, n, k)

    for d in range(len(lev.wmu)):
        mu = lev.mu[d]
        wd = lev.wmu[d]

        def local(k):
            chis, chi, E, S = plane(k)
            return chi, S, (chis, E)

        def boundary(k, mu=mu):
            if mu[2] > 0:
                return lev.cont_B[:, k].copy()
            return np.zeros((nfc, lev.ny, lev.nx))

        def accumulate(k, kind, data):
            if kind == "bc":
                I, _ = data
                Jd, lam = I, None
                Io = I
            else:
                I_u, S_u, ex, psi_u, psi_o, I_o, chi, S, (chis, E) = data
                Jd = I_u * ex + psi_u * S_u
                lam = (chis, chi, psi_o, E)
                Io = I_o
            for t in range(lev.ncont):
                acc[0, t, k] += wd * np.tensordot(wa[t], Jd, axes=(0, 0))
                acc[1, t, k] += wd * np.tensordot(wa[t], lev.cont_g[t][:, k] * Jd, axes=(0, 0))
                if lam is not None:
                    chis, chi, psi_o, E = lam
                    for u in range(nup):
                        acc[2 + u, t, k] += wd * np.tensordot(f * lev.cont_w[t], safe_div(chis[t], chi) * psi_o * E[u],
                                                              axes=(0, 0))
            if want_j:
                Jm[:, k] += wd * Io

        sweep(lev, mu, local, boundary, accumulate)
    if want_j:
        return acc, Jm
    return acc


def emergent_intensity(lev, n, mus):
    """I at the top plane for each upward direction in mus: shape (ndir, nf, ny, nx)."""
    kk, ee = lev.line_coefficients(n)
    lo = lev.line_of
    out = []
    for mu in np.atleast_2d(np.asarray(mus, dtype=np.float64)):
        mu = mu / np.linalg.norm(mu)
        if not mu[2] > 0:
            raise ValueError("emergent directions must point upward")

        def local(k, mu=mu):
            phi = lev.profile(k, mu)
            chi = lev.chi_c[lo, k] + kk[lo, k] * phi
            S = source_function(chi, lev.chi_c[lo, k], lev.eta_c[lo, k], kk[lo, k], ee[lo, k], phi)
            return chi, S, None

        def boundary(k):
            return np.broadcast_to(lev.B[lo, k], (lev.nf, lev.ny, lev.nx)).copy()

        out.append(sweep(lev, mu, local, boundary, None, keep_top=True))
    return np.stack(out)


def continuum_emergent_intensity(lev, n, mus):
    """I at the top plane at every continuum frequency for each upward direction in mus:
    shape (ndir, nfc, ny, nx).  Opacity and source function as in continuum_formal_solution,
    I = B_nu(T) at the lower boundary, bilinear upwind interpolation."""
    _continuum_bilinear_only(lev)
    out = []
    for mu in np.atleast_2d(np.asarray(mus, dtype=np.float64)):
        mu = mu / np.linalg.norm(mu)
        if not mu[2] > 0:
            raise ValueError("emergent directions must point upward")

        def local(k):
            _, chi, _, S = continuum_opacity_source(lev, n, k)
            return chi, S, None

        def boundary(k):
            return lev.cont_B[:, k].copy()

        out.append(sweep(lev, mu, local, boundary, None, keep_top=True))
    return np.stack(out)
