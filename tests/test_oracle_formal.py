"""Pins of the oracle's formal solution: closed forms along rays, the isothermal LTE
invariant, and the diagonal operator against a brute-force Lambda matrix (no GPU)."""
import mpmath
import numpy as np
import pytest

from oracle import physics as ph
from oracle.angles import a4_directions
from oracle.formal import SERIES_DTAU, formal_solution, psi_coefficients, sweep, upwind_interp
from oracle.levels import Level
from oracle.rates import zero_radiation
from paper_1701_01607_amd import synth


class Geom:
    def __init__(self, z, dx=1.0, dy=1.0):
        self.z = np.asarray(z, dtype=np.float64)
        self.nz = len(z)
        self.dx, self.dy = dx, dy


def test_psi_series_and_direct_branches_against_extended_precision():
    mpmath.mp.dps = 40
    for x in (1e-6, 3e-4, 0.5 * SERIES_DTAU, 0.999 * SERIES_DTAU, SERIES_DTAU, 0.3, 5.0, 60.0):
        ex, pu, po = psi_coefficients(np.array([x]))
        X = mpmath.mpf(x)
        e0 = 1 - mpmath.e ** (-X)
        ref_o = 1 - e0 / X
        ref_u = e0 / X - mpmath.e ** (-X)
        assert float(po[0]) == pytest.approx(float(ref_o), rel=5e-14)
        assert float(pu[0]) == pytest.approx(float(ref_u), rel=5e-14)
        assert float(ex[0] + pu[0] + po[0]) == pytest.approx(1.0, rel=1e-15)


def test_upwind_interp_integer_and_half_shifts():
    rng = np.random.default_rng(5)
    Q = rng.random((3, 6, 8))
    assert np.array_equal(upwind_interp(Q, 2.0, -1.0), np.roll(Q, (1, -2), axis=(-2, -1)))
    half = upwind_interp(Q, 0.5, 0.0)
    assert np.allclose(half, 0.5 * (Q + np.roll(Q, -1, axis=-1)), rtol=1e-15)
    # a field linear in x (away from the wrap) is reproduced exactly at fractional shifts
    x = np.arange(8.0)
    L = np.broadcast_to(x, (6, 8)).copy()
    got = upwind_interp(L, 0.3, 0.7)
    assert np.allclose(got[:, :6], x[:6] + 0.3, rtol=1e-14)


def _homog_local(chi_of_k, S_of_k, nf=2, ny=4, nx=4):
    def local(k):
        return (np.full((nf, ny, nx), chi_of_k(k)), np.full((nf, ny, nx), S_of_k(k)), None)
    return local


def test_constant_source_function_closed_form_all_directions():
    # I = I0 exp(-tau) + S (1 - exp(-tau)), tau the trapezoid sum along the ray
    z = np.cumsum(np.concatenate([[0.0], np.random.default_rng(7).uniform(0.5, 2.0, 20)]))
    chi = lambda k: 0.05 * np.exp(0.35 * k)      # spans dtau << 1 to dtau >> 1
    S0, I0 = 2.5, 0.7
    mu, _ = a4_directions()
    for m in mu:
        order = range(len(z)) if m[2] > 0 else range(len(z) - 1, -1, -1)
        order = list(order)
        tau = sum(0.5 * (chi(a) + chi(b)) * abs(z[b] - z[a]) / abs(m[2]) for a, b in zip(order[:-1], order[1:]))
        top = sweep(Geom(z), m, _homog_local(chi, lambda k: S0), lambda k: np.full((2, 4, 4), I0), keep_top=True)
        assert np.allclose(top, I0 * np.exp(-tau) + S0 * (-np.expm1(-tau)), rtol=1e-13)


def test_linear_source_function_in_tau_is_exact():
    # S(t) = alpha + beta t along a vertical ray from t = 0 at the bottom:
    # I(T) = I0 e^-T + alpha (1 - e^-T) + beta (T - 1 + e^-T)
    z = np.linspace(0.0, 40.0, 41)
    chi = lambda k: 1e-3 * 1.4 ** k
    taus = [0.0]
    for k in range(1, len(z)):
        taus.append(taus[-1] + 0.5 * (chi(k - 1) + chi(k)) * (z[k] - z[k - 1]))
    alpha, beta, I0 = 0.4, 0.03, 1.3
    m = np.array([0.0, 0.0, 1.0])
    top = sweep(Geom(z), m, _homog_local(chi, lambda k: alpha + beta * taus[k]),
                lambda k: np.full((2, 4, 4), I0), keep_top=True)
    T = taus[-1]
    exact = I0 * np.exp(-T) + alpha * (1 - np.exp(-T)) + beta * (T - 1 + np.exp(-T))
    assert np.allclose(top, exact, rtol=1e-12)


def _isothermal_six_level(nx=4, ny=4, nz=9, seed=3):
    atom = synth.caii_like_atom(15)
    atm = synth.atmos_stratified(nx=nx, ny=ny, nz=nz, dx=200 * synth.KM, seed=seed)
    atm["T"] = np.full_like(atm["T"], 6000.0)   # isothermal, velocities kept
    return atom, atm


def test_isothermal_lte_gives_planck_everywhere():
    atom, atm = _isothermal_six_level()
    lev = Level(atom, atm)
    lev.top_I = lev.B[lev.line_of, -1]           # prescribed incoming I = B at the top
    n = lev.nstar
    Jeff, omL, Jbar = formal_solution(lev, n, want_jbar=True)
    assert np.allclose(Jbar, lev.B, rtol=1e-12)
    assert np.allclose(Jeff, omL * lev.B, rtol=1e-12)
    assert np.all(omL > 0) and np.all(omL <= 1.0 + 1e-12)


def test_jbar_identity_jeff_plus_lambda_star_times_line_source():
    # Jbar = Jeff + L* S_l for a line without background (two-level atom)
    atom = synth.two_level_atom(1e-2)
    atm = synth.atmos_isothermal(nx=4, ny=4, nz=12)
    rng = np.random.default_rng(11)
    for k in ("vx", "vy", "vz"):
        atm[k] = rng.uniform(-1e5, 1e5, atm[k].shape)
    lev = Level(atom, atm)
    n = zero_radiation(lev)
    Jeff, omL, Jbar = formal_solution(lev, n, want_jbar=True)
    A, B12, B21 = lev.einstein[0]
    S = n[1] * A / (n[0] * B12 - n[1] * B21)
    assert np.allclose(Jbar, Jeff + (1.0 - omL) * S[None], rtol=1e-11)


def test_lambda_star_is_the_diagonal_of_the_brute_force_operator():
    atom = synth.two_level_atom(1e-2)
    atm = synth.atmos_isothermal(nx=4, ny=4, nz=7, dz=150 * synth.KM, dx=120 * synth.KM)
    rng = np.random.default_rng(12)
    for k in ("vx", "vy", "vz"):
        atm[k] = rng.uniform(-1.5e5, 1.5e5, atm[k].shape)
    lev = Level(atom, atm)
    n = zero_radiation(lev)
    lev.top_I = np.zeros((lev.nf, lev.ny, lev.nx))
    kk, _ = lev.line_coefficients(n)
    norm = lev.norm()
    nvox = lev.nz * lev.ny * lev.nx
    # batch of unit source functions, one per voxel
    Lam = np.zeros((nvox, lev.nz, lev.ny, lev.nx))
    for d in range(24):
        mu = lev.mu[d]

        def local(k, mu=mu):
            phi = lev.profile(k, mu)
            chi = kk[0, k][None] * phi
            S = np.zeros((nvox,) + chi.shape)
            for b in range(nvox):
                kb, jb, ib = np.unravel_index(b, (lev.nz, lev.ny, lev.nx))
                if kb == k:
                    S[b, :, jb, ib] = 1.0
            wphi = lev.wmu[d] * lev.wnu[:, None, None] * phi * norm[0, k][None]
            return np.broadcast_to(chi, S.shape), S, wphi

        def acc(k, kind, data):
            if kind == "bc":
                return
            I_o, wphi = data[5], data[8]
            Lam[:, k] += (wphi[None] * I_o).sum(axis=1)

        sweep(lev, mu, local, lambda k: np.zeros((nvox, lev.nf, lev.ny, lev.nx)), acc)
    diag = np.array([Lam[b].reshape(-1)[b] for b in range(nvox)])
    _, omL = formal_solution(lev, n)
    assert np.allclose(diag, 1.0 - omL[0].reshape(-1), rtol=1e-11, atol=1e-15)
    # and the operator is non-negative with row sums below one
    assert Lam.min() >= -1e-15


def test_source_function_is_continuous_where_the_opacity_vanishes():
    """Where the total opacity is zero the source function takes its limit as the
    profile goes to zero: eta_c/chi_c with a background, else the line's e/k, else 0.
    The value at phi = 0 must equal the value an infinitesimal phi away."""
    from oracle.formal import source_function
    tiny = 1e-300
    cases = [  # chi_c, eta_c, k, e
        (2.0, 3.0, 5.0, 7.0),     # background and line
        (0.0, 0.0, 5.0, 7.0),     # line only: S = e/k at any phi > 0
        (2.0, 3.0, 0.0, 0.0),     # background only
        (0.0, 0.0, 0.0, 0.0),     # nothing: S = 0
    ]
    for chi_c, eta_c, k, e in cases:
        chi_c, eta_c, k, e = (np.array([x]) for x in (chi_c, eta_c, k, e))
        at0 = source_function(chi_c + k * 0.0, chi_c, eta_c, k, e, np.array([0.0]))
        near = source_function(chi_c + k * tiny, chi_c, eta_c, k, e, np.array([tiny]))
        if chi_c[0] + k[0] > 0.0:
            np.testing.assert_allclose(at0, near, rtol=1e-12)
        else:
            assert at0[0] == 0.0
    # away from the limit it is the plain ratio (eta_c + e phi)/(chi_c + k phi)
    phi = np.array([0.3])
    s = source_function(np.array([2.0 + 5.0 * 0.3]), np.array([2.0]), np.array([3.0]), np.array([5.0]),
                        np.array([7.0]), phi)
    np.testing.assert_allclose(s, (3.0 + 7.0 * 0.3) / (2.0 + 5.0 * 0.3), rtol=1e-15)


def _fb(sl, sr):
    return sl * sr / (0.5 * sr + 0.5 * sl) if sl * sr > 0.0 else 0.0


def _cubic_value(v0, v1, v2, v3, t):
    """Cubic through (0, v1), (1, v2) with the monotone slopes at 0 and 1, evaluated at t
    from its power-basis coefficients."""
    d1, d2 = _fb(v1 - v0, v2 - v1), _fb(v2 - v1, v3 - v2)
    A = np.array([[1, 0, 0, 0], [1, 1, 1, 1], [0, 1, 0, 0], [0, 1, 2, 3]], dtype=float)
    c = np.linalg.solve(A, np.array([v1, v2, d1, d2]))
    return c[0] + c[1] * t + c[2] * t ** 2 + c[3] * t ** 3


def test_hermite_upwind_interp_matches_the_cubic_point_by_point():
    rng = np.random.default_rng(51)
    Q = rng.random((5, 7))
    for sx, sy in ((-1.3, 0.4), (0.75, -2.2), (2.0, 0.5)):
        got = upwind_interp(Q, sx, sy, "hermite")
        ix, iy = int(np.floor(sx)), int(np.floor(sy))
        fx, fy = sx - ix, sy - iy
        for j in range(5):
            for i in range(7):
                rows = []
                for r in (-1, 0, 1, 2):
                    v = [Q[(j + iy + r) % 5, (i + ix + c) % 7] for c in (-1, 0, 1, 2)]
                    rows.append(_cubic_value(*v, fx))
                assert got[j, i] == pytest.approx(_cubic_value(*rows, fy), rel=1e-12, abs=1e-14)


def test_hermite_upwind_interp_stays_in_its_cell_and_keeps_simple_fields():
    rng = np.random.default_rng(52)
    Q = rng.random((2, 8, 9)) ** 3
    sx, sy = -0.62, 1.37
    got = upwind_interp(Q, sx, sy, "hermite")
    ix, iy = int(np.floor(sx)), int(np.floor(sy))
    cell = np.stack([np.roll(Q, (-iy - a, -ix - b), axis=(-2, -1)) for a in (0, 1) for b in (0, 1)])
    assert np.all(got >= cell.min(axis=0) - 1e-15) and np.all(got <= cell.max(axis=0) + 1e-15)
    assert np.allclose(upwind_interp(np.full((3, 4), 2.5), 0.3, -0.8, "hermite"), 2.5, rtol=1e-15)
    # integer shifts are pure moves, and a field linear in x (away from the wrap) stays exact
    assert np.array_equal(upwind_interp(Q, 2.0, -1.0, "hermite"), np.roll(Q, (1, -2), axis=(-2, -1)))
    x = np.arange(9.0)
    L = np.broadcast_to(x, (8, 9)).copy()
    assert np.allclose(upwind_interp(L, 0.3, 0.7, "hermite")[:, 1:6], x[1:6] + 0.3, rtol=1e-14)
    with pytest.raises(ValueError):
        upwind_interp(Q, 0.3, 0.3, "spline")


def test_hermite_upwind_diffuses_a_beam_less_than_bilinear():
    # A searchlight beam in a transparent medium crossing planes along an inclined ray:
    # the exact solution moves the boundary pattern without change.  Both schemes
    # smear it (short characteristics interpolate at every plane); the monotone cubic
    # keeps more of the peak and never overshoots.
    nz, nx = 25, 48
    z = np.arange(nz, dtype=float)
    mu = np.array([0.6, 0.0, 0.8])                  # shift 0.75 cells per plane along x
    xs = np.arange(nx)
    beam = np.exp(-0.5 * ((xs - 8.0) / 1.5) ** 2)
    I0 = np.broadcast_to(beam, (1, 2, nx)).copy()

    class G:
        def __init__(self, op):
            self.nz, self.dx, self.dy, self.z, self.sc_interp = nz, 1.0, 1.0, z, op

    def local(k):
        return np.full((1, 2, nx), 1e-30), np.zeros((1, 2, nx)), None

    peaks = {}
    for op in ("bilinear", "hermite"):
        top = sweep(G(op), mu, local, lambda k: I0.copy(), keep_top=True)[0, 0]
        assert top.min() >= -1e-15 and top.max() <= 1.0 + 1e-15
        peaks[op] = top.max()
        # the centre moved by 0.75 cells per plane
        assert abs(np.sum(xs * top) / np.sum(top) - (8.0 + 0.75 * (nz - 1))) < 0.5
    assert peaks["hermite"] > 1.3 * peaks["bilinear"]
