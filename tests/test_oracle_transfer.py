"""Pins of the oracle's grid-transfer operators and angle set (no GPU)."""
import numpy as np
import pytest

from oracle.angles import a4_directions
from oracle.transfer import coarsen_atmosphere, prolong, restrict


def trapezoid_sum(q, z_index_step=1.0):
    """Index-space trapezoid sum in z, plain sums over periodic x and y."""
    w = np.ones(q.shape[-3])
    w[0] = w[-1] = 0.5
    return z_index_step * np.einsum("k,...kji->...", w, q)


def test_a4_moments_and_symmetry():
    mu, w = a4_directions()
    assert mu.shape == (24, 3)
    assert np.allclose(np.linalg.norm(mu, axis=1), 1.0, rtol=1e-15)
    assert w.sum() == pytest.approx(1.0, rel=1e-15)
    assert np.allclose(w @ mu, 0.0, atol=1e-16)
    for a in range(3):
        assert (w * mu[:, a] ** 2).sum() == pytest.approx(1.0 / 3.0, rel=1e-14)
    up = mu[:, 2] > 0
    assert (w[up] * mu[up, 2]).sum() == pytest.approx((2.0 + np.sqrt(7.0)) / 18.0, rel=1e-14)
    # octant reflections map the set onto itself
    for s in ((-1, 1, 1), (1, -1, 1), (1, 1, -1)):
        ref = mu * np.array(s)
        for m in ref:
            assert np.min(np.linalg.norm(mu - m, axis=1)) < 1e-15
    assert np.all(mu[:12, 2] > 0) and np.all(mu[12:, 2] < 0)
    assert np.allclose(mu[12:], -mu[:12])


def test_restriction_conserves_trapezoid_sum():
    rng = np.random.default_rng(1)
    q = rng.random((3, 17, 8, 12))
    qc = restrict(q)
    assert qc.shape == (3, 9, 4, 6)
    # coarse cells have twice the spacing along every axis: volume factor 8
    assert np.allclose(8.0 * trapezoid_sum(qc), trapezoid_sum(q), rtol=1e-13)


def test_restriction_of_constant_and_weights():
    q = np.full((9, 4, 4), 3.25)
    assert np.allclose(restrict(q), 3.25, rtol=1e-15)
    # a delta at an even fine point spreads with weights 1/2 (self) and 1/4 (neighbours) per axis
    q = np.zeros((9, 8, 8))
    q[4, 4, 4] = 1.0
    qc = restrict(q)
    assert qc[2, 2, 2] == pytest.approx(0.125)
    q = np.zeros((9, 8, 8))
    q[5, 4, 4] = 1.0     # odd z index: shared by coarse planes 2 and 3
    qc = restrict(q)
    assert qc[2, 2, 2] == pytest.approx(0.0625) and qc[3, 2, 2] == pytest.approx(0.0625)
    q = np.zeros((9, 8, 8))
    q[0, 0, 0] = 1.0     # boundary plane: weight 1/2 in z
    assert restrict(q)[0, 0, 0] == pytest.approx(0.5 * 0.25)


def test_prolongation_exact_for_multilinear_and_identity_at_coincident_points():
    zf = np.cumsum(np.concatenate([[0.0], np.random.default_rng(2).uniform(1, 3, 16)]))
    nx, ny = 8, 6
    xc = np.arange(nx // 2) * 2.0
    yc = np.arange(ny // 2) * 2.0
    zc = zf[::2]
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    # linear in z (physical) times a function of x, y that is linear between coarse
    # nodes and wraps periodically: use a constant plus z-linear term, and check x/y
    # midpoint averaging separately
    qc = 2.0 + 0.5 * Z
    qf = prolong(qc, zf)
    assert np.allclose(qf, (2.0 + 0.5 * zf)[:, None, None], rtol=1e-14)
    rng = np.random.default_rng(3)
    qc = rng.random((9, 3, 4))
    qf = prolong(qc, zf)
    assert np.allclose(qf[::2, ::2, ::2], qc, rtol=0, atol=0)
    assert np.allclose(qf[::2, ::2, 1::2], 0.5 * (qc + np.roll(qc, -1, axis=2)), rtol=1e-15)
    assert np.allclose(qf[::2, 1::2, ::2], 0.5 * (qc + np.roll(qc, -1, axis=1)), rtol=1e-15)
    t = (zf[1::2] - zf[0:-1:2]) / (zf[2::2] - zf[0:-1:2])
    exp = (1 - t)[:, None, None] * qc[:-1] + t[:, None, None] * qc[1:]
    assert np.allclose(qf[1::2, ::2, ::2], exp, rtol=1e-14)


def test_coarsen_atmosphere_keeps_every_second_height():
    z = np.linspace(0, 1, 9) ** 2
    atm = {"nx": 4, "ny": 4, "nz": 9, "dx": 1.0, "dy": 1.0, "z": z, "chi_c": None}
    for k in ("T", "ne", "nH", "ntot", "vx", "vy", "vz"):
        atm[k] = np.ones((9, 4, 4))
    c = coarsen_atmosphere(atm)
    assert c["nz"] == 5 and c["nx"] == 2 and c["dx"] == 2.0
    assert np.array_equal(c["z"], z[::2])


def _half_weighting_by_points(q):
    """Brute force: each coarse value written out from the 7-point definition, the
    vertical neighbour outside the grid replaced by its mirror image."""
    nz, ny, nx = q.shape
    out = np.empty(((nz - 1) // 2 + 1, ny // 2, nx // 2))
    for K in range(out.shape[0]):
        for J in range(out.shape[1]):
            for I in range(out.shape[2]):
                k, j, i = 2 * K, 2 * J, 2 * I
                below = q[k - 1, j, i] if k > 0 else q[k + 1, j, i]
                above = q[k + 1, j, i] if k < nz - 1 else q[k - 1, j, i]
                s = (q[k, j, (i - 1) % nx] + q[k, j, (i + 1) % nx] + q[k, (j - 1) % ny, i]
                     + q[k, (j + 1) % ny, i] + below + above)
                out[K, J, I] = q[k, j, i] / 2.0 + s / 12.0
    return out


def test_half_weighting_matches_its_definition_point_by_point():
    q = np.random.default_rng(11).random((9, 6, 8))
    assert np.allclose(restrict(q, "half"), _half_weighting_by_points(q), rtol=1e-15, atol=0)
    # several fields at once restrict independently
    qq = np.stack([q, 2.0 * q + 1.0])
    assert np.allclose(restrict(qq, "half")[1], 2.0 * restrict(q, "half") + 1.0, rtol=1e-14)


def test_half_weighting_of_constants_and_fourier_modes():
    assert np.allclose(restrict(np.full((9, 4, 6), -1.75), "half"), -1.75, rtol=1e-15)
    # a periodic Fourier mode along x is an eigenfunction of the stencil: the four
    # neighbours along y and z repeat the point, so the coarse value is
    # (1/2 + 4/12 + 2 cos(2 pi m / nx) / 12) times the mode at the coarse point
    nz, ny, nx, m = 9, 4, 16, 3
    x = np.arange(nx)
    f = np.broadcast_to(np.cos(2 * np.pi * m * x / nx), (nz, ny, nx))
    lam = 0.5 + 4.0 / 12.0 + 2.0 * np.cos(2 * np.pi * m / nx) / 12.0
    assert np.allclose(restrict(f, "half"), lam * f[::2, ::2, ::2], rtol=1e-14, atol=1e-15)
    # the same along y
    f = np.broadcast_to(np.sin(2 * np.pi * np.arange(8) / 8)[:, None], (nz, 8, 4))
    lam = 0.5 + 4.0 / 12.0 + 2.0 * np.cos(2 * np.pi / 8) / 12.0
    assert np.allclose(restrict(f, "half"), lam * f[::2, ::2, ::2], rtol=1e-14, atol=1e-15)


def test_half_weighting_vertical_boundary_fold():
    # a field linear in the plane index k: interior coarse planes reproduce it (the
    # stencil is symmetric), the boundary planes see the mirrored neighbour
    nz = 9
    f = np.broadcast_to(np.arange(nz, dtype=float)[:, None, None], (nz, 4, 4))
    qc = restrict(f, "half")
    assert np.allclose(qc[1:-1], f[2:-2:2, ::2, ::2], rtol=1e-15)
    assert qc[0, 0, 0] == pytest.approx(0.0 / 2 + (4 * 0.0 + 1.0 + 1.0) / 12.0, rel=1e-15)
    top = nz - 1
    assert qc[-1, 0, 0] == pytest.approx(top / 2 + (4 * top + 2 * (top - 1)) / 12.0, rel=1e-15)


def test_injection_keeps_coincident_points():
    q = np.random.default_rng(12).random((2, 9, 6, 8))
    qc = restrict(q, "inject")
    assert qc.shape == (2, 5, 3, 4)
    for K, J, I in ((0, 0, 0), (4, 2, 3), (2, 1, 1)):
        assert qc[1, K, J, I] == q[1, 2 * K, 2 * J, 2 * I]
    with pytest.raises(ValueError):
        restrict(q, "quarter")


def test_coarsen_atmosphere_by_injection():
    rng = np.random.default_rng(13)
    atm = {"nx": 8, "ny": 4, "nz": 9, "dx": 1.0, "dy": 1.0, "z": np.arange(9.0), "chi_c": rng.random((2, 9, 4, 8))}
    for k in ("T", "ne", "nH", "ntot", "vx", "vy", "vz"):
        atm[k] = rng.random((9, 4, 8))
    c = coarsen_atmosphere(atm, "inject")
    for k in ("T", "vz"):
        assert np.array_equal(c[k], atm[k][::2, ::2, ::2])
    assert np.array_equal(c["chi_c"], atm["chi_c"][:, ::2, ::2, ::2])
    f = coarsen_atmosphere(atm)
    assert not np.array_equal(f["T"], c["T"])


def _fb_derivative(sl, sr, hl, hr):
    """Fritsch-Butland derivative at a node, written out for one node."""
    if sl * sr <= 0.0:
        return 0.0
    a = (1.0 + hr / (hl + hr)) / 3.0
    return sl * sr / (a * sr + (1.0 - a) * sl)


def _cubic_through(x0, x1, y0, y1, d0, d1, x):
    """Value at x of the cubic with the given values and derivatives at x0 and x1,
    from the 4x4 linear system of its coefficients."""
    A = np.array([[1, x0, x0 ** 2, x0 ** 3], [1, x1, x1 ** 2, x1 ** 3],
                  [0, 1, 2 * x0, 3 * x0 ** 2], [0, 1, 2 * x1, 3 * x1 ** 2]], dtype=float)
    c = np.linalg.solve(A, np.array([y0, y1, d0, d1]))
    return c[0] + c[1] * x + c[2] * x ** 2 + c[3] * x ** 3


def test_hermite_z_matches_the_cubic_through_values_and_monotone_slopes():
    rng = np.random.default_rng(21)
    zf = np.cumsum(np.concatenate([[0.0], rng.uniform(0.5, 2.0, 8)]))
    zc = zf[::2]
    qc = rng.normal(size=(5, 1, 2))
    qf = prolong(qc, zf, "hermite")
    for j in range(2):
        y = qc[:, 0, j]
        s = np.diff(y) / np.diff(zc)
        d = [s[0]] + [_fb_derivative(s[i - 1], s[i], zc[i] - zc[i - 1], zc[i + 1] - zc[i])
                      for i in range(1, 4)] + [s[-1]]
        for K in range(4):
            exp = _cubic_through(zc[K], zc[K + 1], y[K], y[K + 1], d[K], d[K + 1], zf[2 * K + 1])
            assert qf[2 * K + 1, 0, 2 * j] == pytest.approx(exp, rel=1e-11, abs=1e-12)
        assert np.array_equal(qf[::2, 0, 2 * j], y)


def test_hermite_xy_periodic_midpoints():
    rng = np.random.default_rng(22)
    qc = rng.normal(size=(1, 3, 6))
    qf = prolong(qc, np.array([0.0]), "hermite")
    y = qc[0, 0]
    n = len(y)
    for i in range(n):
        sl, sr, srr = y[i] - y[i - 1], y[(i + 1) % n] - y[i], y[(i + 2) % n] - y[(i + 1) % n]
        d0, d1 = _fb_derivative(sl, sr, 1.0, 1.0), _fb_derivative(sr, srr, 1.0, 1.0)
        exp = _cubic_through(0.0, 1.0, y[i], y[(i + 1) % n], d0, d1, 0.5)
        assert qf[0, 0, 2 * i + 1] == pytest.approx(exp, rel=1e-12, abs=1e-13)
    assert np.array_equal(qf[0, ::2, ::2], qc[0])


def test_hermite_reproduces_linear_and_keeps_monotone_data_in_range():
    zf = np.cumsum(np.concatenate([[0.0], np.random.default_rng(23).uniform(1, 3, 16)]))
    qc = np.broadcast_to((1.5 - 0.25 * zf[::2])[:, None, None], (9, 2, 4))
    assert np.allclose(prolong(qc, zf, "hermite"), (1.5 - 0.25 * zf)[:, None, None], rtol=1e-13)
    # a steep monotone step: no value leaves its interval's range (a cubic through
    # centred differences overshoots here)
    zc = zf[::2]
    step = np.tanh((zc - zc.mean()) / 2.0)
    qc = np.broadcast_to(step[:, None, None], (9, 2, 2))
    qf = prolong(qc, zf, "hermite")[:, 0, 0]
    for K in range(8):
        lo, hi = sorted((step[K], step[K + 1]))
        assert lo - 1e-15 <= qf[2 * K + 1] <= hi + 1e-15
    assert np.all(np.diff(qf) >= 0)
    # at a local maximum the derivative is zero: the neighbours' midpoints stay below it
    y = np.array([0.0, 1.0, 3.0, 1.0, 0.0])
    d = [float(v) for v in np.ravel(__import__("oracle.transfer", fromlist=["x"]).monotone_slopes(y))]
    assert d[2] == 0.0


def test_hermite_is_third_order_on_smooth_monotone_data():
    # interior intervals: harmonic-mean derivatives make the interpolant at least third
    # order (error ratio >= 8 per halving; trilinear is second order, ratio 4); the two
    # end intervals use the one-sided slope and stay at least second order
    err = {"hermite": [], "trilinear": [], "ends": []}
    for n in (17, 33, 65):
        zf = np.linspace(0.0, 1.0, 2 * n - 1)
        f = np.tanh((zf - 0.4) / 0.15)
        qc = np.broadcast_to(f[::2][:, None, None], (n, 2, 2))
        for op in ("hermite", "trilinear"):
            e = np.abs(prolong(qc, zf, op)[:, 0, 0] - f)
            err[op].append(e[2:-2].max())
            if op == "hermite":
                err["ends"].append(max(e[1], e[-2]))
    assert err["hermite"][1] / err["hermite"][2] > 8.0
    assert 3.5 < err["trilinear"][1] / err["trilinear"][2] < 4.5
    assert err["ends"][1] / err["ends"][2] > 3.5
    assert err["hermite"][2] < 0.01 * err["trilinear"][2]
