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
