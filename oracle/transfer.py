"""Grid-transfer operators (oracle; test infrastructure only).

* Coarsening (Sect. 4.1): the coarse grid keeps every second point along x, y and z,
  both vertical boundaries included (Sect. 4.2: odd N_z at every level).
* Restriction (Sect. 4.4), three operators, all centred on fine index 2c, periodic in x
  and y, weights in index space:
  - full weighting: the 27-point tensor product of the 1D weights [1/4, 1/2, 1/4].  At
    the two vertical boundary planes the reading is [1/2 self, 1/2 inward neighbour],
    which keeps the trapezoid sum of a field exactly (the paper states full weighting
    conserves the domain integral);
  - half weighting: the point itself and its six neighbours along the axes, with the
    standard 7-point weights of the multigrid literature the paper cites (1/2 for the
    point, 1/12 for each neighbour).  At a vertical boundary plane the missing outward
    neighbour's 1/12 goes to the inward one, the same fold as full weighting's boundary
    rows (a mirror of the stencil);
  - injection: the coarse value is the fine value at the same point.
* Prolongation (Sect. 4.5), two operators:
  - trilinear, the 8-point tensor product of 1D linear interpolation.  In x and y
    (uniform, periodic) an odd fine point is the mean of its two coarse neighbours; in z
    the weights are linear in the physical height;
  - cubic Hermite on the 4x4x4 coarse stencil, applied one axis at a time (x, then y,
    then z).  Along an axis a fine point between coarse nodes i and i+1 takes the cubic
    Hermite interpolant of the values and derivatives at those two nodes.  The paper
    cites Auer (2003) for it and gives no derivative formula; the derivatives here are
    the monotone ones of Fritsch & Butland (1984): zero where the slopes s_l, s_r of the
    two adjacent intervals differ in sign
    or one vanishes, else the weighted harmonic mean s_l s_r / (a s_r + (1 - a) s_l) with
    a = (1 + h_r / (h_l + h_r)) / 3 (the plain harmonic mean on a uniform axis).  At the
    two vertical boundary nodes the derivative is the slope of the one adjacent interval.
    Coincident points keep the coarse values; linear data are reproduced exactly; data
    monotone along an axis stay within the range of the two nodes.
"""
from __future__ import annotations

import numpy as np


def _restrict_periodic(q, axis):
    fw = 0.25 * np.roll(q, 1, axis=axis) + 0.5 * q + 0.25 * np.roll(q, -1, axis=axis)
    sl = [slice(None)] * q.ndim
    sl[axis] = slice(0, None, 2)
    return fw[tuple(sl)]


def _restrict_z(q, axis):
    q = np.moveaxis(q, axis, 0)
    nz = q.shape[0]
    ncz = (nz - 1) // 2 + 1
    out = np.empty((ncz,) + q.shape[1:])
    out[0] = 0.5 * q[0] + 0.5 * q[1]
    out[-1] = 0.5 * q[nz - 1] + 0.5 * q[nz - 2]
    for K in range(1, ncz - 1):
        out[K] = 0.25 * q[2 * K - 1] + 0.5 * q[2 * K] + 0.25 * q[2 * K + 1]
    return np.moveaxis(out, 0, axis)


def _half_weighting(q):
    zd = np.concatenate([q[..., 1:2, :, :], q[..., :-1, :, :]], axis=-3)   # value below (mirrored at the bottom)
    zu = np.concatenate([q[..., 1:, :, :], q[..., -2:-1, :, :]], axis=-3)  # value above (mirrored at the top)
    nb = (np.roll(q, 1, axis=-1) + np.roll(q, -1, axis=-1) + np.roll(q, 1, axis=-2) + np.roll(q, -1, axis=-2)
          + zd + zu)
    return (0.5 * q + nb / 12.0)[..., ::2, ::2, ::2]


RESTRICTIONS = ("full", "half", "inject")


def restrict(q, op="full"):
    """Restriction of q[..., nz, ny, nx] to [..., (nz+1)/2, ny/2, nx/2] by full weighting,
    half weighting or injection."""
    q = np.asarray(q, dtype=np.float64)
    assert q.shape[-1] % 2 == 0 and q.shape[-2] % 2 == 0 and q.shape[-3] % 2 == 1
    if op == "inject":
        return q[..., ::2, ::2, ::2].copy()
    if op == "half":
        return _half_weighting(q)
    if op != "full":
        raise ValueError("unknown restriction %r" % (op,))
    q = _restrict_periodic(q, q.ndim - 1)
    q = _restrict_periodic(q, q.ndim - 2)
    return _restrict_z(q, q.ndim - 3)


def _prolong_periodic(q, axis):
    q = np.moveaxis(q, axis, 0)
    n = q.shape[0]
    out = np.empty((2 * n,) + q.shape[1:])
    out[0::2] = q
    out[1::2] = 0.5 * (q + np.roll(q, -1, axis=0))
    return np.moveaxis(out, 0, axis)


def _prolong_z(q, axis, zf):
    q = np.moveaxis(q, axis, 0)
    nzc = q.shape[0]
    nz = 2 * (nzc - 1) + 1
    assert len(zf) == nz
    out = np.empty((nz,) + q.shape[1:])
    out[0::2] = q
    for K in range(nzc - 1):
        t = (zf[2 * K + 1] - zf[2 * K]) / (zf[2 * K + 2] - zf[2 * K])
        out[2 * K + 1] = (1.0 - t) * q[K] + t * q[K + 1]
    return np.moveaxis(out, 0, axis)


def monotone_slopes(y, x=None, periodic=False):
    """Fritsch-Butland derivative estimates at the nodes of y along axis 0.  x: node
    positions (default the index); periodic: y wraps around on a unit-spaced axis."""
    n = y.shape[0]
    if periodic:
        s = np.roll(y, -1, axis=0) - y                    # s[i]: slope on [i, i+1]
        sl, sr = np.roll(s, 1, axis=0), s
        a = 0.5
    else:
        x = np.arange(n, dtype=np.float64) if x is None else np.asarray(x, dtype=np.float64)
        h = np.diff(x)
        s = np.diff(y, axis=0) / h.reshape((n - 1,) + (1,) * (y.ndim - 1))
        sl, sr = s[:-1], s[1:]
        hl = h[:-1].reshape((n - 2,) + (1,) * (y.ndim - 1))
        hr = h[1:].reshape((n - 2,) + (1,) * (y.ndim - 1))
        a = (1.0 + hr / (hl + hr)) / 3.0
    same = sl * sr > 0.0
    d_in = np.where(same, sl * sr / np.where(same, a * sr + (1.0 - a) * sl, 1.0), 0.0)
    if periodic:
        return d_in
    return np.concatenate([s[:1], d_in, s[-1:]], axis=0)


def _hermite(y0, y1, d0, d1, h, t):
    """Cubic Hermite interpolant on [x0, x0 + h] at fraction t."""
    t2, t3 = t * t, t * t * t
    return ((2 * t3 - 3 * t2 + 1) * y0 + (t3 - 2 * t2 + t) * h * d0
            + (-2 * t3 + 3 * t2) * y1 + (t3 - t2) * h * d1)


def _hermite_periodic(q, axis):
    q = np.moveaxis(q, axis, 0)
    n = q.shape[0]
    d = monotone_slopes(q, periodic=True)
    out = np.empty((2 * n,) + q.shape[1:])
    out[0::2] = q
    out[1::2] = _hermite(q, np.roll(q, -1, axis=0), d, np.roll(d, -1, axis=0), 1.0, 0.5)
    return np.moveaxis(out, 0, axis)


def _hermite_z(q, axis, zf):
    q = np.moveaxis(q, axis, 0)
    nzc = q.shape[0]
    nz = 2 * (nzc - 1) + 1
    zf = np.asarray(zf, dtype=np.float64)
    assert len(zf) == nz
    zc = zf[::2]
    d = monotone_slopes(q, zc)
    out = np.empty((nz,) + q.shape[1:])
    out[0::2] = q
    for K in range(nzc - 1):
        h = zc[K + 1] - zc[K]
        t = (zf[2 * K + 1] - zc[K]) / h
        out[2 * K + 1] = _hermite(q[K], q[K + 1], d[K], d[K + 1], h, t)
    return np.moveaxis(out, 0, axis)


PROLONGATIONS = ("trilinear", "hermite")


def prolong(qc, zf, op="trilinear"):
    """Prolongation of qc[..., nzc, nyc, nxc] to the fine grid with heights zf, trilinear
    or cubic Hermite."""
    qc = np.asarray(qc, dtype=np.float64)
    if op == "hermite":
        q = _hermite_periodic(qc, qc.ndim - 1)
        q = _hermite_periodic(q, q.ndim - 2)
        return _hermite_z(q, q.ndim - 3, zf)
    if op != "trilinear":
        raise ValueError("unknown prolongation %r" % (op,))
    q = _prolong_periodic(qc, qc.ndim - 1)
    q = _prolong_periodic(q, q.ndim - 2)
    return _prolong_z(q, q.ndim - 3, np.asarray(zf))


PRIMITIVES = ("T", "ne", "nH", "ntot", "vx", "vy", "vz")


def coarsen_atmosphere(atmos, op="full"):
    """Coarse-grid model atmosphere by restriction of the primitives (Sect. 4.7: full
    weighting by default; injection was the paper's alternative)."""
    out = {
        "nx": atmos["nx"] // 2, "ny": atmos["ny"] // 2, "nz": (atmos["nz"] - 1) // 2 + 1,
        "dx": 2.0 * atmos["dx"], "dy": 2.0 * atmos["dy"], "z": np.asarray(atmos["z"])[::2].copy(),
    }
    for k in PRIMITIVES:
        out[k] = restrict(atmos[k], op)
    out["chi_c"] = None if atmos.get("chi_c") is None else restrict(atmos["chi_c"], op)
    return out
