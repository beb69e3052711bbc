"""Seeded synthetic inputs: model atoms and model atmospheres.

This module holds input data only.  It contains none of the method's arithmetic:
no Planck function, no line profile, no rates, no formal solution.  Both the HIP
library and the CPU oracle receive their inputs from here.

The paper's own inputs (two radiation-MHD snapshots, a plane-parallel semi-empirical
model and published model atoms; Sect. 3.1 and 3.2) are not available, so seeded
synthetic stand-ins take their shapes and grid spacings but none of their values:

* ``two_level_atom`` / ``atmos_isothermal``: the isothermal two-level test problem
  (16x16x32, T = 5000 K, exponential density, constant destruction probability).
* ``caii_like_atom``: a six-level atom (5 bound levels + continuum, 5 lines) with
  round-number energies and strengths, lines between 390 and 870 nm.
* ``atmos_stratified``: a stratified atmosphere with a photosphere-to-chromosphere
  temperature rise and Gaussian random-field perturbations (10 % in T, 30 % log-normal
  in density, velocities clipped to +-10 km/s).
* ``atmos_rmhd_like``: the same plus granulation-scale fields and shock fronts.

Units are CGS throughout.  Arrays are C-ordered ``[z][y][x]`` with x fastest.
"""
from __future__ import annotations

import numpy as np

KM = 1.0e5          # cm
MM = 1.0e8          # cm

# --------------------------------------------------------------------------- atoms


def doppler_grid_two_level():
    """21 velocity offsets from -5 to +5 km/s in steps of 0.5 km/s (cm/s).

    With the atomic mass chosen below the thermal Doppler width at 5000 K is
    1 km/s, so this spans +-5 Doppler widths.
    """
    return np.linspace(-5.0, 5.0, 21) * KM


def line_grid(n, q_core, q_max, n_core):
    """Symmetric velocity-offset grid (cm/s) with ``n`` (odd) points.

    ``n_core`` points per half (including 0) are spaced linearly up to ``q_core``;
    the remaining points per half are spaced logarithmically out to ``q_max``.
    """
    assert n % 2 == 1
    half = (n - 1) // 2
    n_wing = half + 1 - n_core
    core = np.linspace(0.0, q_core, n_core)
    step = core[1] - core[0]
    wing = np.geomspace(q_core + step, q_max, n_wing) if n_wing > 0 else np.zeros(0)
    pos = np.concatenate([core, wing])
    return np.concatenate([-pos[:0:-1], pos])


def two_level_atom(epsilon=1.0e-4, q_max=5.0 * KM, nfreq=21):
    """Two-level atom with a pure Doppler line and a constant destruction probability.

    The lower level has g = 1, the upper g = 3, the line sits at 500 nm
    (20000 cm^-1).  The atomic mass 83.14 amu makes the thermal Doppler width at
    5000 K equal to 1 km/s.  No damping, no continuum, no background.  The default
    grid (21 points over +-5 km/s) suits a static atmosphere; moving atmospheres need
    q_max beyond the largest velocity plus a few Doppler widths.
    """
    return {
        "name": "two-level",
        "mass_amu": 83.14,
        "xi": 0.0,
        "levels": [
            {"E": 0.0, "g": 1.0, "stage": 1},
            {"E": 20000.0, "g": 3.0, "stage": 1},
        ],
        "lines": [
            {"lower": 0, "upper": 1, "A": 1.0e7, "gamma_rad": 0.0, "gamma_vdw": 0.0,
             "q": doppler_grid_two_level() if (q_max == 5.0 * KM and nfreq == 21)
             else np.linspace(-q_max, q_max, nfreq)},
        ],
        "continua": [],
        "collisions": [],
        "epsilon": float(epsilon),
    }


def caii_like_atom(nfreq=101):
    """Synthetic six-level atom: 5 bound levels of one ion plus the next ion's ground state.

    Topology: two resonance lines from the ground level, three subordinate lines
    from two metastable levels, five fixed bound-free transitions, and collisional
    coupling between every pair of levels.  All numbers are round synthetic values.
    """
    q_res = line_grid(nfreq, 25.0 * KM, 200.0 * KM, 31 if nfreq >= 61 else (nfreq + 1) // 4)
    q_sub = line_grid(nfreq, 25.0 * KM, 60.0 * KM, 31 if nfreq >= 61 else (nfreq + 1) // 4)
    levels = [
        {"E": 0.0, "g": 2.0, "stage": 1},
        {"E": 13700.0, "g": 4.0, "stage": 1},
        {"E": 13800.0, "g": 6.0, "stage": 1},
        {"E": 25200.0, "g": 2.0, "stage": 1},
        {"E": 25400.0, "g": 4.0, "stage": 1},
        {"E": 96000.0, "g": 1.0, "stage": 2},
    ]
    lines = [
        {"lower": 0, "upper": 3, "A": 1.4e8, "gamma_rad": 1.5e8, "gamma_vdw": 2.0e-8, "q": q_res},
        {"lower": 0, "upper": 4, "A": 1.5e8, "gamma_rad": 1.5e8, "gamma_vdw": 2.0e-8, "q": q_res},
        {"lower": 1, "upper": 3, "A": 1.1e7, "gamma_rad": 1.5e8, "gamma_vdw": 2.0e-8, "q": q_sub},
        {"lower": 1, "upper": 4, "A": 1.0e6, "gamma_rad": 1.5e8, "gamma_vdw": 2.0e-8, "q": q_sub},
        {"lower": 2, "upper": 4, "A": 9.0e6, "gamma_rad": 1.5e8, "gamma_vdw": 2.0e-8, "q": q_sub},
    ]
    continua = [
        {"lower": i, "upper": 5, "alpha0": a0}
        for i, a0 in zip(range(5), (2.0e-19, 6.0e-18, 6.0e-18, 2.0e-18, 2.0e-18))
    ]
    collisions = []
    for u in range(6):
        for l in range(u):
            if u == 5:
                c = 2.0e-9
            elif (l, u) in ((0, 3), (0, 4), (1, 3), (1, 4), (2, 4)):
                c = 3.0e-7
            else:
                c = 1.0e-7
            collisions.append({"lower": l, "upper": u, "c_ul": c, "T_ref": 5000.0, "beta": -0.5})
    return {
        "name": "caii-like-6",
        "mass_amu": 40.0,
        "xi": 2.0 * KM,
        "levels": levels,
        "lines": lines,
        "continua": continua,
        "collisions": collisions,
        "epsilon": None,
    }


def two_ion_level_atom(nfreq=101):
    """caii_like_atom() plus the next ion's first excited level (level 6), reached by two
    more bound-free transitions, from levels 3 and 4, and by collisions, so that the
    continua end on two upper levels.  Round synthetic values."""
    atom = caii_like_atom(nfreq)
    atom = dict(atom, name="caii-like-7",
                levels=atom["levels"] + [{"E": 96000.0 + 13650.0, "g": 4.0, "stage": 2}],
                continua=atom["continua"] + [{"lower": 3, "upper": 6, "alpha0": 1.5e-18},
                                             {"lower": 4, "upper": 6, "alpha0": 1.5e-18}])
    atom["collisions"] = [dict(c) for c in atom["collisions"]] + [
        {"lower": l, "upper": 6, "c_ul": 3.0e-7 if l == 5 else 2.0e-9, "T_ref": 5000.0, "beta": -0.5}
        for l in range(6)]
    return atom


def continuum_grid(atom, n_seg=6, n_top=16, top=1.6):
    """Frequencies (Hz) for treating the atom's continua as active transitions: every
    edge, n_seg geometric steps between consecutive edges and n_top from the highest edge
    to `top` times it."""
    c_light = 2.99792458e10
    lv = atom["levels"]
    edges = sorted({c_light * (lv[c["upper"]]["E"] - lv[c["lower"]]["E"]) for c in atom["continua"]})
    pts = []
    for a, b in zip(edges[:-1], edges[1:]):
        pts.extend(np.geomspace(a, b, n_seg + 1)[:-1])
    pts.extend(np.geomspace(edges[-1], top * edges[-1], n_top + 1))
    return np.array(pts)


def with_active_continua(atom, **kw):
    """A copy of `atom` whose continua are swept as active transitions on continuum_grid()."""
    out = dict(atom)
    out["continuum_nu"] = continuum_grid(atom, **kw)
    return out


# --------------------------------------------------------------------- atmospheres


def z_grid(nz, zmin, zmax, ratio=2.67, zfine=0.3):
    """Non-uniform heights (cm), increasing, with spacing growing quadratically away
    from the relative position ``zfine``; ``ratio`` is the largest/smallest spacing."""
    s = (np.arange(nz - 1) + 0.5) / (nz - 1)
    w = 1.0 + (ratio - 1.0) * ((s - zfine) / max(zfine, 1.0 - zfine)) ** 2
    dz = w * (zmax - zmin) / w.sum()
    z = np.concatenate([[zmin], zmin + np.cumsum(dz)])
    z[-1] = zmax
    return z


def _workers():
    """Threads for the plane-parallel parts of the generators (NumPy and SciPy release the
    GIL inside their array loops)."""
    import os
    return max(1, min(16, os.cpu_count() or 1))


def _by_chunks(fn, n, chunk=None):
    """Call fn(i0, i1) over [0, n) in contiguous chunks on a thread pool.  Every chunk
    writes its own slice, so the result does not depend on the chunking."""
    from concurrent.futures import ThreadPoolExecutor
    w = _workers()
    step = chunk or max(1, -(-n // (4 * w)))
    if w == 1 or n <= step:
        fn(0, n)
        return
    with ThreadPoolExecutor(w) as ex:
        list(ex.map(lambda i: fn(i, min(n, i + step)), range(0, n, step)))


def gaussian_random_field(rng, nx, ny, nz, corr_xy, corr_z):
    """Unit-variance Gaussian random field, periodic in x and y.

    White noise is filtered with a Gaussian spectrum of correlation length
    ``corr_xy`` cells horizontally (FFT, hence periodic) and smoothed with a Gaussian of
    ``corr_z`` cells vertically (truncated at 3 sigma, mirrored ends).  Planes (for the
    FFT) and columns (for the vertical smoothing) are processed on a thread pool; each
    is transformed on its own, so the values are those of the whole-array calls.
    """
    from scipy.ndimage import gaussian_filter1d

    noise = rng.standard_normal((nz, ny, nx))
    kx = np.fft.rfftfreq(nx)[None, :]
    ky = np.fft.fftfreq(ny)[:, None]
    filt = np.exp(-2.0 * (np.pi * corr_xy) ** 2 * (kx ** 2 + ky ** 2))
    out = np.empty_like(noise)

    def planes(k0, k1):
        out[k0:k1] = np.fft.irfft2(np.fft.rfft2(noise[k0:k1], axes=(-2, -1)) * filt[None], s=(ny, nx),
                                   axes=(-2, -1))

    _by_chunks(planes, nz)
    del noise
    if corr_z > 0 and nz > 1:
        src = out
        out = np.empty_like(src)

        def columns(j0, j1):
            # the column block with z last (contiguous), smoothed along z, written back
            blk = np.ascontiguousarray(np.moveaxis(src[:, j0:j1, :], 0, -1))
            out[:, j0:j1, :] = np.moveaxis(gaussian_filter1d(blk, corr_z, axis=-1, mode="mirror", truncate=3.0),
                                           -1, 0)

        _by_chunks(columns, ny)
        del src
    sd = out.std()
    if sd > 0:
        def scale(k0, k1):
            out[k0:k1] /= sd

        _by_chunks(scale, nz)
    return out


def atmos_isothermal(nx=16, ny=16, nz=32, dx=100.0 * KM, dz=100.0 * KM, T=5000.0,
                     ntot0=7.5e10, scale_height=150.0 * KM):
    """Isothermal, horizontally homogeneous two-level atmosphere.

    Heights z_k = k * dz.  The total atom density falls as exp(-z / scale_height);
    ``ntot0`` (the density at z = 0) puts the line-centre vertical optical depth near
    1e-3 at the top plane of the default 32-plane grid.
    """
    z = np.arange(nz) * dz
    shape = (nz, ny, nx)
    ntot = ntot0 * np.exp(-z / scale_height)[:, None, None] * np.ones(shape)
    return {
        "nx": nx, "ny": ny, "nz": nz, "dx": float(dx), "dy": float(dx), "z": z,
        "T": np.full(shape, float(T)),
        "ne": np.zeros(shape), "nH": np.zeros(shape), "ntot": ntot,
        "vx": np.zeros(shape), "vy": np.zeros(shape), "vz": np.zeros(shape),
        "chi_c": None,
    }


_T_CTRL_Z = np.array([-0.5, 0.0, 0.5, 1.0, 2.0, 3.0, 6.0]) * MM
_T_CTRL_T = np.array([8000.0, 6000.0, 4200.0, 5000.0, 6500.0, 8000.0, 9000.0])


def _mean_structure(z):
    """Round-number mean stratification: T(z), n_H(z) (hydrostatic, mu = 1.3) and the
    electron fraction n_e / n_H(z)."""
    T = np.interp(z, _T_CTRL_Z, _T_CTRL_T)
    k_b, m_h, g = 1.380649e-16, 1.6735575e-24, 2.74e4
    H = k_b * T / (1.3 * m_h * g)
    zi = np.argmin(np.abs(z))
    lnn = np.zeros_like(z)
    for i in range(1, len(z)):
        lnn[i] = lnn[i - 1] - (z[i] - z[i - 1]) * 0.5 * (1.0 / H[i] + 1.0 / H[i - 1])
    nH = 1.0e17 * np.exp(lnn - lnn[zi])
    frac = 1.0e-4 + 0.05 / (1.0 + np.exp(-(z - 1.5 * MM) / (0.3 * MM)))
    return T, nH, frac


_BACKGROUND_SCALE = np.array([1.0, 1.0, 2.2, 2.2, 2.2, 2.0, 2.0, 2.0])


def _background_base(nH, ne, T):
    return 1.0e-24 * nH * (ne / 1.0e13) * (T / 5000.0) ** 2


def _background(nH, ne, T, nline):
    """Background continuum opacity per line (cm^-1), a round-number scaling with
    n_H * n_e that puts continuum optical depth unity near z = 0."""
    scale = _BACKGROUND_SCALE[:nline]
    base = _background_base(nH, ne, T)
    return np.stack([s * base for s in scale], axis=0)


def atmos_stratified(nx=64, ny=64, nz=129, dx=48.0 * KM, zmin=-0.5 * MM, zmax=3.0 * MM,
                     seed=1607002, nline=5, dT=0.10, drho=0.30, vmax=10.0 * KM,
                     corr_xy=1.0 * MM, corr_z=0.3 * MM):
    """Stratified atmosphere with seeded Gaussian random-field perturbations."""
    rng = np.random.default_rng(seed)
    z = z_grid(nz, zmin, zmax)
    T0, nH0, frac = _mean_structure(z)
    dzm = (zmax - zmin) / (nz - 1)
    f1 = gaussian_random_field(rng, nx, ny, nz, corr_xy / dx, corr_z / dzm)
    f2 = gaussian_random_field(rng, nx, ny, nz, corr_xy / dx, corr_z / dzm)
    vel = [gaussian_random_field(rng, nx, ny, nz, corr_xy / dx, corr_z / dzm) for _ in range(3)]
    T = T0[:, None, None] * (1.0 + dT * f1)
    T = np.clip(T, 0.5 * T0.min(), None)
    nH = nH0[:, None, None] * np.exp(drho * f2 - 0.5 * drho ** 2)
    ne = nH * frac[:, None, None] * (T / T0[:, None, None]) ** 2
    v = [np.clip(0.4 * vmax * f, -vmax, vmax) for f in vel]
    return {
        "nx": nx, "ny": ny, "nz": nz, "dx": float(dx), "dy": float(dx), "z": z,
        "T": T, "ne": ne, "nH": nH, "ntot": 2.0e-6 * nH,
        "vx": v[0], "vy": v[1], "vz": v[2],
        "chi_c": _background(nH, ne, T, nline),
    }


def atmos_rmhd_like(nx=256, ny=256, nz=257, dx=48.0 * KM, zmin=-0.5 * MM, zmax=6.0 * MM,
                    seed=1607003, nline=5, nshock=6, vmax=10.0 * KM):
    """Stratified atmosphere with granulation-scale photospheric fields (1-1.5 Mm,
    amplitude decaying with height) and seeded step-like shock fronts in the
    chromosphere (T x 1.5-2.5 and density x 2-4 across a 1-2 cell front).  The fields
    are assembled slab by slab in z on a thread pool (element-wise, so the values do
    not depend on the slabs)."""
    rng = np.random.default_rng(seed)
    z = z_grid(nz, zmin, zmax)
    T0, nH0, frac = _mean_structure(z)
    dzm = (zmax - zmin) / (nz - 1)
    gran = gaussian_random_field(rng, nx, ny, nz, 1.2 * MM / dx, 0.2 * MM / dzm)
    chrom = gaussian_random_field(rng, nx, ny, nz, 0.8 * MM / dx, 0.3 * MM / dzm)
    vel = [gaussian_random_field(rng, nx, ny, nz, 1.0 * MM / dx, 0.3 * MM / dzm) for _ in range(3)]
    decay = np.exp(-np.clip(z, 0.0, None) / (0.4 * MM))[:, None, None]
    rise = (1.0 / (1.0 + np.exp(-(z - 1.0 * MM) / (0.2 * MM))))[:, None, None]
    # shock fronts: planes or spherical caps above 1 Mm (parameters drawn in order first)
    Lx = nx * dx
    shocks = []
    for _ in range(nshock):
        cx, cy = rng.uniform(0, Lx), rng.uniform(0, Lx)
        zc = rng.uniform(1.2 * MM, min(zmax, 4.0 * MM))
        rad = rng.uniform(1.0 * MM, 3.0 * MM)
        width = rng.uniform(1.0, 2.0) * dx
        tfac = rng.uniform(1.5, 2.5)
        rfac = rng.uniform(2.0, 4.0)
        shocks.append((cx, cy, zc, rad, width, tfac, rfac))
    xs = (np.arange(nx) * dx)[None, None, :]
    ys = (np.arange(ny) * dx)[None, :, None]
    shape = (nz, ny, nx)
    T, nH, ne = np.empty(shape), np.empty(shape), np.empty(shape)
    v = [np.empty(shape) for _ in range(3)]
    chi_c = np.empty((nline,) + shape)
    scale = _BACKGROUND_SCALE[:nline]

    def slab(k0, k1):
        sl = slice(k0, k1)
        t0 = T0[sl, None, None]
        Ts = t0 * (1.0 + 0.10 * gran[sl] * decay[sl] + 0.08 * chrom[sl] * rise[sl])
        nHs = nH0[sl, None, None] * np.exp(0.3 * gran[sl] * decay[sl] + 0.2 * chrom[sl] * rise[sl] - 0.1)
        zs = z[sl, None, None]
        for cx, cy, zc, rad, width, tfac, rfac in shocks:
            ddx = (xs - cx + 0.5 * Lx) % Lx - 0.5 * Lx
            ddy = (ys - cy + 0.5 * Lx) % Lx - 0.5 * Lx
            r = np.sqrt(ddx ** 2 + ddy ** 2 + (zs - (zc - rad)) ** 2)
            inside = 1.0 / (1.0 + np.exp((r - rad) / (0.5 * width)))
            cap = inside * (zs > zc - 0.5 * rad)
            Ts = Ts * (1.0 + (tfac - 1.0) * cap)
            nHs = nHs * (1.0 + (rfac - 1.0) * cap)
        T[sl], nH[sl] = Ts, nHs
        ne[sl] = nHs * frac[sl, None, None] * (Ts / t0) ** 2
        for c in range(3):
            v[c][sl] = np.clip(0.4 * vmax * vel[c][sl], -vmax, vmax)
        base = _background_base(nHs, ne[sl], Ts)
        for l in range(nline):
            chi_c[l, sl] = scale[l] * base

    _by_chunks(slab, nz)
    return {
        "nx": nx, "ny": ny, "nz": nz, "dx": float(dx), "dy": float(dx), "z": z,
        "T": T, "ne": ne, "nH": nH, "ntot": 2.0e-6 * nH,
        "vx": v[0], "vy": v[1], "vz": v[2],
        "chi_c": chi_c,
    }


# ------------------------------------------------------------------ named configs

WORKLOADS = {
    "two_level_16x16x32": dict(desc="two-level atom, plain FP64 MALI, 16x16x32, T=5000 K, eps=1e-4"),
    "caii6_64x64x129": dict(desc="six-level atom, 64x64x129 stratified, 3-level FAS, FP32 sweep"),
    "caii6_256x256x257": dict(desc="six-level atom, 256x256x257 rmhd-like, 4-level FMG"),
    "caii6_504x504x497": dict(desc="six-level atom, 504x504x497 rmhd-like (20 km), 4-level FMG"),
}


# Grid (nx, ny, nz) of each named workload.
GRIDS = {
    "two_level_16x16x32": (16, 16, 32),
    "caii6_64x64x129": (64, 64, 129),
    "caii6_256x256x257": (256, 256, 257),
    "caii6_504x504x497": (504, 504, 497),
}


def workload(name, **kw):
    """(atom, atmosphere) for a named workload; keyword arguments override sizes/seeds."""
    nx, ny, nz = GRIDS[name]
    args = dict(nx=nx, ny=ny, nz=nz)
    if name == "two_level_16x16x32":
        args.update(kw)
        return two_level_atom(), atmos_isothermal(**args)
    nf = kw.pop("nfreq", 101)
    if name == "caii6_64x64x129":
        args.update(kw)
        return caii_like_atom(nf), atmos_stratified(**args)
    if name == "caii6_256x256x257":
        args.update(kw)
        return caii_like_atom(nf), atmos_rmhd_like(**args)
    args.update(dx=20.0 * KM, seed=1607004)
    args.update(kw)
    return caii_like_atom(nf), atmos_rmhd_like(**args)
