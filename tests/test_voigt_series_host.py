"""The small-damping Voigt series that FP32 sweeps evaluate for a < 0.04 and |u| < 5, checked
on the CPU against the Faddeeva function (its definition), independently of the GPU:

* the Taylor coefficients of w about the real axis follow from w' = -2 z w + 2i/sqrt(pi);
  the closed form through a^4 (in exp(-u^2) and G = 1 - 2uF with Dawson's F) is summed
  here in FP64 and must stay within 2e-7 of Re w(u + i a) in relative terms;
* G from the cubic Hermite table of 80 intervals of width 1/16 (nodes from fourth-order
  Runge-Kutta integration of F' = 1 - 2uF) must match 1 - 2u dawsn(u) to 1.5e-6 absolute
  (the interpolation error, h^4/384 times the fourth derivative of G, is largest near u = 0,
  where H ~ 1 and G enters multiplied by a < 0.04) and to 5e-7 relative beyond u = 2.5,
  where G is small; through the series the table costs at most 5e-7 relative in H."""
import numpy as np
from scipy.special import dawsn, wofz


def series(a, u, G):
    t = u * u
    a2, a3, a4 = a * a, a ** 3, a ** 4
    even = np.exp(-t) * (1.0 + a2 + 0.5 * a4 - 2.0 * (a2 + a4) * t + (2.0 / 3.0) * a4 * t * t)
    odd = ((2.0 / 3.0) * a3 - (2.0 * a + 2.0 * a3 - (4.0 / 3.0) * a3 * t) * G) / np.sqrt(np.pi)
    return even + odd


def test_series_truncation_below_2e7():
    u = np.linspace(-4.999, 4.999, 20001)
    G = 1.0 - 2.0 * np.abs(u) * dawsn(np.abs(u))
    for a in (0.0, 1e-5, 1e-3, 0.01, 0.03, 0.0399):
        ref = wofz(u + 1j * a).real
        err = np.max(np.abs(series(a, u, G) / ref - 1.0))
        assert err < 2e-7, (a, err)


def test_hermite_table_of_G():
    h, sub = 1.0 / 16.0, 64
    dt = h / sub
    F, u, Fn = 0.0, 0.0, [0.0]
    f = lambda x, y: 1.0 - 2.0 * x * y   # noqa: E731
    for i in range(80):
        for j in range(sub):
            k1 = f(u, F)
            k2 = f(u + dt / 2, F + dt / 2 * k1)
            k3 = f(u + dt / 2, F + dt / 2 * k2)
            k4 = f(u + dt, F + dt * k3)
            F += dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
            u = (i * sub + j + 1) * dt
        Fn.append(F)
    Fn = np.array(Fn)
    un = np.arange(81) * h
    assert np.max(np.abs(Fn - dawsn(un))) < 1e-12
    G = 1.0 - 2.0 * un * Fn
    D = h * (-2.0 * Fn - 2.0 * un * G)
    x = np.linspace(0.0, 4.9999, 50001) * 16.0
    i = np.minimum(x.astype(int), 79)
    s = x - i
    val = (G[i] * (2 * s ** 3 - 3 * s ** 2 + 1) + D[i] * (s ** 3 - 2 * s ** 2 + s)
           + G[i + 1] * (-2 * s ** 3 + 3 * s ** 2) + D[i + 1] * (s ** 3 - s ** 2))
    uu = x / 16.0
    exact = 1.0 - 2.0 * uu * dawsn(uu)
    assert np.max(np.abs(val - exact)) < 1.5e-6
    far = uu > 2.5
    assert np.max(np.abs(val[far] / exact[far] - 1.0)) < 5e-7
    for a in (1e-5, 1e-3, 0.0399):
        assert np.max(np.abs(series(a, uu, val) / series(a, uu, exact) - 1.0)) < 5e-7
