"""The line profile's Voigt function H(a, u) as the sweeps evaluate it (nlte_voigt), against
the oracle's (the Faddeeva function's real part), point by point.

FP64: Weideman's 32-term series everywhere, relative error <= 2.6e-8 for a >= 1e-4.
FP32: the small-damping Taylor series (a < 0.04, |u| < 5), the FP64 series (a >= 0.04,
|u| < 5) and the FP32 asymptotic wing (|u| >= 5); compared at the FP32-rounded inputs, so
the bound covers the evaluation only (about 5e-7 each, from rounding u^2 before the
exponential and from the truncated series)."""
import numpy as np
import pytest

from oracle import physics as ph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_1701_01607_amd import nlte
    c = nlte.Context(0, torch.cuda.current_stream().cuda_stream)
    yield nlte, c
    c.close()


def grid(a_values):
    u = np.concatenate([np.linspace(-6.0, 6.0, 2401), np.linspace(6.0, 40.0, 341), -np.linspace(6.0, 40.0, 341),
                        [5.0, -5.0, np.nextafter(np.float32(5.0), np.float32(0.0)), 0.0, 4.96875, 3.0625]])
    A, U = np.meshgrid(np.asarray(a_values, dtype=np.float64), u, indexing="ij")
    return A.ravel(), U.ravel()


def on_device(nl, c, precision, a, u):
    import torch
    ad = torch.tensor(a, dtype=torch.float64, device="cuda")
    ud = torch.tensor(u, dtype=torch.float64, device="cuda")
    hd = torch.empty_like(ad)
    c.voigt(precision, a.size, ad.data_ptr(), ud.data_ptr(), hd.data_ptr())
    return hd.cpu().numpy()


def test_voigt_fp64(ctx):
    nl, c = ctx
    a, u = grid([1e-4, 1e-3, 0.01, 0.039, 0.04, 0.1, 0.5, 1.0, 2.5, 10.0])
    H = on_device(nl, c, nl.FP64, a, u)
    ref = ph.voigt_H(a, u)
    err = np.abs(H / ref - 1.0)
    i = int(np.argmax(err))
    print(f"FP64 Voigt: max rel err {err[i]:.2e} at a={a[i]}, u={u[i]}")
    assert err[i] <= 5e-8


def test_voigt_fp32(ctx):
    nl, c = ctx
    a, u = grid([1e-5, 1e-4, 1e-3, 3e-3, 0.01, 0.02, 0.0399, 0.04, 0.1, 0.5, 1.0, 2.5, 10.0])
    H = on_device(nl, c, nl.MIXED, a, u)
    a32, u32 = a.astype(np.float32).astype(np.float64), u.astype(np.float32).astype(np.float64)
    ref = ph.voigt_H(a32, u32)
    err = np.abs(H / ref - 1.0)
    for lo, hi, name in ((0.0, 0.04, "small damping"), (0.04, np.inf, "larger damping")):
        m = (a32 >= lo) & (a32 < hi)
        core, wing = m & (np.abs(u32) < 5.0), m & (np.abs(u32) >= 5.0)
        print(f"FP32 Voigt, {name}: core max rel err {err[core].max():.2e}, wing {err[wing].max():.2e}")
    i = int(np.argmax(err))
    print(f"FP32 Voigt: max rel err {err[i]:.2e} at a={a32[i]}, u={u32[i]}")
    assert err[i] <= 2e-6


def test_voigt_undamped_limit_and_empty(ctx):
    nl, c = ctx
    # a = 0 inside the core is the Gaussian; the small-damping series reduces to exp(-u^2)
    u = np.linspace(-4.9, 4.9, 981)
    a = np.zeros_like(u)
    H = on_device(nl, c, nl.MIXED, a, u)
    u32 = u.astype(np.float32).astype(np.float64)
    assert np.max(np.abs(H / np.exp(-u32 * u32) - 1.0)) <= 2e-6
    c.voigt(nl.MIXED, 0, 0, 0, 0)   # n = 0: nothing to do
    with pytest.raises(nl.NlteError):
        c.voigt(7, 4, 0, 0, 0)
