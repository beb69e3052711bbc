"""The compiled-in Weideman coefficients of the sweep kernels (csrc/voigt_coef.h): the
header is what its generator writes, and the series it defines reproduces the Faddeeva
function of SciPy (an independent evaluation) over the line core the kernels use it in."""
import importlib.util
import os
import re

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1701_01607_amd", "csrc")


def table():
    s = open(os.path.join(CSRC, "voigt_coef.h")).read()
    L = float.fromhex(re.search(r"kVoigtLd = (\S+);", s).group(1))
    body = s[s.index("kVoigtCoefD[kVoigtNd] = {"):]
    body = body[:body.index("};")]
    coef = [float.fromhex(x) for x in re.findall(r"(-?0x[0-9a-f.]+p[+-]\d+)", body)]
    n = int(re.search(r"kVoigtNd = (\d+);", s).group(1))
    return L, coef, n


def test_header_is_the_generators_output():
    spec = importlib.util.spec_from_file_location("voigt_coef", os.path.join(CSRC, "voigt_coef.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    assert open(os.path.join(CSRC, "voigt_coef.h")).read() == gen.header()


def test_series_matches_the_faddeeva_function():
    special = pytest.importorskip("scipy.special")
    L, coef, n = table()
    assert len(coef) == n == 32 and L == np.sqrt(n / np.sqrt(2.0))
    a = np.array([1e-4, 1e-2, 0.04, 0.1, 1.0, 5.0, 30.0])[:, None]
    u = np.linspace(0.0, 5.0, 101)[None, :]
    z = u + 1j * a
    Z = (L + 1j * z) / (L - 1j * z)
    w = 2.0 * np.polyval(coef, Z) / (L - 1j * z) ** 2 + 1.0 / (np.sqrt(np.pi) * (L - 1j * z))
    ref = special.wofz(z).real
    rel = np.abs(w.real / ref - 1.0)
    assert rel.max() < 3e-8                        # H down to ~1e-11 at |u| = 5, a << 1
    assert rel[:, u[0] <= 3.0].max() < 5e-10
    assert rel[:, u[0] <= 1.5].max() < 1e-12
