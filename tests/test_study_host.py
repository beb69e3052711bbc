"""Host-side metrics of the multigrid study (no GPU)."""
import numpy as np

from paper_1701_01607_amd.study import rel_error, smoothing_number


def test_relative_error_is_the_max_norm_of_n_over_ref_minus_one():
    ref = np.full((2, 5, 3, 4), 2.0)
    n = ref.copy()
    n[1, 2, 1, 3] = 2.5
    n[0, 0, 0, 0] = 1.0
    assert rel_error(n, ref) == 0.5


def test_smoothing_number_is_the_largest_second_difference_along_z():
    ref = np.full((1, 7, 2, 2), 4.0)
    k = np.arange(7.0)[None, :, None, None]
    # a relative error quadratic in the plane index has second difference 2 a everywhere
    n = ref * (1.0 + 0.01 * k ** 2)
    assert np.isclose(smoothing_number(n, ref), 0.02, rtol=1e-12)
    # linear errors are perfectly smooth
    assert smoothing_number(ref * (1.0 + 0.3 * k), ref) < 1e-14
    # a spike of height h gives 2 h
    n = ref.copy()
    n[0, 3, 1, 0] *= 1.1
    assert np.isclose(smoothing_number(n, ref), 0.2, rtol=1e-12)
