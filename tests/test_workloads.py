"""Input generators: shapes, ranges, determinism (CPU only)."""
import math

import numpy as np

from paper_2601_18548_amd import workloads as wl


def test_knots_ranges_and_determinism():
    k = wl.knots(1000, 3)
    assert k.shape == (1000, 9) and k.dtype == np.float32
    assert np.all(np.abs(k[:, :2]) <= 2) and np.all(np.abs(k[:, 2:]) <= math.pi + 1e-6)
    assert np.array_equal(k, wl.knots(1000, 3))
    assert not np.array_equal(k, wl.knots(1000, 4))


def test_patch_cloud_fraction_and_box():
    p = wl.points_patches(4096, 1)
    assert p.shape == (4096, 3) and p.dtype == np.float32
    lo, hi = wl.BOX_LO - 0.05, wl.BOX_HI + 0.05
    assert np.all(p >= lo) and np.all(p <= hi)
    assert np.array_equal(p, wl.points_patches(4096, 1))


def test_weights_he_scale_and_bf16_grid():
    w = wl.weights(512, 0)
    assert [m.shape for m in w.mats] == [(512, 9), (512, 512), (512, 512), (512, 512), (1, 512)]
    for li in (1, 2, 3):
        m = w.mats[li]
        assert np.array_equal(m, wl.round_to_bf16_grid(m))
        assert abs(m.std() - math.sqrt(2 / 512)) < 0.002
    assert not np.array_equal(w.mats[0], wl.round_to_bf16_grid(w.mats[0]))


def test_bf16_rounding_ties_to_even():
    one = np.float32(1.0)
    ulp = np.float32(2.0 ** -7)
    x = np.array([one + ulp / 2, one + ulp + ulp / 2, one + ulp / 4], np.float32)
    np.testing.assert_array_equal(wl.round_to_bf16_grid(x), [1.0, 1.0 + 2 * ulp, 1.0])


def test_serving_trace():
    tr = wl.serving_trace(500, 2000.0, 1)
    gaps = np.diff([r.arrival_s for r in tr])
    assert abs(gaps.mean() - 1 / 2000.0) < 0.1 / 2000.0
    assert all(16 <= r.K <= 256 and 512 <= r.Np <= 32768 for r in tr)
