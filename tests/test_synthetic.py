"""Checks of the seeded input generators (synthetic/): determinism, value
ranges, coil normalisation and the mask line counts of each recipe."""
import numpy as np
import pytest

from synthetic import batch_inputs, coil_maps, pe_mask, phantom, vn_params


def test_phantom_range_and_determinism():
    a = phantom(3, 64, 48)
    b = phantom(3, 64, 48)
    assert a.dtype == np.complex64 and a.shape == (64, 48)
    assert np.array_equal(a, b)
    mag = np.abs(a)
    assert mag.max() <= 1.0 + 1e-6 and mag.max() > 0.99
    assert not np.array_equal(a, phantom(4, 64, 48))


def test_coils_sum_of_squares_is_one():
    S = coil_maps(5, 8, 32, 40).astype(np.complex128)
    assert np.max(np.abs(np.sum(np.abs(S) ** 2, axis=0) - 1.0)) < 1e-6


@pytest.mark.parametrize("H,R,nc,kind,expect", [
    (128, 4, 16, "uniform", 32), (320, 4, 24, "vd", 80), (256, 6, 24, "vd", 42),
    (384, 8, 24, "vd", 48)])
def test_mask_line_counts(H, R, nc, kind, expect):
    m = pe_mask(11, H, R, nc, kind)
    assert m.dtype == np.float32 and set(np.unique(m)) <= {0.0, 1.0}
    assert int(m.sum()) == expect
    c0 = H // 2 - nc // 2
    assert np.all(m[c0:c0 + nc] == 1)


def test_regular_mask_has_every_rth_line_and_acs():
    m = pe_mask(0, 384, 4, 28, "regular")
    assert np.all(m[::4] == 1)
    assert np.all(m[192 - 14:192 + 14] == 1)


def test_batch_shapes():
    d = batch_inputs([1, 2], 32, 24, 3, 4, 8)
    assert d["x"].shape == (2, 32, 24) and d["S"].shape == (2, 3, 32, 24)
    assert d["mask"].shape == (2, 32) and d["noise"].shape == (2, 3, 32, 24)


def test_vn_params_shapes():
    p = vn_params(1)
    assert p["k"].shape == (10, 24, 11, 11) and p["w"].shape == (10, 24, 31)
    assert np.max(np.abs(p["k"].mean(axis=(2, 3)))) < 1e-6
