"""Pins of the oracle's weight normalisation (section on partially
overlapping data): hand-computed voxels, the never-increase rule, the
summed-weight bound, the choice of the overlap number, and agreement with the
synthetic generator's own minimal-overlap weights."""
import numpy as np
import pytest

from oracle import mvd_oracle as O
from paper_1308_0730_amd import synth


def test_hand_computed_voxels():
    # three views over four voxels
    w = [np.array([1.0, 1.0, 0.5, 0.0]), np.array([1.0, 0.0, 0.5, 0.0]), np.array([1.0, 0.0, 1.0, 0.0])]
    np.testing.assert_array_equal(O.contributing_views(w), [3, 1, 3, 0])
    out, m = O.normalize_weights(w, O.OVERLAP_MIN)
    assert m == 1.0  # the second voxel is covered by one view only
    np.testing.assert_allclose([x[0] for x in out], [1 / 3] * 3)
    np.testing.assert_allclose([x[2] for x in out], [0.25, 0.25, 0.5])
    np.testing.assert_allclose([x[1] for x in out], [1.0, 0.0, 0.0])
    out, m = O.normalize_weights(w, O.OVERLAP_AVG)
    assert m == pytest.approx(7 / 3)
    np.testing.assert_allclose([x[0] for x in out], [7 / 9] * 3)
    np.testing.assert_allclose([x[2] for x in out], [0.5, 0.5, 1.0])  # sum 2 <= 7/3: unchanged
    out, m = O.normalize_weights(w, O.OVERLAP_USER, 1.5)
    np.testing.assert_allclose([x[0] for x in out], [0.5] * 3)


@pytest.mark.parametrize("mode,value", [(O.OVERLAP_ONE, 0), (O.OVERLAP_MIN, 0), (O.OVERLAP_AVG, 0),
                                        (O.OVERLAP_USER, 2.5)])
def test_bound_and_never_increase(mode, value):
    rng = np.random.default_rng(3)
    w = [np.clip(rng.uniform(-0.5, 1.3, size=(6, 7, 8)), 0, 1) for _ in range(4)]
    out, m = O.normalize_weights(w, mode, value)
    s_in, s_out = np.sum(w, axis=0), np.sum(out, axis=0)
    assert m > 0
    assert np.all(s_out <= m * (1 + 1e-12))
    for a, b in zip(w, out):
        assert np.all(b <= a + 1e-15) and np.all(b >= 0)
    keep = s_in <= m
    for a, b in zip(w, out):
        np.testing.assert_array_equal(a[keep], b[keep])
    # one factor per voxel: ratios between views are kept
    k = s_in > 0
    np.testing.assert_allclose((out[0] * w[1])[k], (out[1] * w[0])[k], atol=1e-15)


def test_generator_weights_are_min_overlap_normalised():
    dims, angles = (40, 32, 24), [0.0, 60.0, 120.0, 180.0, 240.0, 300.0]
    w = synth.overlap_weights(dims, angles)
    out, m = O.normalize_weights(w, O.OVERLAP_MIN)
    for a, b in zip(w, out):
        np.testing.assert_allclose(a, b, atol=1e-6)
