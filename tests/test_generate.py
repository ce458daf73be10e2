"""Seeded generator: determinism, normalisation, weight bounds, and the
analytic rendering of views against an explicit FP64 blur of the truth."""
import numpy as np

from oracle import mvd_oracle as O
from paper_1308_0730_amd import synth


def test_deterministic_per_seed():
    a = synth.make_problem((24, 20, 16), 6, [0, 90], (7, 7, 9), 1.0, 2.0, 99, weights=True)
    b = synth.make_problem((24, 20, 16), 6, [0, 90], (7, 7, 9), 1.0, 2.0, 99, weights=True)
    for x, y in zip(a.views + a.psfs + a.weights, b.views + b.psfs + b.weights):
        np.testing.assert_array_equal(x, y)
    c = synth.make_problem((24, 20, 16), 6, [0, 90], (7, 7, 9), 1.0, 2.0, 100)
    assert not np.array_equal(a.views[0], c.views[0])


def test_psf_normalised_and_rotated():
    p0 = synth.gaussian_psf((9, 9, 13), 1.2, 4.0, 0.0, dtype=np.float64)
    p90 = synth.gaussian_psf((13, 9, 9), 1.2, 4.0, 90.0, dtype=np.float64)
    assert abs(p0.sum() - 1) < 1e-12 and abs(p90.sum() - 1) < 1e-12
    # at 90 deg the long axis lies along x: transposing z and x maps one onto the other
    np.testing.assert_allclose(p90, np.transpose(p0, (2, 1, 0)), atol=1e-12)


def test_weights_bounds():
    dims = (64, 8, 48)
    ws = synth.overlap_weights(dims, [0, 60, 120, 180, 240, 300], band=8, ramp=6)
    W = np.stack(ws)
    assert W.min() >= 0 and W.max() <= 1
    S = W.sum(0)
    assert S.max() <= S.min() + 1e-5 or S.max() <= np.round(S.min()) + 1e-5


def test_views_match_blurred_truth():
    """A blob seen through the PSF rendered analytically agrees with the FP64
    circular blur of the sampled truth up to sampling error."""
    s = synth.make_problem((32, 32, 32), 12, [0.0, 90.0], (15, 15, 21), 1.0, 2.5, 7, noise="none")
    for v, p in zip(s.views, s.psfs):
        ref = O.circ_conv(s.truth.astype(np.float64), O.prepare_psf(p))
        assert O.rel_l2(v, ref) < 5e-3  # 4-sigma windows and point sampling
