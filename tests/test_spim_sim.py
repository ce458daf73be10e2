"""The SPIM acquisition simulator's pieces against closed forms: the
Beer-Lambert attenuation, the rotation convention of the analytic PSF, the
object's support, determinism, and the intensity budget of a view."""
import math

import numpy as np

from paper_1308_0730_amd import spim_sim as S


def test_attenuation_closed_form():
    vol = np.zeros((1, 6, 2), np.float32)
    vol[0, :, 0] = 1.0
    vol[0, :, 1] = 0.5
    got = S.attenuate(vol, delta=0.1)
    # column 0: unit density, the k-th voxel has crossed k units
    np.testing.assert_allclose(got[0, :, 0], np.exp(-0.1 * np.arange(6)), rtol=1e-6)
    # column 1: density 0.5 relative to the maximum 1
    np.testing.assert_allclose(got[0, :, 1], 0.5 * np.exp(-0.1 * 0.5 * np.arange(6)), rtol=1e-6)


def test_psf_rotation_matches_volume_rotation():
    p0 = S.gaussian_psf_x((21, 21, 21), 1.0, 3.5, 0.0)
    for th in (30.0, -50.0):
        same = S.correlation(S.rotate_x(p0, th), S.gaussian_psf_x((21, 21, 21), 1.0, 3.5, th))
        mirror = S.correlation(S.rotate_x(p0, th), S.gaussian_psf_x((21, 21, 21), 1.0, 3.5, -th))
        assert same > 0.99 and mirror < 0.8


def test_psf_normalised_and_axis():
    p = S.gaussian_psf_x((9, 9, 21), 1.0, 3.0, 0.0)
    assert abs(float(p.sum()) - 1.0) < 1e-6
    # elongated along z (axis 0 of (kz, ky, kx))
    prof_z = p[:, 4, 4] / p[10, 4, 4]
    prof_x = p[10, 4, :] / p[10, 4, 4]
    assert prof_z[13] > prof_x[7]  # 3 voxels out: z wider than x
    np.testing.assert_allclose(prof_z[13], math.exp(-0.5 * 9 / 9.0), rtol=1e-5)


def test_object_support_and_determinism():
    dims = (32, 32, 32)
    obj = S.sphere_object(dims, 60, 5)
    z, y, x = np.meshgrid(*[np.arange(n) + 0.5 - n / 2 for n in (32, 32, 32)], indexing="ij")
    r = np.sqrt(x * x + y * y + z * z)
    R = 0.36 * 32 + 2.2 + 1
    assert obj[r > R].max() == 0 and obj.max() > 0
    a = S.simulate((32, 32, 32), n_spheres=40, psf_extent=(7, 7, 11), seed=3)
    b = S.simulate((32, 32, 32), n_spheres=40, psf_extent=(7, 7, 11), seed=3)
    for u, v in zip(a.views, b.views):
        np.testing.assert_array_equal(u, v)


def test_views_keep_the_intensity_budget():
    """Without attenuation the PSF is normalised and the Poisson counts are
    unbiased, so a view's total stays close to the ground truth's."""
    a = S.simulate((48, 48, 48), n_spheres=120, psf_extent=(7, 7, 13), delta=0.0, seed=9)
    t = float(a.truth.sum())
    for v in a.views:
        assert abs(float(v.sum()) - t) < 0.05 * t
        assert v.min() >= 0
