"""C ABI on the host: the library loads, exports what include/mvd.h declares,
rejects bad arguments before touching a device, and its FP64 host
preparation (compound kernels, kernel spectra) matches the oracle."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import mvd_oracle as O
from paper_1308_0730_amd import mvd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "mvd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mvd_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = mvd.lib()
    names = declared_symbols()
    assert "mvd_create" in names and "mvd_iterate" in names and "mvd_get_estimate" in names
    for n in names:
        assert hasattr(L, n), n
    assert L.mvd_version().startswith(b"mvd")


def small_problem(rng, dims=(8, 6, 4), n=2, weights=False):
    nx, ny, nz = dims
    views = [rng.uniform(1, 5, size=(nz, ny, nx)).astype(np.float32) for _ in range(n)]
    psfs = [rng.uniform(0, 1, size=(3, 3, 3)).astype(np.float32) for _ in range(n)]
    w = [rng.uniform(0, 1, size=(nz, ny, nx)).astype(np.float32) for _ in range(n)] if weights else None
    return views, psfs, w


def expect_einval(blocks, needle, options=None):
    rc, h, msg = mvd.create_raw(blocks, options)
    assert rc == mvd.MVD_EINVAL, (rc, msg)
    assert h is None
    assert needle in msg, msg


def test_rejects_bad_shapes():
    rng = np.random.default_rng(0)
    v, p, w = small_problem(rng, (7, 6, 4))
    expect_einval([(v, p, w)], "nx must be even")
    v, p, w = small_problem(rng, (14, 6, 4))
    expect_einval([(v, p, w)], "5-smooth")
    v, p, w = small_problem(rng, (8, 1080, 4))
    expect_einval([(v, p, w)], "ny and nz must be in [2, 1024]")
    v, p, w = small_problem(rng, (8, 6, 4))
    p = [np.ones((9, 3, 3), np.float32)] * 2
    expect_einval([(v, p, w)], "larger than the volume")
    v, p, w = small_problem(rng, (8, 6, 4))
    expect_einval([(v, p, w), small_problem(rng, (8, 6, 4), n=3)], "same number of views")


def test_rejects_bad_values():
    rng = np.random.default_rng(1)
    v, p, w = small_problem(rng, weights=True)
    v[1][0, 0, 3] = -1.0
    expect_einval([(v, p, w)], "negative or non-finite")
    v, p, w = small_problem(rng)
    v[0][1, 2, 3] = np.nan
    expect_einval([(v, p, w)], "negative or non-finite")
    v, p, w = small_problem(rng)
    p[1] = np.zeros_like(p[1])
    expect_einval([(v, p, w)], "sum must be positive")
    v, p, w = small_problem(rng)
    p[0][0, 0, 0] = np.inf
    expect_einval([(v, p, w)], "finite")
    v, p, w = small_problem(rng, weights=True)
    w[0][0, 0, 0] = 1.5
    expect_einval([(v, p, w)], "outside [0, 1]")


def test_rejects_bad_options_and_nulls():
    rng = np.random.default_rng(2)
    v, p, w = small_problem(rng)
    expect_einval([(v, p, w)], "lambda", mvd.Options(-1.0, 0.0, None, mvd.ALLOC_FN(), mvd.FREE_FN(), None, 1, 0))
    L = mvd.lib()
    h = C.c_void_p(123)
    assert L.mvd_create(C.byref(h), None, None) == mvd.MVD_EINVAL
    assert h.value is None
    assert L.mvd_create(None, None, None) == mvd.MVD_EINVAL
    assert L.mvd_iterate(None, 1, 0) == mvd.MVD_EINVAL
    assert L.mvd_get_estimate(None, None, 0, 0) == mvd.MVD_EINVAL
    assert L.mvd_destroy(None) == mvd.MVD_OK
    assert b"NULL" in L.mvd_last_error(None)


def rand_kernel(rng, shape, off):
    kz, ky, kx = shape
    z, y, x = np.meshgrid(np.arange(kz) - (kz - 1) / 2, np.arange(ky) - (ky - 1) / 2,
                          np.arange(kx) - (kx - 1) / 2, indexing="ij")
    g = np.exp(-0.5 * ((x - off[2]) ** 2 / 1.5 + (y - off[1]) ** 2 / 0.7 + (z - off[0]) ** 2 / 2.5))
    g += 0.04 * rng.uniform(size=shape)
    return (g / g.sum()).astype(np.float32)


@pytest.mark.parametrize("variant", [O.RL, O.EFF, O.OPT1, O.OPT2])
def test_compound_kernel_matches_oracle(variant):
    """Host FP64 compound kernels (direct DFT on a padded grid) equal the
    oracle's (direct convolution of the small kernels); unequal and even
    extents included."""
    rng = np.random.default_rng(3)
    psfs = [rand_kernel(rng, (5, 3, 7), (0.4, -0.2, 0.6)), rand_kernel(rng, (4, 5, 3), (-0.5, 0.3, 0.1)),
            rand_kernel(rng, (3, 3, 5), (0.2, 0.4, -0.3))]
    for v in range(3):
        got = mvd.compound_kernel(psfs, v, variant)
        ref = O.compound_kernel([p.astype(np.float64) for p in psfs], v, variant)
        assert got.shape == ref.shape
        np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-14 * ref.max())


@pytest.mark.parametrize("variant", [O.RL, O.EFF, O.OPT1, O.OPT2])
def test_compound_kernel_vjp_matches_oracle(variant):
    """The host adjoint of the compound-kernel construction (direct DFTs on a
    padded grid) equals the oracle's (correlations of the small kernels),
    for every view's kernel, unequal and even extents included."""
    rng = np.random.default_rng(5)
    psfs = [rand_kernel(rng, (5, 3, 7), (0.4, -0.2, 0.6)), rand_kernel(rng, (4, 5, 3), (-0.5, 0.3, 0.1)),
            rand_kernel(rng, (3, 3, 5), (0.2, 0.4, -0.3))]
    P = [O.prepare_psf(p.astype(np.float64)) for p in psfs]
    for v in range(3):
        kbar = rng.normal(size=P[v].shape)
        got = mvd.compound_kernel_vjp(psfs, v, variant, kbar)
        ref = O.compound_kernel_vjp(P, v, variant, kbar)
        for g, r in zip(got, ref):
            assert g.shape == r.shape
            np.testing.assert_allclose(g, r, rtol=1e-9, atol=1e-12 * max(np.abs(r).max(), 1e-300))


def test_kernel_spectrum_matches_fft_of_embedded_kernel():
    rng = np.random.default_rng(4)
    K = O.prepare_psf(rand_kernel(rng, (5, 3, 7), (0.3, 0.2, -0.4)))
    dims = (20, 12, 10)
    main, nyq = mvd.kernel_spectrum(K, dims)
    shape = (dims[2], dims[1], dims[0])
    ref = np.fft.rfftn(O.embed(K, shape)) / np.prod(shape)
    np.testing.assert_allclose(main, ref[:, :, :dims[0] // 2], rtol=0, atol=1e-7 * np.abs(ref).max())
    np.testing.assert_allclose(nyq, ref[:, :, dims[0] // 2], rtol=0, atol=1e-7 * np.abs(ref).max())
