"""Weight normalisation on the GPU against the oracle: the overlap number of
every mode, the contributing-view image, and an iteration with the
normalised weights."""
import numpy as np
import pytest
import torch

from oracle import mvd_oracle as O
from tests.test_gpu_parity import ONE_STEP, problem, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mvd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1308_0730_amd import mvd as m
    return m


def sparse_weights(shape, n, seed):
    rng = np.random.default_rng(seed)
    return [np.clip(rng.uniform(-0.6, 1.4, size=shape), 0, 1).astype(np.float32) for _ in range(n)]


def test_contributing_views_image(mvd):
    views, psfs, _ = problem((40, 36, 30), 3, 51)
    w = sparse_weights(views[0].shape, 3, 52)
    with mvd.Deconvolver(views, psfs, w) as d:
        got = d.contributing_views().cpu().numpy()
    np.testing.assert_array_equal(got, O.contributing_views(w))


@pytest.mark.parametrize("mode,value", [("one", 0.0), ("min", 0.0), ("avg", 0.0), ("user", 1.7)])
def test_normalised_weights_iterate_like_the_oracle(mvd, mode, value):
    views, psfs, _ = problem((40, 36, 30), 3, 53)
    w = sparse_weights(views[0].shape, 3, 54)
    omode = {"one": O.OVERLAP_ONE, "min": O.OVERLAP_MIN, "avg": O.OVERLAP_AVG, "user": O.OVERLAP_USER}[mode]
    wn, m_ref = O.normalize_weights(w, omode, value)
    pb = O.Problem(views, psfs, wn, 0.01)
    ref = pb.iterate(pb.psi0(), 1, O.OPT1)
    with mvd.Deconvolver(views, psfs, w, lam=0.01) as d:
        m = d.normalize_weights(mode, value)
        d.iterate(1, O.OPT1)
        got = d.estimate().cpu().numpy()
    assert m[0] == pytest.approx(m_ref, rel=1e-12)
    e = rel(got, ref)
    print(f"mode {mode}: m={m[0]:.6f} rel_l2={e:.3e}")
    assert e <= ONE_STEP


def test_batched_overlap_numbers_per_block(mvd):
    blocks = []
    refs = []
    for i, dims in enumerate([(40, 36, 30), (32, 48, 20)]):
        v, p, _ = problem(dims, 2, 55 + i, psf_shape=(5, 5, 5))
        w = sparse_weights(v[0].shape, 2, 60 + i)
        blocks.append((v, p, w))
        refs.append(O.normalize_weights(w, O.OVERLAP_AVG)[1])
    with mvd.Deconvolver.batch(blocks) as d:
        m = d.normalize_weights("avg")
    np.testing.assert_allclose(m, refs, rtol=1e-12)


def test_weights_required(mvd):
    views, psfs, _ = problem((16, 12, 10), 2, 56, psf_shape=(3, 3, 3))
    with mvd.Deconvolver(views, psfs) as d:
        with pytest.raises(mvd.MVDError) as e:
            d.normalize_weights("min")
        assert e.value.code == mvd.MVD_ESTATE
        with pytest.raises(mvd.MVDError):
            d.contributing_views()
    views, psfs, w = problem((16, 12, 10), 2, 57, weights=True, psf_shape=(3, 3, 3))
    with mvd.Deconvolver(views, psfs, w) as d:
        with pytest.raises(mvd.MVDError) as e:
            d.normalize_weights("user", -1.0)
        assert e.value.code == mvd.MVD_EINVAL
