"""The linear boundary on the GPU against the linear-boundary oracle: the
volume's estimate after one and several iterations, with weights and lambda,
for every variant; plus the reductions and the handle's bookkeeping."""
import numpy as np
import pytest
import torch

from oracle import mvd_oracle as O
from tests.test_gpu_parity import ONE_STEP, TRAJ, problem, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mvd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1308_0730_amd import mvd as m
    return m


CASES = [(v, wt, lam) for v in (O.RL, O.EFF, O.OPT1, O.OPT2) for wt in (False, True) for lam in (0.0, 0.02)]


@pytest.mark.parametrize("variant,weighted,lam", CASES)
def test_linear_iterations_match_the_oracle(mvd, variant, weighted, lam):
    """(40, 36, 30) with (9, 7, 7) PSFs: the grid is the volume plus margins
    (4, 3, 3) per side rounded up to transform lengths (48, 45, 40)."""
    views, psfs, w = problem((40, 36, 30), 3, 71, weighted)
    pb = O.ProblemLinear(views, psfs, w, lam)
    psi = pb.psi0()
    with mvd.Deconvolver(views, psfs, w, lam=lam, boundary="linear") as d:
        for it in range(3):
            psi = pb.iterate(psi, 1, variant)
            d.iterate(1, variant)
            e = rel(d.estimate().cpu().numpy(), pb.interior(psi))
            print(f"iteration {it + 1}: rel_l2={e:.3e}")
            assert e <= (ONE_STEP if it == 0 else TRAJ), (it, e)


@pytest.mark.parametrize("dims", [(64, 64, 64), (150, 54, 50)])
def test_linear_sizes(mvd, dims):
    views, psfs, w = problem(dims, 2, 72, True, psf_shape=(7, 7, 9))
    pb = O.ProblemLinear(views, psfs, w, 0.01)
    ref = pb.interior(pb.iterate(pb.psi0(), 2, O.OPT1))
    with mvd.Deconvolver(views, psfs, w, lam=0.01, boundary="linear") as d:
        d.iterate(2, O.OPT1)
        e = rel(d.estimate().cpu().numpy(), ref)
    print(f"{dims}: rel_l2={e:.3e}")
    assert e <= TRAJ


def test_delta_psfs_equal_the_circular_path(mvd):
    """With 1x1x1 PSFs there is no margin and every sensitivity is one: the
    linear and circular handles compute the same numbers."""
    rng = np.random.default_rng(73)
    views = [rng.uniform(1, 9, size=(30, 36, 40)).astype(np.float32) for _ in range(2)]
    d1 = [np.ones((1, 1, 1), np.float32)] * 2
    out = []
    for b in ("circular", "linear"):
        with mvd.Deconvolver(views, d1, lam=0.01, boundary=b) as d:
            d.iterate(2, O.RL)
            out.append(d.estimate().cpu().numpy())
    np.testing.assert_array_equal(out[0], out[1])


def test_batched_linear_equals_plain(mvd):
    blocks = [problem(dims, 2, 74 + i, psf_shape=(5, 5, 7)) for i, dims in enumerate([(40, 36, 30), (32, 48, 20)])]
    with mvd.Deconvolver.batch([(b[0], b[1]) for b in blocks], boundary="linear") as d:
        d.iterate(2, O.EFF)
        got = [d.estimate(block=i).cpu().numpy() for i in range(2)]
    for i, b in enumerate(blocks):
        with mvd.Deconvolver(b[0], b[1], boundary="linear") as p:
            p.set_tiles(*d_tiles_like(mvd, p))
            p.iterate(2, O.EFF)
            np.testing.assert_array_equal(got[i], p.estimate().cpu().numpy())


def d_tiles_like(mvd, d):
    """The per-length compile-time plans for every kind (what a batch of
    unequal blocks uses)."""
    out = []
    for kind in range(3):
        for c in mvd.tile_candidates(kind, d.max_lengths()[kind]):
            if mvd.tile_shape(kind, c)["exact_len"] == -1:
                out.append(c)
                break
    return out


def test_estimate_round_trip_and_rejections(mvd):
    views, psfs, w = problem((24, 20, 16), 2, 75, True, psf_shape=(5, 5, 5))
    rng = np.random.default_rng(76)
    x = rng.uniform(1, 5, size=views[0].shape).astype(np.float32)
    with mvd.Deconvolver(views, psfs, w, boundary="linear") as d:
        d.set_estimate(x)
        np.testing.assert_array_equal(d.estimate().cpu().numpy(), x)
        d.set_estimate(torch.from_numpy(x).cuda())
        np.testing.assert_array_equal(d.estimate().cpu().numpy(), x)
        for call in (lambda: d.iterate_combined(1, O.RL), lambda: d.normalize_weights("min")):
            with pytest.raises(mvd.MVDError) as e:
                call()
            assert e.value.code == mvd.MVD_ESTATE
