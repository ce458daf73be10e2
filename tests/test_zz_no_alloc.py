"""mvd_iterate_noalloc (every device buffer in the library's static scratch
array) against the allocating entry points (mvd_create, mvd_set_estimate,
mvd_iterate, mvd_get_estimate) on the same inputs: two calls in a row, the
second on a smaller volume, then a problem too large for the array (a clear
error) followed by a call that still computes the right result."""
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


def allocating(mvd, views, psfs, w, lam, n, variant, psi0=None, boundary="circular"):
    with mvd.Deconvolver(views, psfs, w, lam=lam, boundary=boundary) as d:
        if psi0 is not None:
            d.set_estimate(psi0)
        d.iterate(n, variant)
        return d.estimate().cpu().numpy()


def test_two_calls_in_a_row_the_second_smaller(mvd):
    # first call: 48x40x30, three views with weights and lambda, OPT1, 3 iterations
    views, psfs, w = problem((48, 40, 30), 3, 301, True)
    print("no-alloc call 1: 48x40x30, 3 views, weights, lambda 0.01, OPT1, 3 iterations", flush=True)
    got = mvd.iterate_noalloc(views, psfs, 3, "opt1", weights=w, lam=0.01).cpu().numpy()
    ref = allocating(mvd, views, psfs, w, 0.01, 3, O.OPT1)
    np.testing.assert_array_equal(got, ref)
    pb = O.Problem(views, psfs, w, 0.01)
    e = rel(got, pb.iterate(pb.psi0(), 3, O.OPT1))
    print(f"  rel_l2 vs oracle {e:.2e}")
    assert e <= TRAJ
    # second call, smaller: 32x24x20, two views, EFF, from a given estimate
    views2, psfs2, _ = problem((32, 24, 20), 2, 302, psf_shape=(7, 5, 5))
    pb2 = O.Problem(views2, psfs2)
    start = np.random.default_rng(303).uniform(0.5, 2.0, size=views2[0].shape) * pb2.s
    psi0 = torch.from_numpy(start.astype(np.float32)).cuda()
    print("no-alloc call 2: 32x24x20, 2 views, EFF, 1 iteration from a given estimate", flush=True)
    got2 = mvd.iterate_noalloc(views2, psfs2, 1, "eff", psi0=psi0).cpu().numpy()
    ref2 = allocating(mvd, views2, psfs2, None, 0.0, 1, O.EFF, psi0=psi0)
    np.testing.assert_array_equal(got2, ref2)
    e2 = rel(got2, pb2.iterate(start.astype(np.float32).astype(np.float64), 1, O.EFF))
    print(f"  rel_l2 vs oracle {e2:.2e}")
    assert e2 <= ONE_STEP


def test_out_may_be_psi0(mvd):
    views, psfs, _ = problem((40, 36, 30), 2, 304)
    print("no-alloc: 40x36x30, 2 views, RL, out = psi0", flush=True)
    psi = mvd.iterate_noalloc(views, psfs, 2, "rl")
    mvd.iterate_noalloc(views, psfs, 2, "rl", psi0=psi, out=psi)
    with mvd.Deconvolver(views, psfs) as d:
        d.iterate(2, O.RL)
        d.set_estimate(d.estimate())
        d.iterate(2, O.RL)
        ref = d.estimate().cpu().numpy()
    np.testing.assert_array_equal(psi.cpu().numpy(), ref)


def test_linear_boundary(mvd):
    views, psfs, w = problem((40, 36, 30), 2, 305, True, psf_shape=(7, 5, 5))
    print("no-alloc: 40x36x30 linear boundary, 2 views, weights, OPT2, 2 iterations", flush=True)
    got = mvd.iterate_noalloc(views, psfs, 2, "opt2", weights=w, boundary="linear").cpu().numpy()
    ref = allocating(mvd, views, psfs, w, 0.0, 2, O.OPT2, boundary="linear")
    np.testing.assert_array_equal(got, ref)


def test_too_large_is_rejected_then_a_small_call_still_works(mvd):
    dims = (256, 256, 160)  # four views alone take 168 MB
    rng = np.random.default_rng(306)
    views = [torch.full((dims[2], dims[1], dims[0]), 3.0, device="cuda") for _ in range(4)]
    psfs = [np.ones((3, 3, 3), np.float32)] * 4
    print("no-alloc: 256x256x160 with 4 views (beyond the scratch array): expect MVD_EINVAL", flush=True)
    with pytest.raises(mvd.MVDError) as e:
        mvd.iterate_noalloc(views, psfs, 1, "rl")
    assert e.value.code == mvd.MVD_EINVAL
    assert "scratch" in str(e.value)
    del views, rng
    views2, psfs2, _ = problem((24, 20, 16), 2, 307, psf_shape=(5, 5, 5))
    print("no-alloc: 24x20x16 after the rejection", flush=True)
    got = mvd.iterate_noalloc(views2, psfs2, 2, "eff").cpu().numpy()
    np.testing.assert_array_equal(got, allocating(mvd, views2, psfs2, None, 0.0, 2, O.EFF))


def test_argument_errors(mvd):
    views, psfs, _ = problem((24, 20, 16), 2, 308, psf_shape=(5, 5, 5))
    with pytest.raises(mvd.MVDError) as e:
        mvd.iterate_noalloc(views, psfs, -1, "eff")
    assert e.value.code == mvd.MVD_EINVAL
    with pytest.raises(ValueError):
        mvd.iterate_noalloc(views, psfs, 1, "eff", out=torch.empty(3, device="cuda"))
