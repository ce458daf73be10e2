"""Pins of the oracle's block-wise form: with a halo of twice the kernel
radius on each side the pasted blocks equal the whole-volume update (itself
pinned by direct summation) and direct summation on the blocks' grids, for
volumes of any extents, uneven tilings, every variant, weights and
lambda; a thinner halo gives a different result, and one block whose grid is
the volume itself is the whole-volume update."""
import numpy as np
import pytest

from oracle import mvd_oracle as O
from tests.test_oracle_pins import rand_kernel, rand_volume


def case(rng, n=(13, 17, 22), kshapes=((3, 5, 3), (5, 3, 3)), weights=True, lam=0.05):
    psfs = [rand_kernel(rng, k, offset=(0.3 * (-1) ** i, 0.4, -0.2 * i)) for i, k in enumerate(kshapes)]
    views = [rand_volume(rng, n, 1.0, 30.0) for _ in psfs]
    w = [rng.uniform(0.1, 1.0, size=n) for _ in psfs] if weights else None
    return O.Problem(views, psfs, w, lam)


def radius(pb):
    return tuple(max(P.shape[a] for P in pb.P) // 2 for a in range(3))


@pytest.mark.parametrize("variant", [O.RL, O.EFF, O.OPT1, O.OPT2])
@pytest.mark.parametrize("tiles", [(2, 3, 2), (1, 2, 4), (3, 1, 1)])
def test_halo_of_twice_the_radius_gives_the_whole_volume_update(variant, tiles):
    rng = np.random.default_rng(81)
    pb = case(rng)
    R = radius(pb)
    halo = tuple(2 * r for r in R)
    grid = tuple(-(-n // t) + 2 * h + 1 for n, t, h in zip(pb.shape, tiles, halo))  # one spare plane
    ref = pb.iterate(pb.psi0(), 2, variant)
    got = O.iterate_blocked(pb, pb.psi0(), 2, variant, tiles, halo, grid)
    np.testing.assert_allclose(got, ref, rtol=1e-12)


def test_blocks_equal_direct_summation():
    """The same blocked view-update with every convolution done by direct
    circular summation on the block grids, against the whole-volume update
    by direct summation."""
    rng = np.random.default_rng(82)
    pb = case(rng, n=(9, 11, 10), lam=0.0)
    R = radius(pb)
    halo = tuple(2 * r for r in R)
    tiles = (2, 2, 3)
    grid = tuple(-(-n // t) + 2 * h for n, t, h in zip(pb.shape, tiles, halo))
    K = pb.kernels(O.OPT1)
    psi = rand_volume(rng, pb.shape, 2.0, 20.0)
    whole = O.view_update(psi, pb.views[0], pb.P[0], K[0], pb.weights[0], pb.lam_p, pb.eps,
                          conv=O.circ_conv_direct)
    blocked = O.view_update_blocked(psi, pb.views[0], pb.P[0], K[0], tiles, halo, grid, pb.weights[0],
                                    pb.lam_p, pb.eps, conv=O.circ_conv_direct)
    np.testing.assert_allclose(blocked, whole, rtol=1e-12)


def test_a_thinner_halo_changes_the_result():
    rng = np.random.default_rng(83)
    pb = case(rng)
    R = radius(pb)
    tiles = (2, 2, 2)
    ref = pb.iterate(pb.psi0(), 1, O.RL)
    for halo in (R, tuple(2 * r - 1 for r in R)):
        grid = tuple(-(-n // t) + 2 * h for n, t, h in zip(pb.shape, tiles, halo))
        got = O.iterate_blocked(pb, pb.psi0(), 1, O.RL, tiles, halo, grid)
        assert np.max(np.abs(got - ref) / ref) > 1e-6, halo


def test_one_block_whose_grid_is_the_volume():
    rng = np.random.default_rng(84)
    pb = case(rng)
    ref = pb.iterate(pb.psi0(), 2, O.EFF)
    got = O.iterate_blocked(pb, pb.psi0(), 2, O.EFF, (1, 1, 1), (0, 0, 0), pb.shape)
    np.testing.assert_array_equal(got, ref)


def test_halo_wider_than_the_volume_wraps_again():
    """Tiny volume, several blocks, a halo longer than the volume along an
    axis: the grid reads the period more than once and stays exact."""
    rng = np.random.default_rng(85)
    pb = case(rng, n=(5, 6, 7), kshapes=((5, 5, 5), (3, 5, 3)))
    halo = (4, 4, 4)
    tiles = (2, 3, 1)
    grid = (3 + 8, 2 + 8, 7 + 8)
    ref = pb.iterate(pb.psi0(), 1, O.OPT2)
    got = O.iterate_blocked(pb, pb.psi0(), 1, O.OPT2, tiles, halo, grid)
    np.testing.assert_allclose(got, ref, rtol=1e-12)


def test_block_layout_covers_the_axis():
    for n in (1, 7, 100, 1070):
        for t in range(1, min(n, 9) + 1):
            lay = O.block_layout(n, t)
            assert lay[0][0] == 0 and sum(e for _, e in lay) == n
            assert all(o2 == o1 + e1 for (o1, e1), (o2, _) in zip(lay, lay[1:]))
            assert max(e for _, e in lay) - min(e for _, e in lay) <= 1
