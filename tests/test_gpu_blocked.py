"""The block-wise form on the GPU: each block of the volume computes the
view-update on its own grid (the block and a halo read periodically from the
volume) and pastes its voxels back.  Against the oracle's whole-volume
circular update (exact for a halo of twice the PSF radius) on volumes of
extents that are not transform lengths, against the oracle's own block-wise
form for a thinner halo, beyond the transform-length limits, and at the
size of the paper's largest four-view dataset on sampled voxels."""
import numpy as np
import pytest
import torch

from oracle import mvd_oracle as O
from paper_1308_0730_amd import synth
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
def test_blocks_equal_the_whole_volume(mvd, variant, weighted, lam):
    """45x38x27 (no extent a transform length), 3 views, 9x7x7 PSFs (radius
    3, 3, 4; halo 6, 6, 8), 2x2x2 blocks on 36x32x30 grids."""
    views, psfs, w = problem((45, 38, 27), 3, 401, weighted)
    pb = O.Problem(views, psfs, w, lam)
    psi = pb.psi0()
    with mvd.Deconvolver.blocked(views, psfs, w, tiles=(2, 2, 2), lam=lam) as d:
        tiles, halo, dims = d.blocking()
        assert tiles == (2, 2, 2) and halo == (6, 6, 8) and dims == (45, 38, 27)
        assert d.grid_dims(0) == (36, 32, 30)
        for it in range(2):
            psi = pb.iterate(psi, 1, variant)
            d.iterate(1, variant)
            got = d.estimate().cpu().numpy()
            e = rel(got, psi)
            emax = float(np.max(np.abs(got - psi) / np.maximum(np.abs(psi), pb.s)))
            print(f"iteration {it + 1}: rel_l2={e:.3e} max rel={emax:.3e}")
            assert e <= (ONE_STEP if it == 0 else TRAJ), (it, e)
            if it == 0:
                assert emax <= 1e-5


@pytest.mark.parametrize("variant", [O.RL, O.OPT1])
def test_thin_halo_follows_the_oracles_blocked_form(mvd, variant):
    """A halo of one radius: the grids' wrap-around reaches the pasted voxels;
    the GPU follows the oracle's block-wise form with the same tiles, halo and
    grid, and differs from the whole-volume update."""
    views, psfs, w = problem((45, 38, 27), 2, 402, True)
    pb = O.Problem(views, psfs, w, 0.01)
    halo_xyz = (3, 3, 4)
    with mvd.Deconvolver.blocked(views, psfs, w, tiles=(2, 3, 2), halo=halo_xyz, lam=0.01) as d:
        g = d.grid_dims(0)
        d.iterate(1, variant)
        got = d.estimate().cpu().numpy()
    ref = O.iterate_blocked(pb, pb.psi0(), 1, variant, (2, 3, 2), halo_xyz[::-1], g[::-1])
    whole = pb.iterate(pb.psi0(), 1, variant)
    e = rel(got, ref)
    print(f"grid {g}: rel_l2 vs the oracle's blocks {e:.3e}, blocks vs whole volume {rel(ref, whole):.3e}")
    assert e <= ONE_STEP
    assert rel(ref, whole) > 1e-3


def test_beyond_the_transform_lengths(mvd):
    """2050x1030x8: x beyond 2048 and y beyond 1024 points.  The default
    blocking takes three blocks along x and y (720x360x8 grids: half-rows
    and columns within 512 points; z, one block of a transform length, needs
    no halo); two blocks along each give the longest grids (1080x540x8).
    One iteration of each against the whole-volume oracle."""
    views, psfs, _ = problem((2050, 1030, 8), 2, 403, psf_shape=(3, 5, 5))
    pb = O.Problem(views, psfs, None, 0.0)
    ref = pb.iterate(pb.psi0(), 1, O.EFF)
    for tiles_in, tiles_out, grid in ((None, (3, 3, 1), (720, 360, 8)), ((2, 2, 1), (2, 2, 1), (1080, 540, 8))):
        with mvd.Deconvolver.blocked(views, psfs, tiles=tiles_in) as d:
            tiles, halo, _ = d.blocking()
            print("tiles", tiles, "halo", halo, "grid", d.grid_dims(0))
            assert tiles == tiles_out and d.grid_dims(0) == grid
            d.iterate(1, O.EFF)
            got = d.estimate().cpu().numpy()
        e = rel(got, ref)
        print(f"rel_l2={e:.3e}")
        assert e <= ONE_STEP


def test_one_block_is_the_plain_run(mvd):
    views, psfs, w = problem((48, 40, 30), 2, 404, True)
    with mvd.Deconvolver(views, psfs, w, lam=0.01) as d:
        d.iterate(3, O.OPT1)
        plain = d.estimate().cpu().numpy()
    with mvd.Deconvolver.blocked(views, psfs, w, tiles=(1, 1, 1), halo=(0, 0, 0), lam=0.01) as d:
        assert d.grid_dims(0) == (48, 40, 30)
        d.iterate(3, O.OPT1)
        got = d.estimate().cpu().numpy()
    e = rel(got, plain)
    print(f"rel_l2 vs the plain handle {e:.3e}")
    assert e <= 1e-6


def test_graph_replay_equals_direct_launches_and_flux(mvd):
    views, psfs, _ = problem((45, 38, 27), 2, 405)
    out = []
    for graphs in (True, False):
        with mvd.Deconvolver.blocked(views, psfs, tiles=(3, 2, 2), use_graphs=graphs) as d:
            d.iterate(2, O.RL)
            out.append(d.estimate().cpu().numpy())
            st = d.stats()
    np.testing.assert_array_equal(out[0], out[1])
    # RL, normalised PSFs, lambda 0, no weights: after view v the volume's flux is sum phi_v
    for v in range(2):
        target = float(np.sum(views[v], dtype=np.float64))
        print(f"flux after view {v}: {st['flux'][v]:.6e} (sum phi {target:.6e})")
        assert abs(st["flux"][v] - target) <= 2e-6 * target


def test_estimate_round_trip_and_rejections(mvd):
    views, psfs, w = problem((25, 21, 17), 2, 406, True, psf_shape=(5, 5, 5))
    rng = np.random.default_rng(407)
    x = rng.uniform(1, 5, size=views[0].shape).astype(np.float32)
    with mvd.Deconvolver.blocked(views, psfs, w, tiles=(2, 2, 1)) as d:
        d.set_estimate(x)
        np.testing.assert_array_equal(d.estimate().cpu().numpy(), x)
        d.set_estimate(torch.from_numpy(x).cuda())
        np.testing.assert_array_equal(d.estimate().cpu().numpy(), x)
        for call in (lambda: d.iterate_combined(1, O.RL), lambda: d.normalize_weights("min"),
                     lambda: d.loss_grad(1, psf_shapes=[p.shape for p in psfs])):
            with pytest.raises(mvd.MVDError) as e:
                call()
            assert e.value.code == mvd.MVD_ESTATE
    for kw in (dict(tiles=(26, 1, 1)), dict(tiles=(1, 1, 1), halo=(0, 600, 0)), dict(halo=(-1, 0, 0))):
        with pytest.raises(mvd.MVDError) as e:
            mvd.Deconvolver.blocked(views, psfs, **kw)
        assert e.value.code == mvd.MVD_EINVAL


@pytest.fixture(scope="module")
def larva():
    return synth.larva()


def test_larva_scale_sampled(mvd, larva):
    """1640x1070x345 with four views (Optimization II, lambda 0): two blocks
    along x and three along y on 864x400x405 grids; after one iteration, view
    1's update at sampled voxels (near the block seams and the wrap-around
    too) against the oracle's windowed evaluation."""
    s = larva
    v = 1
    dev = [torch.from_numpy(x).cuda() for x in s.views]
    with mvd.Deconvolver.blocked(dev, s.psfs) as d:
        tiles, halo, dims = d.blocking()
        print("tiles", tiles, "halo", halo, "grid", d.grid_dims(0), flush=True)
        assert tiles == (2, 3, 1) and dims == (1640, 1070, 345) and d.grid_dims(0) == (864, 400, 405)
        d.iterate(1, O.OPT2)
        psi = d.estimate().cpu().numpy()
        d.view_update(v, O.OPT2)
        out = d.estimate().cpu().numpy()
    del dev
    scale = float(np.mean([np.mean(x, dtype=np.float64) for x in s.views]))
    P = O.prepare_psf(s.psfs[v])
    K = O.compound_kernel(s.psfs, v, O.OPT2)
    rng = np.random.default_rng(408)
    nz, ny, nx = psi.shape
    pts = [tuple(int(a) for a in p) for p in rng.integers(0, [nz, ny, nx], size=(30, 3))]
    # the seams between the y blocks (y = 356, 713), the x blocks (x = 820)
    # and the wrap-around
    pts += [(int(z), y, int(x)) for y in (355, 356, 357, 712, 713, 714) for z, x in rng.integers(0, [nz, nx], size=(2, 2))]
    pts += [(int(z), int(y), x) for x in (819, 820, 821) for z, y in rng.integers(0, [nz, ny], size=(2, 2))]
    pts += [(0, 0, 0), (nz - 1, ny - 1, nx - 1), (nz - 1, 0, 5), (3, ny - 1, nx - 2)]
    bright = np.argwhere(s.truth[::4, ::4, ::4] > np.percentile(s.truth[::4, ::4, ::4], 99.9)) * 4
    pts += [tuple(int(a) for a in bright[i]) for i in rng.integers(0, len(bright), size=10)]
    ref = O.view_update_at(psi, s.views[v], P, K, pts, None, 0.0, O.EPS_SCALE * scale)
    got = np.array([out[p] for p in pts], np.float64)
    e = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    emax = float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), scale)))
    print(f"sampled view-update: rel_l2={e:.3e} max rel={emax:.3e} over {len(pts)} voxels")
    assert e <= 1e-5 and emax <= 1e-5


@pytest.mark.parametrize("dims,psf_shape,tiles,halo", [((10, 12, 9), (9, 9, 9), (1, 1, 1), (8, 8, 8)),
                                                       ((3, 5, 4), (3, 3, 3), (1, 1, 1), (2, 2, 2)),
                                                       ((21, 17, 13), (7, 5, 9), (3, 2, 2), None)])
def test_windows_wider_than_the_volume(mvd, dims, psf_shape, tiles, halo):
    """Windows that wrap around the volume several times along x (a 30-point
    grid on a 10-voxel volume), the smallest grid (8 points along x for a
    3-voxel volume), and blocks thinner than their halo: still the
    whole-volume update, two iterations with weights and lambda."""
    views, psfs, w = problem(dims, 2, 409, True, psf_shape=psf_shape)
    pb = O.Problem(views, psfs, w, 0.01)
    psi = pb.psi0()
    with mvd.Deconvolver.blocked(views, psfs, w, tiles=tiles, halo=halo, lam=0.01) as d:
        g = d.grid_dims(0)
        print("grid", g, "blocking", d.blocking())
        assert g[0] >= 8
        for it in range(2):
            psi = pb.iterate(psi, 1, O.OPT1)
            d.iterate(1, O.OPT1)
            e = rel(d.estimate().cpu().numpy(), psi)
            print(f"iteration {it + 1}: rel_l2={e:.3e}")
            assert e <= (ONE_STEP if it == 0 else TRAJ), (it, e)


def test_single_block_axes_of_transform_length_take_no_halo(mvd):
    """64x45x32 in one block along x and z (transform lengths: the grid is
    the volume's period there, no halo) and two along y (45 is not a
    transform length; halo of twice the radius): the whole-volume update,
    two iterations with weights and lambda."""
    views, psfs, w = problem((64, 45, 32), 2, 410, True)
    pb = O.Problem(views, psfs, w, 0.01)
    psi = pb.psi0()
    with mvd.Deconvolver.blocked(views, psfs, w, tiles=(1, 2, 1), lam=0.01) as d:
        tiles, halo, _ = d.blocking()
        g = d.grid_dims(0)
        print("halo", halo, "grid", g)
        assert halo == (0, 6, 0) and g[0] == 64 and g[2] == 32
        for it in range(2):
            psi = pb.iterate(psi, 1, O.OPT1)
            d.iterate(1, O.OPT1)
            e = rel(d.estimate().cpu().numpy(), psi)
            print(f"iteration {it + 1}: rel_l2={e:.3e}")
            assert e <= (ONE_STEP if it == 0 else TRAJ), (it, e)
