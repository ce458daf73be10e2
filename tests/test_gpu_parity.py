"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (relative L2): one iteration from the oracle's own estimate
<= 1e-5; whole runs from the flat start <= 1e-4, checked after every
iteration; the fixed point and the flux identity at FP32 round-off.  PSFs
are asymmetric wherever the test allows, so a wrong mirror cannot pass.
"""
import numpy as np
import pytest
import torch

from oracle import mvd_oracle as O
from paper_1308_0730_amd import synth

pytestmark = pytest.mark.gpu

ONE_STEP = 1e-5
TRAJ = 1e-4


@pytest.fixture(scope="module")
def mvd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1308_0730_amd import mvd as m
    return m


def asym_psf(rng, shape, off, tail=0.3):
    kz, ky, kx = shape
    z, y, x = np.meshgrid(np.arange(kz) - (kz - 1) / 2, np.arange(ky) - (ky - 1) / 2,
                          np.arange(kx) - (kx - 1) / 2, indexing="ij")
    g = np.exp(-0.5 * ((x - off[2]) ** 2 / 1.7 + (y - off[1]) ** 2 / 1.1 + (z - off[0]) ** 2 / 3.0))
    g += tail * np.exp(-0.5 * ((x + 1.5) ** 2 + (y - 1) ** 2 + (z + 2) ** 2) / 0.8)
    g += 0.02 * rng.uniform(size=shape)
    return (g / g.sum()).astype(np.float32)


def problem(dims, n_views, seed, weights=False, psf_shape=(9, 7, 7)):
    s = synth.make_problem(dims, max(4, int(40 * np.prod(dims) / 64 ** 3)), [0.0, 70.0, 130.0, 200.0][:n_views],
                           (5, 5, 7), 1.0, 2.0, seed, weights=False)
    rng = np.random.default_rng(seed + 7)
    offs = [(0.6, -0.4, 0.3), (-0.5, 0.5, 0.7), (0.3, 0.2, -0.6), (-0.2, -0.6, 0.4)]
    psfs = [asym_psf(rng, psf_shape, offs[v]) for v in range(n_views)]
    w = None
    if weights:
        w = [np.clip(rng.uniform(-0.2, 1.2, size=s.views[0].shape), 0, 1).astype(np.float32)
             for _ in range(n_views)]
    return s.views, psfs, w


def rel(a, b):
    return O.rel_l2(np.asarray(a, np.float64), b)


def max_rel(a, b, scale):
    """Largest element-wise error relative to max(|b|, scale) (scale: the
    views' mean, so voxels near zero do not divide by ~0)."""
    a = np.asarray(a, np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), scale)))


# element-wise bound of one iteration (measured 1e-6 to 3e-6)
ONE_STEP_MAX = 1e-5


CASES = [(v, wt, lam) for v in (O.RL, O.EFF, O.OPT1, O.OPT2) for wt in (False, True) for lam in (0.0, 0.02)]


@pytest.mark.parametrize("variant,weighted,lam", CASES)
def test_one_iteration_from_oracle_estimate(mvd, variant, weighted, lam):
    """dims (40, 36, 30): x has 20 complex columns (a ragged tile), y and z
    lengths use radices 2, 3 and 5."""
    views, psfs, w = problem((40, 36, 30), 3, 11, weighted)
    pb = O.Problem(views, psfs, w, lam)
    psi_r = pb.iterate(pb.psi0(), 2, variant).astype(np.float32)
    ref = pb.iterate(psi_r.astype(np.float64), 1, variant)
    with mvd.Deconvolver(views, psfs, w, lam=lam) as d:
        d.set_estimate(psi_r)
        d.iterate(1, variant)
        got = d.estimate().cpu().numpy()
    em = max_rel(got, ref, pb.s)
    print(f"rel_l2={rel(got, ref):.3e} max rel={em:.3e}")
    assert rel(got, ref) <= ONE_STEP, rel(got, ref)
    assert em <= ONE_STEP_MAX, em


@pytest.mark.parametrize("dims", [(150, 54, 50), (64, 100, 48), (4, 2, 2), (250, 24, 18), (1024, 6, 4),
                                  (2048, 6, 4), (1000, 6, 4), (16, 1024, 6), (8, 6, 1000)])
def test_one_iteration_odd_and_mixed_radix_sizes(mvd, dims):
    """Odd half-row length (nx/2 = 75 = 3*5*5), radix-5 lengths, the
    smallest valid volume, long rows (nx = 1000, 1024 and the largest,
    2048: half-rows of 500, 512 and 1024) and column lengths above 512
    (1024 along y, 1000 along z: compile-time plans on 8-line tiles)."""
    k = tuple(min(5, n if n % 2 else n - 1) for n in (dims[2], dims[1], dims[0]))
    views, psfs, _ = problem(dims, 2, 12, psf_shape=k)
    pb = O.Problem(views, psfs)
    psi_r = pb.iterate(pb.psi0(), 1, O.EFF).astype(np.float32)
    ref = pb.iterate(psi_r.astype(np.float64), 1, O.EFF)
    with mvd.Deconvolver(views, psfs) as d:
        d.set_estimate(psi_r)
        d.iterate(1, O.EFF)
        got = d.estimate().cpu().numpy()
    em = max_rel(got, ref, pb.s)
    print(f"rel_l2={rel(got, ref):.3e} max rel={em:.3e}")
    assert rel(got, ref) <= ONE_STEP, rel(got, ref)
    assert em <= ONE_STEP_MAX, em


def test_trajectory_config1(mvd):
    """64^3, two views, 17^3 PSFs, efficient update, 5 iterations."""
    s = synth.config1()
    pb = O.Problem(s.views, s.psfs)
    psi = pb.psi0()
    with mvd.Deconvolver(s.views, s.psfs) as d:
        for it in range(s.n_iter):
            psi = pb.iterate(psi, 1, O.EFF)
            d.iterate(1, O.EFF)
            e = rel(d.estimate().cpu().numpy(), psi)
            print(f"iteration {it}: rel_l2={e:.3e}")
            assert e <= (ONE_STEP if it == 0 else TRAJ), (it, e)
        st = d.stats()
    assert st["iterations"] == s.n_iter and not st["nonfinite"]


@pytest.mark.parametrize("variant", [O.RL, O.EFF])
def test_trajectory_config2(mvd, variant):
    """128^3, four views, 25^3 PSFs, 20 iterations of RL and of the efficient update."""
    s = synth.config2()
    pb = O.Problem(s.views, s.psfs)
    psi = pb.psi0()
    with mvd.Deconvolver(s.views, s.psfs) as d:
        for it in range(20):
            psi = pb.iterate(psi, 1, variant)
            d.iterate(1, variant)
            e = rel(d.estimate().cpu().numpy(), psi)
            print(f"iteration {it}: rel_l2={e:.3e}")
            assert e <= (ONE_STEP if it == 0 else TRAJ), (it, e)


@pytest.mark.parametrize("variant", [O.RL, O.EFF, O.OPT1, O.OPT2])
def test_fixed_point(mvd, variant):
    views, psfs, w = problem((48, 40, 36), 3, 13, weights=True)
    rng = np.random.default_rng(3)
    truth = rng.uniform(1.0, 20.0, size=views[0].shape)
    clean = [O.circ_conv(truth, O.prepare_psf(p)).astype(np.float32) for p in psfs]
    t32 = truth.astype(np.float32)
    with mvd.Deconvolver(clean, psfs, w) as d:
        d.set_estimate(t32)
        d.iterate(2, variant)
        got = d.estimate().cpu().numpy()
    assert rel(got, t32.astype(np.float64)) <= 2e-6


def test_flux_identity_rl(mvd):
    """RL, lambda = 0, no weights: after view v the total equals sum(phi_v)."""
    views, psfs, _ = problem((48, 40, 36), 3, 14)
    with mvd.Deconvolver(views, psfs) as d:
        d.iterate(3, O.RL)
        st = d.stats()
    for v in range(3):
        tot = float(np.sum(views[v], dtype=np.float64))
        assert abs(st["flux"][v] - tot) <= 2e-6 * tot, (v, st["flux"][v], tot)
    assert st["ratio_clamps"] == 0 and st["neg_clamps"] == 0


def test_graph_replay_equals_direct_launches(mvd):
    views, psfs, w = problem((40, 36, 30), 3, 15, weights=True)
    outs = []
    for g in (True, False):
        with mvd.Deconvolver(views, psfs, w, lam=0.01, use_graphs=g) as d:
            d.iterate(3, O.OPT1)
            outs.append(d.estimate().cpu().numpy())
    np.testing.assert_array_equal(outs[0], outs[1])


def test_single_view_delta_psf_returns_the_view(mvd):
    """A 1x1x1 PSF makes both convolutions the identity: one RL step from any
    estimate gives phi back."""
    rng = np.random.default_rng(5)
    phi = rng.uniform(1, 9, size=(6, 10, 12)).astype(np.float32)
    with mvd.Deconvolver([phi], [np.ones((1, 1, 1), np.float32)]) as d:
        d.iterate(1, O.RL)
        got = d.estimate().cpu().numpy()
    np.testing.assert_allclose(got, phi, rtol=2e-6)


def test_device_inputs_equal_host_inputs(mvd):
    views, psfs, w = problem((40, 36, 30), 2, 16, weights=True)
    with mvd.Deconvolver(views, psfs, w) as d:
        d.iterate(2, O.EFF)
        a = d.estimate().cpu().numpy()
    dv = [torch.from_numpy(v).cuda() for v in views]
    dp = [torch.from_numpy(p).cuda() for p in psfs]
    dw = [torch.from_numpy(x).cuda() for x in w]
    with mvd.Deconvolver(dv, dp, dw) as d:
        d.iterate(2, O.EFF)
        b = d.estimate().cpu().numpy()
    np.testing.assert_array_equal(a, b)


def test_device_value_checks(mvd):
    views, psfs, _ = problem((8, 6, 4), 2, 17, psf_shape=(3, 3, 3))
    dv = [torch.from_numpy(v).cuda() for v in views]
    dv[1][0, 0, 0] = -1.0
    with pytest.raises(mvd.MVDError) as e:
        mvd.Deconvolver(dv, psfs)
    assert e.value.code == mvd.MVD_EINVAL


SHAPE_DIMS = [(64, 64, 64), (512, 64, 32), (32, 512, 64), (32, 64, 256), (64, 128, 512), (150, 96, 100), (128, 128, 64),
              (256, 32, 128)]


@pytest.mark.parametrize("dims", SHAPE_DIMS)
def test_every_launch_shape(mvd, dims):
    """Every launch-shape candidate of every pass kind (runtime-plan and
    compile-time-plan) gives the oracle's iteration: the autotuner may pick
    any of them."""
    views, psfs, w = problem(dims, 2, 21, weights=True, psf_shape=(5, 5, 5))
    pb = O.Problem(views, psfs, w, 0.01)
    psi_r = pb.iterate(pb.psi0(), 1, O.OPT1).astype(np.float32)
    ref = pb.iterate(psi_r.astype(np.float64), 1, O.OPT1)
    with mvd.Deconvolver(views, psfs, w, lam=0.01) as d:
        base = d.tiles()
        lens = d.max_lengths()
        tried = 0
        for kind in range(3):
            for c in mvd.tile_candidates(kind, lens[kind]):
                cfg = list(base)
                cfg[kind] = c
                d.set_tiles(*cfg)
                d.set_estimate(psi_r)
                d.iterate(1, O.OPT1)
                e = rel(d.estimate().cpu().numpy(), ref)
                print(f"kind {kind} candidate {c} {mvd.tile_shape(kind, c)}: rel_l2={e:.3e}")
                assert e <= ONE_STEP, (kind, c, e)
                tried += 1
    assert tried >= 3


def test_zero_iterations_change_nothing(mvd):
    """mvd_iterate with n = 0 is a no-op: the estimate and the statistics
    stay as they were."""
    views, psfs, w = problem((40, 36, 30), 3, 41, weights=True)
    with mvd.Deconvolver(views, psfs, w) as d:
        d.iterate(2, O.OPT1)
        before = d.estimate().cpu().numpy()
        st = d.stats()
        d.iterate(0, O.OPT1)
        np.testing.assert_array_equal(d.estimate().cpu().numpy(), before)
        assert d.stats()["iterations"] == st["iterations"]


def test_all_zero_views_are_rejected(mvd):
    """Views without any signal have no mean intensity to start from (the
    flat start and the ratio guard are both scaled by it): create fails
    with MVD_EINVAL and names the block."""
    views, psfs, _ = problem((16, 12, 10), 2, 43)
    zero = [np.zeros_like(v) for v in views]
    with pytest.raises(mvd.MVDError) as e:
        mvd.Deconvolver(zero, psfs)
    assert e.value.code == mvd.MVD_EINVAL and "all zero" in str(e.value)



@pytest.mark.parametrize("variant", [O.RL, O.EFF, O.OPT1, O.OPT2])
def test_even_psf_extents(mvd, variant):
    """PSFs of even extents (8x6x6 and 6x8x7, asymmetric): each gets one
    trailing zero plane per even axis and its centre at (k - 1) / 2 of the
    padded box; one iteration from the oracle's estimate and a three-iteration
    run, with weights and lambda."""
    rng = np.random.default_rng(61)
    views, _, w = problem((40, 36, 30), 2, 62, True)
    psfs = [asym_psf(rng, (8, 6, 6), (0.5, -0.5, 0.5)), asym_psf(rng, (6, 8, 7), (-0.5, 0.5, 0.0))]
    pb = O.Problem(views, psfs, w, 0.02)
    psi_r = pb.iterate(pb.psi0(), 2, variant).astype(np.float32)
    ref = pb.iterate(psi_r.astype(np.float64), 1, variant)
    with mvd.Deconvolver(views, psfs, w, lam=0.02) as d:
        d.set_estimate(psi_r)
        d.iterate(1, variant)
        got = d.estimate().cpu().numpy()
        e1, em = rel(got, ref), max_rel(got, ref, pb.s)
        d.set_estimate(pb.psi0().astype(np.float32))
        d.iterate(3, variant)
        e3 = rel(d.estimate().cpu().numpy(), pb.iterate(pb.psi0(), 3, variant))
    print(f"one step rel_l2={e1:.3e} max rel={em:.3e}; three iterations rel_l2={e3:.3e}")
    assert e1 <= ONE_STEP and em <= ONE_STEP_MAX and e3 <= TRAJ


@pytest.mark.parametrize("variant", [O.RL, O.OPT1])
def test_active_clamps(mvd, variant):
    """Views that are zero on a box much larger than the PSFs: the estimate
    goes to zero there, the blur falls below eps (ratio clamps) and the
    back-projection's round-off goes negative (negativity clamps).  Both
    sides take those branches; the estimates agree, and inside the box the
    GPU estimate is zero up to round-off."""
    views, psfs, _ = problem((48, 40, 36), 2, 63)
    box = (slice(8, 28), slice(10, 32), slice(12, 38))
    for v in views:
        v[box] = 0.0
    pb = O.Problem(views, psfs)
    stats = {}
    psi = pb.iterate(pb.psi0(), 4, variant)
    ref = pb.iterate(psi, 1, variant, stats=stats)
    with mvd.Deconvolver(views, psfs) as d:
        d.iterate(5, variant)
        st = d.stats()
        got = d.estimate().cpu().numpy()
    e = rel(got, ref)
    inner = got[10:26, 12:30, 14:36]
    print(f"rel_l2={e:.3e}; GPU clamps in the last iteration: ratio {st['ratio_clamps']} neg {st['neg_clamps']}; "
          f"oracle {stats}; largest inner value {float(inner.max()):.3e} (s = {pb.s:.3e})")
    assert e <= TRAJ
    assert st["ratio_clamps"] > 0 and st["neg_clamps"] > 0
    assert stats["ratio_clamps"] > 0
    assert float(inner.max()) <= 1e-3 * pb.s
