"""Batched form: blocks of different sizes deconvolved together equal the
plain form run on each block alone, and the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import mvd_oracle as O
from paper_1308_0730_amd import synth

pytestmark = pytest.mark.gpu

DIMS = [(40, 36, 30), (48, 40, 36), (64, 64, 48), (60, 54, 50), (32, 32, 32), (96, 24, 20)]


@pytest.fixture(scope="module")
def mvd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1308_0730_amd import mvd as m
    return m


def block(dims, seed):
    s = synth.make_problem(dims, max(4, int(40 * np.prod(dims) / 64 ** 3)), [0.0, 45.0, 90.0, 135.0],
                           (7, 7, 9), 1.0 * (1 + 0.05 * (seed % 3)), 2.5, seed, weights=False)
    rng = np.random.default_rng(seed)
    w = [np.clip(rng.uniform(-0.2, 1.2, size=s.views[0].shape), 0, 1).astype(np.float32) for _ in range(4)]
    return s.views, s.psfs, w


def tiles_of(mvd, lens, exact_len):
    """The first candidate of each pass kind with the given exact_len field:
    0 = runtime plan (any length), -1 = the per-length compile-time plans."""
    out = []
    for kind in range(3):
        for c in mvd.tile_candidates(kind, lens[kind]):
            if mvd.tile_shape(kind, c)["exact_len"] == exact_len:
                out.append(c)
                break
    return out


@pytest.mark.parametrize("mode", [0, -1])
@pytest.mark.parametrize("variant", [O.RL, O.EFF])
def test_batched_equals_plain_per_block(mvd, variant, mode):
    """With the same kind of plan on both sides (runtime plans, or the
    compile-time plan of each length launched per group of equal length) the
    batched form gives every block's plain result bitwise."""
    blocks = [block(d, 100 + i) for i, d in enumerate(DIMS)]
    with mvd.Deconvolver.batch(blocks, lam=0.01) as b:
        b.set_tiles(*tiles_of(mvd, b.max_lengths(), mode))
        b.iterate(3, variant)
        got = [b.estimate(i).cpu().numpy() for i in range(len(DIMS))]
        st = b.stats()
    assert st["n_blocks"] == len(DIMS) and not st["nonfinite"]
    for i, (v, p, w) in enumerate(blocks):
        with mvd.Deconvolver(v, p, w, lam=0.01) as d:
            d.set_tiles(*tiles_of(mvd, d.max_lengths(), mode))
            d.iterate(3, variant)
            ref = d.estimate().cpu().numpy()
        # same per-line arithmetic (the same plans of the same lengths): bitwise
        np.testing.assert_array_equal(got[i], ref)


def test_batched_matches_oracle(mvd):
    blocks = [block(d, 200 + i) for i, d in enumerate(DIMS[:4])]
    with mvd.Deconvolver.batch(blocks) as b:
        b.iterate(2, O.OPT1)
        got = [b.estimate(i).cpu().numpy() for i in range(4)]
    for i, (v, p, w) in enumerate(blocks):
        ref = O.run(v, p, 2, O.OPT1, weights=w)
        e = O.rel_l2(got[i], ref)
        print(f"block {i} {DIMS[i]}: rel_l2={e:.3e}")
        assert e <= 1e-5


def test_batched_every_launch_shape(mvd):
    """Every runtime-plan shape of every kind, on blocks of unequal lengths,
    gives the same result bitwise (the same radix plans of the same lengths)."""
    blocks = [block(d, 300 + i) for i, d in enumerate(DIMS[:3])]
    with mvd.Deconvolver.batch(blocks) as b:
        base = tiles_of(mvd, b.max_lengths(), 0)
        b.set_tiles(*base)
        b.iterate(1, O.EFF)
        ref = [b.estimate(i).cpu().numpy() for i in range(3)]
        psi1 = [r.copy() for r in ref]
        b.iterate(1, O.EFF)
        ref2 = [b.estimate(i).cpu().numpy() for i in range(3)]
        lens = b.max_lengths()
        for kind in range(3):
            for c in mvd.tile_candidates(kind, lens[kind]):
                if mvd.tile_shape(kind, c)["exact_len"]:
                    continue
                cfg = list(base)
                cfg[kind] = c
                b.set_tiles(*cfg)
                for i in range(3):
                    b.set_estimate(psi1[i], block=i)
                b.iterate(1, O.EFF)
                for i in range(3):
                    np.testing.assert_array_equal(b.estimate(i).cpu().numpy(), ref2[i])


def test_autotune_restores_estimates(mvd):
    """The autotuner runs passes and whole iterations on the handle; every
    block's estimate is as before afterwards, and the chosen shapes are set."""
    from paper_1308_0730_amd import tune
    blocks = [block(d, 400 + i) for i, d in enumerate(DIMS[:4])]
    with mvd.Deconvolver.batch(blocks) as b:
        b.iterate(1, O.EFF)
        before = [b.estimate(i).cpu().numpy() for i in range(4)]
        tiles, _ = tune.autotune(b, "eff", iters=1, cache_path=None)
        assert tuple(b.tiles()) == tuple(tiles)
        for i in range(4):
            np.testing.assert_array_equal(b.estimate(i).cpu().numpy(), before[i])


def test_batched_repeated_sizes_over_lanes(mvd):
    """Blocks of repeated and different sizes (equal lengths on several
    stream lanes, several lengths in one length class, and the column
    passes' class launches beside per-length row launches) give every
    block's plain result bitwise."""
    dims = [(40, 36, 30), (40, 36, 30), (64, 64, 48), (40, 36, 30), (48, 40, 36), (64, 64, 48), (20, 18, 16)]
    blocks = [block(d, 500 + i) for i, d in enumerate(dims)]
    with mvd.Deconvolver.batch(blocks, lam=0.01) as b:
        b.set_tiles(*tiles_of(mvd, b.max_lengths(), -1))
        b.iterate(2, O.OPT1)
        got = [b.estimate(i).cpu().numpy() for i in range(len(dims))]
    for i, (v, p, w) in enumerate(blocks):
        with mvd.Deconvolver(v, p, w, lam=0.01) as d:
            d.set_tiles(*tiles_of(mvd, d.max_lengths(), -1))
            d.iterate(2, O.OPT1)
            np.testing.assert_array_equal(got[i], d.estimate().cpu().numpy())


def test_batched_columns_above_512(mvd):
    """Blocks with y lengths above 512 (their own length class, 8-line
    tiles) beside ordinary ones give every block's plain result bitwise."""
    dims = [(16, 720, 10), (16, 1000, 12), (20, 36, 30), (16, 720, 10)]
    blocks = [block(d, 600 + i) for i, d in enumerate(dims)]
    with mvd.Deconvolver.batch(blocks) as b:
        b.set_tiles(*tiles_of(mvd, b.max_lengths(), -1))
        b.iterate(2, O.EFF)
        got = [b.estimate(i).cpu().numpy() for i in range(len(dims))]
    for i, (v, p, w) in enumerate(blocks):
        with mvd.Deconvolver(v, p, w) as d:
            d.set_tiles(*tiles_of(mvd, d.max_lengths(), -1))
            d.iterate(2, O.EFF)
            np.testing.assert_array_equal(got[i], d.estimate().cpu().numpy())



@pytest.mark.parametrize("graphs", [True, False])
def test_schedules_give_the_same_results(mvd, graphs):
    """Pass-major, block-major and run-major schedules (blocks on several
    lanes, repeated and different sizes) give the same estimates bitwise,
    over runs of one and of three iterations, with and without graphs; the
    flux statistics of the last iteration agree too."""
    dims = [(40, 36, 30), (48, 40, 36), (40, 36, 30), (64, 64, 48), (20, 18, 16), (32, 32, 32)]
    blocks = [block(d, 700 + i) for i, d in enumerate(dims)]
    out = {}
    with mvd.Deconvolver.batch(blocks, lam=0.01, use_graphs=graphs) as b:
        b.set_tiles(*tiles_of(mvd, b.max_lengths(), -1))
        start = [b.estimate(i).clone() for i in range(len(dims))]
        for sch in ("pass", "block", "run"):
            b.set_schedule(sch)
            assert b.schedule() == sch
            for i in range(len(dims)):
                b.set_estimate(start[i], block=i)
            b.iterate(1, O.OPT1)
            b.iterate(3, O.OPT1)
            out[sch] = ([b.estimate(i).cpu().numpy() for i in range(len(dims))], b.stats()["flux"])
    for sch in ("block", "run"):
        for a, r in zip(out[sch][0], out["pass"][0]):
            np.testing.assert_array_equal(a, r)
        np.testing.assert_allclose(out[sch][1], out["pass"][1], rtol=1e-12)


def test_shuffled_blocks_and_schedules_give_the_same_blocks(mvd):
    """Scheduler stress: 20 blocks of mixed dims (repeated dims share a lane
    and a launch; up to sixteen stream lanes), handed over in three seeded
    random orders and run under every schedule with the per-length plans:
    every block's estimate is bitwise the same as in the first order."""
    dims = [DIMS[i % len(DIMS)] for i in range(20)]
    blocks = [block(d, 300 + i) for i, d in enumerate(dims)]
    rng = np.random.default_rng(311)
    ref = None
    for trial in range(3):
        order = list(range(len(blocks))) if trial == 0 else list(rng.permutation(len(blocks)))
        with mvd.Deconvolver.batch([blocks[i] for i in order], lam=0.01) as b:
            b.set_tiles(*tiles_of(mvd, b.max_lengths(), -1))
            for sch in ("pass", "block", "run"):
                b.set_schedule(sch)
                for j, i in enumerate(order):
                    b.set_estimate(np.full(blocks[i][0][0].shape, 3.0, np.float32), j)
                b.iterate(2, O.EFF)
                got = {i: b.estimate(j).cpu().numpy() for j, i in enumerate(order)}
                if ref is None:
                    ref = got
                    continue
                for i in range(len(blocks)):
                    np.testing.assert_array_equal(got[i], ref[i], err_msg=f"trial {trial} schedule {sch} block {i}")
