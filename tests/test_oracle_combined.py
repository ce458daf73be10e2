"""Pins of the oracle's combined updates (eq. 51, geometric and arithmetic
means) against facts that do not depend on the oracle's own code: the
explicit-matrix ML-EM iteration of Shepp and Vardi on stacked data, closed
forms for delta kernels, the reduction to single-view RL, the fixed point,
the flux identity of ML-EM, the AM-GM order of the two means, and the ML-EM
likelihood property."""
import numpy as np
import pytest

from oracle import mvd_oracle as O
from tests.test_oracle_pins import conv_matrix, rand_kernel, rand_volume


def test_arithmetic_rl_is_explicit_matrix_mlem():
    """With the mirrored PSFs and the arithmetic mean, a combined update is
    Shepp-Vardi EM on the stacked system [A_1; ...; A_N]:
    psi <- psi . sum_v A_v^T (phi_v / A_v psi) / sum_v A_v^T 1."""
    rng = np.random.default_rng(21)
    shape = (4, 5, 6)
    psfs = [rand_kernel(rng, (3, 3, 3), offset=(0.4, -0.3, 0.2)),
            rand_kernel(rng, (3, 5, 3), offset=(-0.5, 0.6, 0.1)),
            rand_kernel(rng, (5, 3, 3), offset=(0.2, 0.0, -0.6))]
    truth = rand_volume(rng, shape, 1.0, 20.0)
    views = [O.circ_conv(truth, O.prepare_psf(p)) * rng.uniform(0.9, 1.1, size=shape) for p in psfs]
    pb = O.Problem(views, psfs)
    got = pb.iterate_combined(pb.psi0(), 3, O.RL, O.ARITHMETIC)
    A = [conv_matrix(O.prepare_psf(p), shape) for p in psfs]
    x = pb.psi0().ravel().copy()
    ones = np.ones_like(x)
    for _ in range(3):
        num = sum(Av.T @ (phi.ravel() / (Av @ x)) for Av, phi in zip(A, views))
        den = sum(Av.T @ ones for Av in A)
        x = x * num / den
    np.testing.assert_allclose(got.ravel(), x, rtol=1e-11)


def test_geometric_rl_with_explicit_matrices():
    """The geometric mean of eq. 51 written with explicit matrices:
    psi <- psi . (prod_v A_v^T (phi_v / A_v psi))^(1/N)."""
    rng = np.random.default_rng(22)
    shape = (4, 5, 6)
    psfs = [rand_kernel(rng, (3, 3, 3), offset=(0.4, -0.3, 0.2)),
            rand_kernel(rng, (5, 3, 3), offset=(0.2, 0.0, -0.6))]
    truth = rand_volume(rng, shape, 1.0, 20.0)
    views = [O.circ_conv(truth, O.prepare_psf(p)) * rng.uniform(0.9, 1.1, size=shape) for p in psfs]
    pb = O.Problem(views, psfs)
    got = pb.iterate_combined(pb.psi0(), 2, O.RL, O.GEOMETRIC)
    A = [conv_matrix(O.prepare_psf(p), shape) for p in psfs]
    x = pb.psi0().ravel().copy()
    for _ in range(2):
        prod = np.ones_like(x)
        for Av, phi in zip(A, views):
            prod = prod * (Av.T @ (phi.ravel() / (Av @ x)))
        x = x * prod ** 0.5
    np.testing.assert_allclose(got.ravel(), x, rtol=1e-11)


@pytest.mark.parametrize("variant", [O.RL, O.EFF, O.OPT1, O.OPT2])
def test_delta_kernels_give_the_means_of_the_views(variant):
    """With delta PSFs every blur is the identity, so one combined update maps
    any psi to the geometric (eq. 51 with the |V|-th root) or arithmetic mean
    of the views, voxel by voxel."""
    rng = np.random.default_rng(23)
    shape = (5, 6, 7)
    views = [rand_volume(rng, shape, 1.0, 30.0) for _ in range(3)]
    d = np.ones((1, 1, 1))
    pb = O.Problem(views, [d, d, d])
    psi = rand_volume(rng, shape, 2.0, 9.0)
    g = pb.iterate_combined(psi, 1, variant, O.GEOMETRIC)
    a = pb.iterate_combined(psi, 1, variant, O.ARITHMETIC)
    np.testing.assert_allclose(g, np.cbrt(views[0] * views[1] * views[2]), rtol=1e-13)
    np.testing.assert_allclose(a, (views[0] + views[1] + views[2]) / 3.0, rtol=1e-13)


@pytest.mark.parametrize("mean", [O.GEOMETRIC, O.ARITHMETIC])
@pytest.mark.parametrize("variant", [O.RL, O.EFF, O.OPT1])
def test_one_view_reduces_to_the_sequential_step(mean, variant):
    """N = 1: both means of one factor are that factor, so a combined update
    is the single-view step (lambda included)."""
    rng = np.random.default_rng(24)
    shape = (8, 10, 12)
    P = rand_kernel(rng, (5, 3, 3), offset=(0.3, -0.2, 0.4))
    phi = rng.poisson(10.0, size=shape).astype(float) + 0.5
    pb = O.Problem([phi], [P], lam=0.02)
    psi = pb.psi0()
    np.testing.assert_allclose(pb.iterate_combined(psi, 2, variant, mean), pb.iterate(psi, 2, variant), rtol=1e-13)


@pytest.mark.parametrize("mean", [O.GEOMETRIC, O.ARITHMETIC])
def test_identical_views_equal_single_view_rl(mean):
    """N identical views with identical PSFs: every factor is the same, so
    one combined update equals one single-view RL step."""
    rng = np.random.default_rng(25)
    shape = (8, 10, 12)
    P = rand_kernel(rng, (3, 5, 3), offset=(0.3, -0.2, 0.4))
    phi = rng.poisson(10.0, size=shape).astype(float) + 0.5
    multi = O.Problem([phi] * 4, [P] * 4).iterate_combined(O.Problem([phi], [P]).psi0(), 2, O.RL, mean)
    single = O.run([phi], [P], 2, O.RL)
    np.testing.assert_allclose(multi, single, rtol=1e-12)


@pytest.mark.parametrize("mean", [O.GEOMETRIC, O.ARITHMETIC])
@pytest.mark.parametrize("variant", [O.RL, O.EFF, O.OPT1, O.OPT2])
def test_combined_fixed_point(mean, variant):
    """Noise-free views and psi = psi*: every factor is one (normalised
    kernels), so psi is unchanged."""
    rng = np.random.default_rng(26)
    shape = (8, 10, 12)
    psfs = [rand_kernel(rng, (3, 5, 3), offset=(0.3, 0.4, -0.2)), rand_kernel(rng, (5, 3, 5), offset=(-0.4, 0, 0.5)),
            rand_kernel(rng, (3, 3, 5))]
    truth = rand_volume(rng, shape)
    views = [O.circ_conv(truth, O.prepare_psf(p)) for p in psfs]
    got = O.Problem(views, psfs).iterate_combined(truth, 2, variant, mean)
    np.testing.assert_allclose(got, truth, rtol=1e-11)


def test_arithmetic_rl_flux_is_mean_view_flux():
    """ML-EM identity: with mirrored normalised PSFs and lambda = 0,
    sum psi' = (1/N) sum_v sum_x psi (q_v x P_v*) = (1/N) sum_v sum phi_v."""
    rng = np.random.default_rng(27)
    shape = (8, 10, 12)
    psfs = [rand_kernel(rng, (3, 5, 3), offset=(0.3, 0.4, -0.2)), rand_kernel(rng, (5, 3, 5)),
            rand_kernel(rng, (3, 3, 3), offset=(0, -0.5, 0.3))]
    views = [rng.poisson(20.0, size=shape).astype(float) + 1 for _ in psfs]
    flux = []
    pb = O.Problem(views, psfs)
    pb.iterate_combined(pb.psi0(), 3, O.RL, O.ARITHMETIC, flux=flux)
    target = np.mean([v.sum() for v in views])
    for f in flux:
        assert abs(f - target) < 1e-10 * target


def test_geometric_never_exceeds_arithmetic():
    """AM-GM: from the same psi (lambda = 0) the geometric update is at most
    the arithmetic one at every voxel, with equality only where the factors
    agree."""
    rng = np.random.default_rng(28)
    shape = (8, 10, 12)
    psfs = [rand_kernel(rng, (3, 5, 3), offset=(0.3, 0.4, -0.2)), rand_kernel(rng, (5, 3, 5))]
    views = [rng.poisson(15.0, size=shape).astype(float) + 1 for _ in psfs]
    pb = O.Problem(views, psfs)
    psi = rand_volume(rng, shape, 5.0, 25.0)
    g = pb.iterate_combined(psi, 1, O.EFF, O.GEOMETRIC)
    a = pb.iterate_combined(psi, 1, O.EFF, O.ARITHMETIC)
    assert np.all(g <= a * (1 + 1e-14))
    assert np.mean(a - g) > 0


def test_arithmetic_rl_likelihood_monotone():
    """ML-EM on Poisson data: the summed log-likelihood over all views,
    sum_v sum(phi_v log b_v - b_v), b_v = psi x P_v, never decreases."""
    rng = np.random.default_rng(29)
    shape = (8, 10, 12)
    psfs = [rand_kernel(rng, (5, 3, 5), offset=(0.3, 0.1, -0.4)), rand_kernel(rng, (3, 5, 3))]
    truth = rand_volume(rng, shape, 1, 50)
    views = [rng.poisson(O.circ_conv(truth, O.prepare_psf(p))).astype(float) for p in psfs]
    pb = O.Problem(views, psfs)
    psi = pb.psi0()
    prev = -np.inf
    for _ in range(12):
        ll = sum(float(np.sum(phi * np.log(O.circ_conv(psi, P)) - O.circ_conv(psi, P))) for phi, P in zip(views, pb.P))
        assert ll >= prev - 1e-9 * abs(ll)
        prev = ll
        psi = pb.iterate_combined(psi, 1, O.RL, O.ARITHMETIC)


def test_combined_rejects_weights():
    rng = np.random.default_rng(30)
    shape = (4, 5, 6)
    v = [rand_volume(rng, shape)]
    pb = O.Problem(v, [np.ones((1, 1, 1))], [np.ones(shape)])
    with pytest.raises(ValueError):
        pb.iterate_combined(pb.psi0(), 1, O.RL)
