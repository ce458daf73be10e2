"""Pins of the linear-boundary oracle: EM with explicit restricted system
matrices, the fixed point, the sensitivity-weighted flux identity of EM,
delta kernels, and the margin's bookkeeping."""
import numpy as np
import pytest

from oracle import mvd_oracle as O
from tests.test_oracle_pins import rand_kernel, rand_volume


def restricted_matrix(P, n, p):
    """A: psi on the extended domain (n + 2p) -> (psi * P) on the volume, as
    an explicit matrix built from the definition b(x) = sum_d P[c+d] psi(x-d)."""
    ne = tuple(n[a] + 2 * p[a] for a in range(3))
    A = np.zeros((int(np.prod(n)), int(np.prod(ne))))
    K = np.asarray(P, np.float64)
    c = [(k - 1) // 2 for k in K.shape]
    for z in range(n[0]):
        for y in range(n[1]):
            for x in range(n[2]):
                row = (z * n[1] + y) * n[2] + x
                for a in range(K.shape[0]):
                    for b in range(K.shape[1]):
                        for e in range(K.shape[2]):
                            d = (a - c[0], b - c[1], e - c[2])
                            ze, ye, xe = z - d[0] + p[0], y - d[1] + p[1], x - d[2] + p[2]
                            A[row, (ze * ne[1] + ye) * ne[2] + xe] += K[a, b, e]
    return A


def test_rl_equals_restricted_matrix_em():
    rng = np.random.default_rng(41)
    n = (4, 5, 6)
    psfs = [rand_kernel(rng, (3, 3, 3), offset=(0.4, -0.3, 0.2)), rand_kernel(rng, (3, 5, 3), offset=(-0.5, 0.6, 0.1))]
    views = [rand_volume(rng, n, 1.0, 20.0) for _ in psfs]
    pb = O.ProblemLinear(views, psfs)
    got = pb.iterate(pb.psi0(), 2, O.RL)
    A = [restricted_matrix(P, n, pb.p) for P in pb.P]
    x = pb.psi0().ravel().copy()
    for _ in range(2):
        for Av, phi in zip(A, views):
            sens = Av.T @ np.ones(Av.shape[0])
            x = np.where(sens >= O.SENS_MIN, x * (Av.T @ (phi.ravel() / (Av @ x))) / np.maximum(sens, 1e-300), x)
    np.testing.assert_allclose(got.ravel(), x, rtol=1e-10)


@pytest.mark.parametrize("variant", [O.RL, O.EFF, O.OPT1, O.OPT2])
def test_linear_fixed_point(variant):
    """Views that are exactly the restricted blur of psi*: every variant keeps
    psi* (the back-projection of ones is the sensitivity)."""
    rng = np.random.default_rng(42)
    n = (6, 7, 8)
    psfs = [rand_kernel(rng, (3, 5, 3), offset=(0.3, 0.4, -0.2)), rand_kernel(rng, (5, 3, 3))]
    pb0 = O.ProblemLinear([np.ones(n)] * 2, psfs)
    truth = rand_volume(rng, pb0.shape_e, 1.0, 9.0)
    views = [O.lin_blur(truth, P, pb0.p) for P in pb0.P]
    pb = O.ProblemLinear(views, psfs)
    np.testing.assert_allclose(pb.iterate(truth, 2, variant), truth, rtol=1e-11)


def test_sensitivity_weighted_flux():
    """EM identity: after an RL view-update sum_xi N(xi) psi'(xi) = sum phi
    (every voxel live, lambda 0, no weights)."""
    rng = np.random.default_rng(43)
    n = (6, 7, 8)
    P = rand_kernel(rng, (3, 3, 3), offset=(0.3, -0.2, 0.1)) + 0.05  # no tiny tails: every margin voxel live
    phi = rng.poisson(20.0, size=n).astype(float) + 1
    pb = O.ProblemLinear([phi], [P])
    psi = pb.iterate(pb.psi0(), 1, O.RL)
    N = O.lin_back(np.ones(n), pb.kernels(O.RL)[0], pb.p)  # A^T 1: the back-projection kernel P*
    assert np.all(N >= O.SENS_MIN)
    assert abs(float(np.sum(N * psi)) - phi.sum()) < 1e-10 * phi.sum()


def test_delta_kernel_returns_the_view():
    rng = np.random.default_rng(44)
    phi = rand_volume(rng, (5, 6, 7), 1.0, 9.0)
    pb = O.ProblemLinear([phi], [np.ones((1, 1, 1))])
    assert pb.p == (0, 0, 0)
    np.testing.assert_allclose(pb.iterate(pb.psi0(), 1, O.RL), phi, rtol=1e-13)


def test_margin_weights_and_interior():
    rng = np.random.default_rng(45)
    n = (4, 5, 6)
    psfs = [rand_kernel(rng, (3, 3, 5))]
    w = [rng.uniform(0, 1, size=n)]
    pb = O.ProblemLinear([rand_volume(rng, n)], psfs, w)
    assert pb.shape_e == (6, 7, 10)
    we = pb.weights_e[0]
    np.testing.assert_array_equal(pb.interior(we), w[0])
    assert we.sum() - w[0].sum() == pytest.approx(we.size - w[0].size)
