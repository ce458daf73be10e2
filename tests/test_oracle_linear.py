"""Pins of the linear-boundary oracle.

The oracle takes the neutral ratio (q = 1 where a view has no data) and
back-projects it over the extended domain.  These tests check it against a
different formulation built from explicit matrices: the restricted-matrix EM
step psi K^T q / N taken as the fraction N of a full step (N = K^T 1, the
voxel's sensitivity), plus the fixed point, a flux identity, delta kernels
and the margin's bookkeeping.  No test uses a threshold on N."""
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


def weighted_em_step(x, A, B, phi, w=None, lam_p=0.0):
    """Restricted-matrix EM with back-projector B (B = A^T for RL), applied as
    the fraction N = B 1 of a full step, then Tikhonov and the user weight:
    t = T(x + N (x B q / N - x)), x <- x + w (t - x).  Voxels with N = 0 keep
    their value (their fraction is zero)."""
    q = phi.ravel() / (A @ x)
    N = B @ np.ones(B.shape[1])
    full = np.divide(x * (B @ q), N, out=np.zeros_like(x), where=N > 0)
    step = x + N * (full - x)
    t = step if lam_p == 0.0 else 2 * step / (1 + np.sqrt(1 + 4 * lam_p * step))
    return t if w is None else x + w * (t - x)


@pytest.mark.parametrize("variant", [O.RL, O.EFF, O.OPT1, O.OPT2])
def test_matches_sensitivity_weighted_restricted_em(variant):
    """Two views, two iterations, every variant: the oracle equals the
    explicit-matrix step.  The back-projector of view v is the matrix of the
    mirrored K_v (c(xi) = sum_x K[c + xi - x] q(x)); for RL that is A_v^T."""
    rng = np.random.default_rng(41)
    n = (4, 5, 6)
    psfs = [rand_kernel(rng, (3, 3, 3), offset=(0.4, -0.3, 0.2)), rand_kernel(rng, (3, 5, 3), offset=(-0.5, 0.6, 0.1))]
    views = [rand_volume(rng, n, 1.0, 20.0) for _ in psfs]
    pb = O.ProblemLinear(views, psfs)
    got = pb.iterate(pb.psi0(), 2, variant)
    A = [restricted_matrix(P, n, pb.p) for P in pb.P]
    B = [restricted_matrix(O.mirror(K), n, pb.p).T for K in pb.kernels(variant)]
    if variant == O.RL:
        for a, b in zip(A, B):
            np.testing.assert_allclose(b, a.T, rtol=0, atol=1e-15)
    x = pb.psi0().ravel().copy()
    for _ in range(2):
        for a, b, phi in zip(A, B, views):
            x = weighted_em_step(x, a, b, phi)
    np.testing.assert_allclose(got.ravel(), x, rtol=1e-11)


def test_weights_and_tikhonov_apply_after_the_weighted_step():
    rng = np.random.default_rng(46)
    n = (4, 5, 6)
    psfs = [rand_kernel(rng, (3, 3, 5), offset=(0.2, 0.1, -0.4)), rand_kernel(rng, (5, 3, 3))]
    views = [rand_volume(rng, n, 1.0, 20.0) for _ in psfs]
    w = [rng.uniform(0.1, 0.9, size=n) for _ in psfs]
    pb = O.ProblemLinear(views, psfs, w, lam=0.3)
    got = pb.iterate(pb.psi0(), 1, O.OPT1)
    A = [restricted_matrix(P, n, pb.p) for P in pb.P]
    B = [restricted_matrix(O.mirror(K), n, pb.p).T for K in pb.kernels(O.OPT1)]
    x = pb.psi0().ravel().copy()
    for v in range(2):
        x = weighted_em_step(x, A[v], B[v], views[v], pb.weights_e[v].ravel(), pb.lam_p)
    np.testing.assert_allclose(got.ravel(), x, rtol=1e-11)


@pytest.mark.parametrize("variant", [O.RL, O.EFF, O.OPT1, O.OPT2])
def test_linear_fixed_point(variant):
    """Views that are exactly the restricted blur of psi*: every variant keeps
    psi* (the ratio is one on the volume and, by definition, outside it)."""
    rng = np.random.default_rng(42)
    n = (6, 7, 8)
    psfs = [rand_kernel(rng, (3, 5, 3), offset=(0.3, 0.4, -0.2)), rand_kernel(rng, (5, 3, 3))]
    pb0 = O.ProblemLinear([np.ones(n)] * 2, psfs)
    truth = rand_volume(rng, pb0.shape_e, 1.0, 9.0)
    A = [restricted_matrix(P, n, pb0.p) for P in pb0.P]
    views = [(a @ truth.ravel()).reshape(n) for a in A]
    pb = O.ProblemLinear(views, psfs)
    np.testing.assert_allclose(pb.iterate(truth, 2, variant), truth, rtol=1e-11)


def test_flux_identity():
    """RL, lambda 0, no weights, no clamps: sum psi' = sum psi + sum phi -
    sum b (sum_xi psi (1 - N + A^T q) with sum_xi psi A^T q = sum_x q b = sum phi
    and sum_xi psi N = sum_x b), with b from the explicit matrix."""
    rng = np.random.default_rng(43)
    n = (6, 7, 8)
    P = rand_kernel(rng, (3, 3, 5), offset=(0.3, -0.2, 0.1))
    phi = rng.poisson(20.0, size=n).astype(float) + 1
    pb = O.ProblemLinear([phi], [P])
    psi = rand_volume(rng, pb.shape_e, 2.0, 30.0)
    stats = {}
    out = pb.iterate(psi, 1, O.RL, stats=stats)
    assert stats["ratio_clamps"] == 0 and stats["neg_clamps"] == 0
    b = restricted_matrix(pb.P[0], n, pb.p) @ psi.ravel()
    assert abs(out.sum() - (psi.sum() + phi.sum() - b.sum())) < 1e-11 * phi.sum()


def test_sensitivity_is_one_inside_and_falls_off_in_the_margin():
    rng = np.random.default_rng(47)
    n = (6, 7, 8)
    P = O.prepare_psf(rand_kernel(rng, (3, 5, 3)))
    pb = O.ProblemLinear([np.ones(n)], [P])
    N = O.sensitivity(n, O.mirror(P), pb.p)
    A = restricted_matrix(P, n, pb.p)
    np.testing.assert_allclose(N.ravel(), A.T @ np.ones(A.shape[0]), atol=1e-14)
    np.testing.assert_allclose(pb.interior(N)[1:-1, 2:-2, 1:-1], 1.0, atol=1e-14)
    assert N.min() >= -1e-15 and N.max() <= 1 + 1e-14


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


def test_mistakes_in_the_update_fail_the_matrix_pin():
    """A ratio of zero outside the volume, or the restricted-EM step taken in
    full, both differ from the oracle: the matrix pin tells them apart."""
    rng = np.random.default_rng(48)
    n = (4, 5, 6)
    psfs = [rand_kernel(rng, (3, 3, 3), offset=(0.4, -0.3, 0.2))]
    views = [rand_volume(rng, n, 1.0, 20.0)]
    pb = O.ProblemLinear(views, psfs)
    got = pb.iterate(pb.psi0(), 1, O.RL).ravel()
    A = restricted_matrix(pb.P[0], n, pb.p)
    x = pb.psi0().ravel()
    q = views[0].ravel() / (A @ x)
    zero_outside = x * (A.T @ q)
    N = A.T @ np.ones(A.shape[0])
    full_step = x * (A.T @ q) / N
    for wrong in (zero_outside, full_step):
        assert np.max(np.abs(wrong - got) / got) > 1e-3
