"""Pins of the oracle's gradient of the unrolled sequential RL run:
adjoint dot-product identities of its building blocks and central finite
differences of the loss in psi^0 and in the raw PSF values."""
import numpy as np
import pytest

from oracle import mvd_oracle as O


def rand_kernel(rng, shape, off):
    kz, ky, kx = shape
    z, y, x = np.meshgrid(np.arange(kz) - (kz - 1) / 2, np.arange(ky) - (ky - 1) / 2,
                          np.arange(kx) - (kx - 1) / 2, indexing="ij")
    g = np.exp(-0.5 * ((x - off[2]) ** 2 / 1.4 + (y - off[1]) ** 2 / 0.9 + (z - off[0]) ** 2 / 2.2))
    return g + 0.05 * rng.uniform(size=shape)


def test_convolution_adjoint_identity():
    """<f (x) K, g> = <f, g (x) K*>  and  <f (x) K, g> = <K, corr(g, f)>."""
    rng = np.random.default_rng(1)
    f = rng.normal(size=(8, 10, 12))
    g = rng.normal(size=(8, 10, 12))
    K = rng.normal(size=(3, 5, 3))
    lhs = np.sum(O.circ_conv(f, K) * g)
    assert abs(lhs - np.sum(f * O.circ_conv(g, O.mirror(K)))) < 1e-10 * abs(lhs)
    assert abs(lhs - np.sum(K * O.circ_corr_window(g, f, K.shape))) < 1e-10 * abs(lhs)


def small_case(rng, weights, lam):
    shape = (6, 8, 10)
    psfs = [rand_kernel(rng, (3, 5, 3), (0.4, -0.3, 0.2)), rand_kernel(rng, (5, 3, 4), (-0.2, 0.5, 0.1)),
            rand_kernel(rng, (3, 3, 5), (0.1, 0.2, -0.4))]
    truth = rng.uniform(2, 20, size=shape)
    views = [np.maximum(O.circ_conv(truth, O.prepare_psf(p)) + rng.normal(0, 0.3, size=shape), 0.1)
             for p in psfs]
    w = [rng.uniform(0.2, 1, size=shape) for _ in psfs] if weights else None
    psi0 = rng.uniform(5, 10, size=shape)
    return views, psfs, w, psi0


@pytest.mark.parametrize("weights,lam", [(False, 0.0), (True, 0.05)])
def test_gradient_matches_finite_differences(weights, lam):
    rng = np.random.default_rng(2)
    views, psfs, w, psi0 = small_case(rng, weights, lam)
    n = 2
    L, gpsi, gP = O.loss_and_grad(views, psfs, n, psi0, w, lam)
    assert abs(L - O.loss_of(views, psfs, n, psi0, w, lam)) < 1e-10 * L
    # psi0 along a random direction
    d = rng.normal(size=psi0.shape)
    h = 1e-4
    fd = (O.loss_of(views, psfs, n, psi0 + h * d, w, lam) - O.loss_of(views, psfs, n, psi0 - h * d, w, lam)) / (2 * h)
    an = float(np.sum(gpsi * d))
    assert abs(fd - an) < 1e-6 * max(abs(an), 1e-3 * L), (fd, an)
    # every PSF along a random direction, and single entries
    for v in range(3):
        dP = rng.normal(size=psfs[v].shape)
        hp = 1e-5 * psfs[v].max()
        p1 = [p.copy() for p in psfs]
        p2 = [p.copy() for p in psfs]
        p1[v] = p1[v] + hp * dP
        p2[v] = p2[v] - hp * dP
        fd = (O.loss_of(views, p1, n, psi0, w, lam) - O.loss_of(views, p2, n, psi0, w, lam)) / (2 * hp)
        an = float(np.sum(gP[v] * dP))
        assert abs(fd - an) < 1e-5 * max(abs(an), 1e-3 * L), (v, fd, an)
