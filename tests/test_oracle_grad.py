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


def _psi_n(views, psfs, n, psi0, w, lam):
    pb = O.Problem(views, psfs, w, lam)
    return pb.iterate(np.asarray(psi0, np.float64), n, O.RL)


@pytest.mark.parametrize("weights,lam", [(False, 0.0), (True, 0.05)])
def test_vjp_matches_finite_differences(weights, lam):
    """The vector-Jacobian product against central differences of
    <gbar, psi_n> computed with the forward iteration alone."""
    rng = np.random.default_rng(3)
    views, psfs, w, psi0 = small_case(rng, weights, lam)
    n = 2
    gbar = rng.normal(size=psi0.shape)
    psi_n, gpsi, gP = O.vjp(views, psfs, n, psi0, gbar, w, lam)
    assert O.rel_l2(psi_n, _psi_n(views, psfs, n, psi0, w, lam)) < 1e-13

    def f(p, s0):
        return float(np.sum(gbar * _psi_n(views, p, n, s0, w, lam)))

    d = rng.normal(size=psi0.shape)
    h = 1e-4
    fd = (f(psfs, psi0 + h * d) - f(psfs, psi0 - h * d)) / (2 * h)
    an = float(np.sum(gpsi * d))
    assert abs(fd - an) < 1e-6 * max(abs(an), 1.0), (fd, an)
    for v in range(3):
        dP = rng.normal(size=psfs[v].shape)
        hp = 1e-5 * psfs[v].max()
        p1 = [p.copy() for p in psfs]
        p2 = [p.copy() for p in psfs]
        p1[v] = p1[v] + hp * dP
        p2[v] = p2[v] - hp * dP
        fd = (f(p1, psi0) - f(p2, psi0)) / (2 * hp)
        an = float(np.sum(gP[v] * dP))
        assert abs(fd - an) < 1e-5 * max(abs(an), 1.0), (v, fd, an)


def test_vjp_is_linear_and_zero_seed_gives_zero():
    rng = np.random.default_rng(4)
    views, psfs, w, psi0 = small_case(rng, True, 0.05)
    g1 = rng.normal(size=psi0.shape)
    g2 = rng.normal(size=psi0.shape)
    _, a1, b1 = O.vjp(views, psfs, 2, psi0, g1, w, 0.05)
    _, a2, b2 = O.vjp(views, psfs, 2, psi0, g2, w, 0.05)
    _, a3, b3 = O.vjp(views, psfs, 2, psi0, 2.0 * g1 - 3.0 * g2, w, 0.05)
    assert O.rel_l2(a3, 2.0 * a1 - 3.0 * a2) < 1e-12
    for x, y, z in zip(b1, b2, b3):
        assert O.rel_l2(z, 2.0 * x - 3.0 * y) < 1e-12
    _, a0, b0 = O.vjp(views, psfs, 2, psi0, np.zeros_like(g1), w, 0.05)
    assert not a0.any() and not any(x.any() for x in b0)


@pytest.mark.parametrize("variant", [O.EFF, O.OPT1, O.OPT2])
def test_compound_kernel_vjp_matches_finite_differences(variant):
    """<Kbar, K_v(G)> for raw PSFs G of odd and even extents: the
    construction's adjoint (then the normalisation of eq. 3) against central
    differences along random directions, for every view's kernel and every
    PSF it depends on."""
    rng = np.random.default_rng(11)
    psfs = [rand_kernel(rng, (3, 5, 3), (0.4, -0.3, 0.2)), rand_kernel(rng, (5, 3, 4), (-0.2, 0.5, 0.1)),
            rand_kernel(rng, (3, 3, 5), (0.1, 0.2, -0.4))]
    P = [O.prepare_psf(p) for p in psfs]
    for v in range(3):
        Kbar = rng.normal(size=P[v].shape)
        gP = O.compound_kernel_vjp(P, v, variant, Kbar)

        def f(ps):
            return float(np.sum(Kbar * O.compound_kernel(ps, v, variant)))

        for w in range(3):
            G = psfs[w]
            gG = ((gP[w] - np.sum(gP[w] * P[w])) / G.sum())[:G.shape[0], :G.shape[1], :G.shape[2]]
            d = rng.normal(size=G.shape)
            h = 1e-6 * G.max()
            p1 = [p.copy() for p in psfs]
            p2 = [p.copy() for p in psfs]
            p1[w] = p1[w] + h * d
            p2[w] = p2[w] - h * d
            fd = (f(p1) - f(p2)) / (2 * h)
            an = float(np.sum(gG * d))
            assert abs(fd - an) < 1e-6 * max(abs(an), 1e-3), (v, w, fd, an)
            if variant == O.OPT2 and w != v:
                assert not gP[w].any()


def test_compound_kernel_vjp_of_rl_is_the_mirror():
    rng = np.random.default_rng(12)
    P = [O.prepare_psf(rand_kernel(rng, (3, 5, 3), (0.4, -0.3, 0.2))) for _ in range(2)]
    Kbar = rng.normal(size=P[0].shape)
    g = O.compound_kernel_vjp(P, 0, O.RL, Kbar)
    np.testing.assert_array_equal(g[0], O.mirror(Kbar))
    assert not g[1].any()


@pytest.mark.parametrize("variant", [O.EFF, O.OPT1])
def test_compound_variant_gradient_matches_finite_differences(variant):
    """Loss and vector-Jacobian product of runs with compound kernels (with
    weights and lambda): central differences in psi^0 and in every PSF."""
    rng = np.random.default_rng(13)
    views, psfs, w, psi0 = small_case(rng, True, 0.05)
    n = 2
    L, gpsi, gP = O.loss_and_grad(views, psfs, n, psi0, w, 0.05, variant)
    assert abs(L - O.loss_of(views, psfs, n, psi0, w, 0.05, variant)) < 1e-10 * L
    d = rng.normal(size=psi0.shape)
    h = 1e-4
    fd = (O.loss_of(views, psfs, n, psi0 + h * d, w, 0.05, variant)
          - O.loss_of(views, psfs, n, psi0 - h * d, w, 0.05, variant)) / (2 * h)
    an = float(np.sum(gpsi * d))
    assert abs(fd - an) < 1e-6 * max(abs(an), 1e-3 * L), (fd, an)
    for v in range(3):
        dP = rng.normal(size=psfs[v].shape)
        hp = 1e-5 * psfs[v].max()
        p1 = [p.copy() for p in psfs]
        p2 = [p.copy() for p in psfs]
        p1[v] = p1[v] + hp * dP
        p2[v] = p2[v] - hp * dP
        fd = (O.loss_of(views, p1, n, psi0, w, 0.05, variant) - O.loss_of(views, p2, n, psi0, w, 0.05, variant)) / (2 * hp)
        an = float(np.sum(gP[v] * dP))
        assert abs(fd - an) < 1e-5 * max(abs(an), 1e-3 * L), (v, fd, an)
    # the vector-Jacobian product against <gbar, psi_n> from the forward alone
    gbar = rng.normal(size=psi0.shape)
    psi_n, gpsi2, gP2 = O.vjp(views, psfs, n, psi0, gbar, w, 0.05, variant)

    def g(p, s0):
        pb = O.Problem(views, p, w, 0.05)
        return float(np.sum(gbar * pb.iterate(np.asarray(s0, np.float64), n, variant)))

    for v in range(3):
        dP = rng.normal(size=psfs[v].shape)
        hp = 1e-5 * psfs[v].max()
        p1 = [p.copy() for p in psfs]
        p2 = [p.copy() for p in psfs]
        p1[v] = p1[v] + hp * dP
        p2[v] = p2[v] - hp * dP
        fd = (g(p1, psi0) - g(p2, psi0)) / (2 * hp)
        an = float(np.sum(gP2[v] * dP))
        assert abs(fd - an) < 1e-5 * max(abs(an), 1.0), (v, fd, an)
