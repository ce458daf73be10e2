"""Differentiated form on the GPU: loss and gradients through the unrolled
sequential RL run (hand-written adjoint passes) against the FP64 oracle
gradient, and the PSF-parameter gradient against finite differences.

Tolerances (relative L2 against the FP64 oracle gradient): GRAD = 5e-5 on
the small cases, where the measured errors are 1e-7 to 6e-6 (an order of
magnitude of margin, half the 1e-4 target); 1e-4 at the 128^3 workload."""
import numpy as np
import pytest
import torch

from oracle import mvd_oracle as O
from paper_1308_0730_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mvd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1308_0730_amd import mvd as m
    return m


def asym_psf(rng, shape, off):
    kz, ky, kx = shape
    z, y, x = np.meshgrid(np.arange(kz) - (kz - 1) / 2, np.arange(ky) - (ky - 1) / 2,
                          np.arange(kx) - (kx - 1) / 2, indexing="ij")
    g = np.exp(-0.5 * ((x - off[2]) ** 2 / 1.7 + (y - off[1]) ** 2 / 1.1 + (z - off[0]) ** 2 / 3.0))
    g += 0.3 * np.exp(-0.5 * ((x + 1.5) ** 2 + (y - 1) ** 2 + (z + 2) ** 2) / 0.8)
    return (g / g.sum() * 3.0).astype(np.float32)  # not normalised: the gradient includes eq. 3


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


GRAD = 5e-5


@pytest.mark.parametrize("weighted,lam,dims", [(False, 0.0, (40, 36, 30)), (True, 0.02, (40, 36, 30)),
                                               (True, 0.02, (64, 20, 24))])
def test_gradient_matches_oracle(mvd, weighted, lam, dims):
    s = synth.make_problem(dims, 8, [0.0, 70.0, 130.0], (5, 5, 7), 1.0, 2.0, 31)
    rng = np.random.default_rng(5)
    psfs = [asym_psf(rng, (9, 7, 7), off) for off in ((0.6, -0.4, 0.3), (-0.5, 0.5, 0.7), (0.3, 0.2, -0.6))]
    w = [np.clip(rng.uniform(-0.2, 1.2, size=s.views[0].shape), 0, 1).astype(np.float32) for _ in range(3)] \
        if weighted else None
    psi0 = rng.uniform(5, 25, size=s.views[0].shape).astype(np.float32)
    n = 3
    L, gpsi, gP = O.loss_and_grad(s.views, psfs, n, psi0.astype(np.float64), w, lam)
    with mvd.Deconvolver(s.views, psfs, w, lam=lam) as d:
        l2, gp2, gpsi2 = d.loss_grad(n, psi0)
        gpsi2 = gpsi2.cpu().numpy()
    print(f"loss {l2:.8e} vs {L:.8e}; psi0 grad rel {rel(gpsi2, gpsi):.2e}; "
          f"psf grad rel {[f'{rel(a, b):.2e}' for a, b in zip(gp2, gP)]}")
    assert abs(l2 - L) <= 1e-5 * L
    assert rel(gpsi2, gpsi) <= GRAD
    for a, b in zip(gp2, gP):
        assert rel(a, b) <= GRAD


def grad_case(weighted, seed=5, dims=(40, 36, 30)):
    s = synth.make_problem(dims, 8, [0.0, 70.0, 130.0], (5, 5, 7), 1.0, 2.0, 31)
    rng = np.random.default_rng(seed)
    psfs = [asym_psf(rng, (9, 7, 7), off) for off in ((0.6, -0.4, 0.3), (-0.5, 0.5, 0.7), (0.3, 0.2, -0.6))]
    w = [np.clip(rng.uniform(-0.2, 1.2, size=s.views[0].shape), 0, 1).astype(np.float32) for _ in range(3)] \
        if weighted else None
    psi0 = rng.uniform(5, 25, size=s.views[0].shape).astype(np.float32)
    return s, psfs, w, psi0, rng


@pytest.mark.parametrize("weighted,lam,dims", [(False, 0.0, (40, 36, 30)), (True, 0.02, (40, 36, 30)),
                                               (True, 0.02, (32, 36, 30)), (False, 0.0, (64, 20, 24)),
                                               (False, 0.0, (16, 720, 10)), (True, 0.02, (2048, 8, 10))])
def test_backward_matches_oracle_vjp(mvd, weighted, lam, dims):
    """mvd_backward with a random upstream gradient against the oracle's
    vector-Jacobian product; the handle is left at psi_n.  Half-rows of 20
    and 8 use the runtime-plan adjoint x passes, 16, 32 and 1024 the
    compile-time ones; 720 along y exceeds the runtime plans' lengths."""
    s, psfs, w, psi0, rng = grad_case(weighted, dims=dims)
    gbar = rng.normal(size=psi0.shape).astype(np.float32)
    n = 3
    psi_n, gpsi, gP = O.vjp(s.views, psfs, n, psi0.astype(np.float64), gbar.astype(np.float64), w, lam)
    with mvd.Deconvolver(s.views, psfs, w, lam=lam) as d:
        gp2, gpsi2 = d.backward(n, psi0, gbar)
        gpsi2 = gpsi2.cpu().numpy()
        e = d.estimate().cpu().numpy()
        # host seed, PSF gradients only
        gp3, none = d.backward(n, torch.from_numpy(psi0).cuda(), gbar, grad_psi0=False)
    print(f"psi0 grad rel {rel(gpsi2, gpsi):.2e}; psf grad rel {[f'{rel(a, b):.2e}' for a, b in zip(gp2, gP)]}; "
          f"psi_n rel {rel(e, psi_n):.2e}")
    assert none is None
    assert rel(e, psi_n) <= 1e-5
    assert rel(gpsi2, gpsi) <= GRAD
    for a, b, c in zip(gp2, gP, gp3):
        assert rel(a, b) <= GRAD
        assert np.array_equal(a, c)


def test_deconvolve_layer_under_a_torch_loss(mvd):
    """MVDDeconvolve (psi_n as a differentiable torch output) under a loss
    written in torch, L = sum (psi_n - truth)^2 over a mask: the gradients
    torch receives in psi0 and the PSFs against the oracle's vector-Jacobian
    product seeded with that loss's dL/dpsi_n."""
    from paper_1308_0730_amd.autograd import MVDDeconvolve
    s, psfs, w, psi0, rng = grad_case(False, seed=6)
    truth = torch.from_numpy(s.truth.astype(np.float32)).cuda()
    mask = torch.from_numpy((rng.uniform(size=psi0.shape) < 0.5).astype(np.float32)).cuda()
    n = 2
    with mvd.Deconvolver(s.views, psfs) as d:
        p0 = torch.from_numpy(psi0).cuda().requires_grad_(True)
        ps = [torch.from_numpy(p.astype(np.float64)).requires_grad_(True) for p in psfs]
        out = MVDDeconvolve.apply(d, n, p0, *ps)
        L = (((out - truth) ** 2) * mask).sum()
        L.backward()
        gbar = (2.0 * (out.detach() - truth) * mask).cpu().numpy().astype(np.float64)
    psi_n, gpsi, gP = O.vjp(s.views, psfs, n, psi0.astype(np.float64), gbar)
    assert rel(out.detach().cpu().numpy(), psi_n) <= 1e-5
    assert rel(p0.grad.cpu().numpy(), gpsi) <= GRAD
    for a, b in zip(ps, gP):
        assert a.grad.dtype == torch.float64
        assert rel(a.grad.numpy(), b) <= GRAD


def test_forward_only_loss(mvd):
    dims = (40, 36, 30)
    s = synth.make_problem(dims, 8, [0.0, 90.0], (5, 5, 7), 1.0, 2.0, 32)
    with mvd.Deconvolver(s.views, s.psfs) as d:
        l1, g1, g2 = d.loss_grad(4, None, grad_psf=False, grad_psi0=False)
        assert g1 is None and g2 is None
        pb = O.Problem(s.views, s.psfs)
        ref = O.loss_value(pb.iterate(pb.psi0(), 4, O.RL), pb.views, pb.P)
        assert abs(l1 - ref) <= 1e-5 * ref
        # the handle is left at the end of the run
        e = d.estimate().cpu().numpy()
        assert O.rel_l2(e, pb.iterate(pb.psi0(), 4, O.RL)) <= 1e-4


def test_config5_theta_gradient(mvd):
    """128^3, four views, 25^3 PSFs from (sigma_xy, sigma_z) per view, start
    perturbed by U[0.8, 1.2], 8 iterations: the library's PSF-parameter
    gradient against central finite differences (step 1e-3) of the library's
    own loss, and its PSF gradient against the FP64 oracle gradient."""
    from paper_1308_0730_amd.autograd import loss_and_theta_grad, psf_from_theta
    s = synth.config5()
    true, start = synth.config5_theta()
    psi0 = np.full(s.views[0].shape, float(np.mean([v.mean() for v in s.views])), np.float32)
    ext = (25, 25, 25)
    with mvd.Deconvolver(s.views, s.psfs) as d:
        L, g = loss_and_theta_grad(d, 8, torch.from_numpy(psi0).cuda(), start, s.angles, ext)

        def loss_at(th):
            ps = [psf_from_theta(torch.tensor(th[v, 0]), torch.tensor(th[v, 1]), s.angles[v], ext).numpy()
                  for v in range(4)]
            d.set_psfs(ps)
            return d.loss_grad(8, psi0, grad_psf=False, grad_psi0=False)[0]

        h = 1e-3
        fd = np.zeros_like(g)
        for v in range(4):
            for k in range(2):
                tp, tm = start.copy(), start.copy()
                tp[v, k] += h
                tm[v, k] -= h
                fd[v, k] = (loss_at(tp) - loss_at(tm)) / (2 * h)
        print("theta grad", g.ravel(), "fd", fd.ravel())
        assert rel(g, fd) <= 5e-3
        # PSF and psi0 gradients against the FP64 oracle at the start point
        ps = [psf_from_theta(torch.tensor(start[v, 0]), torch.tensor(start[v, 1]), s.angles[v], ext).numpy()
              for v in range(4)]
        d.set_psfs(ps)
        L2, gP2, gpsi2 = d.loss_grad(8, psi0)
        gpsi2 = gpsi2.cpu().numpy()
    Lo, gpsio, gPo = O.loss_and_grad(s.views, ps, 8, psi0.astype(np.float64))
    print(f"loss {L2:.8e} vs {Lo:.8e}; psi0 grad rel {rel(gpsi2, gpsio):.2e}; "
          f"psf grad rel {[f'{rel(a, b):.2e}' for a, b in zip(gP2, gPo)]}")
    assert abs(L - Lo) <= 1e-4 * Lo and abs(L2 - Lo) <= 1e-4 * Lo
    assert rel(gpsi2, gpsio) <= 1e-4
    for a, b in zip(gP2, gPo):
        assert rel(a, b) <= 1e-4


def test_autograd_gradients_follow_each_inputs_device(mvd):
    """PSFs as CUDA tensors and psi0 as a CPU tensor: MVDLoss and
    MVDDeconvolve return every gradient on its input's device and dtype,
    with the values of the run on the default devices."""
    from paper_1308_0730_amd.autograd import MVDDeconvolve, MVDLoss
    s, psfs, _, psi0, _ = grad_case(False, seed=7)
    n = 2
    with mvd.Deconvolver(s.views, psfs) as d:
        for fn in (MVDLoss, MVDDeconvolve):
            grads = []
            for psi_dev, psf_dev in (("cuda", "cpu"), ("cpu", "cuda")):
                p0 = torch.from_numpy(psi0).to(psi_dev).requires_grad_(True)
                ps = [torch.from_numpy(p.astype(np.float64)).to(psf_dev).requires_grad_(True) for p in psfs]
                out = fn.apply(d, n, p0, *ps)
                (out if fn is MVDLoss else (out * out).sum()).backward()
                assert p0.grad.device.type == psi_dev and p0.grad.dtype == torch.float32
                assert all(p.grad.device.type == psf_dev and p.grad.dtype == torch.float64 for p in ps)
                grads.append([p0.grad.cpu().numpy()] + [p.grad.cpu().numpy() for p in ps])
            for a, b in zip(*grads):
                np.testing.assert_allclose(a, b, rtol=1e-6, atol=0)


def test_recorded_backward_equals_backward(mvd):
    """mvd_forward_recorded + mvd_backward_recorded (no forward run from psi0
    in the backward) give mvd_backward's psi_n and gradients bitwise; the
    record serves a second seed; a call that changes the estimate voids it
    (MVD_ESTATE)."""
    s, psfs, w, psi0, rng = grad_case(True)
    n = 3
    g1 = rng.normal(size=psi0.shape).astype(np.float32)
    g2 = rng.normal(size=psi0.shape).astype(np.float32)
    with mvd.Deconvolver(s.views, psfs, w, lam=0.02) as d:
        ref1 = d.backward(n, psi0, g1)
        psi_ref = d.estimate().cpu().numpy()
        ref2 = d.backward(n, psi0, g2)
        psi_n, tok = d.forward_recorded(n, psi0)
        np.testing.assert_array_equal(psi_n.cpu().numpy(), psi_ref)
        for g, ref in ((g1, ref1), (g2, ref2)):
            gp, gpsi = d.backward_recorded(tok, g)
            np.testing.assert_array_equal(gpsi.cpu().numpy(), ref[1].cpu().numpy())
            for a, b in zip(gp, ref[0]):
                np.testing.assert_array_equal(a, b)
            np.testing.assert_array_equal(d.estimate().cpu().numpy(), psi_ref)
        d.iterate(1, O.RL)
        with pytest.raises(mvd.MVDError) as e:
            d.backward_recorded(tok, g1)
        assert e.value.code == mvd.MVD_ESTATE


@pytest.mark.parametrize("variant", [O.EFF, O.OPT1, O.OPT2])
def test_compound_variant_gradients_match_oracle(mvd, variant):
    """Runs with compound back-projection kernels: loss and gradients, and
    the vector-Jacobian product, against the oracle's (whose kernel
    gradients go through the construction of eq. 222/230/240; pinned by
    finite differences), with weights and lambda."""
    s, psfs, w, psi0, rng = grad_case(True)
    n = 2
    L, gpsi, gP = O.loss_and_grad(s.views, psfs, n, psi0.astype(np.float64), w, 0.02, variant)
    gbar = rng.normal(size=psi0.shape).astype(np.float32)
    psi_n, vpsi, vP = O.vjp(s.views, psfs, n, psi0.astype(np.float64), gbar.astype(np.float64), w, 0.02, variant)
    with mvd.Deconvolver(s.views, psfs, w, lam=0.02) as d:
        l2, gp2, gpsi2 = d.loss_grad(n, psi0, variant=variant)
        vp2, vpsi2 = d.backward(n, psi0, gbar, variant=variant)
        e = d.estimate().cpu().numpy()
    print(f"loss {l2:.8e} vs {L:.8e}; psi0 grad rel {rel(gpsi2.cpu().numpy(), gpsi):.2e}; "
          f"psf grad rel {[f'{rel(a, b):.2e}' for a, b in zip(gp2, gP)]}; "
          f"vjp psi0 {rel(vpsi2.cpu().numpy(), vpsi):.2e} psf {[f'{rel(a, b):.2e}' for a, b in zip(vp2, vP)]}")
    assert abs(l2 - L) <= 1e-5 * L
    assert rel(e, psi_n) <= 1e-5
    assert rel(gpsi2.cpu().numpy(), gpsi) <= GRAD and rel(vpsi2.cpu().numpy(), vpsi) <= GRAD
    for a, b in zip(gp2 + vp2, gP + vP):
        assert rel(a, b) <= GRAD


def test_config5_efficient_update_gradient(mvd):
    """The 128^3 four-view workload with 25^3 PSFs, 8 iterations of the
    efficient update (EFF, eq. 222): loss, PSF and psi0 gradients against the
    FP64 oracle (<= 1e-4)."""
    s = synth.config5()
    psi0 = np.full(s.views[0].shape, float(np.mean([v.mean() for v in s.views])), np.float32)
    with mvd.Deconvolver(s.views, s.psfs) as d:
        L2, gP2, gpsi2 = d.loss_grad(8, psi0, variant=O.EFF)
        gpsi2 = gpsi2.cpu().numpy()
    Lo, gpsio, gPo = O.loss_and_grad(s.views, s.psfs, 8, psi0.astype(np.float64), variant=O.EFF)
    print(f"loss {L2:.8e} vs {Lo:.8e}; psi0 grad rel {rel(gpsi2, gpsio):.2e}; "
          f"psf grad rel {[f'{rel(a, b):.2e}' for a, b in zip(gP2, gPo)]}")
    assert abs(L2 - Lo) <= 1e-4 * Lo
    assert rel(gpsi2, gpsio) <= 1e-4
    for a, b in zip(gP2, gPo):
        assert rel(a, b) <= 1e-4
