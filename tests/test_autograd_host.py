"""Host-side pieces of the differentiated form: the torch PSF model equals
the generator's sampled Gaussian, and its parameter derivatives match
finite differences."""
import numpy as np
import torch

from paper_1308_0730_amd import synth


def test_psf_from_theta_matches_generator():
    from paper_1308_0730_amd.autograd import psf_from_theta
    for th in (0.0, 45.0, 90.0, 135.0):
        g = psf_from_theta(torch.tensor(1.2, dtype=torch.float64), torch.tensor(4.0, dtype=torch.float64), th,
                           (9, 9, 13)).numpy()
        ref = synth.gaussian_psf((9, 9, 13), 1.2, 4.0, th, dtype=np.float64)
        np.testing.assert_allclose(g / g.sum(), ref, rtol=1e-12, atol=1e-15)


def test_psf_from_theta_parameter_derivative():
    from paper_1308_0730_amd.autograd import psf_from_theta
    s = torch.tensor([1.3, 3.7], dtype=torch.float64, requires_grad=True)
    w = torch.from_numpy(np.random.default_rng(0).normal(size=(11, 9, 9)))
    T = lambda x: torch.tensor(x, dtype=torch.float64)
    f = lambda a, b: float((psf_from_theta(T(a), T(b), 30.0, (9, 9, 11)) * w).sum())
    (psf_from_theta(s[0], s[1], 30.0, (9, 9, 11)) * w).sum().backward()
    h = 1e-6
    fd0 = (f(1.3 + h, 3.7) - f(1.3 - h, 3.7)) / (2 * h)
    fd1 = (f(1.3, 3.7 + h) - f(1.3, 3.7 - h)) / (2 * h)
    np.testing.assert_allclose(s.grad.numpy(), [fd0, fd1], rtol=1e-6)
