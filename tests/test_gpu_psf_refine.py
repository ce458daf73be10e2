"""PSF refinement driven by the differentiated form: from widths perturbed by
up to 25 %, gradient descent on the views' misfit after four RL iterations
lowers the loss many-fold and moves the widths toward the true ones."""
import numpy as np
import pytest
import torch

from paper_1308_0730_amd import synth

pytestmark = pytest.mark.gpu


def test_refinement_moves_toward_the_true_psfs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1308_0730_amd import psf_refine
    angles = [0.0, 45.0, 90.0, 135.0]
    s = synth.make_problem((64, 64, 64), 40, angles, (17, 17, 17), 1.2, 4.0, 77, noise="none")
    true = np.array([[1.2, 4.0]] * 4)
    th0 = true * np.random.default_rng(5).uniform(0.75, 1.25, size=true.shape)
    th, hist = psf_refine.refine(s.views, angles, (17, 17, 17), th0, n_iter=4, steps=25)
    e0 = np.abs(th0 / true - 1)
    e1 = np.abs(th / true - 1)
    print("loss", hist[0][0], "->", hist[-1][0], "max rel error", e0.max(), "->", e1.max())
    assert all(b[0] < a[0] for a, b in zip(hist, hist[1:]))  # every accepted step lowers the loss
    assert hist[-1][0] < hist[0][0] / 10
    assert e1.max() < 0.6 * e0.max()
    assert np.abs(th[:, 1] / true[:, 1] - 1).max() < 0.1  # axial widths within 10 %
