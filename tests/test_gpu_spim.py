"""Deconvolution of a simulated SPIM acquisition: it beats the views'
correlation to the ground truth by a wide margin, tolerates a moderately
misrotated PSF with a small loss, and Optimization I reaches its best in
fewer iterations than RL."""
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def acq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1308_0730_amd import spim_sim
    return spim_sim.simulate((64, 64, 64), n_spheres=150)


def test_robustness_to_psf_rotation(acq):
    from paper_1308_0730_amd import spim_sim
    r = spim_sim.psf_robustness(acq, errors=(0.0, 20.0), variant="opt1", n_iter=8)
    print(r)
    c0, c20 = r["results"][0]["best_correlation"], r["results"][1]["best_correlation"]
    assert c0 > 0.9 and c0 > r["views_correlation"] + 0.2
    assert r["views_correlation"] < c20 < c0


def test_optimisation_one_needs_fewer_iterations(acq):
    from paper_1308_0730_amd import spim_sim
    rl = spim_sim.psf_robustness(acq, errors=(0.0,), variant="rl", n_iter=16)["results"][0]
    o1 = spim_sim.psf_robustness(acq, errors=(0.0,), variant="opt1", n_iter=16)["results"][0]
    print(rl, o1)
    assert o1["at_iteration"] < rl["at_iteration"]
    assert abs(o1["best_correlation"] - rl["best_correlation"]) < 0.01
