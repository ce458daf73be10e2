"""The convergence harness on a noise-free synthetic problem with its ground
truth: the orderings the paper reports for reaching the same quality (its
benchmark section and main figure 1d-f) hold, and the reference method meets
its own target exactly where it was taken."""
import pytest
import torch

from paper_1308_0730_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def result():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1308_0730_amd import convergence
    s = synth.make_problem((64, 64, 64), 40, [0.0, 45.0, 90.0, 135.0], (17, 17, 17), 1.2, 4.0, 99, noise="none")
    r = convergence.compare(s, ref_iters=60, max_iter=300)
    for m in r["methods"]:
        print(m)
    return {(m["scheme"], m["variant"]): m for m in r["methods"]}


def test_every_method_reaches_the_target(result):
    for k, m in result.items():
        assert m["iterations"] is not None, k


def test_reference_is_met_where_it_was_taken(result):
    """Noise-free ML-EM approaches the truth monotonically, so it first meets
    the distance it had after 60 iterations at iteration 60."""
    assert result[("combined-arithmetic", "rl")]["iterations"] == 60


def test_sequential_updates_cut_iterations(result):
    """Sequential (OS-EM) updates of the same derivation need several times
    fewer iterations than combined ones (the paper: about N-fold)."""
    for v in ("rl", "eff", "opt1", "opt2"):
        seq = result[("sequential", v)]["iterations"]
        comb = result[("combined-geometric", v)]["iterations"]
        assert 2 * seq <= comb, (v, seq, comb)


def test_virtual_views_and_optimisations_cut_iterations(result):
    """Efficient < RL, and Optimization I and II no slower than efficient, for
    both schemes."""
    for scheme in ("combined-geometric", "sequential"):
        it = {v: result[(scheme, v)]["iterations"] for v in ("rl", "eff", "opt1", "opt2")}
        assert it["eff"] < it["rl"], (scheme, it)
        assert it["opt1"] <= it["eff"] and it["opt2"] <= it["opt1"], (scheme, it)
