"""The GPU parity classifier itself, checked on the CPU.

Stand-in "device" results come from the oracle under a rounding perturbation
it does not use as a probe (multiply-add contraction plus u0 moved by two
ulps): they must pass.  Corrupted results must fail."""
import numpy as np
import pytest

from _helpers import MAX_SENSITIVE, classify, grid_batch, run_oracle, sensitive_mask
from paper_2403_16341_amd import inputs


def _standin(b):
    return run_oracle(b, variant="fma", u0=np.nextafter(np.nextafter(b.u0, np.inf), np.inf))


def _grid_case(fam, alg, n):
    return grid_batch(fam, n, alg, seed=1000 + 10 * n + fam)


@pytest.mark.parametrize("b", [inputs.config(2, M=300), inputs.config(3, M=200), inputs.config(4, M=800),
                               _grid_case(1, 2, 1), _grid_case(1, 1, 40), _grid_case(1, 0, 24),
                               _grid_case(1, 4, 64), _grid_case(1, 3, 40),
                               inputs.rosenbrock(60, 10, seed=5)],
                         ids=["w2", "w3", "w4", "tanh-dogleg-n1", "tanh-armijo-n40", "tanh-newton-n24",
                              "tanh-potra-n64", "tanh-poly-n40", "rosenbrock"])
def test_rounding_perturbed_results_pass(b):
    rep, _ = classify(b, _standin(b))
    assert not rep["strict_fail"], rep


def test_pooled_grid_caps_sensitive_share():
    """A grid case whose plain draw is mostly chaotic (tanh Newton, n = 64,
    far starts) is drawn from a pool: at most MAX_SENSITIVE of it is
    rounding-sensitive, so the strict bar covers the rest."""
    b = _grid_case(1, 0, 64)
    _, _, sens = sensitive_mask(b)
    assert sens.sum() <= MAX_SENSITIVE * b.M


def test_safeguard_codes_fail():
    """A system ended by a kernel safeguard (trip guard or group
    disagreement) fails the comparison, sensitive or not."""
    b = inputs.config(3, M=120)
    for rc, it in ((6, -100000), (6, -4), (1, -100000)):
        g = run_oracle(b)
        g["retcode"][11], g["iters"][11] = rc, it
        with pytest.raises(AssertionError, match="safeguard"):
            classify(b, g)


def test_sensitive_outcomes_capped():
    """On rounding-sensitive systems the device may differ from the oracle
    only about as often as a perturbed oracle does: a device that fails
    every sensitive system fails the comparison."""
    b = grid_batch(1, 40, 0, seed=4040, M=150)
    g = run_oracle(b)
    _, _, sens = sensitive_mask(b)
    assert sens.sum() >= 20
    rc = g["retcode"].copy()
    g["retcode"][sens & (rc == 0)] = 1
    g["retcode"][sens & (rc != 0)] = np.where(rc[sens & (rc != 0)] == 1, 4, 1)
    with pytest.raises(AssertionError, match="sensitive"):
        classify(b, g)


def test_corrupted_results_fail():
    b = inputs.config(2, M=200)
    g = run_oracle(b)
    g["u"] = g["u"] * (1 + 1e-7)
    with pytest.raises(AssertionError):
        classify(b, g)
    g = run_oracle(b)
    g["retcode"][7] = 1
    rep, _ = classify(b, g)
    assert rep["strict_fail"] and rep["strict_fail"][0][0] == 7
    g = run_oracle(b)
    g["iters"][9] += 2
    rep, _ = classify(b, g)
    assert rep["strict_fail"] and rep["strict_fail"][0][0] == 9
