"""The GPU parity classifier itself, checked on the CPU.

Stand-in "device" results come from the oracle under a rounding perturbation
it does not use as a probe (multiply-add contraction plus u0 moved by two
ulps): they must pass.  Corrupted results must fail."""
import numpy as np
import pytest

from _helpers import classify, run_oracle
from paper_2403_16341_amd import inputs


def _standin(b):
    return run_oracle(b, variant="fma", u0=np.nextafter(np.nextafter(b.u0, np.inf), np.inf))


def _grid_case(fam, alg, n):
    rng = np.random.Generator(np.random.PCG64(1000 + 10 * n + fam))
    M = 70 if n <= 16 else 23
    p = inputs.cubic_params(rng, M, n) if fam == 0 else inputs.tanh_params(rng, M, n)
    u0 = rng.uniform(-3, 3, (M, n)) if fam == 0 else rng.uniform(-4, 4, (M, n))
    return inputs.homogeneous(fam, n, alg, p, u0, 1e-10, 40)


@pytest.mark.parametrize("b", [inputs.config(2, M=300), inputs.config(3, M=200), inputs.config(4, M=800),
                               _grid_case(1, 2, 1), _grid_case(1, 1, 40), _grid_case(1, 0, 24),
                               inputs.rosenbrock(60, 10, seed=5)],
                         ids=["w2", "w3", "w4", "tanh-dogleg-n1", "tanh-armijo-n40", "tanh-newton-n24",
                              "rosenbrock"])
def test_rounding_perturbed_results_pass(b):
    rep, _ = classify(b, _standin(b))
    assert not rep["strict_fail"] and rep["other_root"] == 0, rep


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
