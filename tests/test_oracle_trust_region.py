"""Pins of the oracle's trust-region radius update and of the Sec. 2.3 example.

Sec. 2.2.2 states three regimes for the ratio rho_k of actual to predicted
reduction: a large ratio expands the radius, a moderate one keeps it, and a
small one shrinks it and rejects the trial.  The reading used here is
eta1 = 1e-4 (accept when rho > eta1), eta2 = 0.75 (expand x2, capped at 1e8,
when rho >= eta2), shrink to a quarter of the step length on rejection, and
TR_COLLAPSED when the radius falls below 1e-14 max(1, ||u||_2).

The pins:
* scalar instances whose first ratio is computed in 50-digit arithmetic,
  independently of the oracle, and placed in each regime (reject, keep,
  expand); the oracle's ratio must match and its decision and next radius
  must follow the regime;
* a start so large that a unit step is absorbed by rounding (u + s == u), so
  that the actual reduction is exactly zero, the trial is rejected and the
  radius collapses at the first iteration;
* the regime rules checked on every trial of the dogleg traces of the tanh and
  mixed workloads, with each regime required to occur;
* the worked example of Sec. 2.3, f(u, p) = u^2 - p with u0 = (1, 2),
  p = (2, 5): the root sqrt(p) and dg/dp = (1, 1) for g = sum u^2.
"""
import json
import os

import mpmath
import numpy as np
import pytest

import oracle
from paper_2403_16341_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ETA1, ETA2, DMAX = 1e-4, 0.75, 1e8

# scalar cubic F(u) = a u + 0.1 u^3 - b (family CUBIC, N = 1) with a < 0, so
# that a Newton step can overshoot and the ratio can take any value
A_S, B_S = -1.0, 0.3


def _mp_F(u):
    return mpmath.mpf(A_S) * u + mpmath.mpf("0.1") * u ** 3 - mpmath.mpf(B_S)


def _mp_J(u):
    return mpmath.mpf(A_S) + mpmath.mpf("0.3") * u ** 2


def _mp_rho(u, s):
    """rho = (F(u)^2 - F(u+s)^2) / (F(u)^2 - (F(u) + J(u) s)^2), 50 digits."""
    f0, f1 = _mp_F(u), _mp_F(u + s)
    return (f0 ** 2 - f1 ** 2) / (f0 ** 2 - (f0 + _mp_J(u) * s) ** 2)


def _start_with_ratio(target, lo, hi):
    """u0 in [lo, hi] whose full Newton step has ratio `target` (bisection in
    50 digits), rounded to a double."""
    mpmath.mp.dps = 50

    def g(u):
        u = mpmath.mpf(u)
        return _mp_rho(u, -_mp_F(u) / _mp_J(u)) - target

    return float(mpmath.findroot(g, (mpmath.mpf(lo), mpmath.mpf(hi)), solver="bisect", tol=1e-40))


@pytest.mark.parametrize("target,bracket,regime", [
    (5e-5, (-2.421, -2.42), "reject"),
    (0.5, (-2.494, -2.493), "keep"),
    (0.9, (-2.662, -2.661), "expand"),
])
def test_first_ratio_and_regime_on_scalar_instances(target, bracket, regime):
    u0 = _start_with_ratio(target, *bracket)
    mpmath.mp.dps = 50
    u = mpmath.mpf(u0)
    dN = -_mp_F(u) / _mp_J(u)
    assert abs(dN) < 10.0                      # the Newton step fits in the first region
    rho_exact = float(_mp_rho(u, dN))
    p = np.array([A_S, B_S])
    r = oracle.solve_one(oracle.CUBIC, oracle.DOGLEG, p, np.array([u0]), abstol=1e-300, maxiters=2,
                         opts=dict(tr_delta0=10.0), trace_cap=4)
    t = r["trace"]
    assert len(t["k"]) == 2
    assert t["kind"][0] == 0 and t["delta"][0] == 10.0
    assert abs(t["alpha"][0] - rho_exact) <= 1e-9 * max(1.0, abs(rho_exact))
    assert abs(t["alpha"][0] - target) <= 1e-6 * max(1.0, target)
    if regime == "reject":
        assert t["accepted"][0] == 0
        assert t["delta"][1] == 0.25 * t["step"][0]
        assert abs(t["step"][0] - float(abs(dN))) <= 1e-14 * float(abs(dN))
        # the second trial is the boundary step of the shrunk radius, from the
        # same point: its ratio again from 50 digits
        s1 = mpmath.mpf(t["delta"][1]) * mpmath.sign(dN)
        assert t["kind"][1] != 0
        rho1 = float(_mp_rho(u, s1))
        assert abs(t["alpha"][1] - rho1) <= 1e-9 * max(1.0, abs(rho1))
    elif regime == "keep":
        assert t["accepted"][0] == 1 and t["delta"][1] == 10.0
    else:
        assert t["accepted"][0] == 1 and t["delta"][1] == 20.0


def test_expansion_is_capped():
    """Delta0 just below the cap: an expanding trial sets the radius to the cap."""
    u0 = _start_with_ratio(0.9, -2.662, -2.661)
    r = oracle.solve_one(oracle.CUBIC, oracle.DOGLEG, np.array([A_S, B_S]), np.array([u0]), abstol=1e-300,
                         maxiters=2, opts=dict(tr_delta0=0.75 * DMAX), trace_cap=4)
    t = r["trace"]
    assert t["accepted"][0] == 1 and t["delta"][1] == DMAX


@pytest.mark.parametrize("u0", [1e17, 2.0 ** 60, -3e20])
def test_rounding_absorbed_step_collapses_the_radius_at_once(u0):
    """F(u) = u + 0.1 u^3 at |u| >= 1e17: the Newton step is far outside the
    unit region, the boundary step has length 1 < ulp(u), so u + s == u and
    the actual reduction is exactly 0 (the predicted one rounds away as well,
    rho = -inf): rho <= eta1, rejected, Delta = 1/4, which is below
    1e-14 |u| -> TR_COLLAPSED at iteration 1, u unchanged."""
    p = np.array([1.0, 0.0])
    r = oracle.solve_one(oracle.CUBIC, oracle.DOGLEG, p, np.array([u0]), abstol=1e-10, maxiters=100,
                         trace_cap=4)
    t = r["trace"]
    assert r["retcode"] == oracle.RC_TR_COLLAPSED and r["iters"] == 1
    assert r["u"][0] == u0
    assert t["ared"][0] == 0.0 and t["alpha"][0] <= 0.0 and t["accepted"][0] == 0
    assert t["kind"][0] == 1 and t["step"][0] == 1.0
    assert 0.25 * t["step"][0] < 1e-14 * abs(u0)


@pytest.mark.parametrize("k", [3, 4])
def test_radius_regimes_on_every_dogleg_trial(k):
    """On the tanh (3) and mixed (4) workloads: every trial's decision and the
    next radius follow the regime of its ratio, and each regime occurs."""
    b = inputs.config(k, M=80)
    seen = {"reject": 0, "keep": 0, "expand": 0, "cap": 0}
    for s in range(b.M):
        f, n, _, p, u0 = b.system(s)
        r = oracle.solve_one(f, oracle.DOGLEG, p, u0, abstol=1e-10, maxiters=100, trace_cap=128)
        t = r["trace"]
        L = len(t["k"])
        for i in range(L):
            rho, D, acc = t["alpha"][i], t["delta"][i], t["accepted"][i]
            # the ratio is ared / pred when the model predicts a decrease
            if t["pred"][i] > 0 and np.isfinite(t["merit"][i]) and acc == 1:
                assert rho == t["ared"][i] / t["pred"][i]
            nxt = t["delta"][i + 1] if i + 1 < L else None
            if rho >= ETA2:
                assert acc == 1
                seen["expand"] += 1
                if nxt is not None:
                    assert nxt == min(2.0 * D, DMAX)
                    seen["cap"] += nxt == DMAX
            elif rho > ETA1:
                assert acc == 1
                seen["keep"] += 1
                if nxt is not None:
                    assert nxt == D
            else:
                assert acc == 0
                seen["reject"] += 1
                if nxt is not None:
                    assert nxt == 0.25 * t["step"][i]
        if r["retcode"] == oracle.RC_TR_COLLAPSED:
            assert t["accepted"][-1] == 0
    assert seen["reject"] > 0 and seen["keep"] > 0 and seen["expand"] > 0


def test_sensitivity_worked_example():
    """Sec. 2.3: f(u, p) = u.^2 - p from u0 = (1, 2) at p = (2, 5) has the root
    (sqrt 2, sqrt 5); for g(u*) = sum u*^2 the derivative in p is (1, 1)
    (at the root g = p_1 + p_2)."""
    ex = json.load(open(os.path.join(GOLDEN, "sensitivity_example.json")))
    p, u0 = np.array(ex["p"]), np.array(ex["u0"])
    for alg in (oracle.NEWTON, oracle.ARMIJO, oracle.DOGLEG):
        r = oracle.solve_one(oracle.SQUARE, alg, p, u0, abstol=1e-14, maxiters=50)
        assert r["retcode"] == oracle.RC_SUCCESS
        assert np.allclose(r["u"], ex["known_root"], rtol=1e-14, atol=0)
    u = r["u"]
    # adjoint: lambda = J^-T dg/du with dg/du = 2u, gradient -(dF/dp)^T lambda
    st, lam, grad = oracle.adjoint(oracle.SQUARE, p, u, 2.0 * u)
    assert st == 0
    assert np.allclose(grad, ex["dg_dp"], rtol=0, atol=1e-13)
    # tangent: du*/dp_j = 1 / (2 sqrt(p_j)) e_j, and dg/dp_j = 2 u . du
    for j in range(2):
        v = np.zeros(2)
        v[j] = 1.0
        st, du = oracle.tangent(oracle.SQUARE, p, u, v)
        assert st == 0
        assert np.allclose(du, v / (2.0 * np.sqrt(p)), rtol=1e-13, atol=1e-15)
        assert abs(2.0 * u @ du - ex["dg_dp"][j]) <= 1e-13
