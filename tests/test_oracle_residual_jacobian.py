"""Pins of the oracle's residual families and dual-number Jacobians.

Residuals are checked against exact rational arithmetic (cubic, on dyadic
inputs) and 50-digit mpmath (tanh, Rosenbrock, the workflow example of Sec. 3).
Jacobians are checked against hand-derived closed forms, complex-step
differentiation of an independent numpy residual, and central differences.
"""
import json
import math
import os
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle
from paper_2403_16341_amd import inputs

EPS = np.finfo(np.float64).eps
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dyadic(rng, shape, scale=8, span=4):
    return rng.integers(-span * scale, span * scale + 1, size=shape) / scale


@pytest.mark.parametrize("n", [1, 2, 3, 4, 8, 16, 33])
def test_cubic_residual_matches_exact_rationals(n):
    rng = np.random.default_rng(100 + n)
    for _ in range(5):
        A, b, u = _dyadic(rng, (n, n)), _dyadic(rng, n), _dyadic(rng, n)
        F = oracle.residual(oracle.CUBIC, np.concatenate([A.ravel(), b]), u)
        for i in range(n):
            s = sum(Fraction(A[i, j]) * Fraction(u[j]) for j in range(n))
            exact = s + Fraction(1, 10) * Fraction(u[i]) ** 3 - Fraction(b[i])
            scale = float(sum(abs(Fraction(A[i, j]) * Fraction(u[j])) for j in range(n))
                          + Fraction(1, 10) * abs(Fraction(u[i])) ** 3 + abs(Fraction(b[i])))
            assert abs(F[i] - float(exact)) <= (n + 6) * EPS * scale + 1e-300


def _mp_tanh_residual(A, b, beta, u):
    n = len(u)
    out = []
    for i in range(n):
        s = mpmath.fsum(mpmath.mpf(A[i, j]) * mpmath.tanh(mpmath.mpf(u[j])) for j in range(n))
        out.append(s + mpmath.mpf(beta) * mpmath.mpf(u[i]) - mpmath.mpf(b[i]))
    return out


@pytest.mark.parametrize("n", [1, 2, 5, 16])
def test_tanh_residual_matches_mpmath(n):
    mpmath.mp.dps = 50
    rng = np.random.default_rng(200 + n)
    for _ in range(4):
        A = rng.standard_normal((n, n))
        b = rng.uniform(-2, 2, n)
        beta = rng.uniform(0.05, 0.5)
        u = rng.uniform(-4, 4, n)
        F = oracle.residual(oracle.TANH, np.concatenate([A.ravel(), b, [beta]]), u)
        ref = _mp_tanh_residual(A, b, beta, u)
        for i in range(n):
            scale = np.abs(A[i]).sum() + abs(beta * u[i]) + abs(b[i])
            assert abs(F[i] - float(ref[i])) <= (n + 8) * 2 * EPS * scale


def test_rosenbrock_residual_matches_mpmath_and_root():
    mpmath.mp.dps = 50
    rng = np.random.default_rng(3)
    for n in (2, 3, 10, 64):
        u = rng.uniform(-2, 2, n)
        F = oracle.residual(oracle.ROSENBROCK, np.zeros(0), u)
        assert abs(F[0] - float(1 - mpmath.mpf(u[0]))) <= 2 * EPS
        for i in range(1, n):
            ref = 10 * (mpmath.mpf(u[i]) - mpmath.mpf(u[i - 1]) ** 2)
            assert abs(F[i] - float(ref)) <= 8 * EPS * (10 * (abs(u[i]) + u[i - 1] ** 2))
    g = json.load(open(os.path.join(GOLDEN, "rosenbrock_n10.json")))
    F = oracle.residual(oracle.ROSENBROCK, np.zeros(0), np.array(g["known_root"]))
    assert np.all(F == 0.0)


def test_paper_example_residual_and_known_root():
    mpmath.mp.dps = 50
    g = json.load(open(os.path.join(GOLDEN, "paper_example.json")))
    p = np.array(g["p"])
    F = oracle.residual(oracle.PAPER, p, np.array(g["known_root"]))
    assert np.all(F == 0.0)
    rng = np.random.default_rng(4)
    for _ in range(20):
        u = rng.uniform(-1, 1, 2)
        F = oracle.residual(oracle.PAPER, p, u)
        x1, x2 = mpmath.mpf(u[0]), mpmath.mpf(u[1])
        r1 = (x1 + 3) * (x2 ** 3 - 7) + 18
        r2 = mpmath.sin(x2 * mpmath.exp(x1) - 1)
        assert abs(F[0] - float(r1)) <= 1e-14 * 30
        assert abs(F[1] - float(r2)) <= 1e-15 * 4


@pytest.mark.parametrize("family", [oracle.CUBIC, oracle.TANH, oracle.ROSENBROCK, oracle.PAPER])
def test_dual_value_part_equals_plain_residual(family):
    rng = np.random.default_rng(5 + family)
    for n in ([2] if family == oracle.PAPER else [2, 7, 16]):
        p = _random_params(rng, family, n)
        u = rng.uniform(-2, 2, n)
        a = oracle.residual(family, p, u)
        b = oracle.residual_dual_value(family, p, u)
        assert np.array_equal(a, b)


def _random_params(rng, family, n):
    if family == oracle.CUBIC:
        return inputs.cubic_params(rng, 1, n)[0]
    if family == oracle.TANH:
        return inputs.tanh_params(rng, 1, n)[0]
    if family == oracle.ROSENBROCK:
        return np.zeros(0)
    return np.array([3.0, 7.0, 18.0]) + rng.uniform(-1, 1, 3)


def _np_residual(family, p, u):
    """Independent numpy residual (works on complex u for the complex step)."""
    n = u.size
    if family == oracle.CUBIC:
        A = p[: n * n].reshape(n, n)
        b = p[n * n: n * n + n]
        return A @ u + 0.1 * u ** 3 - b
    if family == oracle.TANH:
        A = p[: n * n].reshape(n, n)
        b = p[n * n: n * n + n]
        beta = p[n * n + n]
        return A @ np.tanh(u) + beta * u - b
    if family == oracle.ROSENBROCK:
        return np.concatenate([[1 - u[0]], 10 * (u[1:] - u[:-1] ** 2)])
    a, b, c = p
    return np.array([(u[0] + a) * (u[1] ** 3 - b) + c, np.sin(u[1] * np.exp(u[0]) - 1)])


def _closed_form_jacobian(family, p, u):
    n = u.size
    if family == oracle.CUBIC:
        return p[: n * n].reshape(n, n) + np.diag(0.3 * u ** 2)
    if family == oracle.TANH:
        A = p[: n * n].reshape(n, n)
        return A * (1 - np.tanh(u) ** 2)[None, :] + p[n * n + n] * np.eye(n)
    if family == oracle.ROSENBROCK:
        J = np.zeros((n, n))
        J[0, 0] = -1.0
        for i in range(1, n):
            J[i, i - 1] = -20.0 * u[i - 1]
            J[i, i] = 10.0
        return J
    a, b, c = p
    arg = u[1] * math.exp(u[0]) - 1
    return np.array([[u[1] ** 3 - b, 3 * u[1] ** 2 * (u[0] + a)],
                     [math.cos(arg) * u[1] * math.exp(u[0]), math.cos(arg) * math.exp(u[0])]])


@pytest.mark.parametrize("family", [oracle.CUBIC, oracle.TANH, oracle.ROSENBROCK, oracle.PAPER])
def test_jacobian_closed_form_complex_step_and_fd(family):
    rng = np.random.default_rng(50 + family)
    for n in ([2] if family == oracle.PAPER else [2, 4, 8, 16]):
        for _ in range(3):
            p = _random_params(rng, family, n)
            u = rng.uniform(-1.5, 1.5, n)
            J = oracle.jacobian(family, p, u)
            Jc = _closed_form_jacobian(family, p, u)
            scale = max(1.0, np.abs(Jc).max())
            assert np.abs(J - Jc).max() <= 64 * EPS * scale
            # complex step: Im F(u + i h e_j) / h, exact to rounding for analytic F
            h = 1e-30
            Jcs = np.empty((n, n))
            for j in range(n):
                z = u.astype(complex)
                z[j] += 1j * h
                Jcs[:, j] = _np_residual(family, p, z).imag / h
            assert np.abs(J - Jcs).max() <= 64 * EPS * scale
            # central differences: O(h^2) truncation
            hf = 1e-6
            Jfd = np.empty((n, n))
            for j in range(n):
                e = np.zeros(n)
                e[j] = hf
                Jfd[:, j] = (oracle.residual(family, p, u + e) - oracle.residual(family, p, u - e)) / (2 * hf)
            assert np.abs(J - Jfd).max() <= 1e-6 * scale


def test_nparams_matches_input_packing():
    for n in (1, 2, 8, 64):
        assert oracle.nparams(oracle.CUBIC, n) == inputs.nparams(inputs.CUBIC, n)
        assert oracle.nparams(oracle.TANH, n) == inputs.nparams(inputs.TANH, n)
    assert oracle.nparams(oracle.PAPER, 2) == 3
    assert oracle.nparams(oracle.PAPER, 3) == -1
    assert oracle.nparams(oracle.ROSENBROCK, 1) == -1
    assert oracle.nparams(oracle.CUBIC, 65) == -1
    assert oracle.nparams(7, 4) == -1
