"""Pins of the oracle's sensitivities at a solution (Sec. 2.3, implicit
function theorem): closed forms on separable systems (implicit
differentiation of a scalar equation, roots by Cardano), central finite
differences of converged solves on general systems, the duality of the
tangent and adjoint forms, numpy's LAPACK solve for the transposed system,
and the singular / non-finite cases."""
import mpmath
import numpy as np
import pytest

import oracle
from paper_2403_16341_amd import inputs


def _cardano_root(a, b):
    """Real root of 0.1 u^3 + a u - b = 0 for a > 0 (depressed cubic in
    trigonometric-hyperbolic form, 40 digits)."""
    mpmath.mp.dps = 40
    P, Q = 10 * mpmath.mpf(a), -10 * mpmath.mpf(b)
    return float(-2 * mpmath.sqrt(P / 3) * mpmath.sinh(mpmath.asinh((3 * Q / (2 * P)) * mpmath.sqrt(3 / P)) / 3))


def _rel(x, y):
    return np.abs(np.asarray(x) - np.asarray(y)).max() / max(np.abs(np.asarray(y)).max(), 1e-300)


@pytest.mark.parametrize("n", [1, 3, 6])
def test_separable_cubic_closed_form(n):
    """F_i = a_i u_i + 0.1 u_i^3 - b_i.  Implicit differentiation of one
    equation: du_i/db_i = 1/(a_i + 0.3 u_i^2), du_i/dA_ij = -u_j/(a_i + 0.3
    u_i^2) (the off-diagonal A_ij enter F_i through u_j).  For g = sum u^2
    (the paper's worked example of Sec. 2.3 differentiates this g), the
    gradient is dg/db_i = 2 u_i/(a_i + 0.3 u_i^2) -- positive, as the minus
    sign of the implicit function theorem requires."""
    b = inputs.separable_cubic(8, n, seed=40 + n)
    for s in range(b.M):
        f, _, _, p, _ = b.system(s)
        a = np.diag(p[: n * n].reshape(n, n)).copy()
        rhs = p[n * n:]
        u = np.array([_cardano_root(a[i], rhs[i]) for i in range(n)])
        d = a + 0.3 * u ** 2
        rc, lam, g = oracle.adjoint(f, p, u, 2 * u)
        assert rc == 0
        gA = g[: n * n].reshape(n, n)
        assert _rel(g[n * n:], 2 * u / d) <= 1e-13
        assert _rel(gA, -np.outer(2 * u / d, u)) <= 1e-13
        assert (g[n * n:] * np.sign(u) > 0).all()
        for i in range(n):
            v = np.zeros(p.size)
            v[n * n + i] = 1.0
            rc, du = oracle.tangent(f, p, u, v)
            ref = np.zeros(n)
            ref[i] = 1.0 / d[i]
            assert rc == 0 and _rel(du, ref) <= 1e-13


def test_cubic_without_linear_term_closed_form():
    """A = 0: 0.1 u^3 = b, u = (10 b)^(1/3), du/db = 1/(0.3 u^2); with
    g = sum u^2, dg/db = 20/(3 u)."""
    n = 3
    bvec = np.array([0.7, 2.5, 8.1])
    p = np.concatenate([np.zeros(n * n), bvec])
    u = np.cbrt(10 * bvec)
    rc, _, g = oracle.adjoint(oracle.CUBIC, p, u, 2 * u)
    # J = diag(0.3 u^2) is nonsingular; only b enters the gradient directly,
    # A_ij through u_j
    assert rc == 0
    assert _rel(g[n * n:], 20 / (3 * u)) <= 1e-13


def _converged(f, p, u0):
    r = oracle.solve_one(f, oracle.NEWTON, p, u0, abstol=1e-14, maxiters=60)
    assert r["retcode"] == oracle.RC_SUCCESS
    return r["u"]


@pytest.mark.parametrize("case", ["cubic", "tanh", "paper"])
def test_finite_differences_of_converged_solves(case):
    """Tangents against central differences of solves at theta +- h v (from
    the root, to 1e-14), on non-separable systems."""
    rng = np.random.default_rng(55)
    if case == "cubic":
        b = inputs.config(1, M=6)
    elif case == "tanh":
        b = inputs.config(3, M=40)
    else:
        b = inputs.paper_example(20, seed=8)
    checked = 0
    for s in range(b.M):
        f, n, _, p, u0 = b.system(s)
        r = oracle.solve_one(f, oracle.NEWTON, p, u0, abstol=1e-14, maxiters=60)
        if r["retcode"] != oracle.RC_SUCCESS:
            continue
        u = r["u"]
        J = oracle.jacobian(f, p, u)
        if np.linalg.cond(J) > 1e4:
            continue
        v = rng.standard_normal(p.size)
        rc, du = oracle.tangent(f, p, u, v)
        assert rc == 0
        h = 1e-6 * max(1.0, np.abs(p).max())
        up = _converged(f, p + h * v, u)
        um = _converged(f, p - h * v, u)
        fd = (up - um) / (2 * h)
        assert _rel(du, fd) <= 1e-6, (s, du, fd)
        checked += 1
        if checked >= 5:
            break
    assert checked >= 3


@pytest.mark.parametrize("k", [1, 3, 4])
def test_tangent_adjoint_duality(k):
    """w^T (D v) = (w^T D) v for random v, w: the adjoint is the transpose
    of the tangent map (catches a transposed solve or a lost sign in one)."""
    rng = np.random.default_rng(60 + k)
    b = inputs.config(k, M=30)
    checked = 0
    for s in range(b.M):
        f, n, _, p, u0 = b.system(s)
        u = oracle.solve_one(f, b.alg[s], p, u0, abstol=1e-12, maxiters=100)["u"]
        v = rng.standard_normal(p.size)
        w = rng.standard_normal(n)
        rt, du = oracle.tangent(f, p, u, v)
        ra, lam, g = oracle.adjoint(f, p, u, w)
        assert rt == ra
        # (near-singular end points of failed solves lose the identity to
        # rounding in proportion to the condition number)
        if rt == 0 and np.linalg.cond(oracle.jacobian(f, p, u)) <= 1e6:
            checked += 1
            lhs, rhs = w @ du, g @ v
            assert abs(lhs - rhs) <= 1e-10 * (np.abs(w).sum() * np.abs(du).max() + abs(rhs) + 1e-300)
    assert checked >= 10


def test_adjoint_vector_is_the_transposed_solve_and_parameter_jacobian():
    """lambda against numpy's LAPACK solve of J^T lambda = w; dF/dtheta
    against the families' derivatives written out by hand."""
    rng = np.random.default_rng(61)
    for f, b in ((oracle.ROSENBROCK, inputs.rosenbrock(5, 8, seed=3)),
                 (oracle.TANH, inputs.config(3, M=5)),
                 (oracle.CUBIC, inputs.config(1, M=5))):
        for s in range(b.M):
            _, n, _, p, u0 = b.system(s)
            u = u0 + 0.1 * rng.standard_normal(n)
            w = rng.standard_normal(n)
            rc, lam, g = oracle.adjoint(f, p, u, w)
            J = oracle.jacobian(f, p, u)
            assert rc == 0
            assert _rel(lam, np.linalg.solve(J.T, w)) <= 1e-11
            Jp = oracle.param_jacobian(f, p, u)
            if f == oracle.CUBIC:
                ref = np.zeros((n, p.size))
                for i in range(n):
                    ref[i, i * n:(i + 1) * n] = u
                    ref[i, n * n + i] = -1.0
                assert np.array_equal(Jp, ref)
            elif f == oracle.TANH:
                ref = np.zeros((n, p.size))
                for i in range(n):
                    ref[i, i * n:(i + 1) * n] = np.tanh(u)
                    ref[i, n * n + i] = -1.0
                    ref[i, -1] = u[i]
                assert _rel(Jp, ref) <= 1e-15  # (libm and numpy tanh may differ by an ulp)
            else:
                assert Jp.shape == (n, 0) and g.size == 0
    # the workflow example's three parameters
    p = np.array([0.3, 1.7, -0.4])
    u = np.array([0.2, 0.9])
    Jp = oracle.param_jacobian(oracle.PAPER, p, u)
    ref = np.array([[u[1] ** 3 - p[1], -(u[0] + p[0]), 1.0], [0.0, 0.0, 0.0]])
    assert _rel(Jp, ref) <= 1e-15


def test_singular_and_nonfinite():
    n = 3
    A = np.array([[1.0, 2.0, 3.0], [2.0, 4.0, 6.0], [0.5, 0.1, 0.2]])  # rank 2
    p = np.concatenate([A.ravel(), np.zeros(n)])
    u = np.zeros(n)  # J = A + diag(0.3 u^2) = A, singular
    rc, du = oracle.tangent(oracle.CUBIC, p, u, np.ones(p.size))
    assert rc == 2 and np.isnan(du).all()
    rc, lam, g = oracle.adjoint(oracle.CUBIC, p, u, np.ones(n))
    assert rc == 2 and np.isnan(lam).all() and np.isnan(g).all()
    u = np.array([0.1, np.nan, 0.2])
    rc, du = oracle.tangent(oracle.CUBIC, p, u, np.ones(p.size))
    assert rc == 3 and np.isnan(du).all()
    p2 = p.copy()
    p2[4] = np.inf
    rc, lam, g = oracle.adjoint(oracle.CUBIC, p2, np.ones(n), np.ones(n))
    assert rc == 3 and np.isnan(g).all()
