"""Pins of the oracle's LU with partial pivoting against LAPACK getrf (scipy)."""
import numpy as np
import pytest
import scipy.linalg

import oracle

EPS = np.finfo(np.float64).eps


def _unpack(lu, piv):
    n = lu.shape[0]
    L = np.tril(lu, -1) + np.eye(n)
    U = np.triu(lu)
    perm = np.arange(n)
    for k in range(n):
        perm[[k, piv[k]]] = perm[[piv[k], k]]
    return L, U, perm


@pytest.mark.parametrize("n", [1, 2, 3, 4, 8, 13, 16, 32, 64])
def test_lu_matches_getrf_pivots_and_reconstructs(n):
    rng = np.random.default_rng(n)
    for _ in range(6):
        A = rng.standard_normal((n, n))
        lu, piv, info = oracle.lu(A)
        assert info == 0
        lu_ref, piv_ref = scipy.linalg.lu_factor(A)
        assert np.array_equal(piv, piv_ref)
        L, U, perm = _unpack(lu, piv)
        R = A[perm] - L @ U
        bound = 4 * n * EPS * (np.abs(L) @ np.abs(U)).max()
        assert np.abs(R).max() <= bound
        assert np.abs(lu - lu_ref).max() <= 1e3 * n * EPS * np.abs(lu_ref).max()
        # |l_ij| <= 1 is the partial-pivoting invariant
        assert np.abs(np.tril(lu, -1)).max(initial=0.0) <= 1.0


def test_lu_tie_break_matches_getrf_on_exact_integer_matrices():
    """Entries in {-1, 0, 1} with every pivot a power of two keep elimination
    exact on both sides (LAPACK scales by the reciprocal pivot, the oracle
    divides), so ties are real ties; the first maximum in current row order
    wins, as in LAPACK's idamax."""
    rng = np.random.default_rng(7)
    checked = 0
    for trial in range(3000):
        n = int(rng.integers(2, 7))
        A = rng.integers(-1, 2, size=(n, n)).astype(float)
        if abs(np.linalg.det(A)) < 0.5:
            continue
        lu, piv, info = oracle.lu(A)
        assert info == 0
        if not np.all(np.log2(np.abs(np.diag(lu))) % 1 == 0):
            continue
        _, piv_ref = scipy.linalg.lu_factor(A)
        assert np.array_equal(piv, piv_ref), (A, piv, piv_ref)
        checked += 1 if np.any(piv != np.arange(n)) else 0
    assert checked > 50


def test_lu_diagonal_needs_no_swaps():
    rng = np.random.default_rng(8)
    for n in (1, 5, 16):
        d = rng.uniform(0.5, 2.0, n) * rng.choice([-1, 1], n)
        lu, piv, info = oracle.lu(np.diag(d))
        assert info == 0
        assert np.array_equal(piv, np.arange(n))
        assert np.array_equal(lu, np.diag(d))


def test_lu_reports_zero_and_nonfinite_pivots():
    A = np.array([[1.0, 2.0, 3.0], [2.0, 4.0, 6.0], [1.0, 1.0, 1.0]])
    lu, piv, info = oracle.lu(A)
    # step 1 pivots on row 1 (|2| > |1|); after elimination column 1 is (0, -1): the
    # pivot of step 2 is the -1, and step 3 hits an exact zero.
    assert info == 3
    Z = np.zeros((4, 4))
    assert oracle.lu(Z)[2] == 1
    N = np.eye(3)
    N[0, 0] = np.nan
    assert oracle.lu(N)[2] == 1
    I = np.eye(3)
    I[2, 0] = np.inf
    assert oracle.lu(I)[2] == 1


@pytest.mark.parametrize("n", [1, 3, 8, 16, 40])
def test_lu_solve_matches_numpy(n):
    rng = np.random.default_rng(10 + n)
    A = rng.standard_normal((n, n)) + n * np.eye(n) * 0.1
    b = rng.standard_normal(n)
    lu, piv, info = oracle.lu(A)
    x = oracle.lu_solve(lu, piv, b)
    xr = np.linalg.solve(A, b)
    cond = np.linalg.cond(A)
    assert np.abs(x - xr).max() <= 50 * n * EPS * cond * np.abs(xr).max()
    assert np.abs(A @ x - b).max() <= 50 * n * EPS * np.abs(A).max() * np.abs(x).max()
