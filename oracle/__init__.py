"""TEST INFRASTRUCTURE ONLY: the CPU oracle of the batched nonlinear solver.

A plain, single-threaded FP64 C implementation (``nls_oracle.c``) of what the
GPU path computes, written from the paper (arXiv 2403.16341):

* residual families and the problem statement ``f(u, theta) = 0`` (Sec. 2),
* Jacobians by forward-mode dual numbers, one JVP per column (Sec. 2.4),
* LU with partial pivoting, LAPACK getrf pivot rule (Sec. 3.2 small dense LU),
* Newton-Raphson (Sec. 2.1), Armijo backtracking (Sec. 2.2.1), Powell dogleg
  trust region (Sec. 2.2.2), the Potra-Ptak two-step scheme (Sec. 2.1),
* the first-order part of the default poly-algorithm (Sec. 3.2): the three
  methods above in turn, each from the starting point, until one succeeds,
* sensitivities at a solution by the implicit function theorem (Sec. 2.3),
  tangent and adjoint forms.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline``
leg may import this package.  It shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nls_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CUBIC, TANH, ROSENBROCK, PAPER = 0, 1, 2, 3
SQUARE = 9  # oracle-only family: F_i = u_i^2 - p_i, the worked example of Sec. 2.3
NEWTON, ARMIJO, DOGLEG, POLY, POTRA_PTAK = 0, 1, 2, 3, 4
RC_SUCCESS, RC_MAXITERS, RC_SINGULAR, RC_NONFINITE, RC_LINESEARCH_FAILED, RC_TR_COLLAPSED = range(6)

# trace columns (mirror of the OR_TR_* enum in nls_oracle.h)
TRACE_FIELDS = [
    "k", "finf", "merit", "merit_before", "alpha", "delta", "step", "pred", "ared",
    "gnorm", "cauchy", "kind", "accepted", "newton_norm",
]

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


# Build variants.  "plain" is the oracle.  The others are rounding-level
# perturbations of the same arithmetic, used only to tell which systems are
# sensitive to rounding: "fma" is the source compiled with multiply-add
# contraction; "jitter1" and "jitter2" scale every step componentwise by
# 1 +- n 2^-53 (the rounding error of a length-n inner product), in two
# complementary up/down patterns, so that the whole trajectory is perturbed
# and not only its start; "pairwise" adds the merit ||F||^2 and the dogleg's
# inner products as a balanced tree instead of in index order.
VARIANTS = {
    "plain": ("liboracle.so", []),
    "fma": ("liboracle_fma.so", ["-mfma", "-ffp-contract=fast"]),
    "jitter1": ("liboracle_jitter1.so", ["-DOR_JITTER=1"]),
    "jitter2": ("liboracle_jitter2.so", ["-DOR_JITTER=2"]),
    "pairwise": ("liboracle_pairwise.so", ["-DOR_PAIRWISE"]),
}


def build(force: bool = False, variant: str = "plain") -> str:
    """Compile the oracle library with gcc (plain: no contraction, no fast-math)."""
    name, extra = VARIANTS[variant]
    out = os.path.join(_HERE, name)
    if (not force and os.path.exists(out)
            and os.path.getmtime(out) >= os.path.getmtime(_SRC)
            and os.path.getmtime(out) >= os.path.getmtime(os.path.join(_HERE, "nls_oracle.h"))):
        return out
    tmp = out + ".tmp%d" % os.getpid()
    contract = "-ffp-contract=fast" in extra
    flags = [f for f in CFLAGS if not (contract and f == "-ffp-contract=off")]
    cmd = ["gcc", *flags, *extra, "-o", tmp, _SRC, "-lm", "-lpthread"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


class _Opts(ctypes.Structure):
    _fields_ = [
        ("armijo_c", ctypes.c_double),
        ("armijo_rho", ctypes.c_double),
        ("armijo_max_halvings", ctypes.c_int32),
        ("tr_delta0", ctypes.c_double),
        ("tr_delta_max", ctypes.c_double),
        ("tr_eta1", ctypes.c_double),
        ("tr_eta2", ctypes.c_double),
        ("tr_expand", ctypes.c_double),
        ("tr_shrink", ctypes.c_double),
        ("tr_collapse", ctypes.c_double),
    ]


class _Result(ctypes.Structure):
    _fields_ = [
        ("retcode", ctypes.c_int32),
        ("iters", ctypes.c_int32),
        ("nfev", ctypes.c_int32),
        ("njev", ctypes.c_int32),
        ("fnorm_inf", ctypes.c_double),
    ]


_libs = {}


def lib(variant: str = "plain"):
    if variant not in _libs:
        # NLS_ORACLE_LIB points the pins at another build of the oracle (the
        # mutation test plants mistakes in a copy and checks the pins fail)
        path = os.environ.get("NLS_ORACLE_LIB") if variant == "plain" else None
        _lib = ctypes.CDLL(path or build(variant=variant))
        _libs[variant] = _lib
        P = ctypes.c_void_p
        _lib.or_default_opts.argtypes = [ctypes.POINTER(_Opts)]
        _lib.or_nparams.argtypes = [ctypes.c_int, ctypes.c_int]
        _lib.or_nparams.restype = ctypes.c_int
        for name in ("or_residual", "or_residual_dual_value", "or_jacobian"):
            getattr(_lib, name).argtypes = [ctypes.c_int, ctypes.c_int, P, P, P]
        _lib.or_lu.argtypes = [ctypes.c_int, P, P]
        _lib.or_lu.restype = ctypes.c_int
        _lib.or_lu_solve.argtypes = [ctypes.c_int, P, P, P]
        _lib.or_solve_one.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P,
                                      ctypes.c_double, ctypes.c_int32, ctypes.POINTER(_Opts), P,
                                      P, ctypes.c_int32, P]
        _lib.or_solve_one.restype = _Result
        _lib.or_param_jacobian.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P]
        _lib.or_tangent.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P]
        _lib.or_tangent.restype = ctypes.c_int
        _lib.or_adjoint.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P]
        _lib.or_adjoint.restype = ctypes.c_int
        _lib.or_solve_batch.argtypes = [ctypes.c_int64, P, P, P, P, P, P, P, ctypes.c_double,
                                        ctypes.c_int32, ctypes.POINTER(_Opts), P, P, P, P, P, P,
                                        ctypes.c_int32]
    return _libs[variant]


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def default_opts() -> dict:
    o = _Opts()
    lib().or_default_opts(ctypes.byref(o))
    return {name: getattr(o, name) for name, _ in _Opts._fields_}


def _make_opts(opts: dict | None) -> _Opts:
    o = _Opts()
    lib().or_default_opts(ctypes.byref(o))
    for k, v in (opts or {}).items():
        setattr(o, k, v)
    return o


def nparams(family: int, n: int) -> int:
    return lib().or_nparams(family, n)


def residual(family: int, p, u) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    F = np.empty_like(u)
    lib().or_residual(family, u.size, _ptr(p), _ptr(u), _ptr(F))
    return F


def residual_dual_value(family: int, p, u) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    F = np.empty_like(u)
    lib().or_residual_dual_value(family, u.size, _ptr(p), _ptr(u), _ptr(F))
    return F


def jacobian(family: int, p, u) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    J = np.empty((u.size, u.size))
    lib().or_jacobian(family, u.size, _ptr(p), _ptr(u), _ptr(J))
    return J


def param_jacobian(family: int, p, u) -> np.ndarray:
    """dF/dtheta (n x P) at (u, theta), from forward-mode duals on the parameters."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    Jp = np.empty((u.size, max(p.size, 0)))
    lib().or_param_jacobian(family, u.size, _ptr(p), _ptr(u), _ptr(Jp) if Jp.size else None)
    return Jp


def tangent(family: int, p, u, v):
    """(rc, du): du = -J^{-1} (dF/dtheta) v at the solution u (Sec. 2.3)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    du = np.empty_like(u)
    rc = lib().or_tangent(family, u.size, _ptr(p), _ptr(u), _ptr(v), _ptr(du))
    return rc, du


def adjoint(family: int, p, u, w):
    """(rc, lambda, grad): lambda = J^{-T} w, grad = -(dF/dtheta)^T lambda (Sec. 2.3)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    lam = np.empty_like(u)
    grad = np.empty_like(p)
    rc = lib().or_adjoint(family, u.size, _ptr(p), _ptr(u), _ptr(w), _ptr(lam), _ptr(grad))
    return rc, lam, grad


def lu(a):
    """Returns (lu, piv, info); info = 0 or the 1-based step of a zero/non-finite pivot."""
    a = np.array(a, dtype=np.float64, order="C", copy=True)
    n = a.shape[0]
    piv = np.zeros(n, dtype=np.int32)
    info = lib().or_lu(n, _ptr(a), _ptr(piv))
    return a, piv, info


def lu_solve(lu_, piv, b) -> np.ndarray:
    lu_ = np.ascontiguousarray(lu_, dtype=np.float64)
    piv = np.ascontiguousarray(piv, dtype=np.int32)
    x = np.array(b, dtype=np.float64, copy=True)
    lib().or_lu_solve(lu_.shape[0], _ptr(lu_), _ptr(piv), _ptr(x))
    return x


def solve_one(family: int, alg: int, p, u0, abstol: float = 1e-10, maxiters: int = 100,
              opts: dict | None = None, trace_cap: int = 0):
    """Solve one system.  Returns dict(u, retcode, iters, nfev, njev, fnorm_inf[, trace])."""
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    u = np.empty_like(u0)
    o = _make_opts(opts)
    tr = np.full((max(trace_cap, 0), len(TRACE_FIELDS)), np.nan)
    tlen = np.zeros(1, dtype=np.int32)
    r = lib().or_solve_one(family, u0.size, alg, _ptr(p), _ptr(u0), float(abstol), int(maxiters),
                           ctypes.byref(o), _ptr(u), _ptr(tr) if trace_cap > 0 else None,
                           int(trace_cap), _ptr(tlen))
    out = dict(u=u, retcode=r.retcode, iters=r.iters, nfev=r.nfev, njev=r.njev,
               fnorm_inf=r.fnorm_inf)
    if trace_cap > 0:
        out["trace"] = {name: tr[: tlen[0], i].copy() for i, name in enumerate(TRACE_FIELDS)}
    return out


def solve_batch(family, n, alg, params, p_off, u0, u_off, abstol: float, maxiters: int,
                opts: dict | None = None, nthreads: int = 1, variant: str = "plain") -> dict:
    """Batch solve.  family/n/alg: uint8[M]; p_off/u_off: int64[M+1] prefix offsets."""
    family = np.ascontiguousarray(family, dtype=np.uint8)
    n = np.ascontiguousarray(n, dtype=np.uint8)
    alg = np.ascontiguousarray(alg, dtype=np.uint8)
    params = np.ascontiguousarray(params, dtype=np.float64)
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    p_off = np.ascontiguousarray(p_off, dtype=np.int64)
    u_off = np.ascontiguousarray(u_off, dtype=np.int64)
    M = family.size
    u = np.empty_like(u0)
    fnorm = np.empty(M)
    iters = np.empty(M, dtype=np.int32)
    rc = np.empty(M, dtype=np.int32)
    nfev = np.empty(M, dtype=np.int32)
    njev = np.empty(M, dtype=np.int32)
    o = _make_opts(opts)
    lib(variant).or_solve_batch(M, _ptr(family), _ptr(n), _ptr(alg), _ptr(params), _ptr(p_off),
                         _ptr(u0), _ptr(u_off), float(abstol), int(maxiters), ctypes.byref(o),
                         _ptr(u), _ptr(fnorm), _ptr(iters), _ptr(rc), _ptr(nfev), _ptr(njev),
                         int(nthreads))
    return dict(u=u, fnorm_inf=fnorm, iters=iters, retcode=rc, nfev=nfev, njev=njev)
