"""Seeded synthetic inputs for the batched nonlinear solver.

This module only *draws* inputs (numpy ``Generator(PCG64(seed))``); it holds
none of the solver's arithmetic, and both the GPU path and the CPU oracle
consume what it produces.

Parameter packing per system (row-major ``A`` first):

* CUBIC       ``[A (N*N), b (N)]``           F_i = sum_j A_ij u_j + 0.1 u_i^3 - b_i
* TANH        ``[A (N*N), b (N), beta]``     F_i = sum_j A_ij tanh(u_j) + beta u_i - b_i
* ROSENBROCK  ``[]``                         generalized Rosenbrock (Sec. 2.2.1)
* PAPER       ``[a, b, c]``                  workflow example of Sec. 3 (N = 2)

The paper has no public inputs for this path; the workloads below are
synthetic stand-ins with the sizes and value distributions of the five
benchmark configurations (batch sizes, N mix, families, algorithms).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

CUBIC, TANH, ROSENBROCK, PAPER = 0, 1, 2, 3
NEWTON, ARMIJO, DOGLEG, POLY, POTRA_PTAK = 0, 1, 2, 3, 4
PREC_FP64, PREC_FP32_INNER = 0, 1

SEED_BASE = 20240316
NMAX = 64

CFG4_NS = np.array([2, 3, 4, 6, 8, 12, 16, 24, 32])
CFG4_WEIGHTS = np.array([0.2, 0.15, 0.15, 0.1, 0.15, 0.1, 0.08, 0.04, 0.03])


def nparams(family: int, n: int) -> int:
    if family == CUBIC:
        return n * n + n
    if family == TANH:
        return n * n + n + 1
    if family == ROSENBROCK:
        return 0
    if family == PAPER:
        return 3
    raise ValueError("unknown family %r" % family)


@dataclasses.dataclass
class Batch:
    """A batch of independent systems in the library's host layout."""
    family: np.ndarray       # uint8[M]
    n: np.ndarray            # uint8[M]
    alg: np.ndarray          # uint8[M]
    params: np.ndarray       # float64[p_off[-1]]
    p_off: np.ndarray        # int64[M+1]
    u0: np.ndarray           # float64[u_off[-1]]
    u_off: np.ndarray        # int64[M+1]
    abstol: float = 1e-10
    maxiters: int = 100
    precision: int = PREC_FP64
    name: str = ""

    @property
    def M(self) -> int:
        return int(self.family.size)

    def uniform(self):
        """(family, n, alg) if every system shares them, else None."""
        if self.M == 0:
            return None
        f, n, a = int(self.family[0]), int(self.n[0]), int(self.alg[0])
        if (self.family == f).all() and (self.n == n).all() and (self.alg == a).all():
            return f, n, a
        return None

    def system(self, s: int):
        """(family, n, alg, params, u0) of system s."""
        return (int(self.family[s]), int(self.n[s]), int(self.alg[s]),
                self.params[self.p_off[s]:self.p_off[s + 1]], self.u0[self.u_off[s]:self.u_off[s + 1]])

    def subset(self, idx) -> "Batch":
        """A new batch holding the systems ``idx`` (copied, re-packed)."""
        idx = np.asarray(idx, dtype=np.int64)
        fam, n, alg = self.family[idx], self.n[idx], self.alg[idx]
        plen = self.p_off[idx + 1] - self.p_off[idx]
        ulen = self.u_off[idx + 1] - self.u_off[idx]
        p_off = np.zeros(idx.size + 1, dtype=np.int64)
        u_off = np.zeros(idx.size + 1, dtype=np.int64)
        np.cumsum(plen, out=p_off[1:])
        np.cumsum(ulen, out=u_off[1:])
        params = _gather(self.params, self.p_off, idx, p_off)
        u0 = _gather(self.u0, self.u_off, idx, u_off)
        return Batch(fam, n, alg, params, p_off, u0, u_off, self.abstol, self.maxiters,
                     self.precision, self.name + "[subset]")


def _gather(arr: np.ndarray, off: np.ndarray, idx: np.ndarray, new_off: np.ndarray) -> np.ndarray:
    """The spans arr[off[s]:off[s+1]] of the systems idx, back to back (new_off:
    their prefix offsets)."""
    lens = off[idx + 1] - off[idx]
    shift = np.repeat(off[idx] - new_off[:-1], lens)
    return arr[np.arange(new_off[-1], dtype=np.int64) + shift] if idx.size else np.zeros(0)


def homogeneous(family: int, n: int, alg: int, params2d: np.ndarray, u02d: np.ndarray,
                abstol: float, maxiters: int, precision: int = PREC_FP64, name: str = "") -> Batch:
    M = u02d.shape[0]
    P = nparams(family, n)
    params2d = np.ascontiguousarray(params2d, dtype=np.float64).reshape(M, P)
    u02d = np.ascontiguousarray(u02d, dtype=np.float64).reshape(M, n)
    return Batch(
        family=np.full(M, family, dtype=np.uint8), n=np.full(M, n, dtype=np.uint8),
        alg=np.full(M, alg, dtype=np.uint8), params=params2d.reshape(-1),
        p_off=np.arange(M + 1, dtype=np.int64) * P, u0=u02d.reshape(-1),
        u_off=np.arange(M + 1, dtype=np.int64) * n, abstol=abstol, maxiters=maxiters,
        precision=precision, name=name)


def concat(batches) -> Batch:
    """Concatenate batches (systems kept in order)."""
    batches = list(batches)
    fam = np.concatenate([b.family for b in batches])
    n = np.concatenate([b.n for b in batches])
    alg = np.concatenate([b.alg for b in batches])
    params = np.concatenate([b.params for b in batches])
    u0 = np.concatenate([b.u0 for b in batches])
    plen = np.concatenate([np.diff(b.p_off) for b in batches])
    ulen = np.concatenate([np.diff(b.u_off) for b in batches])
    p_off = np.zeros(fam.size + 1, dtype=np.int64)
    u_off = np.zeros(fam.size + 1, dtype=np.int64)
    np.cumsum(plen, out=p_off[1:])
    np.cumsum(ulen, out=u_off[1:])
    b0 = batches[0]
    return Batch(fam, n, alg, params, p_off, u0, u_off, b0.abstol, b0.maxiters, b0.precision,
                 "+".join(b.name for b in batches))


# --------------------------------------------------------------------------
# parameter draws (fixed order: A (via G), then b, then beta, then u0)
# --------------------------------------------------------------------------
def cubic_params(rng: np.random.Generator, M: int, n: int) -> np.ndarray:
    """A = 4 I + 0.5 G with G_ij ~ N(0,1); b ~ U(-1, 1)."""
    G = rng.standard_normal((M, n, n))
    A = 0.5 * G
    A[:, np.arange(n), np.arange(n)] += 4.0
    b = rng.uniform(-1.0, 1.0, (M, n))
    return np.concatenate([A.reshape(M, n * n), b], axis=1)


def tanh_params(rng: np.random.Generator, M: int, n: int) -> np.ndarray:
    """A_ij ~ N(0,1)/sqrt(N); b ~ U(-2, 2); beta ~ U(0.05, 0.5)."""
    A = rng.standard_normal((M, n, n)) / math.sqrt(n)
    b = rng.uniform(-2.0, 2.0, (M, n))
    beta = rng.uniform(0.05, 0.5, (M, 1))
    return np.concatenate([A.reshape(M, n * n), b, beta], axis=1)


def _u0_for(rng, family: int, M: int, n: int) -> np.ndarray:
    if family == CUBIC:
        return rng.uniform(-3.0, 3.0, (M, n))
    return rng.uniform(-4.0, 4.0, (M, n))


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------
def config(k: int, M: int | None = None, seed: int | None = None,
           precision: int = PREC_FP64) -> Batch:
    """Workload k (1..4) at its full size, or with M systems for parity cases."""
    seed = SEED_BASE + k if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    if k == 1:
        # 1,024 systems, N = 4, cubic, u0 = 0, Newton, abstol 1e-10, maxiters 50
        M = 1024 if M is None else M
        p = cubic_params(rng, M, 4)
        u0 = np.zeros((M, 4))
        return homogeneous(CUBIC, 4, NEWTON, p, u0, 1e-10, 50, precision, "cubic-n4-newton")
    if k == 2:
        # 1,048,576 systems, N = 8, cubic, u0 ~ U(-3, 3), Newton + Armijo backtracking
        M = 1 << 20 if M is None else M
        p = cubic_params(rng, M, 8)
        u0 = rng.uniform(-3.0, 3.0, (M, 8))
        return homogeneous(CUBIC, 8, ARMIJO, p, u0, 1e-10, 100, precision, "cubic-n8-armijo")
    if k == 3:
        # 262,144 systems, N = 16, tanh, u0 ~ U(-4, 4), Powell dogleg, radius 1
        M = 1 << 18 if M is None else M
        p = tanh_params(rng, M, 16)
        u0 = rng.uniform(-4.0, 4.0, (M, 16))
        return homogeneous(TANH, 16, DOGLEG, p, u0, 1e-10, 100, precision, "tanh-n16-dogleg")
    if k == 4:
        # 500,000 systems, N from the weighted set, family and algorithm 50/50 each.
        # Choices are drawn first (N, then family, then algorithm), then the
        # parameters group by group in ascending (N, family) order.
        M = 500_000 if M is None else M
        ns = rng.choice(CFG4_NS, size=M, p=CFG4_WEIGHTS).astype(np.uint8)
        fam = rng.integers(0, 2, size=M).astype(np.uint8)          # 0 cubic, 1 tanh
        alg = np.where(rng.integers(0, 2, size=M) == 0, ARMIJO, DOGLEG).astype(np.uint8)
        plen = np.array([nparams(int(f), int(n)) for f, n in zip(fam, ns)], dtype=np.int64) \
            if M < 4096 else _plen_vec(fam, ns)
        p_off = np.zeros(M + 1, dtype=np.int64)
        np.cumsum(plen, out=p_off[1:])
        u_off = np.zeros(M + 1, dtype=np.int64)
        np.cumsum(ns.astype(np.int64), out=u_off[1:])
        params = np.empty(p_off[-1])
        u0 = np.empty(u_off[-1])
        for n in CFG4_NS:
            for f in (CUBIC, TANH):
                idx = np.nonzero((ns == n) & (fam == f))[0]
                if idx.size == 0:
                    continue
                P = nparams(f, int(n))
                pp = cubic_params(rng, idx.size, int(n)) if f == CUBIC else tanh_params(rng, idx.size, int(n))
                uu = _u0_for(rng, f, idx.size, int(n))
                pidx = p_off[idx][:, None] + np.arange(P)[None, :]
                uidx = u_off[idx][:, None] + np.arange(int(n))[None, :]
                params[pidx] = pp
                u0[uidx] = uu
        return Batch(fam, ns, alg, params, p_off, u0, u_off, 1e-10, 100, precision, "mixed-uneven")
    raise ValueError("workload %r" % k)


def _plen_vec(fam: np.ndarray, ns: np.ndarray) -> np.ndarray:
    n = ns.astype(np.int64)
    return n * n + n + (fam == TANH).astype(np.int64)


@dataclasses.dataclass
class Request:
    """One serving request: a homogeneous batch and its arrival time (s)."""
    rid: int
    arrival: float
    batch: Batch


def serving_requests(count: int, rate_hz: float, seed: int = SEED_BASE * 100,
                     max_systems: int = 65536, n_range=(2, 64),
                     precision: int = PREC_FP32_INNER) -> list:
    """Poisson arrivals; request size log-uniform on [1, max_systems]; N ~ U{lo..hi}
    per request; family 50/50 (cubic with Newton+Armijo, tanh with dogleg).
    Request r draws its payload from seed ``seed + r``."""
    arr_rng = np.random.Generator(np.random.PCG64(seed - 1))
    gaps = arr_rng.exponential(1.0 / rate_hz, size=count) if rate_hz > 0 else np.zeros(count)
    t = np.cumsum(gaps)
    out = []
    for r in range(count):
        rng = np.random.Generator(np.random.PCG64(seed + r))
        size = int(min(max_systems, math.floor(math.exp(rng.uniform(0.0, math.log(max_systems + 1))))))
        size = max(1, size)
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        fam = int(rng.integers(0, 2))
        if fam == CUBIC:
            p = cubic_params(rng, size, n)
            u0 = rng.uniform(-3.0, 3.0, (size, n))
            b = homogeneous(CUBIC, n, ARMIJO, p, u0, 1e-10, 100, precision, "req%d" % r)
        else:
            p = tanh_params(rng, size, n)
            u0 = rng.uniform(-4.0, 4.0, (size, n))
            b = homogeneous(TANH, n, DOGLEG, p, u0, 1e-10, 100, precision, "req%d" % r)
        out.append(Request(r, float(t[r]), b))
    return out


# --------------------------------------------------------------------------
# structured test families (edge cases and closed-form instances)
# --------------------------------------------------------------------------
def separable_cubic(M: int, n: int, seed: int, alg: int = NEWTON) -> Batch:
    """Diagonal A with a_ii ~ U(0.5, 5): every component solves 0.1u^3 + a u - b = 0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.uniform(0.5, 5.0, (M, n))
    A = np.zeros((M, n, n))
    A[:, np.arange(n), np.arange(n)] = a
    b = rng.uniform(-5.0, 5.0, (M, n))
    u0 = rng.uniform(-3.0, 3.0, (M, n))
    p = np.concatenate([A.reshape(M, n * n), b], axis=1)
    return homogeneous(CUBIC, n, alg, p, u0, 1e-12, 100, name="separable-cubic")


def separable_tanh(M: int, n: int, seed: int, alg: int = DOGLEG) -> Batch:
    """Diagonal A with a_ii > -beta: each component a tanh(u) + beta u = b has one root."""
    rng = np.random.Generator(np.random.PCG64(seed))
    beta = rng.uniform(0.2, 1.0, (M, 1))
    a = rng.uniform(-0.15, 2.0, (M, n))
    A = np.zeros((M, n, n))
    A[:, np.arange(n), np.arange(n)] = a
    b = rng.uniform(-2.0, 2.0, (M, n))
    u0 = rng.uniform(-2.0, 2.0, (M, n))
    p = np.concatenate([A.reshape(M, n * n), b, beta], axis=1)
    return homogeneous(TANH, n, alg, p, u0, 1e-12, 200, name="separable-tanh")


def no_root_tanh(M: int, n: int, seed: int, alg: int = ARMIJO) -> Batch:
    """beta = 0 and b_1 = sum_j |A_1j| + 1: |F_1| >= 1 everywhere, so no root exists."""
    rng = np.random.Generator(np.random.PCG64(seed))
    A = rng.standard_normal((M, n, n)) / math.sqrt(n)
    b = rng.uniform(-2.0, 2.0, (M, n))
    b[:, 0] = np.abs(A[:, 0, :]).sum(axis=1) + 1.0
    beta = np.zeros((M, 1))
    u0 = rng.uniform(-4.0, 4.0, (M, n))
    p = np.concatenate([A.reshape(M, n * n), b, beta], axis=1)
    return homogeneous(TANH, n, alg, p, u0, 1e-10, 30, name="no-root-tanh")


def singular_cubic(M: int, n: int, alg: int = NEWTON) -> Batch:
    """A = 0, u0 = 0, b != 0: J(u0) = 0, so the first factorisation is singular."""
    A = np.zeros((M, n * n))
    b = np.ones((M, n))
    p = np.concatenate([A, b], axis=1)
    return homogeneous(CUBIC, n, alg, p, np.zeros((M, n)), 1e-10, 20, name="singular-cubic")


def rosenbrock(M: int, n: int, seed: int, alg: int = NEWTON, u0: str = "uniform") -> Batch:
    """Generalized Rosenbrock; u0 ~ U(0,1) ("uniform") or (-1.2, 1, ..., 1) ("paper")."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if u0 == "paper":
        x = np.ones((M, n))
        x[:, 0] = -1.2
    else:
        x = rng.uniform(0.0, 1.0, (M, n))
    return homogeneous(ROSENBROCK, n, alg, np.zeros((M, 0)), x, 1e-8, 1000, name="rosenbrock")


def paper_gpu_workload(alg: int = NEWTON) -> Batch:
    """The batch of the paper's GPU kernel example (Sec. 3.3): 1,024 generalized
    Rosenbrock systems of 10 unknowns, each started from U(0,1)^10, Newton."""
    b = rosenbrock(1024, 10, seed=SEED_BASE + 6, alg=alg)
    b.name = "paper-gpu-rosenbrock"
    return b


def paper_example(M: int, seed: int, alg: int = NEWTON) -> Batch:
    """Workflow example of Sec. 3: p = (3, 7, 18) for system 0, random nearby p otherwise."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = np.tile(np.array([3.0, 7.0, 18.0]), (M, 1))
    if M > 1:
        p[1:] += rng.uniform(-0.5, 0.5, (M - 1, 3))
    u0 = np.zeros((M, 2))
    if M > 1:
        u0[1:] = rng.uniform(-0.3, 0.3, (M - 1, 2))
    return homogeneous(PAPER, 2, alg, p, u0, 1e-10, 100, name="paper-example")
