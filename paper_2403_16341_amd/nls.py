"""Python binding of the C ABI in ``include/nls.h`` (argument marshalling only).

Every step of the solve runs in the HIP library ``_lib/libnls.so``; this module
only converts arguments.  torch is imported before the library is loaded so
that both share one HIP runtime, and torch tensors provide device memory and
the stream the work is enqueued on.  If the library is missing, loading fails
with an error: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

import torch  # noqa: F401  (must precede the library: one HIP runtime per process)

from . import inputs as _inputs

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libnls.so")

OK, PENDING = 0, 1
E_INVALID, E_NOMEM, E_DEVICE, E_NOTFOUND = -1, -2, -3, -4
FAMILY_CUBIC, FAMILY_TANH, FAMILY_ROSENBROCK, FAMILY_PAPER_EXAMPLE = 0, 1, 2, 3
ALG_NEWTON, ALG_NEWTON_ARMIJO, ALG_DOGLEG, ALG_POLY, ALG_POTRA_PTAK = 0, 1, 2, 3, 4
PREC_FP64, PREC_FP32_INNER = 0, 1
MEM_HOST, MEM_DEVICE = 0, 1
RC_SUCCESS, RC_MAXITERS, RC_SINGULAR, RC_NONFINITE, RC_LINESEARCH_FAILED, RC_TR_COLLAPSED, RC_INVALID = range(7)
CTX_THREADSAFE = 1
CTX_AUTOTUNE = 2

# every symbol include/nls.h declares
EXPORTS = ("nls_create", "nls_destroy", "nls_solve_batch", "nls_query", "nls_validate",
           "nls_last_error", "nls_get_mapping", "nls_nparams", "nls_default_options", "nls_abi_version",
           "nls_server_create", "nls_server_submit", "nls_server_poll", "nls_server_stats_get",
           "nls_server_destroy", "nls_sensitivity_batch", "nls_solve_batch_noalloc")
# fixed limits of nls_solve_batch_noalloc (include/nls.h)
NOALLOC_MAX_CHAIN_SYSTEMS, NOALLOC_MAX_CHAIN_UNKNOWNS = 65536, 1048576
SENS_TANGENT, SENS_ADJOINT = 0, 1


class ContextDesc(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("mem_budget_bytes", ctypes.c_uint64), ("stream", ctypes.c_void_p)]


class AlgOptions(ctypes.Structure):
    _fields_ = [("armijo_c", ctypes.c_double), ("armijo_rho", ctypes.c_double),
                ("armijo_max_halvings", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("tr_delta0", ctypes.c_double), ("tr_delta_max", ctypes.c_double),
                ("tr_eta1", ctypes.c_double), ("tr_eta2", ctypes.c_double),
                ("tr_expand", ctypes.c_double), ("tr_shrink", ctypes.c_double),
                ("tr_collapse", ctypes.c_double)]


class Batch(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int64),
                ("family", ctypes.c_void_p), ("n", ctypes.c_void_p), ("alg", ctypes.c_void_p),
                ("family_all", ctypes.c_uint8), ("n_all", ctypes.c_uint8),
                ("alg_all", ctypes.c_uint8), ("precision", ctypes.c_uint8),
                ("mem_kind", ctypes.c_uint32), ("maxiters", ctypes.c_int32),
                ("abstol", ctypes.c_double),
                ("params", ctypes.c_void_p), ("p_offset", ctypes.c_void_p),
                ("u0", ctypes.c_void_p), ("u_offset", ctypes.c_void_p),
                ("opts", ctypes.POINTER(AlgOptions))]


class Results(ctypes.Structure):
    _fields_ = [("u", ctypes.c_void_p), ("fnorm_inf", ctypes.c_void_p), ("iters", ctypes.c_void_p),
                ("retcode", ctypes.c_void_p), ("nfev", ctypes.c_void_p), ("njev", ctypes.c_void_p)]


class SensBatch(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int64), ("family", ctypes.c_void_p), ("n", ctypes.c_void_p),
                ("family_all", ctypes.c_uint8), ("n_all", ctypes.c_uint8), ("mode", ctypes.c_uint8),
                ("reserved", ctypes.c_uint8), ("mem_kind", ctypes.c_uint32),
                ("params", ctypes.c_void_p), ("p_offset", ctypes.c_void_p),
                ("u", ctypes.c_void_p), ("u_offset", ctypes.c_void_p), ("seed", ctypes.c_void_p)]


class SensResults(ctypes.Structure):
    _fields_ = [("out", ctypes.c_void_p), ("lambda_", ctypes.c_void_p), ("status", ctypes.c_void_p)]


class TicketInfo(ctypes.Structure):
    _fields_ = [("done", ctypes.c_int32), ("status", ctypes.c_int32), ("gpu_ms", ctypes.c_double),
                ("systems", ctypes.c_int64)]


class ServerDesc(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("streams", ctypes.c_int32),
                ("mem_budget_bytes", ctypes.c_uint64), ("max_inflight", ctypes.c_int32),
                ("max_admit", ctypes.c_int32)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("status", ctypes.c_int32), ("merged", ctypes.c_int32),
                ("systems", ctypes.c_int64), ("t_submit_ms", ctypes.c_double),
                ("t_admit_ms", ctypes.c_double), ("t_done_ms", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_int64), ("inflight_launches", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("resident_bytes", ctypes.c_uint64), ("peak_resident_bytes", ctypes.c_uint64),
                ("budget_bytes", ctypes.c_uint64)]


class NLSError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("nls error %d: %s" % (code, msg))
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """Load ``libnls.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("HIP library %s is missing: build it with __graft_entry__.build() "
                           "(there is no CPU fallback)" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH, mode=ctypes.RTLD_GLOBAL)
    P = ctypes.c_void_p
    L.nls_create.argtypes = [ctypes.POINTER(ContextDesc), ctypes.POINTER(P)]
    L.nls_create.restype = ctypes.c_int
    L.nls_destroy.argtypes = [P]
    L.nls_destroy.restype = ctypes.c_int
    L.nls_solve_batch.argtypes = [P, ctypes.POINTER(Batch), ctypes.POINTER(Results),
                                  ctypes.POINTER(ctypes.c_uint64)]
    L.nls_solve_batch.restype = ctypes.c_int
    L.nls_query.argtypes = [P, ctypes.c_uint64, ctypes.c_int32, ctypes.POINTER(TicketInfo)]
    L.nls_query.restype = ctypes.c_int
    L.nls_validate.argtypes = [ctypes.POINTER(Batch), ctypes.POINTER(ctypes.c_int64)]
    L.nls_validate.restype = ctypes.c_int
    L.nls_last_error.argtypes = [P]
    L.nls_last_error.restype = ctypes.c_char_p
    L.nls_get_mapping.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_int32)]
    L.nls_get_mapping.restype = ctypes.c_int
    L.nls_nparams.argtypes = [ctypes.c_int, ctypes.c_int]
    L.nls_nparams.restype = ctypes.c_int
    L.nls_default_options.argtypes = [ctypes.POINTER(AlgOptions)]
    L.nls_default_options.restype = None
    L.nls_abi_version.argtypes = []
    L.nls_abi_version.restype = ctypes.c_int
    L.nls_server_create.argtypes = [ctypes.POINTER(ServerDesc), ctypes.POINTER(P)]
    L.nls_server_create.restype = ctypes.c_int
    L.nls_server_submit.argtypes = [P, ctypes.POINTER(Batch), ctypes.POINTER(Results),
                                    ctypes.POINTER(ctypes.c_uint64)]
    L.nls_server_submit.restype = ctypes.c_int
    L.nls_server_poll.argtypes = [P, ctypes.c_int32, ctypes.POINTER(RequestInfo), ctypes.c_int32,
                                  ctypes.POINTER(ctypes.c_int32)]
    L.nls_server_poll.restype = ctypes.c_int
    L.nls_server_stats_get.argtypes = [P, ctypes.POINTER(ServerStats)]
    L.nls_server_stats_get.restype = ctypes.c_int
    L.nls_server_destroy.argtypes = [P]
    L.nls_server_destroy.restype = ctypes.c_int
    L.nls_sensitivity_batch.argtypes = [P, ctypes.POINTER(SensBatch), ctypes.POINTER(SensResults),
                                        ctypes.POINTER(ctypes.c_uint64)]
    L.nls_sensitivity_batch.restype = ctypes.c_int
    L.nls_solve_batch_noalloc.argtypes = [ctypes.POINTER(Batch), ctypes.POINTER(Results), P]
    L.nls_solve_batch_noalloc.restype = ctypes.c_int
    _lib = L
    return L


def last_error(ctx=None) -> str:
    return lib().nls_last_error(ctx).decode()


def default_options() -> AlgOptions:
    o = AlgOptions()
    lib().nls_default_options(ctypes.byref(o))
    return o


def make_options(**kw) -> AlgOptions:
    o = default_options()
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, torch.Tensor):
        return ctypes.c_void_p(x.data_ptr())
    if isinstance(x, np.ndarray):
        return x.ctypes.data_as(ctypes.c_void_p)
    raise TypeError(type(x))


def _host_u8(x, M):
    """uint8 host array of length M, or None for a scalar descriptor."""
    if x is None or np.isscalar(x):
        return None
    a = np.ascontiguousarray(x, dtype=np.uint8)
    assert a.size == M
    return a


class Context:
    """An ``nls_context`` on one GPU, enqueuing on a torch stream."""

    def __init__(self, device: int = 0, stream: "torch.cuda.Stream | None" = None,
                 mem_budget_bytes: int = 0, flags: int = 0):
        L = lib()
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        d = ContextDesc(device, flags, mem_budget_bytes, ctypes.c_void_p(self.stream.cuda_stream))
        h = ctypes.c_void_p()
        rc = L.nls_create(ctypes.byref(d), ctypes.byref(h))
        if rc != OK:
            raise NLSError(rc, last_error(None))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().nls_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def mapping(self, family: int, n: int, alg: int, precision: int = PREC_FP64) -> int:
        """Lanes per system the context uses for a combination (0 = not tuned yet)."""
        v = ctypes.c_int32(0)
        rc = lib().nls_get_mapping(self.handle, family, n, alg, precision, ctypes.byref(v))
        if rc != OK:
            raise NLSError(rc, last_error(None))
        return v.value

    def error(self) -> str:
        return lib().nls_last_error(self.handle).decode()

    # --- raw submission ----------------------------------------------------
    def submit(self, *, count, family, n, alg, params, u0, p_offset=None, u_offset=None,
               abstol=1e-10, maxiters=100, precision=PREC_FP64, opts=None, mem_kind=MEM_DEVICE,
               out=None, keep=None):
        """Enqueue one batch; returns (ticket, out, keepalive).  ``family``/``n``/
        ``alg`` are ints (every system) or host arrays; ``params``/``u0`` and the
        arrays in ``out`` are device tensors (MEM_DEVICE) or numpy arrays (MEM_HOST)."""
        b = Batch()
        b.count = int(count)
        fa, na, aa = _host_u8(family, count), _host_u8(n, count), _host_u8(alg, count)
        b.family, b.n, b.alg = _ptr(fa), _ptr(na), _ptr(aa)
        b.family_all = 0 if fa is not None else int(family)
        b.n_all = 0 if na is not None else int(n)
        b.alg_all = 0 if aa is not None else int(alg)
        b.precision = int(precision)
        b.mem_kind = int(mem_kind)
        b.maxiters = int(maxiters)
        b.abstol = float(abstol)
        po = None if p_offset is None else np.ascontiguousarray(p_offset, dtype=np.int64)
        uo = None if u_offset is None else np.ascontiguousarray(u_offset, dtype=np.int64)
        b.params, b.u0 = _ptr(params), _ptr(u0)
        b.p_offset, b.u_offset = _ptr(po), _ptr(uo)
        if opts is not None:
            b.opts = ctypes.pointer(opts)
        r = Results(*[_ptr(out.get(k)) for k in ("u", "fnorm_inf", "iters", "retcode", "nfev", "njev")])
        t = ctypes.c_uint64(0)
        rc = lib().nls_solve_batch(self.handle, ctypes.byref(b), ctypes.byref(r), ctypes.byref(t))
        if rc != OK:
            raise NLSError(rc, self.error())
        return t.value, (fa, na, aa, po, uo, params, u0, keep)

    def submit_sensitivity(self, *, count, family, n, mode, params, u, seed, p_offset=None,
                           u_offset=None, mem_kind=MEM_DEVICE, out=None, lam=None, status=None):
        """Enqueue sensitivities of solved systems (tangent: du for direction
        ``seed``; adjoint: the gradient of seed . u* and, if ``lam`` is given,
        J^{-T} seed); returns (ticket, keepalive)."""
        b = SensBatch()
        b.count = int(count)
        fa, na = _host_u8(family, count), _host_u8(n, count)
        b.family, b.n = _ptr(fa), _ptr(na)
        b.family_all = 0 if fa is not None else int(family)
        b.n_all = 0 if na is not None else int(n)
        b.mode = int(mode)
        b.mem_kind = int(mem_kind)
        po = None if p_offset is None else np.ascontiguousarray(p_offset, dtype=np.int64)
        uo = None if u_offset is None else np.ascontiguousarray(u_offset, dtype=np.int64)
        b.params, b.u, b.seed = _ptr(params), _ptr(u), _ptr(seed)
        b.p_offset, b.u_offset = _ptr(po), _ptr(uo)
        r = SensResults(_ptr(out), _ptr(lam), _ptr(status))
        t = ctypes.c_uint64(0)
        rc = lib().nls_sensitivity_batch(self.handle, ctypes.byref(b), ctypes.byref(r), ctypes.byref(t))
        if rc != OK:
            raise NLSError(rc, self.error())
        return t.value, (fa, na, po, uo, params, u, seed, out, lam, status)

    def query(self, ticket: int, wait_ms: int = -1):
        info = TicketInfo()
        rc = lib().nls_query(self.handle, ctypes.c_uint64(ticket), int(wait_ms), ctypes.byref(info))
        if rc == PENDING:
            return None
        if rc != OK:
            raise NLSError(rc, self.error())
        return info

    # --- convenience -------------------------------------------------------
    def solve(self, batch: "DeviceBatch", out: dict | None = None, opts=None, wait: bool = True,
              precision: int | None = None):
        """Solve a DeviceBatch; returns the result dict (device tensors)."""
        out = out if out is not None else batch.alloc_results()
        t, keep = self.submit(
            count=batch.M, family=batch.family, n=batch.n, alg=batch.alg, params=batch.params,
            u0=batch.u0, p_offset=batch.p_offset, u_offset=batch.u_offset, abstol=batch.abstol,
            maxiters=batch.maxiters, precision=batch.precision if precision is None else precision,
            opts=opts, mem_kind=MEM_DEVICE, out=out)
        if wait:
            info = self.query(t, -1)
            out["gpu_ms"] = info.gpu_ms
        else:
            out["ticket"] = t
            out["_keep"] = keep
        return out


class DeviceBatch:
    """A batch whose payload (params, u0) lives in device memory."""

    def __init__(self, b: "_inputs.Batch", device="cuda"):
        self.M = b.M
        self.abstol, self.maxiters, self.precision = b.abstol, b.maxiters, b.precision
        uni = b.uniform()
        plen = np.diff(b.p_off)
        ulen = np.diff(b.u_off)
        packed = (b.p_off[0] == 0 and b.u_off[0] == 0)
        if uni is not None and packed and (plen == plen[0]).all() and (ulen == uni[1]).all():
            self.family, self.n, self.alg = uni
            self.p_offset = self.u_offset = None
        else:
            self.family, self.n, self.alg = b.family, b.n, b.alg
            self.p_offset, self.u_offset = b.p_off, b.u_off
        self.params = torch.from_numpy(np.ascontiguousarray(b.params)).to(device)
        self.u0 = torch.from_numpy(np.ascontiguousarray(b.u0)).to(device)
        if self.params.numel() == 0:
            self.params = torch.zeros(1, dtype=torch.float64, device=device)
        self.device = device

    def alloc_results(self) -> dict:
        dev = self.device
        return dict(u=torch.empty_like(self.u0), fnorm_inf=torch.empty(self.M, dtype=torch.float64, device=dev),
                    iters=torch.empty(self.M, dtype=torch.int32, device=dev),
                    retcode=torch.empty(self.M, dtype=torch.int32, device=dev),
                    nfev=torch.empty(self.M, dtype=torch.int32, device=dev),
                    njev=torch.empty(self.M, dtype=torch.int32, device=dev))


def solve_noalloc(batch: "DeviceBatch", out: dict | None = None, precision: int | None = None, opts=None,
                  stream: "torch.cuda.Stream | None" = None) -> dict:
    """Enqueue a uniform DeviceBatch through nls_solve_batch_noalloc on a torch
    stream (default: the current one) and return the result tensors; the work
    is stream-ordered, so synchronise the stream before reading them."""
    if not np.isscalar(batch.family) or batch.p_offset is not None:
        raise NLSError(E_INVALID, "nls_solve_batch_noalloc takes uniform, packed batches")
    out = out if out is not None else batch.alloc_results()
    st = stream if stream is not None else torch.cuda.current_stream()
    b = Batch()
    b.count = int(batch.M)
    b.family_all, b.n_all, b.alg_all = int(batch.family), int(batch.n), int(batch.alg)
    b.precision = int(batch.precision if precision is None else precision)
    b.mem_kind = MEM_DEVICE
    b.maxiters = int(batch.maxiters)
    b.abstol = float(batch.abstol)
    b.params, b.u0 = _ptr(batch.params), _ptr(batch.u0)
    if opts is not None:
        b.opts = ctypes.pointer(opts)
    r = Results(*[_ptr(out.get(k)) for k in ("u", "fnorm_inf", "iters", "retcode", "nfev", "njev")])
    rc = lib().nls_solve_batch_noalloc(ctypes.byref(b), ctypes.byref(r), ctypes.c_void_p(st.cuda_stream))
    if rc != OK:
        raise NLSError(rc, last_error(None))
    return out


def results_to_numpy(out: dict) -> dict:
    return {k: (v.cpu().numpy() if isinstance(v, torch.Tensor) else v) for k, v in out.items()
            if not k.startswith("_")}


def sensitivities(ctx: Context, b: "_inputs.Batch", u, seed, mode: int, mem_kind: int = MEM_DEVICE,
                  want_lambda: bool = True) -> dict:
    """Sensitivities of the systems of ``b`` at the solutions ``u`` (laid out
    like ``b.u0``) through the device (MEM_DEVICE) or host (MEM_HOST) payload
    path; returns numpy arrays out, lambda (adjoint), status and gpu_ms."""
    M = b.M
    uni = b.uniform()
    packed = M > 0 and uni is not None and b.p_off[0] == 0 and b.u_off[0] == 0 and \
        (np.diff(b.p_off) == nls_params(uni[0], uni[1])).all() and (np.diff(b.u_off) == uni[1]).all()
    fam, n = (uni[0], uni[1]) if packed else (b.family, b.n)
    po, uo = (None, None) if packed else (b.p_off, b.u_off)
    u = np.ascontiguousarray(u, dtype=np.float64)
    seed = np.ascontiguousarray(seed, dtype=np.float64)
    params = b.params if b.params.size else np.zeros(1)
    out_len = b.u0.size if mode == SENS_TANGENT else max(b.params.size, 1)
    adj = mode == SENS_ADJOINT and want_lambda
    if mem_kind == MEM_DEVICE:
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda(ctx.device)
        dp, du_, ds = dev(params), dev(u), dev(seed if seed.size else np.zeros(1))
        out = torch.full((out_len,), float("nan"), dtype=torch.float64, device="cuda")
        lam = torch.full((max(b.u0.size, 1),), float("nan"), dtype=torch.float64, device="cuda") if adj else None
        st = torch.full((max(M, 1),), -1, dtype=torch.int32, device="cuda")
        t, keep = ctx.submit_sensitivity(count=M, family=fam, n=n, mode=mode, params=dp, u=du_, seed=ds,
                                         p_offset=po, u_offset=uo, mem_kind=MEM_DEVICE, out=out, lam=lam,
                                         status=st)
        info = ctx.query(t, -1)
        res = dict(out=out.cpu().numpy(), status=st.cpu().numpy()[:M], gpu_ms=info.gpu_ms)
        if adj:
            res["lambda"] = lam.cpu().numpy()[: b.u0.size]
        return res
    out = np.full(out_len, np.nan)
    lam = np.full(max(b.u0.size, 1), np.nan) if adj else None
    st = np.full(max(M, 1), -1, dtype=np.int32)
    t, keep = ctx.submit_sensitivity(count=M, family=fam, n=n, mode=mode, params=params, u=u,
                                     seed=seed if seed.size else np.zeros(1), p_offset=po, u_offset=uo,
                                     mem_kind=MEM_HOST, out=out, lam=lam, status=st)
    info = ctx.query(t, -1)
    res = dict(out=out, status=st[:M], gpu_ms=info.gpu_ms)
    if adj:
        res["lambda"] = lam[: b.u0.size]
    return res


def solve_host(ctx: Context, b: "_inputs.Batch", precision: int | None = None, opts=None) -> dict:
    """Solve a host-memory batch through the MEM_HOST path (copies in and out)."""
    M = b.M
    out = dict(u=np.empty_like(b.u0), fnorm_inf=np.empty(M), iters=np.empty(M, np.int32),
               retcode=np.empty(M, np.int32), nfev=np.empty(M, np.int32), njev=np.empty(M, np.int32))
    params = b.params if b.params.size else np.zeros(1)
    t, _ = ctx.submit(count=M, family=b.family, n=b.n, alg=b.alg, params=params, u0=b.u0,
                      p_offset=b.p_off, u_offset=b.u_off, abstol=b.abstol, maxiters=b.maxiters,
                      precision=b.precision if precision is None else precision, opts=opts,
                      mem_kind=MEM_HOST, out=out)
    ctx.query(t, -1)
    return out


class Server:
    """An ``nls_server``: continuous batching of host-memory solve requests.

    ``submit`` queues a request (an ``inputs.Batch`` of one family, size and
    algorithm) and returns its id; the arrays of a request are held here until
    ``poll`` reports it, together with its results and host-clock stamps."""

    def __init__(self, device: int = 0, mem_budget_bytes: int = 1 << 30, streams: int = 4,
                 max_inflight: int = 0, max_admit: int = 0):
        L = lib()
        d = ServerDesc(device, streams, mem_budget_bytes, max_inflight, max_admit)
        h = ctypes.c_void_p()
        rc = L.nls_server_create(ctypes.byref(d), ctypes.byref(h))
        if rc != OK:
            raise NLSError(rc, last_error(None))
        self.handle = h
        self._live = {}

    def submit(self, b: "_inputs.Batch", precision: int | None = None, opts=None) -> int:
        M = b.M
        uni = b.uniform() if M else (FAMILY_CUBIC, 1, ALG_NEWTON)
        if uni is None:
            raise NLSError(E_INVALID, "server requests have one family, size and algorithm")
        fam, n, alg = uni
        P = nls_params(fam, n)
        packed = (np.array_equal(b.p_off, np.arange(M + 1) * P)
                  and np.array_equal(b.u_off, np.arange(M + 1) * n))
        po = None if packed else np.ascontiguousarray(b.p_off, dtype=np.int64)
        uo = None if packed else np.ascontiguousarray(b.u_off, dtype=np.int64)
        params = np.ascontiguousarray(b.params) if b.params.size else np.zeros(1)
        u0 = np.ascontiguousarray(b.u0)
        out = dict(u=u0.copy(), fnorm_inf=np.empty(M), iters=np.empty(M, np.int32),
                   retcode=np.empty(M, np.int32), nfev=np.empty(M, np.int32), njev=np.empty(M, np.int32))
        bb = Batch()
        bb.count = M
        bb.family_all, bb.n_all, bb.alg_all = fam, n, alg
        bb.precision = int(b.precision if precision is None else precision)
        bb.mem_kind = MEM_HOST
        bb.maxiters = int(b.maxiters)
        bb.abstol = float(b.abstol)
        bb.params, bb.u0 = _ptr(params), _ptr(u0)
        bb.p_offset, bb.u_offset = _ptr(po), _ptr(uo)
        if opts is not None:
            bb.opts = ctypes.pointer(opts)
        r = Results(*[_ptr(out[k]) for k in ("u", "fnorm_inf", "iters", "retcode", "nfev", "njev")])
        i = ctypes.c_uint64(0)
        rc = lib().nls_server_submit(self.handle, ctypes.byref(bb), ctypes.byref(r), ctypes.byref(i))
        if rc != OK:
            raise NLSError(rc, last_error(None))
        self._live[i.value] = (out, (params, u0, po, uo, opts))
        return i.value

    def poll(self, wait_ms: int = 0, max_out: int = 256) -> list:
        """Completed requests as (info dict, results dict), oldest completion first."""
        buf = (RequestInfo * max_out)()
        k = ctypes.c_int32(0)
        rc = lib().nls_server_poll(self.handle, int(wait_ms), buf, max_out, ctypes.byref(k))
        if rc != OK:
            raise NLSError(rc, last_error(None))
        done = []
        for j in range(k.value):
            x = buf[j]
            info = dict(id=x.id, status=x.status, merged=x.merged, systems=x.systems,
                        t_submit_ms=x.t_submit_ms, t_admit_ms=x.t_admit_ms, t_done_ms=x.t_done_ms)
            out, _keep = self._live.pop(x.id)
            done.append((info, out))
        return done

    def drain(self) -> list:
        """Wait for every outstanding request; returns them as ``poll`` does."""
        done = []
        while self._live:
            done += self.poll(-1)
        return done

    def stats(self) -> dict:
        st = ServerStats()
        lib().nls_server_stats_get(self.handle, ctypes.byref(st))
        return {name: getattr(st, name) for name, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "handle", None):
            lib().nls_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def nls_params(family: int, n: int) -> int:
    return lib().nls_nparams(family, n)
