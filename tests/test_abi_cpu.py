"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and host-side validation rejects bad batches."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def nls():
    from paper_2403_16341_amd import nls as _nls
    _nls.lib()
    return _nls


def test_header_declarations_are_exported(nls):
    hdr = open(os.path.join(ROOT, "include", "nls.h")).read()
    declared = set(re.findall(r"^\s*(?:int|void|const char\*)\s+(nls_\w+)\s*\(", hdr, re.M))
    assert declared == set(nls.EXPORTS)
    L = nls.lib()
    for name in declared:
        assert hasattr(L, name), name


def test_abi_constants(nls):
    L = nls.lib()
    assert L.nls_abi_version() == 1
    assert L.nls_nparams(nls.FAMILY_CUBIC, 8) == 72
    assert L.nls_nparams(nls.FAMILY_TANH, 16) == 16 * 16 + 17
    assert L.nls_nparams(nls.FAMILY_ROSENBROCK, 10) == 0
    assert L.nls_nparams(nls.FAMILY_PAPER_EXAMPLE, 2) == 3
    assert L.nls_nparams(nls.FAMILY_PAPER_EXAMPLE, 3) == -1
    assert L.nls_nparams(nls.FAMILY_CUBIC, 65) == -1
    o = nls.default_options()
    assert (o.armijo_c, o.armijo_rho, o.armijo_max_halvings) == (1e-4, 0.5, 10)
    assert (o.tr_delta0, o.tr_eta1, o.tr_eta2, o.tr_shrink) == (1.0, 1e-4, 0.75, 0.25)
    # struct layout matches the header (sizes)
    assert ctypes.sizeof(nls.Batch) == 8 + 8 * 3 + 4 + 4 + 4 + 4 + 8 * 5 + 8
    assert ctypes.sizeof(nls.AlgOptions) == 8 * 2 + 4 * 2 + 8 * 7


def _batch(nls, **kw):
    b = nls.Batch()
    u0 = np.zeros(64)
    p = np.zeros(64 * 80)
    b.count = kw.get("count", 4)
    b.family_all = kw.get("family", 0)
    b.n_all = kw.get("n", 4)
    b.alg_all = kw.get("alg", 0)
    b.precision = kw.get("precision", 0)
    b.mem_kind = kw.get("mem_kind", 0)
    b.maxiters = kw.get("maxiters", 10)
    b.abstol = kw.get("abstol", 1e-10)
    b.u0 = u0.ctypes.data_as(ctypes.c_void_p) if kw.get("u0", True) else None
    b.params = p.ctypes.data_as(ctypes.c_void_p) if kw.get("params", True) else None
    return b, (u0, p)


@pytest.mark.parametrize("bad,msg", [
    (dict(n=0), "n = 0"), (dict(n=65), "n = 65"), (dict(family=9), "family 9"),
    (dict(alg=5), "algorithm 5"), (dict(family=3, n=3), "family 3"), (dict(family=2, n=1), "family 2"),
    (dict(precision=2), "precision"), (dict(mem_kind=5), "mem_kind"), (dict(abstol=-1.0), "abstol"),
    (dict(abstol=float("nan")), "abstol"), (dict(maxiters=-1), "maxiters"), (dict(count=-1), "count"),
    (dict(u0=False), "u0"), (dict(params=False), "params"),
])
def test_validation_rejects(nls, bad, msg):
    b, keep = _batch(nls, **bad)
    fb = ctypes.c_int64(123)
    rc = nls.lib().nls_validate(ctypes.byref(b), ctypes.byref(fb))
    assert rc == nls.E_INVALID
    assert msg in nls.last_error()


def test_validation_accepts_and_reports_first_bad_system(nls):
    b, keep = _batch(nls)
    assert nls.lib().nls_validate(ctypes.byref(b), None) == nls.OK
    b.count = 0
    assert nls.lib().nls_validate(ctypes.byref(b), None) == nls.OK
    ns = np.array([4, 8, 70, 3], dtype=np.uint8)
    b, keep = _batch(nls)
    b.n = ns.ctypes.data_as(ctypes.c_void_p)
    fb = ctypes.c_int64(0)
    assert nls.lib().nls_validate(ctypes.byref(b), ctypes.byref(fb)) == nls.E_INVALID
    assert fb.value == 2 and "system 2" in nls.last_error()
    # offsets: spans shorter than the parameter count are rejected
    po = np.array([0, 20, 39, 60, 80], dtype=np.int64)
    b, keep = _batch(nls)
    b.p_offset = po.ctypes.data_as(ctypes.c_void_p)
    assert nls.lib().nls_validate(ctypes.byref(b), ctypes.byref(fb)) == nls.E_INVALID and fb.value == 1
    po = np.array([0, 25, 50, 75, 100], dtype=np.int64)       # gaps are fine
    b.p_offset = po.ctypes.data_as(ctypes.c_void_p)
    assert nls.lib().nls_validate(ctypes.byref(b), None) == nls.OK


def test_option_validation(nls):
    for field, val in (("armijo_c", 0.0), ("armijo_rho", 1.0), ("armijo_max_halvings", -1),
                       ("tr_delta0", 0.0), ("tr_eta1", 0.9), ("tr_shrink", 1.5), ("tr_expand", 0.5)):
        o = nls.default_options()
        setattr(o, field, val)
        b, keep = _batch(nls)
        b.opts = ctypes.pointer(o)
        assert nls.lib().nls_validate(ctypes.byref(b), None) == nls.E_INVALID, field


def test_context_calls_reject_null(nls):
    L = nls.lib()
    t = ctypes.c_uint64(0)
    assert L.nls_solve_batch(None, None, None, ctypes.byref(t)) == nls.E_INVALID
    assert L.nls_query(None, 1, 0, None) == nls.E_INVALID
    assert L.nls_create(None, None) == nls.E_INVALID
    assert L.nls_destroy(None) == nls.OK
    assert isinstance(L.nls_last_error(None), bytes)


def test_fp32_inner_accepted_everywhere(nls):
    """FP32-inner is a precision form of every kernel: validation accepts it
    for every family, size and algorithm, uniform or mixed."""
    for fam, n, alg in ((0, 4, 0), (0, 8, 2), (0, 24, 1), (1, 8, 2), (1, 64, 2), (2, 10, 1), (3, 2, 0)):
        b, keep = _batch(nls, family=fam, n=n, alg=alg, precision=1)
        assert nls.lib().nls_validate(ctypes.byref(b), None) == nls.OK, (fam, n, alg)
    ns = np.array([4, 4, 8, 4], dtype=np.uint8)
    b, keep = _batch(nls, precision=1)
    b.n = ns.ctypes.data_as(ctypes.c_void_p)
    assert nls.lib().nls_validate(ctypes.byref(b), None) == nls.OK


def test_fallback_chain_is_an_algorithm(nls):
    """POLY (the Newton -> line search -> trust region chain) and the
    Potra-Ptak scheme validate like the other algorithms for every family and
    size; the next value does not."""
    assert nls.ALG_POLY == 3
    for fam, n in ((0, 4), (0, 24), (1, 8), (1, 64), (2, 10), (3, 2)):
        for prec in (0, 1):
            b, keep = _batch(nls, family=fam, n=n, alg=nls.ALG_POLY, precision=prec)
            assert nls.lib().nls_validate(ctypes.byref(b), None) == nls.OK, (fam, n, prec)
    b, keep = _batch(nls, alg=nls.ALG_POTRA_PTAK)
    assert nls.lib().nls_validate(ctypes.byref(b), None) == nls.OK
    b, keep = _batch(nls, alg=5)
    assert nls.lib().nls_validate(ctypes.byref(b), None) == nls.E_INVALID
    algs = np.array([0, 3, 3, 1], dtype=np.uint8)
    b, keep = _batch(nls)
    b.alg = algs.ctypes.data_as(ctypes.c_void_p)
    assert nls.lib().nls_validate(ctypes.byref(b), None) == nls.OK


def test_sensitivity_entry_rejects_null_context(nls):
    """The sensitivity entry point checks its context before anything else
    (no device needed)."""
    L = nls.lib()
    b = nls.SensBatch()
    r = nls.SensResults()
    t = ctypes.c_uint64(0)
    assert L.nls_sensitivity_batch(None, ctypes.byref(b), ctypes.byref(r), ctypes.byref(t)) == nls.E_INVALID
    assert nls.SENS_TANGENT == 0 and nls.SENS_ADJOINT == 1


def test_noalloc_entry_validates_before_any_device_work(nls):
    """nls_solve_batch_noalloc refuses host payloads, mixed batches and
    fallback-chain batches beyond its fixed scratch without touching a
    device (this process has none)."""
    L = nls.lib()
    r = nls.Results()
    b, keep = _batch(nls)  # host memory
    u = np.zeros(64)
    r.u = r.fnorm_inf = r.iters = r.retcode = u.ctypes.data_as(ctypes.c_void_p)
    assert L.nls_solve_batch_noalloc(ctypes.byref(b), ctypes.byref(r), None) == nls.E_INVALID
    assert "device memory" in nls.last_error()
    b, keep = _batch(nls, mem_kind=nls.MEM_DEVICE)
    ns = np.array([4, 8, 4, 4], dtype=np.uint8)
    b.n = ns.ctypes.data_as(ctypes.c_void_p)
    assert L.nls_solve_batch_noalloc(ctypes.byref(b), ctypes.byref(r), None) == nls.E_INVALID
    assert "uniform" in nls.last_error()
    b, keep = _batch(nls, mem_kind=nls.MEM_DEVICE, alg=nls.ALG_POLY, count=nls.NOALLOC_MAX_CHAIN_SYSTEMS + 1)
    assert L.nls_solve_batch_noalloc(ctypes.byref(b), ctypes.byref(r), None) == nls.E_NOMEM
    assert "scratch" in nls.last_error()
