"""nls_solve_batch_noalloc: the solve for callers that cannot allocate.

Through the C ABI, two calls in a row on one stream (the second with a
smaller batch, so the fixed scratch holds the first call's leftovers) must
give bitwise the results of nls_solve_batch on the same inputs, for a lane and
a group mapping and for the fallback chain, whose later stages run entirely
in the fixed scratch; and the first batch is checked against the oracle.
Requests beyond the scratch's stated limits are refused before any work."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2403_16341_amd import inputs

from _helpers import classify

pytestmark = pytest.mark.gpu

KEYS = ("u", "fnorm_inf", "iters", "retcode", "nfev", "njev")


@pytest.fixture(scope="module")
def nls():
    from paper_2403_16341_amd import nls as _nls
    _nls.lib()
    return _nls


def _noalloc(nls, b):
    import torch
    db = nls.DeviceBatch(b)
    out = nls.solve_noalloc(db)
    torch.cuda.current_stream().synchronize()
    return nls.results_to_numpy(out)


@pytest.mark.parametrize("k,alg,M1,M2", [
    (2, inputs.ARMIJO, 64 * 40 + 7, 64 * 3 + 5),     # lane mapping, n = 8
    (3, inputs.DOGLEG, 64 * 6 + 9, 101),             # 16-lane groups, n = 16
    (3, inputs.POLY, 64 * 6 + 9, 77),                # fallback chain in the fixed scratch
])
def test_noalloc_matches_batch_path(nls, k, alg, M1, M2):
    print("case: noalloc workload %d alg %d M %d then %d" % (k, alg, M1, M2), flush=True)
    ctx = nls.Context(0)
    try:
        b1 = inputs.config(k, M=M1)
        b1.alg[:] = alg
        b2 = inputs.config(k, M=M2, seed=4242)
        b2.alg[:] = alg
        g1 = _noalloc(nls, b1)
        g2 = _noalloc(nls, b2)
        for b, g in ((b1, g1), (b2, g2)):
            ref = nls.results_to_numpy(ctx.solve(nls.DeviceBatch(b)))
            for key in KEYS:
                assert np.array_equal(g[key], ref[key], equal_nan=True), (k, alg, b.M, key)
        rep, _ = classify(b1, g1)
        assert not rep["strict_fail"], rep["strict_fail"][:5]
    finally:
        ctx.close()


def test_noalloc_refuses_beyond_limits(nls):
    import torch
    b = inputs.config(1, M=nls.NOALLOC_MAX_CHAIN_SYSTEMS + 1)
    b.alg[:] = inputs.POLY
    db = nls.DeviceBatch(b)
    with pytest.raises(nls.NLSError) as e:
        nls.solve_noalloc(db)
    assert e.value.code == nls.E_NOMEM and "scratch" in str(e.value)
    # a mixed batch is not accepted (it would need a planning step that allocates)
    m = inputs.config(4, M=50)
    dm = nls.DeviceBatch(m)
    with pytest.raises(nls.NLSError):
        nls.solve_noalloc(dm)
    torch.cuda.synchronize()
