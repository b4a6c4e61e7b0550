"""GPU tests of the request server (continuous batching behind nls_server_*).

* every request's results meet the parity bar against the oracle;
* each request's results are bitwise the same alone (one request on the
  server) and in a mix (many requests submitted together, merged into shared
  launches, spread over streams), and the same as the direct batch path;
* admission never holds more device memory than the budget and admits in
  arrival order; requests that can never fit, or break the request rules,
  are refused.
"""
import numpy as np
import pytest

from paper_2403_16341_amd import inputs

pytestmark = pytest.mark.gpu

from _helpers import classify

KEYS = ("u", "fnorm_inf", "iters", "retcode", "nfev", "njev")


@pytest.fixture(scope="module")
def nls():
    from paper_2403_16341_amd import nls as _nls
    _nls.lib()
    return _nls


@pytest.fixture(scope="module")
def requests():
    # sizes up to 300 systems, n in 2..40: every mapping (lane, 16/32/64-lane
    # groups), both families, Armijo and dogleg
    return inputs.serving_requests(24, rate_hz=0.0, seed=777000, max_systems=300, n_range=(2, 40),
                                   precision=inputs.PREC_FP64)


def _same(a, b):
    return all(np.array_equal(a[k], b[k]) for k in KEYS)


def test_server_parity_alone_vs_mix(nls, requests):
    print("case: 24 requests alone, then in a mix with duplicates", flush=True)
    alone = {}
    srv = nls.Server(0, mem_budget_bytes=256 << 20)
    for rq in requests:
        i = srv.submit(rq.batch)
        (info, out), = srv.drain()
        assert info["id"] == i and info["status"] == 0 and info["merged"] == 1
        alone[rq.rid] = out
    srv.close()

    # the mix: every request twice (the copies share a key, so they merge)
    srv = nls.Server(0, mem_budget_bytes=256 << 20, streams=4)
    ids = {}
    for rep in range(2):
        for rq in requests:
            ids[srv.submit(rq.batch)] = (rq.rid, rep)
    done = srv.drain()
    st = srv.stats()
    srv.close()
    assert len(done) == 2 * len(requests)
    assert max(info["merged"] for info, _ in done) > 1, "no launch was shared"
    assert st["launches"] < 2 * len(requests) and st["completed"] == 2 * len(requests)
    for info, out in done:
        rid, _ = ids[info["id"]]
        assert info["status"] == 0
        assert _same(out, alone[rid]), "request %d differs alone and in the mix" % rid

    # the direct batch path runs the same kernels: bitwise the same
    ctx = nls.Context(0)
    for rq in requests[:8]:
        ref = nls.results_to_numpy(ctx.solve(nls.DeviceBatch(rq.batch)))
        assert _same(alone[rq.rid], ref), rq.rid
    ctx.close()

    # parity with the oracle on every request
    for rq in requests:
        b = rq.batch
        print("case: request %d family %d n %d M %d" % (rq.rid, b.family[0], b.n[0], b.M), flush=True)
        rep, _ = classify(b, alone[rq.rid], u_tol="bound" if b.family[0] == inputs.TANH else "strict")
        assert not rep["strict_fail"], (rq.rid, rep["strict_fail"][:5])


def test_server_budget_and_order(nls, requests):
    """A budget that holds only a few requests at once: the server never holds
    more, admits in arrival order, and every result is still the same."""
    foot = max(nls_region_bytes(rq.batch) for rq in requests)
    budget = 3 * foot + 4096
    print("case: budget %d bytes, 40 requests" % budget, flush=True)
    srv = nls.Server(0, mem_budget_bytes=budget, streams=2)
    ref = {}
    ctx = nls.Context(0)
    order = []
    for j in range(40):
        rq = requests[j % len(requests)]
        order.append((srv.submit(rq.batch), rq.rid))
        if rq.rid not in ref:
            ref[rq.rid] = nls.results_to_numpy(ctx.solve(nls.DeviceBatch(rq.batch)))
    done = srv.drain()
    st = srv.stats()
    srv.close()
    ctx.close()
    assert st["peak_resident_bytes"] <= st["budget_bytes"] <= budget
    assert st["resident_bytes"] == 0 and st["queued"] == 0 and st["inflight_launches"] == 0
    by_id = {info["id"]: (info, out) for info, out in done}
    admits = [by_id[i][0]["t_admit_ms"] for i, _ in order]
    assert all(x <= y for x, y in zip(admits, admits[1:])), "admission out of arrival order"
    for i, rid in order:
        info, out = by_id[i]
        assert info["t_submit_ms"] <= info["t_admit_ms"] <= info["t_done_ms"]
        assert _same(out, ref[rid])


def nls_region_bytes(b):
    """Device bytes of one request's launch region (inputs and outputs)."""
    n, M = int(b.n[0]), b.M
    P = int(b.p_off[1] - b.p_off[0])
    r16 = lambda x: (x + 15) // 16 * 16
    return (r16(8 * M * P) + r16(8 * M * n) + r16(8 * M * n) + r16(8 * M) + 4 * r16(4 * M) + 255) // 256 * 256


def test_server_offsets_empty_and_refusals(nls, requests):
    b = requests[3].batch
    p_off = b.p_off + 5 * np.arange(b.M + 1, dtype=np.int64)
    u_off = b.u_off + 3 * np.arange(b.M + 1, dtype=np.int64)
    params = np.full(p_off[-1], np.nan)
    u0 = np.full(u_off[-1], 9.0)
    for s in range(b.M):
        P = b.p_off[s + 1] - b.p_off[s]
        params[p_off[s]:p_off[s] + P] = b.params[b.p_off[s]:b.p_off[s + 1]]
        u0[u_off[s]:u_off[s] + b.n[s]] = b.u0[b.u_off[s]:b.u_off[s + 1]]
    gb = inputs.Batch(b.family, b.n, b.alg, params, p_off, u0, u_off, b.abstol, b.maxiters)
    srv = nls.Server(0, mem_budget_bytes=64 << 20)
    i_gap = srv.submit(gb)
    i_ref = srv.submit(b)
    empty = inputs.homogeneous(inputs.CUBIC, 4, inputs.NEWTON, np.zeros((0, 20)), np.zeros((0, 4)), 1e-10, 10)
    i_empty = srv.submit(empty)
    done = {info["id"]: (info, out) for info, out in srv.drain()}
    assert done[i_empty][0]["systems"] == 0 and done[i_empty][0]["status"] == 0
    g, r = done[i_gap][1], done[i_ref][1]
    for s in range(b.M):
        assert np.array_equal(g["u"][u_off[s]:u_off[s] + b.n[s]], r["u"][b.u_off[s]:b.u_off[s + 1]])
    gaps = np.ones(u_off[-1], bool)
    for s in range(b.M):
        gaps[u_off[s]:u_off[s] + b.n[s]] = False
    assert (g["u"][gaps] == 9.0).all()
    for k in KEYS[1:]:
        assert np.array_equal(g[k], r[k])

    # refusals: larger than the whole budget, several sizes in one request,
    # a size outside 1..64
    small = nls.Server(0, mem_budget_bytes=1 << 16)
    big = inputs.homogeneous(inputs.CUBIC, 8, inputs.ARMIJO, np.zeros((2000, 72)), np.zeros((2000, 8)),
                             1e-10, 10)
    with pytest.raises(nls.NLSError) as ei:
        small.submit(big)
    assert ei.value.code == nls.E_NOMEM
    small.close()
    mixed = inputs.concat([requests[0].batch, requests[1].batch])
    if mixed.uniform() is None:
        with pytest.raises(nls.NLSError):
            srv.submit(mixed)
    c70 = inputs.homogeneous(inputs.CUBIC, 70, inputs.ARMIJO, np.zeros((2, 70 * 71)), np.zeros((2, 70)), 1e-10, 10)
    with pytest.raises(nls.NLSError) as ei:
        srv.submit(c70)
    assert ei.value.code == nls.E_INVALID
    srv.close()


def test_server_sliced_launches(nls, requests, monkeypatch):
    """With slicing switched on (NLS_SERVE_SLICE_WORK, read at server
    creation) every launch of more than 64 systems runs as several persistent
    launches; results stay bitwise those of the direct batch path."""
    monkeypatch.setenv("NLS_SERVE_SLICE_WORK", "65536")
    print("case: sliced launches, 12 requests", flush=True)
    srv = nls.Server(0, mem_budget_bytes=128 << 20)
    ids = {srv.submit(rq.batch): rq for rq in requests[:12]}
    done = srv.drain()
    srv.close()
    ctx = nls.Context(0)
    for info, out in done:
        rq = ids[info["id"]]
        ref = nls.results_to_numpy(ctx.solve(nls.DeviceBatch(rq.batch)))
        assert info["status"] == 0 and _same(out, ref), rq.rid
    ctx.close()


def test_server_fp32_inner_alone_vs_mix(nls):
    """FP32-inner requests (the serving workload's form): each request's
    results are bitwise the same alone and in a mix, and every success passes
    the FP64 stopping test."""
    reqs = inputs.serving_requests(12, rate_hz=0.0, seed=778000, max_systems=200, n_range=(2, 64),
                                   precision=inputs.PREC_FP32_INNER)
    print("case: 12 fp32-inner requests alone, then mixed", flush=True)
    srv = nls.Server(0, mem_budget_bytes=128 << 20)
    alone = {}
    for rq in reqs:
        srv.submit(rq.batch)
        (info, out), = srv.drain()
        alone[rq.rid] = out
    ids = {srv.submit(rq.batch): rq for rq in reqs}
    done = srv.drain()
    srv.close()
    for info, out in done:
        rq = ids[info["id"]]
        assert info["status"] == 0 and _same(out, alone[rq.rid]), rq.rid
        succ = out["retcode"] == 0
        assert (out["retcode"] != nls.RC_INVALID).all()
        assert (out["fnorm_inf"][succ] <= rq.batch.abstol).all()


def test_server_potra_ptak_requests_match_the_batch_path(nls):
    """Potra-Ptak requests (lane and group kernels) through the server give
    bitwise the results of the direct batch path, alone and merged."""
    rng = np.random.Generator(np.random.PCG64(4242))
    batches = []
    for n, M in ((4, 150), (8, 90), (12, 60), (24, 20)):
        p, u0 = inputs.cubic_params(rng, M, n), rng.uniform(-3, 3, (M, n))
        batches.append(inputs.homogeneous(inputs.CUBIC, n, inputs.POTRA_PTAK, p, u0, 1e-10, 50))
    ctx = nls.Context(0)
    ref = [nls.solve_host(ctx, b) for b in batches]
    ctx.close()
    srv = nls.Server(0, mem_budget_bytes=64 << 20, streams=2)
    ids = {}
    for rep in range(2):
        for j, b in enumerate(batches):
            ids[srv.submit(b)] = j
    done = srv.drain()
    srv.close()
    assert len(done) == 2 * len(batches)
    for info, out in done:
        assert info["status"] == 0
        assert _same(out, ref[ids[info["id"]]])
    assert all((r["retcode"] == 0).mean() > 0.9 for r in ref)


def test_server_fallback_chain_requests_match_the_batch_path(nls):
    """Fallback-chain requests (lane and group kernels, both families) through
    the server give bitwise the results of the direct batch path, alone and
    merged; their regions carry the chain's scratch."""
    rng = np.random.Generator(np.random.PCG64(4343))
    batches = []
    for fam, n, M in ((inputs.TANH, 3, 120), (inputs.TANH, 16, 70), (inputs.CUBIC, 8, 90), (inputs.TANH, 40, 12)):
        if fam == inputs.CUBIC:
            p, u0 = inputs.cubic_params(rng, M, n), rng.uniform(-6, 6, (M, n))
        else:
            p, u0 = inputs.tanh_params(rng, M, n), rng.uniform(-4, 4, (M, n))
        batches.append(inputs.homogeneous(fam, n, inputs.POLY, p, u0, 1e-10, 30))
    ctx = nls.Context(0)
    ref = [nls.solve_host(ctx, b) for b in batches]
    ctx.close()
    srv = nls.Server(0, mem_budget_bytes=64 << 20, streams=2)
    ids = {}
    for rep in range(2):
        for j, b in enumerate(batches):
            ids[srv.submit(b)] = j
    done = srv.drain()
    srv.close()
    assert len(done) == 2 * len(batches)
    for info, out in done:
        assert info["status"] == 0
        assert _same(out, ref[ids[info["id"]]])
    # the chain did run past its Newton stage somewhere
    assert any((r["nfev"] > r["iters"] + 1).any() for r in ref)


def _with_gaps(b, pg, ug):
    """The same batch with pg unused doubles after each system's parameters
    and ug after each starting point (NaN / 9.0 in the gaps)."""
    p_off = b.p_off + pg * np.arange(b.M + 1, dtype=np.int64)
    u_off = b.u_off + ug * np.arange(b.M + 1, dtype=np.int64)
    params = np.full(p_off[-1], np.nan)
    u0 = np.full(u_off[-1], 9.0)
    for s in range(b.M):
        P = b.p_off[s + 1] - b.p_off[s]
        params[p_off[s]:p_off[s] + P] = b.params[b.p_off[s]:b.p_off[s + 1]]
        u0[u_off[s]:u_off[s] + b.n[s]] = b.u0[b.u_off[s]:b.u_off[s + 1]]
    return inputs.Batch(b.family, b.n, b.alg, params, p_off, u0, u_off, b.abstol, b.maxiters), u_off


def test_server_copy_threads(nls, requests, monkeypatch):
    """Host copies handed to the copy threads (thresholds lowered through
    NLS_SERVE_INLINE_COPY_BYTES / NLS_SERVE_COPY_JOB_BYTES, read at server
    creation, so that every launch is staged and scattered in several jobs
    with a ragged last one): results bitwise those of the inline copies, for
    contiguous requests and for requests with gaps between systems, merged
    and alone."""
    monkeypatch.setenv("NLS_SERVE_INLINE_COPY_BYTES", "0")
    monkeypatch.setenv("NLS_SERVE_COPY_JOB_BYTES", "3000")
    print("case: copy threads, 24 requests twice plus 4 with gaps", flush=True)
    ctx = nls.Context(0)
    ref = {rq.rid: nls.results_to_numpy(ctx.solve(nls.DeviceBatch(rq.batch))) for rq in requests}
    ctx.close()
    gapped = [(rq.rid,) + _with_gaps(rq.batch, 7, 3) for rq in requests[:4]]
    srv = nls.Server(0, mem_budget_bytes=256 << 20, streams=4)
    ids = {}
    for rep in range(2):
        for rq in requests:
            ids[srv.submit(rq.batch)] = ("plain", rq.rid)
    for rid, gb, u_off in gapped:
        ids[srv.submit(gb)] = ("gaps", rid, u_off)
    done = srv.drain()
    st = srv.stats()
    srv.close()
    assert len(done) == 2 * len(requests) + len(gapped)
    assert st["resident_bytes"] == 0 and st["inflight_launches"] == 0
    for info, out in done:
        tag = ids[info["id"]]
        assert info["status"] == 0
        r = ref[tag[1]]
        if tag[0] == "plain":
            assert _same(out, r), tag
            continue
        b = [rq.batch for rq in requests if rq.rid == tag[1]][0]
        u_off = tag[2]
        for s in range(b.M):
            assert np.array_equal(out["u"][u_off[s]:u_off[s] + b.n[s]], r["u"][b.u_off[s]:b.u_off[s + 1]])
        gaps = np.ones(u_off[-1], bool)
        for s in range(b.M):
            gaps[u_off[s]:u_off[s] + b.n[s]] = False
        assert (out["u"][gaps] == 9.0).all()
        for k in KEYS[1:]:
            assert np.array_equal(out[k], r[k])
