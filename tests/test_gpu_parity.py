"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bar for the plain FP64 form: identical return codes, iteration counts within
+-1, and ||u_gpu - u_oracle||_inf / ||u_oracle||_inf <= 1e-9 on every system
both sides solve.  Inputs come from the seeded generators only.
"""
import numpy as np
import pytest

import oracle
from paper_2403_16341_amd import inputs

pytestmark = pytest.mark.gpu

from _helpers import REL, classify, grid_batch, rel_err, run_oracle


@pytest.fixture(scope="module")
def nls():
    from paper_2403_16341_amd import nls as _nls
    _nls.lib()
    return _nls


@pytest.fixture(scope="module")
def ctx(nls):
    c = nls.Context(0)
    yield c
    c.close()


def run_gpu(nls, ctx, b, precision=None, opts=None):
    db = nls.DeviceBatch(b)
    out = ctx.solve(db, precision=precision, opts=opts)
    return nls.results_to_numpy(out)


def compare(b, g, label, opts=None, strict_all=False, u_tol="strict"):
    """Parity bar on one batch (see _helpers.classify: strict bar on every
    system that is not rounding-sensitive, derived caps on the sensitive ones,
    no safeguard codes); returns the report."""
    rep, o = classify(b, g, opts=opts, strict_all=strict_all, u_tol=u_tol)
    rep["label"] = label
    print({k: (v[:5] if isinstance(v, list) else v) for k, v in rep.items()}, flush=True)
    assert not rep["strict_fail"], (label, rep["strict_fail"][:5])
    return rep


# ---------------------------------------------------------------------------
# the workloads at oracle-friendly sizes (several wavefronts plus a ragged tail)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("k,M", [(1, 1024), (2, 64 * 9 + 13), (3, 64 * 5 + 21), (4, 1500)])
def test_workload_parity_fp64(nls, ctx, k, M):
    b = inputs.config(k, M=M)
    print("case: workload %d M=%d" % (k, M), flush=True)
    g = run_gpu(nls, ctx, b)
    rep = compare(b, g, "workload%d" % k)
    if k in (1, 2):
        assert rep["sensitive"] == 0


@pytest.mark.parametrize("fam", [inputs.CUBIC, inputs.TANH])
@pytest.mark.parametrize("alg", [inputs.NEWTON, inputs.ARMIJO, inputs.DOGLEG, inputs.POTRA_PTAK])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 9, 12, 16, 20, 24, 32, 40, 64])
def test_family_alg_size_grid(nls, ctx, fam, alg, n):
    b = grid_batch(fam, n, alg, seed=1000 + 10 * n + fam)
    print("case: fam=%d alg=%d n=%d" % (fam, alg, n), flush=True)
    g = run_gpu(nls, ctx, b)
    compare(b, g, "fam%d-alg%d-n%d" % (fam, alg, n))


@pytest.mark.parametrize("seed", [11, 12])
@pytest.mark.parametrize("fam", [inputs.CUBIC, inputs.TANH])
@pytest.mark.parametrize("alg", [inputs.NEWTON, inputs.ARMIJO, inputs.DOGLEG, inputs.POTRA_PTAK, inputs.POLY])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 9, 12, 16, 20, 24, 32, 40, 64])
def test_wide_seed_sweep(nls, ctx, seed, fam, alg, n):
    """The same grid on two more seeds and with the fallback chain: every
    mapping, family and algorithm under the same bar."""
    b = grid_batch(fam, n, alg, seed=seed * 100000 + 10 * n + fam)
    print("case: seed=%d fam=%d alg=%d n=%d" % (seed, fam, alg, n), flush=True)
    g = run_gpu(nls, ctx, b)
    compare(b, g, "seed%d-fam%d-alg%d-n%d" % (seed, fam, alg, n))


def test_edge_families_and_cases(nls, ctx):
    cases = [
        inputs.rosenbrock(100, 10, seed=5, alg=inputs.NEWTON),
        inputs.rosenbrock(100, 10, seed=5, alg=inputs.POTRA_PTAK),
        inputs.rosenbrock(60, 6, seed=15, alg=inputs.POTRA_PTAK),
        inputs.paper_example(64, seed=8, alg=inputs.POTRA_PTAK),
        inputs.singular_cubic(5, 3, alg=inputs.POTRA_PTAK),
        inputs.singular_cubic(5, 12, alg=inputs.POTRA_PTAK),
        inputs.rosenbrock(100, 8, seed=6, alg=inputs.DOGLEG),
        inputs.rosenbrock(7, 10, seed=7, alg=inputs.ARMIJO, u0="paper"),
        inputs.paper_example(64, seed=8, alg=inputs.NEWTON),
        inputs.paper_example(64, seed=9, alg=inputs.DOGLEG),
        inputs.singular_cubic(5, 3),
        inputs.singular_cubic(5, 12, alg=inputs.DOGLEG),
        inputs.no_root_tanh(20, 5, seed=10),
        inputs.no_root_tanh(20, 11, seed=11, alg=inputs.DOGLEG),
        inputs.separable_cubic(30, 4, seed=12),
        inputs.separable_tanh(30, 6, seed=13),
    ]
    for b in cases:
        print("case:", b.name, b.M, int(b.n[0]), int(b.alg[0]), flush=True)
        compare(b, run_gpu(nls, ctx, b), b.name,
                u_tol="bound" if b.name in ("rosenbrock", "paper-example") else "strict")


@pytest.mark.parametrize("n", [4, 8, 16, 32])
def test_pivot_ties(nls, ctx, n):
    """Exact ties among the pivot candidates at every elimination step: cubic
    systems whose matrix is a Hadamard matrix (entries +-1, rows permuted and
    rows and columns sign-flipped at random), solved from u0 = 0, where the
    first Jacobian is the matrix itself; its elimination keeps producing
    columns of equal magnitudes.  The first maximum in current row order must
    win in every mapping (lane at n = 4 and 8, two rows per lane at 16, one
    row per lane at 32): FP64 meets the parity bar against the oracle, and the
    FP32-inner form keeps the FP64 stopping test on every success."""
    rng = np.random.Generator(np.random.PCG64(4100 + n))
    M = 200
    H = np.array([[1.0]])
    while H.shape[0] < n:
        H = np.block([[H, H], [H, -H]])
    A = np.empty((M, n, n))
    for m in range(M):
        perm, s1, s2 = rng.permutation(n), rng.choice([-1.0, 1.0], n), rng.choice([-1.0, 1.0], n)
        A[m] = s1[:, None] * H[perm] * s2[None, :]
    b = rng.integers(-3, 4, (M, n)).astype(np.float64)
    p = np.concatenate([A.reshape(M, n * n), b], axis=1)
    for alg in (inputs.NEWTON, inputs.ARMIJO):
        bt = inputs.homogeneous(inputs.CUBIC, n, alg, p, np.zeros((M, n)), 1e-10, 40, name="pivot-ties")
        print("case: pivot ties n=%d alg=%d" % (n, alg), flush=True)
        compare(bt, run_gpu(nls, ctx, bt), "ties-n%d-alg%d" % (n, alg))
        g32 = run_gpu(nls, ctx, bt, precision=inputs.PREC_FP32_INNER)
        assert (g32["retcode"] != nls.RC_INVALID).all()
        succ = g32["retcode"] == oracle.RC_SUCCESS
        assert succ.mean() >= 0.95
        assert (g32["fnorm_inf"][succ] <= bt.abstol).all()


def test_paper_gpu_workload(nls, ctx):
    """The batch of the paper's GPU kernel example (Sec. 3.3): 1,024 x
    generalized Rosenbrock N = 10 from U(0,1)^10, Newton; every system reaches
    the unique root (1, ..., 1)."""
    b = inputs.paper_gpu_workload()
    g = run_gpu(nls, ctx, b)
    compare(b, g, b.name, u_tol="bound")
    assert (g["retcode"] == oracle.RC_SUCCESS).all()
    assert np.abs(g["u"] - 1.0).max() <= 1e-8


def test_potra_ptak_mixed_batch_and_counters(nls, ctx):
    """The two-step scheme among the other algorithms in one mixed batch
    (lane and group kernels, one graph), FP64 and FP32-inner; one
    factorisation and two residuals per iteration."""
    b = inputs.config(4, M=1200)
    rng = np.random.Generator(np.random.PCG64(92))
    # (cubic systems only: the mixed workload's tanh starts are far, see the grid)
    b.alg[(rng.random(b.M) < 0.6) & (b.family == inputs.CUBIC)] = inputs.POTRA_PTAK
    g = run_gpu(nls, ctx, b)
    compare(b, g, "potra-mixed")
    pp = b.alg == inputs.POTRA_PTAK
    done = pp & (g["iters"] > 0) & (g["retcode"] != oracle.RC_SINGULAR)
    assert np.array_equal(g["njev"][done], g["iters"][done])
    ok = done & (g["retcode"] != oracle.RC_NONFINITE)
    assert np.array_equal(g["nfev"][ok], 2 * g["iters"][ok] + 1)
    g32 = run_gpu(nls, ctx, b, precision=inputs.PREC_FP32_INNER)
    o = run_oracle(b)
    succ = g32["retcode"] == oracle.RC_SUCCESS
    assert (g32["fnorm_inf"][succ] <= b.abstol).all()
    cub = pp & (b.family == inputs.CUBIC) & succ & (o["retcode"] == oracle.RC_SUCCESS)
    errs = np.array([rel_err(b, g32["u"], o["u"], s) for s in np.nonzero(cub)[0]])
    assert errs.size > 50 and (errs <= 1e-8).mean() >= 0.95


def test_nonfinite_maxiters_and_empty(nls, ctx):
    b = inputs.config(2, M=130)
    b.u0[8 * 3 + 2] = np.nan          # system 3 starts at NaN
    b.params[72 * 5 + 10] = np.inf    # system 5 has an infinite parameter
    g = run_gpu(nls, ctx, b)
    compare(b, g, "nonfinite")
    assert g["retcode"][3] == oracle.RC_NONFINITE and g["iters"][3] == 0
    assert g["retcode"][5] == oracle.RC_NONFINITE
    b0 = inputs.config(1, M=100)
    b0.maxiters = 0
    g = run_gpu(nls, ctx, b0)
    assert (g["retcode"] == oracle.RC_MAXITERS).all() and (g["iters"] == 0).all()
    e = inputs.config(1, M=0)
    g = run_gpu(nls, ctx, e)
    assert g["retcode"].size == 0


def test_host_and_device_paths_agree_and_repeat_bitwise(nls, ctx):
    b = inputs.config(4, M=900)
    g1 = run_gpu(nls, ctx, b)
    g2 = run_gpu(nls, ctx, b)
    h = nls.solve_host(ctx, b)
    for key in ("u", "fnorm_inf", "iters", "retcode", "nfev", "njev"):
        assert np.array_equal(g1[key], g2[key], equal_nan=True), key
        assert np.array_equal(g1[key], h[key], equal_nan=True), key


def test_ragged_offsets_with_gaps(nls, ctx):
    """Systems placed at offsets with gaps between them (spans longer than the
    parameter and unknown counts), solved through both payload kinds."""
    b = inputs.config(4, M=300)
    p_off = b.p_off + 3 * np.arange(b.M + 1, dtype=np.int64)
    u_off = b.u_off + 2 * np.arange(b.M + 1, dtype=np.int64)
    params = np.full(p_off[-1], np.nan)
    u0 = np.full(u_off[-1], 7.0)
    for s in range(b.M):
        P = b.p_off[s + 1] - b.p_off[s]
        params[p_off[s]:p_off[s] + P] = b.params[b.p_off[s]:b.p_off[s + 1]]
        u0[u_off[s]:u_off[s] + b.n[s]] = b.u0[b.u_off[s]:b.u_off[s + 1]]
    gb = inputs.Batch(b.family, b.n, b.alg, params, p_off, u0, u_off, b.abstol, b.maxiters)
    h = nls.solve_host(ctx, gb)
    d = run_gpu(nls, ctx, gb)
    ref = run_gpu(nls, ctx, b)
    for s in range(b.M):
        a = h["u"][u_off[s]:u_off[s] + b.n[s]]
        assert np.array_equal(a, ref["u"][b.u_off[s]:b.u_off[s + 1]])
        assert np.array_equal(a, d["u"][u_off[s]:u_off[s] + b.n[s]])
    gaps = np.ones(u_off[-1], bool)
    for s in range(b.M):
        gaps[u_off[s]:u_off[s] + b.n[s]] = False
    assert (h["u"][gaps] == 7.0).all()
    for key in ("iters", "retcode", "fnorm_inf", "nfev", "njev"):
        assert np.array_equal(h[key], ref[key]) and np.array_equal(d[key], ref[key])


def test_fp32_inner_classification(nls, ctx):
    """FP32-inner against the FP64 oracle: every GPU success meets the test, the
    unique-root cubic workloads reach the oracle's root, and tanh systems are
    classified same root / other root / failure."""
    for k, M in ((1, 1024), (2, 700), (3, 400)):
        b = inputs.config(k, M=M)
        g = run_gpu(nls, ctx, b, precision=inputs.PREC_FP32_INNER)
        o = run_oracle(b)
        succ = g["retcode"] == oracle.RC_SUCCESS
        assert (g["fnorm_inf"][succ] <= b.abstol).all()
        if k in (1, 2):
            assert succ.all()
            errs = np.array([rel_err(b, g["u"], o["u"], s) for s in range(M)])
            # a root of a strongly monotone map: error <= ||J^-1|| abstol, ~1e-10
            assert errs.max() <= 1e-8, errs.max()
        else:
            both = succ & (o["retcode"] == oracle.RC_SUCCESS)
            errs = np.array([rel_err(b, g["u"], o["u"], s) for s in np.nonzero(both)[0]])
            same = (errs <= 1e-8).sum()
            print("fp32-inner workload3: gpu success %d, oracle success %d, same root %d of %d"
                  % (succ.sum(), (o["retcode"] == 0).sum(), same, both.sum()), flush=True)
            assert same >= 0.9 * both.sum()


def test_full_size_headline_sampled(nls, ctx):
    """The 2^20 x N=8 Armijo workload in the launch the benchmark times: sampled
    systems against the oracle one by one, plus properties on every system."""
    b = inputs.config(2)
    g = run_gpu(nls, ctx, b)
    assert (g["retcode"] == oracle.RC_SUCCESS).all()
    assert (g["fnorm_inf"] <= b.abstol).all()
    assert g["iters"].min() >= 1 and g["iters"].max() <= 10
    rng = np.random.Generator(np.random.PCG64(77))
    idx = np.sort(rng.choice(b.M, 3000, replace=False))
    sub = b.subset(idx)
    gs = {k: (v[idx] if k != "u" else np.concatenate([v[b.u_off[s]:b.u_off[s + 1]] for s in idx]))
          for k, v in g.items() if isinstance(v, np.ndarray)}
    rep = compare(sub, gs, "headline-sampled")
    assert rep["sensitive"] == 0


def test_group_mapping_for_small_systems(nls, monkeypatch):
    """The group kernels of the n <= 16 bucket also solve n <= 8 systems (the
    autotuner's alternatives); forced through NLS_MAPPING, they meet the same
    bar."""
    monkeypatch.setenv("NLS_MAPPING", "group")
    c = nls.Context(0)
    try:
        assert c.mapping(inputs.CUBIC, 8, inputs.ARMIJO) == 8
        for k, M in ((1, 300), (2, 333)):
            b = inputs.config(k, M=M)
            compare(b, run_gpu(nls, c, b), "group-mapped workload %d" % k)
        b = inputs.config(4, M=900)
        compare(b, run_gpu(nls, c, b), "group-mapped mixed")
    finally:
        c.close()


def test_autotuned_mixed_batch(nls):
    c = nls.Context(0, flags=nls.CTX_AUTOTUNE)
    try:
        b = inputs.config(4, M=3000)
        assert c.mapping(inputs.TANH, 8, inputs.DOGLEG) == 0   # not tuned yet
        g1 = run_gpu(nls, c, b)
        lanes = c.mapping(inputs.TANH, 8, inputs.DOGLEG)
        assert lanes in (1, 8, 16)
        assert c.mapping(inputs.TANH, 12, inputs.DOGLEG) in (8, 16)
        print("autotuned lanes per system (tanh, n=8, dogleg):", lanes, flush=True)
        compare(b, g1, "autotuned mixed")
        g2 = run_gpu(nls, c, b)      # same mapping, replayed graph: bitwise equal
        for key in ("u", "iters", "retcode", "fnorm_inf", "nfev", "njev"):
            assert np.array_equal(g1[key], g2[key], equal_nan=True), key
    finally:
        c.close()


def test_fp32_inner_mixed_batch(nls, ctx):
    """FP32-inner on the mixed workload (every lane and group kernel in FP32
    form, one graph of launches): every GPU success meets the stopping test in
    FP64, the cubic systems (unique roots) reach the oracle's root, and tanh
    systems mostly reach the same root as the FP64 oracle."""
    b = inputs.config(4, M=1500)
    g = run_gpu(nls, ctx, b, precision=inputs.PREC_FP32_INNER)
    o = run_oracle(b)
    assert (g["retcode"] != nls.RC_INVALID).all()
    succ = g["retcode"] == oracle.RC_SUCCESS
    assert (g["fnorm_inf"][succ] <= b.abstol).all()
    cub = b.family == inputs.CUBIC
    assert succ[cub].all()
    errs = np.array([rel_err(b, g["u"], o["u"], s) for s in np.nonzero(cub)[0]])
    assert errs.max() <= 1e-8, errs.max()
    both = succ & (o["retcode"] == oracle.RC_SUCCESS) & ~cub
    errs = np.array([rel_err(b, g["u"], o["u"], s) for s in np.nonzero(both)[0]])
    print("fp32-inner mixed: tanh same root %d of %d" % ((errs <= 1e-8).sum(), both.sum()), flush=True)
    assert (errs <= 1e-8).sum() >= 0.9 * both.sum()

@pytest.mark.parametrize("fam,alg", [(inputs.CUBIC, inputs.NEWTON), (inputs.CUBIC, inputs.ARMIJO),
                                     (inputs.TANH, inputs.ARMIJO), (inputs.TANH, inputs.DOGLEG)])
@pytest.mark.parametrize("n", [3, 8, 12, 24, 40, 64])
def test_fp32_inner_grid(nls, ctx, fam, alg, n):
    """FP32-inner on every mapping (lane, 16/32/64-lane groups): every GPU
    success passes the FP64 stopping test; cubic systems (unique roots) reach
    the FP64 oracle's root; tanh successes mostly reach the oracle's root."""
    rng = np.random.Generator(np.random.PCG64(3000 + 10 * n + fam))
    M = 70 if n <= 16 else 23
    if fam == inputs.CUBIC:
        p, u0 = inputs.cubic_params(rng, M, n), rng.uniform(-3, 3, (M, n))
    else:
        p, u0 = inputs.tanh_params(rng, M, n), rng.uniform(-4, 4, (M, n))
    b = inputs.homogeneous(fam, n, alg, p, u0, 1e-10, 40)
    print("case: fp32-inner fam=%d alg=%d n=%d" % (fam, alg, n), flush=True)
    g = run_gpu(nls, ctx, b, precision=inputs.PREC_FP32_INNER)
    o = run_oracle(b)
    assert (g["retcode"] != nls.RC_INVALID).all()
    succ = g["retcode"] == oracle.RC_SUCCESS
    assert (g["fnorm_inf"][succ] <= b.abstol).all()
    both = succ & (o["retcode"] == oracle.RC_SUCCESS)
    errs = np.array([rel_err(b, g["u"], o["u"], s) for s in np.nonzero(both)[0]])
    if fam == inputs.CUBIC:
        assert (succ == (o["retcode"] == oracle.RC_SUCCESS)).all()
        assert errs.max() <= 1e-8, errs.max()
    else:
        assert (errs <= 1e-8).sum() >= 0.8 * both.sum(), ((errs <= 1e-8).sum(), both.sum())


@pytest.mark.parametrize("n", [9, 16])
@pytest.mark.parametrize("rows", [1, 2])
def test_group_rows_per_lane(nls, monkeypatch, n, rows):
    """Systems of 9..16 unknowns run on groups of 8 lanes with two rows per
    lane (the FP64 default) or of 16 lanes with one row per lane (the
    FP32-inner default); NLS_GROUP_ROWS forces either, and both meet the bar
    in both forms."""
    monkeypatch.setenv("NLS_GROUP_ROWS", str(rows))
    c = nls.Context(0)
    try:
        for fam in (inputs.CUBIC, inputs.TANH):
            for alg in (inputs.NEWTON, inputs.ARMIJO, inputs.DOGLEG):
                b = grid_batch(fam, n, alg, seed=8000 + 10 * n + fam + 100 * alg)
                print("case: rows=%d fam=%d alg=%d n=%d" % (rows, fam, alg, n), flush=True)
                compare(b, run_gpu(nls, c, b), "rows%d-fam%d-alg%d-n%d" % (rows, fam, alg, n))
                g32 = run_gpu(nls, c, b, precision=inputs.PREC_FP32_INNER)
                assert (g32["retcode"] != nls.RC_INVALID).all()
                succ = g32["retcode"] == oracle.RC_SUCCESS
                assert (g32["fnorm_inf"][succ] <= b.abstol).all()
    finally:
        c.close()
