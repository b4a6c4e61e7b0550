"""Shared test helpers: an independent numpy residual and the parity
classification of GPU results against the oracle."""
import numpy as np

import oracle

REL = 1e-9
STALLS = (oracle.RC_MAXITERS, oracle.RC_LINESEARCH_FAILED, oracle.RC_TR_COLLAPSED)
RC_INVALID = 6  # the kernels' safeguard code (never an oracle outcome)


def np_residual(family, p, u):
    """Residual families written out in numpy (independent of both sides)."""
    n = u.size
    if family == oracle.CUBIC:
        return p[: n * n].reshape(n, n) @ u + 0.1 * u ** 3 - p[n * n: n * n + n]
    if family == oracle.TANH:
        return p[: n * n].reshape(n, n) @ np.tanh(u) + p[n * n + n] * u - p[n * n: n * n + n]
    if family == oracle.ROSENBROCK:
        return np.concatenate([[1 - u[0]], 10 * (u[1:] - u[:-1] ** 2)])
    a, b_, c = p
    return np.array([(u[0] + a) * (u[1] ** 3 - b_) + c, np.sin(u[1] * np.exp(u[0]) - 1)])


def run_oracle(b, opts=None, variant="plain", u0=None):
    return oracle.solve_batch(b.family, b.n, b.alg, b.params, b.p_off, b.u0 if u0 is None else u0,
                              b.u_off, b.abstol, b.maxiters, opts=opts, nthreads=8, variant=variant)


def rel_err(b, ug, uo, s):
    sl = slice(b.u_off[s], b.u_off[s] + b.n[s])
    den = max(np.abs(uo[sl]).max(), np.finfo(float).tiny)
    return np.abs(ug[sl] - uo[sl]).max() / den


def forward_bound(b, o, s):
    """Relative forward-error bound 2 ||J(u*)^-1||_inf abstol / ||u*||_inf of a
    point that passes the stopping test, at the oracle's solution u*."""
    f_, n, _, p, _ = b.system(s)
    uo = o["u"][b.u_off[s]:b.u_off[s] + n]
    try:
        kappa = np.abs(np.linalg.inv(oracle.jacobian(f_, p, uo))).sum(axis=1).max()
    except np.linalg.LinAlgError:
        return np.inf
    return 2 * kappa * b.abstol / max(np.abs(uo).max(), 1e-300)


def _same(b, x, y, s):
    """Two oracle runs agree on system s: same return code, iterations within
    +-1, and final iterates that did not separate (1e-9 relative for a
    success; 1e-6 for a failure, whose end point tracks the trajectory)."""
    if x["retcode"][s] != y["retcode"][s] or abs(int(x["iters"][s]) - int(y["iters"][s])) > 1:
        return False
    e = rel_err(b, x["u"], y["u"], s)
    if not np.isfinite(e):
        return x["retcode"][s] == y["retcode"][s] == oracle.RC_NONFINITE
    return e <= (REL if x["retcode"][s] == oracle.RC_SUCCESS else 1e-6)


# Rounding-level perturbations of the oracle's own run: the source built with
# multiply-add contraction, u0 moved by one ulp either way, both, every step
# scaled by 1 +- n 2^-53 in two complementary patterns (the whole trajectory
# perturbed, not only its start), the merit and inner products summed as a
# balanced tree (the rounding order of a butterfly reduction), and two starts a
# few ulps from u0 in random directions.
def probe_starts(u0, seeds=(1, 2)):
    """Starting points a few ulps from u0: every component scaled by
    1 + k 2^-52, k in {-4, ..., 4} hashed from the component's own bits and
    the seed, so a system gets the same probes in any batch it sits in."""
    bits = np.ascontiguousarray(u0, dtype=np.float64).view(np.uint64)
    out = []
    for seed in seeds:
        h = (bits ^ np.uint64((seed * 0x632BE59BD9B4E019) & 0xFFFFFFFFFFFFFFFF)) * np.uint64(0x9E3779B97F4A7C15)
        k = ((h >> np.uint64(40)) % np.uint64(9)).astype(np.int64) - 4
        out.append(u0 * (1.0 + k * 2.0 ** -52))
    return out


def probe_runs(b, opts=None):
    up, dn = np.nextafter(b.u0, np.inf), np.nextafter(b.u0, -np.inf)
    r1, r2 = probe_starts(b.u0)
    return [run_oracle(b, opts, variant="fma"), run_oracle(b, opts, u0=up), run_oracle(b, opts, u0=dn),
            run_oracle(b, opts, variant="fma", u0=up), run_oracle(b, opts, variant="fma", u0=dn),
            run_oracle(b, opts, variant="jitter1"), run_oracle(b, opts, variant="jitter2"),
            run_oracle(b, opts, variant="pairwise"), run_oracle(b, opts, u0=r1), run_oracle(b, opts, u0=r2)]


def _poly_attempts_sensitive(b, o, opts):
    """A POLY system's outcome is decided by its attempts: whether a stage
    succeeds decides whether the next one runs, and when all fail the smallest
    residual picks the result.  So the system is rounding-sensitive when any
    attempt the chain makes is (a Newton trajectory stalled at its cap can
    wander anywhere, and may as well land on a root), under the same probes as
    the chain itself."""
    out = np.zeros(b.M, dtype=bool)
    idx = np.nonzero(b.alg == oracle.POLY)[0]
    if idx.size == 0:
        return out
    sub = b.subset(idx)
    running = np.ones(sub.M, dtype=bool)  # the chain reaches this stage
    for alg in (oracle.NEWTON, oracle.ARMIJO, oracle.DOGLEG):
        sub.alg[:] = alg
        base = run_oracle(sub, opts)
        probes = probe_runs(sub, opts)
        for j in np.nonzero(running)[0]:
            if not all(_same(sub, base, q, j) for q in probes):
                out[idx[j]] = True
        running &= base["retcode"] != oracle.RC_SUCCESS
    return out


def sensitive_mask(b, opts=None):
    """(oracle result, probe results, mask of the rounding-sensitive systems)."""
    o = run_oracle(b, opts)
    probes = probe_runs(b, opts)
    sens = np.array([not all(_same(b, o, q, s) for q in probes) for s in range(b.M)], dtype=bool)
    sens |= _poly_attempts_sensitive(b, o, opts)
    return o, probes, sens


# at most this fraction of a parity batch may be rounding-sensitive
MAX_SENSITIVE = 0.2


def pool_batch(make, M, opts=None, max_sensitive=MAX_SENSITIVE):
    """Parity batch of M systems drawn from a pool of candidates (make(count)
    returns a Batch of that many seeded systems; the pool is 2M, doubled up
    to 16M while too few candidates qualify): the candidates in pool order,
    skipping rounding-sensitive ones once the batch holds max_sensitive * M of
    them.  The choice uses the oracle alone, so it is the same for every
    implementation under test; it keeps the strict bar on at least
    (1 - max_sensitive) of the batch also where far starts make many
    trajectories chaotic (local methods on the tanh family)."""
    count = 2 * M
    while True:
        pool = make(count)
        _, _, sens = sensitive_mask(pool, opts)
        keep, ns = [], 0
        for s in range(pool.M):
            if len(keep) == M:
                break
            if sens[s]:
                if ns >= int(max_sensitive * M):
                    continue
                ns += 1
            keep.append(s)
        if len(keep) == M or count >= 16 * M:
            break
        count *= 2
    assert len(keep) == M, ("pool too sensitive", pool.M, int(sens.sum()))
    return pool.subset(np.array(keep))


def classify(b, g, opts=None, strict_all=False, u_tol="strict", max_sensitive=MAX_SENSITIVE):
    """Compare GPU results g with the oracle.

    No system may end with the kernels' safeguard code RC_INVALID (trip guard
    or group disagreement), sensitive or not.

    A system is rounding-sensitive when the oracle's own outcome changes under
    a rounding-level perturbation (probe_runs).  Every other system must meet
    the strict bar (identical return code, iterations within +-1, relative u
    error <= 1e-9), except that two runs stalled at the same non-root point (u
    within 1e-6) count as one outcome whichever stop test ended them.

    Caps: at most max_sensitive of the batch may be sensitive.  On the
    sensitive systems the GPU may differ from the oracle no more often than a
    perturbed oracle does: its return code (sens_rc_diff), and where both
    succeed, its root (other_root: farther apart than the forward-error bound
    below) -- each at most 1.5 times the largest count over the probes, plus 3
    for the sampling noise of small counts.

    u_tol="bound" relaxes the 1e-9 of the strict bar to the forward-error
    bound of the stopping test where that is larger (families whose last step
    comes from far away, e.g. the generalized Rosenbrock from U(0,1) starts).  Sensitive systems must still satisfy the invariants, and where
    both sides succeed, agree within the forward-error bound of the stopping
    test, 2 ||J(u*)^-1||_inf abstol (or have reached another valid root)."""
    M = b.M
    bad = np.nonzero((g["retcode"] == RC_INVALID) | (g["iters"] < 0))[0]
    assert bad.size == 0, ("systems ended by a kernel safeguard", bad[:5], g["retcode"][bad[:5]],
                           g["iters"][bad[:5]])
    o, probes, sens = sensitive_mask(b, opts)
    if strict_all:
        sens[:] = False
    probe_rc_diff = max([int((sens & (q["retcode"] != o["retcode"])).sum()) for q in probes] + [0])
    report = dict(M=M, sensitive=int(sens.sum()), success_gpu=int((g["retcode"] == 0).sum()),
                  success_oracle=int((o["retcode"] == 0).sum()), strict_fail=[], sens_rc_diff=0,
                  probe_rc_diff=probe_rc_diff, other_root=0, same_stall=0, max_rel_strict=0.0)
    fb = {}

    def bound(s):
        if s not in fb:
            fb[s] = forward_bound(b, o, s)
        return fb[s]

    for s in range(M):
        gs, os_ = int(g["retcode"][s]), int(o["retcode"][s])
        f_, n, _, p, _ = b.system(s)
        if gs == oracle.RC_SUCCESS:
            ug = g["u"][b.u_off[s]:b.u_off[s] + n]
            assert g["fnorm_inf"][s] <= b.abstol, (s, g["fnorm_inf"][s])
            Fn = np.abs(np_residual(f_, p, ug)).max()
            assert Fn <= b.abstol * (1 + 1e-6) + 1e-13, (s, Fn)
        if not sens[s]:
            ok = gs == os_ and abs(int(g["iters"][s]) - int(o["iters"][s])) <= 1
            if ok and gs == oracle.RC_SUCCESS:
                e = rel_err(b, g["u"], o["u"], s)
                report["max_rel_strict"] = max(report["max_rel_strict"], e)
                ok = e <= (REL if u_tol == "strict" else max(REL, forward_bound(b, o, s)))
            if not ok and gs in STALLS and os_ in STALLS and rel_err(b, g["u"], o["u"], s) <= 1e-6:
                # both stalled at the same non-root point; which stop test fires
                # first (radius collapse, failed search or the cap) is set by rounding
                report["same_stall"] += 1
                ok = True
            if not ok:
                report["strict_fail"].append((s, gs, int(g["iters"][s]), os_, int(o["iters"][s])))
        else:
            if gs != os_:
                report["sens_rc_diff"] += 1
            if gs == os_ == oracle.RC_SUCCESS:
                if rel_err(b, g["u"], o["u"], s) > bound(s) + REL:
                    report["other_root"] += 1
    probe_other = 0
    for q in probes:
        both = np.nonzero(sens & (q["retcode"] == oracle.RC_SUCCESS) & (o["retcode"] == oracle.RC_SUCCESS))[0]
        probe_other = max(probe_other, sum(1 for s in both if rel_err(b, q["u"], o["u"], s) > bound(s) + REL))
    report["probe_other_root"] = probe_other
    assert report["sensitive"] <= max(max_sensitive * M, 1), ("too many rounding-sensitive systems", report)
    assert report["sens_rc_diff"] <= 1.5 * probe_rc_diff + 3, ("return codes of sensitive systems", report)
    assert report["other_root"] <= 1.5 * probe_other + 3, ("other roots of sensitive systems", report)
    return report, o


def grid_batch(fam, n, alg, seed, M=None, maxiters=40):
    """Parity-grid batch: seeded cubic (u0 ~ U(-3, 3)) or tanh (u0 ~ U(-4, 4))
    systems of size n, drawn through pool_batch."""
    from paper_2403_16341_amd import inputs
    M = M or (70 if n <= 16 else 23)

    def make(count):
        rng = np.random.Generator(np.random.PCG64(seed))
        if fam == inputs.CUBIC:
            p, u0 = inputs.cubic_params(rng, count, n), rng.uniform(-3, 3, (count, n))
        else:
            p, u0 = inputs.tanh_params(rng, count, n), rng.uniform(-4, 4, (count, n))
        return inputs.homogeneous(fam, n, alg, p, u0, 1e-10, maxiters)

    return pool_batch(make, M)
