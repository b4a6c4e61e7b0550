"""The oracle's pins must catch plausible mistakes.

Each mutant is a copy of the oracle source with one planted error (a dropped
term, a wrong sign, a transposed operand, a wrong constant or index), built
on the CPU into a temporary library; the pin suites then run against it in a
subprocess and must fail.
"""
import concurrent.futures
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "nls_oracle.c")
PINS = ["tests/test_oracle_residual_jacobian.py", "tests/test_oracle_lu.py",
        "tests/test_oracle_solvers.py", "tests/test_oracle_sensitivity.py",
        "tests/test_oracle_trust_region.py"]

MUTANTS = {
    "cubic coefficient": ("F[i] = (s + 0.1 * cube) - b[i];", "F[i] = (s + 0.2 * cube) - b[i];"),
    "dual product rule drops a term": ("a.d * b.v + a.v * b.d", "a.d * b.v"),
    "tanh derivative sign": ("(1.0 - t * t) * a.d", "(1.0 + t * t) * a.d"),
    "rosenbrock square dropped": ("F[i] = 10.0 * (u[i] - u[i - 1] * u[i - 1]);",
                                  "F[i] = 10.0 * (u[i] - u[i - 1]);"),
    "tanh residual beta sign": ("F[i] = (s + beta * u[i]) - b[i];", "F[i] = (s - beta * u[i]) - b[i];"),
    "pivot picks the minimum": ("if (v > amax) { amax = v; p = i; }", "if (v < amax) { amax = v; p = i; }"),
    "pivot tie picks the last": ("if (v > amax) { amax = v; p = i; }", "if (v >= amax) { amax = v; p = i; }"),
    "back substitution multiplies": ("b[i] = b[i] / lu[i * n + i];", "b[i] = b[i] * lu[i * n + i];"),
    "forward substitution index": ("for (j = 0; j < i; ++j) b[i] = b[i] - lu[i * n + j] * b[j];",
                                   "for (j = 0; j < i; ++j) b[i] = b[i] - lu[j * n + i] * b[j];"),
    "newton direction sign": ("for (i = 0; i < n; ++i) delta[i] = -F[i];",
                              "for (i = 0; i < n; ++i) delta[i] = F[i];"),
    "armijo bound sign": ("(1.0 - 2.0 * o.armijo_c * alpha) * phi0", "(1.0 + 2.0 * o.armijo_c * alpha) * phi0"),
    "armijo accepts without test": ("if (phit <= bound) { accepted = 1; break; }", "{ accepted = 1; break; }"),
    "gradient uses J not J^T": ("for (i = 0; i < n; ++i) s = s + J[i * n + j] * F[i];",
                                "for (i = 0; i < n; ++i) s = s + J[j * n + i] * F[i];"),
    # (the qb <= 0 branch of the tau formula is not mutated: with exact Newton
    # and Cauchy steps qb = 2 t (||F||^2 - ||g||^4/||Jg||^2) >= 0 by
    # Cauchy-Schwarz, so that branch only runs at qb = 0, where both root
    # formulas give the same tau)
    "dogleg tau other root branch": ("(-2.0 * qc) / (qb + sq)", "(2.0 * qc) / (qb + sq)"),
    "cauchy step length": ("tcauchy = ng2 / nJg2;", "tcauchy = ng2 / sqrt(nJg2);"),
    "radius not shrunk": ("Delta = o.tr_shrink * nstep;", "Delta = nstep;"),
    "radius never expands": ("Delta = fmin(o.tr_expand * Delta, o.tr_delta_max);", "Delta = Delta;"),
    "radius expansion not capped": ("Delta = fmin(o.tr_expand * Delta, o.tr_delta_max);",
                                    "Delta = o.tr_expand * Delta;"),
    "accept threshold eta1 -> 0": ("} else if (rho > o.tr_eta1) {", "} else if (rho > 0.0) {"),
    "expand threshold eta2 -> eta1": ("if (rho >= o.tr_eta2) {", "if (rho >= o.tr_eta1) {"),
    "collapse never fires": ("if (Delta < o.tr_collapse * fmax(1.0, unorm)) {", "if (0) {"),
    "predicted reduction sign": ("lin[i] = F[i] + s;", "lin[i] = F[i] - s;"),
    "norm is last component": ("double v = fabs(x[i]); if (v > m) m = v;", "double v = fabs(x[i]); m = v;"),
    "poly restarts from the failed endpoint": ("r = or_solve_one(family, n, chain[a], p, u0, abstol,",
                                              "r = or_solve_one(family, n, chain[a], p, a ? u_out : u0, abstol,"),
    "poly keeps the last attempt": ("if (!have || r.retcode == OR_RC_SUCCESS || r.fnorm_inf < best.fnorm_inf)",
                                    "if (1)"),
    "poly counts only the reported attempt": ("  best.iters = iters;\n", "  best.iters = best.iters;\n"),
    "poly stage order": ("{OR_ALG_NEWTON, OR_ALG_ARMIJO, OR_ALG_DOGLEG}", "{OR_ALG_NEWTON, OR_ALG_DOGLEG, OR_ALG_ARMIJO}"),
    "tangent sign": ("      du[i] = -s;\n", "      du[i] = s;\n"),
    "adjoint gradient sign": ("      grad[j] = -s;\n", "      grad[j] = s;\n"),
    "adjoint solves with J, not J^T": ("for (j = 0; j < n; ++j) Jt[i * n + j] = J[j * n + i];",
                                       "for (j = 0; j < n; ++j) Jt[i * n + j] = J[i * n + j];"),
    "parameter seed on the wrong entry": ("for (i = 0; i < P; ++i) pd[i] = dl(p[i], i == j ? 1.0 : 0.0);",
                                          "for (i = 0; i < P; ++i) pd[i] = dl(p[i], i == (j + 1) % P ? 1.0 : 0.0);"),
    "tanh parameter derivative uses u": ("s = dadd(s, dmul(A[i * n + j], dconst(tanh(u[j]))));",
                                         "s = dadd(s, dmul(A[i * n + j], dconst(u[j])));"),
    "potra second solve uses f(u_k)": ("      for (i = 0; i < n; ++i) step[i] = -Ft[i];\n      or_lu_solve(n, lu, piv, step);",
                                       "      for (i = 0; i < n; ++i) step[i] = -F[i];\n      or_lu_solve(n, lu, piv, step);"),
    "potra second step subtracted": ("for (i = 0; i < n; ++i) u[i] = ut[i] + step[i];",
                                     "for (i = 0; i < n; ++i) u[i] = ut[i] - step[i];"),
    "iteration count off by one": ("r.retcode = OR_RC_SUCCESS; r.iters = k; goto done; }\n    }\n    r.retcode = OR_RC_MAXITERS; r.iters = maxiters;\n    goto done;\n  }\n\n  if (alg == OR_ALG_ARMIJO)",
                                   "r.retcode = OR_RC_SUCCESS; r.iters = k + 1; goto done; }\n    }\n    r.retcode = OR_RC_MAXITERS; r.iters = maxiters;\n    goto done;\n  }\n\n  if (alg == OR_ALG_ARMIJO)"),
}


def _build_and_run(name, old, new, tmp):
    src = open(SRC).read()
    assert src.count(old) >= 1, name
    mutated = src.replace(old, new, 1)
    d = os.path.join(tmp, name.replace(" ", "_").replace("^", ""))
    os.makedirs(d, exist_ok=True)
    c = os.path.join(d, "nls_oracle.c")
    open(c, "w").write(mutated)
    import shutil
    shutil.copy(os.path.join(ROOT, "oracle", "nls_oracle.h"), d)
    so = os.path.join(d, "liboracle.so")
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-o", so, c,
                    "-lm", "-lpthread"], check=True)
    env = dict(os.environ, NLS_ORACLE_LIB=so, PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-W", "ignore", *PINS], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=900)
    return name, r.returncode, r.stdout[-400:]


def test_every_planted_mistake_fails_a_pin():
    with tempfile.TemporaryDirectory() as tmp:
        jobs = max(1, min(8, os.cpu_count() or 1))
        with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
            res = list(ex.map(lambda kv: _build_and_run(kv[0], kv[1][0], kv[1][1], tmp), MUTANTS.items()))
    survivors = [(n, out) for n, rc, out in res if rc == 0]
    assert not survivors, "mutants not caught by any pin: %s" % [n for n, _ in survivors]
