/*
 * nls_oracle.c -- TEST INFRASTRUCTURE ONLY (see nls_oracle.h).
 *
 * Plain FP64 reference, written for readability: every sum runs in index
 * order, divisions are divisions, and the file is compiled with
 * -ffp-contract=off so that no multiply-add is fused.  Nothing here is
 * blocked, fused or reordered beyond what the paper's definitions state.
 */
#include "nls_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define OR_NMAX 64

void or_default_opts(or_opts* o) {
  o->armijo_c = 1e-4;
  o->armijo_rho = 0.5;
  o->armijo_max_halvings = 10;
  o->tr_delta0 = 1.0;
  o->tr_delta_max = 1e8;
  o->tr_eta1 = 1e-4;
  o->tr_eta2 = 0.75;
  o->tr_expand = 2.0;
  o->tr_shrink = 0.25;
  o->tr_collapse = 1e-14;
}

int or_nparams(int family, int n) {
  if (n < 1 || n > OR_NMAX) return -1;
  switch (family) {
    case OR_FAM_CUBIC: return n * n + n;          /* A (row-major), b        */
    case OR_FAM_TANH: return n * n + n + 1;       /* A (row-major), b, beta  */
    case OR_FAM_ROSENBROCK: return n >= 2 ? 0 : -1;
    case OR_FAM_PAPER: return n == 2 ? 3 : -1;    /* (a, b, c)               */
    case OR_FAM_SQUARE: return n;                 /* p                       */
    default: return -1;
  }
}

/* ------------------------------------------------------------------------ */
/* Residual families.  Problem statement f(u, theta) = 0 (Sec. 2).           */
/*   CUBIC      F_i = sum_j A_ij u_j + 0.1 u_i^3 - b_i                       */
/*   TANH       F_i = sum_j A_ij tanh(u_j) + beta u_i - b_i                  */
/*   ROSENBROCK F_1 = 1 - u_1,  F_i = 10 (u_i - u_{i-1}^2)  (generalized     */
/*              Rosenbrock equation of Sec. 2.2.1)                           */
/*   PAPER      F_1 = (u_1 + a)(u_2^3 - b) + c,  F_2 = sin(u_2 e^{u_1} - 1)  */
/*              (the residual of the workflow example in Sec. 3)             */
/*   SQUARE     F_i = u_i^2 - p_i  (the sensitivity example of Sec. 2.3)     */
/* Order: the j-sum first (j ascending), then the elementwise term, then -b. */
/* ------------------------------------------------------------------------ */
void or_residual(int family, int n, const double* p, const double* u, double* F) {
  int i, j;
  switch (family) {
    case OR_FAM_CUBIC: {
      const double* A = p;
      const double* b = p + n * n;
      for (i = 0; i < n; ++i) {
        double s = 0.0;
        for (j = 0; j < n; ++j) s = s + A[i * n + j] * u[j];
        double cube = u[i] * u[i] * u[i];
        F[i] = (s + 0.1 * cube) - b[i];
      }
      break;
    }
    case OR_FAM_TANH: {
      const double* A = p;
      const double* b = p + n * n;
      double beta = p[n * n + n];
      for (i = 0; i < n; ++i) {
        double s = 0.0;
        for (j = 0; j < n; ++j) s = s + A[i * n + j] * tanh(u[j]);
        F[i] = (s + beta * u[i]) - b[i];
      }
      break;
    }
    case OR_FAM_ROSENBROCK: {
      F[0] = 1.0 - u[0];
      for (i = 1; i < n; ++i) F[i] = 10.0 * (u[i] - u[i - 1] * u[i - 1]);
      break;
    }
    case OR_FAM_PAPER: {
      double a = p[0], b = p[1], c = p[2];
      double cube = u[1] * u[1] * u[1];
      F[0] = (u[0] + a) * (cube - b) + c;
      F[1] = sin(u[1] * exp(u[0]) - 1.0);
      break;
    }
    case OR_FAM_SQUARE: {
      for (i = 0; i < n; ++i) F[i] = u[i] * u[i] - p[i];
      break;
    }
    default:
      for (i = 0; i < n; ++i) F[i] = NAN;
  }
}

/* ------------------------------------------------------------------------ */
/* Dual numbers a + a' eps (Sec. 2.4): the value and one directional          */
/* derivative travel together; eps^2 = 0.                                     */
/* ------------------------------------------------------------------------ */
typedef struct { double v, d; } dual;

static dual dl(double v, double d) { dual r; r.v = v; r.d = d; return r; }
static dual dconst(double c) { return dl(c, 0.0); }
static dual dadd(dual a, dual b) { return dl(a.v + b.v, a.d + b.d); }
static dual dsub(dual a, dual b) { return dl(a.v - b.v, a.d - b.d); }
/* (a, a')(b, b') = (ab, a'b + ab') */
static dual dmul(dual a, dual b) { return dl(a.v * b.v, a.d * b.v + a.v * b.d); }
static dual dtanh(dual a) { double t = tanh(a.v); return dl(t, (1.0 - t * t) * a.d); }
static dual dsin(dual a) { return dl(sin(a.v), cos(a.v) * a.d); }
static dual dexp(dual a) { double e = exp(a.v); return dl(e, e * a.d); }

/* The same residual, evaluated on dual numbers. */
static void residual_dual(int family, int n, const double* p, const dual* u, dual* F) {
  int i, j;
  switch (family) {
    case OR_FAM_CUBIC: {
      const double* A = p;
      const double* b = p + n * n;
      for (i = 0; i < n; ++i) {
        dual s = dconst(0.0);
        for (j = 0; j < n; ++j) s = dadd(s, dmul(dconst(A[i * n + j]), u[j]));
        dual cube = dmul(dmul(u[i], u[i]), u[i]);
        F[i] = dsub(dadd(s, dmul(dconst(0.1), cube)), dconst(b[i]));
      }
      break;
    }
    case OR_FAM_TANH: {
      const double* A = p;
      const double* b = p + n * n;
      double beta = p[n * n + n];
      for (i = 0; i < n; ++i) {
        dual s = dconst(0.0);
        for (j = 0; j < n; ++j) s = dadd(s, dmul(dconst(A[i * n + j]), dtanh(u[j])));
        F[i] = dsub(dadd(s, dmul(dconst(beta), u[i])), dconst(b[i]));
      }
      break;
    }
    case OR_FAM_ROSENBROCK: {
      F[0] = dsub(dconst(1.0), u[0]);
      for (i = 1; i < n; ++i)
        F[i] = dmul(dconst(10.0), dsub(u[i], dmul(u[i - 1], u[i - 1])));
      break;
    }
    case OR_FAM_PAPER: {
      dual a = dconst(p[0]), b = dconst(p[1]), c = dconst(p[2]);
      dual cube = dmul(dmul(u[1], u[1]), u[1]);
      F[0] = dadd(dmul(dadd(u[0], a), dsub(cube, b)), c);
      F[1] = dsin(dsub(dmul(u[1], dexp(u[0])), dconst(1.0)));
      break;
    }
    case OR_FAM_SQUARE: {
      for (i = 0; i < n; ++i) F[i] = dsub(dmul(u[i], u[i]), dconst(p[i]));
      break;
    }
    default:
      for (i = 0; i < n; ++i) F[i] = dl(NAN, NAN);
  }
}

void or_residual_dual_value(int family, int n, const double* p, const double* u, double* F) {
  dual ud[OR_NMAX], Fd[OR_NMAX];
  int i;
  for (i = 0; i < n; ++i) ud[i] = dl(u[i], 0.0);
  residual_dual(family, n, p, ud, Fd);
  for (i = 0; i < n; ++i) F[i] = Fd[i].v;
}

/* Column j of J is the tangent part of F for the seed u_j + eps (one JVP). */
void or_jacobian(int family, int n, const double* p, const double* u, double* J) {
  dual ud[OR_NMAX], Fd[OR_NMAX];
  int i, j;
  for (j = 0; j < n; ++j) {
    for (i = 0; i < n; ++i) ud[i] = dl(u[i], i == j ? 1.0 : 0.0);
    residual_dual(family, n, p, ud, Fd);
    for (i = 0; i < n; ++i) J[i * n + j] = Fd[i].d;
  }
}

/* The residual again, now with dual parameters and a plain u: the tangent  */
/* part is dF/dtheta along the parameters' seeds.                            */
static void residual_dual_params(int family, int n, const dual* p, const double* u, dual* F) {
  int i, j;
  switch (family) {
    case OR_FAM_CUBIC: {
      const dual* A = p;
      const dual* b = p + n * n;
      for (i = 0; i < n; ++i) {
        dual s = dconst(0.0);
        for (j = 0; j < n; ++j) s = dadd(s, dmul(A[i * n + j], dconst(u[j])));
        dual cube = dconst(u[i] * u[i] * u[i]);
        F[i] = dsub(dadd(s, dmul(dconst(0.1), cube)), b[i]);
      }
      break;
    }
    case OR_FAM_TANH: {
      const dual* A = p;
      const dual* b = p + n * n;
      dual beta = p[n * n + n];
      for (i = 0; i < n; ++i) {
        dual s = dconst(0.0);
        for (j = 0; j < n; ++j) s = dadd(s, dmul(A[i * n + j], dconst(tanh(u[j]))));
        F[i] = dsub(dadd(s, dmul(beta, dconst(u[i]))), b[i]);
      }
      break;
    }
    case OR_FAM_ROSENBROCK: {
      F[0] = dconst(1.0 - u[0]);
      for (i = 1; i < n; ++i) F[i] = dconst(10.0 * (u[i] - u[i - 1] * u[i - 1]));
      break;
    }
    case OR_FAM_PAPER: {
      dual a = p[0], b = p[1], c = p[2];
      dual cube = dconst(u[1] * u[1] * u[1]);
      F[0] = dadd(dmul(dadd(dconst(u[0]), a), dsub(cube, b)), c);
      F[1] = dconst(sin(u[1] * exp(u[0]) - 1.0));
      break;
    }
    case OR_FAM_SQUARE: {
      for (i = 0; i < n; ++i) F[i] = dsub(dconst(u[i] * u[i]), p[i]);
      break;
    }
    default:
      for (i = 0; i < n; ++i) F[i] = dl(NAN, NAN);
  }
}

void or_param_jacobian(int family, int n, const double* p, const double* u, double* Jp) {
  const int P = or_nparams(family, n);
  dual* pd = (dual*)malloc(sizeof(dual) * (P > 0 ? P : 1));
  dual Fd[OR_NMAX];
  int i, j;
  for (j = 0; j < P; ++j) {
    for (i = 0; i < P; ++i) pd[i] = dl(p[i], i == j ? 1.0 : 0.0);
    residual_dual_params(family, n, pd, u, Fd);
    for (i = 0; i < n; ++i) Jp[i * P + j] = Fd[i].d;
  }
  free(pd);
}

/* ------------------------------------------------------------------------ */
/* LU with partial pivoting.  Step k: the pivot is the first row (in current */
/* row order, scanning upward from k) whose |a_ik| is strictly larger than   */
/* every earlier candidate; rows k and p are exchanged whole; multipliers    */
/* l = a_ik / a_kk overwrite the strict lower part.                          */
/* ------------------------------------------------------------------------ */
int or_lu(int n, double* a, int32_t* piv) {
  int i, j, k;
  for (k = 0; k < n; ++k) {
    int p = k;
    double amax = fabs(a[k * n + k]);
    for (i = k + 1; i < n; ++i) {
      double v = fabs(a[i * n + k]);
      if (v > amax) { amax = v; p = i; }
    }
    piv[k] = p;
    double pv = a[p * n + k];
    if (pv == 0.0 || !isfinite(pv)) return k + 1;
    if (p != k) {
      for (j = 0; j < n; ++j) {
        double t = a[k * n + j];
        a[k * n + j] = a[p * n + j];
        a[p * n + j] = t;
      }
    }
    for (i = k + 1; i < n; ++i) {
      double l = a[i * n + k] / a[k * n + k];
      a[i * n + k] = l;
      for (j = k + 1; j < n; ++j) a[i * n + j] = a[i * n + j] - l * a[k * n + j];
    }
  }
  return 0;
}

void or_lu_solve(int n, const double* lu, const int32_t* piv, double* b) {
  int i, j, k;
  for (k = 0; k < n; ++k) {
    if (piv[k] != k) { double t = b[k]; b[k] = b[piv[k]]; b[piv[k]] = t; }
  }
  for (i = 0; i < n; ++i)
    for (j = 0; j < i; ++j) b[i] = b[i] - lu[i * n + j] * b[j];
  for (i = n - 1; i >= 0; --i) {
    for (j = i + 1; j < n; ++j) b[i] = b[i] - lu[i * n + j] * b[j];
    b[i] = b[i] / lu[i * n + i];
  }
}

/* ------------------------------------------------------------------------ */
/* Small vector helpers (index order).                                       */
/* ------------------------------------------------------------------------ */
static int all_finite(int n, const double* x) {
  int i;
  for (i = 0; i < n; ++i) if (!isfinite(x[i])) return 0;
  return 1;
}
static double norm_inf(int n, const double* x) {
  double m = 0.0;
  int i;
  for (i = 0; i < n; ++i) { double v = fabs(x[i]); if (v > m) m = v; }
  return m;
}
#ifndef OR_PAIRWISE
static double sumsq(int n, const double* x) {
  double s = 0.0;
  int i;
  for (i = 0; i < n; ++i) s = s + x[i] * x[i];
  return s;
}
static double dot(int n, const double* x, const double* y) {
  double s = 0.0;
  int i;
  for (i = 0; i < n; ++i) s = s + x[i] * y[i];
  return s;
}
#else
/* Rounding probe (classification build only): the same sums added as a
 * balanced binary tree instead of in index order -- another rounding order of
 * the merit ||F||^2 and of the dogleg's inner products. */
static double pw_dot(const double* x, const double* y, int lo, int hi) {
  int mid;
  if (hi - lo == 1) return x[lo] * y[lo];
  mid = lo + (hi - lo) / 2;
  return pw_dot(x, y, lo, mid) + pw_dot(x, y, mid, hi);
}
static double sumsq(int n, const double* x) { return n > 0 ? pw_dot(x, x, 0, n) : 0.0; }
static double dot(int n, const double* x, const double* y) { return n > 0 ? pw_dot(x, y, 0, n) : 0.0; }
#endif
/* the reported residual norm: +inf when the residual is not finite */
static double report_norm(int n, const double* F) {
  return all_finite(n, F) ? norm_inf(n, F) : INFINITY;
}

static void trace_row(double* trace, int32_t cap, int32_t* len, const double* row) {
  if (!trace || !len || *len >= cap) return;
  memcpy(trace + (size_t)(*len) * OR_TRACE_FIELDS, row, sizeof(double) * OR_TRACE_FIELDS);
  *len += 1;
}
static void row_clear(double* row) {
  int i;
  for (i = 0; i < OR_TRACE_FIELDS; ++i) row[i] = NAN;
}

/* Rounding probe (classification builds only, never the oracle itself):
 * built with OR_JITTER = 1 or 2, every step is scaled componentwise by
 * 1 +- n 2^-53 (n times the unit roundoff: the size of the rounding error of
 * an inner product of length n, and so of the solve that made the step), up
 * or down in a pattern of (iteration, component), so that the whole
 * trajectory -- not only its start -- carries a perturbation of the size of
 * the rounding differences between two correct implementations.  A system
 * whose outcome changes under it is sensitive to the rounding order of its
 * arithmetic.  In the oracle build this is a no-op. */
#ifdef OR_JITTER
static void nudge(int n, double* d, int k) {
  int i;
  const double e = ldexp((double)n, -53);
  for (i = 0; i < n; ++i) d[i] = d[i] * (((k + i + OR_JITTER) & 1) ? 1.0 + e : 1.0 - e);
}
#define OR_NUDGE(n, d, k) nudge((n), (d), (k))
#else
#define OR_NUDGE(n, d, k) ((void)0)
#endif

/* Newton direction: J delta = -F (eq. newton_descent).  Returns 0 or singular. */
static int newton_direction(int family, int n, const double* p, const double* u, const double* F,
                            double* J, double* lu, int32_t* piv, double* delta) {
  int i;
  or_jacobian(family, n, p, u, J);
  memcpy(lu, J, sizeof(double) * n * n);
  if (or_lu(n, lu, piv) != 0) return 1;
  for (i = 0; i < n; ++i) delta[i] = -F[i];
  or_lu_solve(n, lu, piv, delta);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Sensitivities at a solution (Sec. 2.3).  Differentiating F(u*(theta),     */
/* theta) = 0 gives J D + dF/dtheta = 0 with D the derivative of u* in theta */
/* (implicit function theorem), so D = -J^{-1} dF/dtheta.  The tangent form  */
/* applies D to one parameter direction v; the adjoint form gives w^T D, the */
/* gradient of w^T u* with respect to theta, from one solve with J^T.        */
/* ------------------------------------------------------------------------ */
static int sens_setup(int family, int n, const double* p, const double* u, double* J, double* Jp, int P) {
  int i;
  for (i = 0; i < n; ++i) if (!isfinite(u[i])) return 3;
  for (i = 0; i < P; ++i) if (!isfinite(p[i])) return 3;
  or_jacobian(family, n, p, u, J);
  for (i = 0; i < n * n; ++i) if (!isfinite(J[i])) return 3;
  if (P > 0) or_param_jacobian(family, n, p, u, Jp);
  return 0;
}

int or_tangent(int family, int n, const double* p, const double* u, const double* v, double* du) {
  const int P = or_nparams(family, n);
  double J[OR_NMAX * OR_NMAX];
  double* Jp = (double*)malloc(sizeof(double) * (size_t)n * (P > 0 ? P : 1));
  int32_t piv[OR_NMAX];
  int i, j, rc = sens_setup(family, n, p, u, J, Jp, P);
  if (rc == 0) {
    /* right-hand side -(dF/dtheta) v */
    for (i = 0; i < n; ++i) {
      double s = 0.0;
      for (j = 0; j < P; ++j) s = s + Jp[i * P + j] * v[j];
      du[i] = -s;
    }
    if (or_lu(n, J, piv) != 0) rc = 2;
    else or_lu_solve(n, J, piv, du);
  }
  if (rc != 0) for (i = 0; i < n; ++i) du[i] = NAN;
  free(Jp);
  return rc;
}

int or_adjoint(int family, int n, const double* p, const double* u, const double* w, double* lambda,
               double* grad) {
  const int P = or_nparams(family, n);
  double J[OR_NMAX * OR_NMAX], Jt[OR_NMAX * OR_NMAX];
  double* Jp = (double*)malloc(sizeof(double) * (size_t)n * (P > 0 ? P : 1));
  int32_t piv[OR_NMAX];
  int i, j, rc = sens_setup(family, n, p, u, J, Jp, P);
  if (rc == 0) {
    /* J^T lambda = w, by LU with partial pivoting of the transposed matrix */
    for (i = 0; i < n; ++i)
      for (j = 0; j < n; ++j) Jt[i * n + j] = J[j * n + i];
    for (i = 0; i < n; ++i) lambda[i] = w[i];
    if (or_lu(n, Jt, piv) != 0) rc = 2;
    else or_lu_solve(n, Jt, piv, lambda);
  }
  if (rc == 0) {
    /* grad_j = -sum_i lambda_i dF_i/dtheta_j */
    for (j = 0; j < P; ++j) {
      double s = 0.0;
      for (i = 0; i < n; ++i) s = s + lambda[i] * Jp[i * P + j];
      grad[j] = -s;
    }
  } else {
    for (i = 0; i < n; ++i) lambda[i] = NAN;
    for (j = 0; j < P; ++j) grad[j] = NAN;
  }
  free(Jp);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* POLY (Sec. 3.2, default poly-algorithm): for small systems the default     */
/* chain skips the quasi-Newton phase and tries Newton-Raphson, then Newton   */
/* with a line search, then a trust-region method, moving on when one fails.  */
/* Readings: each attempt restarts from u0 with the full budget; the first    */
/* success ends the chain; when all fail the smallest final ||F||_inf wins    */
/* (the earliest attempt on ties); the counters add up over the attempts.     */
/* ------------------------------------------------------------------------ */
static or_result solve_poly(int family, int n, const double* p, const double* u0, double abstol,
                            int32_t maxiters, const or_opts* o, double* u_out) {
  static const int chain[3] = {OR_ALG_NEWTON, OR_ALG_ARMIJO, OR_ALG_DOGLEG};
  double ut[OR_NMAX];
  or_result best, r;
  int32_t iters = 0, nfev = 0, njev = 0;
  int a, have = 0;
  best.retcode = OR_RC_MAXITERS; best.iters = 0; best.nfev = 0; best.njev = 0;
  best.fnorm_inf = INFINITY;
  for (a = 0; a < 3; ++a) {
    r = or_solve_one(family, n, chain[a], p, u0, abstol, maxiters, o, ut, NULL, 0, NULL);
    iters += r.iters;
    nfev += r.nfev;
    njev += r.njev;
    if (!have || r.retcode == OR_RC_SUCCESS || r.fnorm_inf < best.fnorm_inf) {
      best = r;
      memcpy(u_out, ut, sizeof(double) * n);
      have = 1;
    }
    if (r.retcode == OR_RC_SUCCESS) break;
  }
  best.iters = iters;
  best.nfev = nfev;
  best.njev = njev;
  return best;
}

or_result or_solve_one(int family, int n, int alg, const double* p, const double* u0,
                       double abstol, int32_t maxiters, const or_opts* o_in, double* u_out,
                       double* trace, int32_t trace_cap, int32_t* trace_len) {
  or_opts o;
  or_result r;
  double u[OR_NMAX], F[OR_NMAX], Ft[OR_NMAX], ut[OR_NMAX], delta[OR_NMAX];
  double J[OR_NMAX * OR_NMAX], lu[OR_NMAX * OR_NMAX];
  double g[OR_NMAX], Jg[OR_NMAX], dN[OR_NMAX], dC[OR_NMAX], step[OR_NMAX], lin[OR_NMAX];
  int32_t piv[OR_NMAX];
  double row[OR_TRACE_FIELDS];
  int i, j, k;

  if (o_in) o = *o_in; else or_default_opts(&o);
  if (trace_len) *trace_len = 0;
  if (alg == OR_ALG_POLY) return solve_poly(family, n, p, u0, abstol, maxiters, &o, u_out);
  r.retcode = OR_RC_MAXITERS; r.iters = 0; r.nfev = 0; r.njev = 0; r.fnorm_inf = INFINITY;

  memcpy(u, u0, sizeof(double) * n);
  or_residual(family, n, p, u, F);
  r.nfev = 1;
  if (!all_finite(n, F)) {
    r.retcode = OR_RC_NONFINITE; r.iters = 0; r.fnorm_inf = INFINITY;
    memcpy(u_out, u, sizeof(double) * n);
    return r;
  }
  if (norm_inf(n, F) <= abstol) {
    r.retcode = OR_RC_SUCCESS; r.iters = 0; r.fnorm_inf = norm_inf(n, F);
    memcpy(u_out, u, sizeof(double) * n);
    return r;
  }

  if (alg == OR_ALG_NEWTON) {
    /* Sec. 2.1: J_k delta = -f(u_k), u_{k+1} = u_k + delta. */
    for (k = 1; k <= maxiters; ++k) {
      double mb = sumsq(n, F);
      r.njev += 1;
      if (newton_direction(family, n, p, u, F, J, lu, piv, delta)) {
        r.retcode = OR_RC_SINGULAR; r.iters = k; goto done;
      }
      OR_NUDGE(n, delta, k);
      for (i = 0; i < n; ++i) u[i] = u[i] + delta[i];
      or_residual(family, n, p, u, F);
      r.nfev += 1;
      row_clear(row);
      row[OR_TR_K] = k; row[OR_TR_MERIT_BEFORE] = mb; row[OR_TR_STEP] = sqrt(sumsq(n, delta));
      row[OR_TR_FINF] = report_norm(n, F); row[OR_TR_MERIT] = sumsq(n, F);
      row[OR_TR_ACCEPTED] = 1;
      trace_row(trace, trace_cap, trace_len, row);
      if (!all_finite(n, F)) { r.retcode = OR_RC_NONFINITE; r.iters = k; goto done; }
      if (norm_inf(n, F) <= abstol) { r.retcode = OR_RC_SUCCESS; r.iters = k; goto done; }
    }
    r.retcode = OR_RC_MAXITERS; r.iters = maxiters;
    goto done;
  }

  if (alg == OR_ALG_POTRA_PTAK) {
    /* Sec. 2.1, multi-step scheme of Potra and Ptak: one Jacobian, two solves.
     *   J_k d1 = -f(u_k),  y_k = u_k + d1,  J_k d2 = -f(y_k),  u_{k+1} = y_k + d2.
     * The stopping test applies to the iterates u_k; a non-finite f(y_k) ends
     * the iteration (NONFINITE, reporting y_k). */
    for (k = 1; k <= maxiters; ++k) {
      double mb = sumsq(n, F);
      r.njev += 1;
      if (newton_direction(family, n, p, u, F, J, lu, piv, delta)) {
        r.retcode = OR_RC_SINGULAR; r.iters = k; goto done;
      }
      OR_NUDGE(n, delta, k);
      for (i = 0; i < n; ++i) ut[i] = u[i] + delta[i];
      or_residual(family, n, p, ut, Ft);
      r.nfev += 1;
      if (!all_finite(n, Ft)) {
        memcpy(u, ut, sizeof(double) * n);
        memcpy(F, Ft, sizeof(double) * n);
        r.retcode = OR_RC_NONFINITE; r.iters = k; goto done;
      }
      /* the same factors, right-hand side -f(y_k) */
      for (i = 0; i < n; ++i) step[i] = -Ft[i];
      or_lu_solve(n, lu, piv, step);
      OR_NUDGE(n, step, k + 1);
      for (i = 0; i < n; ++i) u[i] = ut[i] + step[i];
      or_residual(family, n, p, u, F);
      r.nfev += 1;
      row_clear(row);
      row[OR_TR_K] = k; row[OR_TR_MERIT_BEFORE] = mb;
      row[OR_TR_STEP] = sqrt(sumsq(n, delta)); row[OR_TR_NEWTON_NORM] = sqrt(sumsq(n, step));
      row[OR_TR_FINF] = report_norm(n, F); row[OR_TR_MERIT] = sumsq(n, F);
      row[OR_TR_ACCEPTED] = 1;
      trace_row(trace, trace_cap, trace_len, row);
      if (!all_finite(n, F)) { r.retcode = OR_RC_NONFINITE; r.iters = k; goto done; }
      if (norm_inf(n, F) <= abstol) { r.retcode = OR_RC_SUCCESS; r.iters = k; goto done; }
    }
    r.retcode = OR_RC_MAXITERS; r.iters = maxiters;
    goto done;
  }

  if (alg == OR_ALG_ARMIJO) {
    /* Sec. 2.2.1: backtracking from alpha = 1 by the factor rho until
     * phi(alpha) <= phi(0) + c alpha f^T J delta, with phi = 0.5 ||f||_2^2.
     * Since J delta = -f, f^T J delta = -||f||_2^2, so the test reads
     * ||f(u + alpha delta)||_2^2 <= (1 - 2 c alpha) ||f(u)||_2^2. */
    for (k = 1; k <= maxiters; ++k) {
      r.njev += 1;
      if (newton_direction(family, n, p, u, F, J, lu, piv, delta)) {
        r.retcode = OR_RC_SINGULAR; r.iters = k; goto done;
      }
      OR_NUDGE(n, delta, k);
      double phi0 = sumsq(n, F);
      double alpha = 1.0;
      int accepted = 0, m;
      double phit = NAN;
      for (m = 0; m <= o.armijo_max_halvings; ++m) {
        for (i = 0; i < n; ++i) ut[i] = u[i] + alpha * delta[i];
        or_residual(family, n, p, ut, Ft);
        r.nfev += 1;
        if (all_finite(n, Ft)) {
          phit = sumsq(n, Ft);
          double bound = (1.0 - 2.0 * o.armijo_c * alpha) * phi0;
          if (phit <= bound) { accepted = 1; break; }
        }
        alpha = alpha * o.armijo_rho;
      }
      row_clear(row);
      row[OR_TR_K] = k; row[OR_TR_MERIT_BEFORE] = phi0;
      row[OR_TR_NEWTON_NORM] = sqrt(sumsq(n, delta));
      if (!accepted) {
        row[OR_TR_ALPHA] = 0.0; row[OR_TR_ACCEPTED] = 0;
        row[OR_TR_FINF] = norm_inf(n, F); row[OR_TR_MERIT] = phi0;
        trace_row(trace, trace_cap, trace_len, row);
        r.retcode = OR_RC_LINESEARCH_FAILED; r.iters = k; goto done;
      }
      memcpy(u, ut, sizeof(double) * n);
      memcpy(F, Ft, sizeof(double) * n);
      row[OR_TR_ALPHA] = alpha; row[OR_TR_ACCEPTED] = 1;
      row[OR_TR_STEP] = alpha * row[OR_TR_NEWTON_NORM];
      row[OR_TR_ARED] = phi0 - phit;
      row[OR_TR_FINF] = norm_inf(n, F); row[OR_TR_MERIT] = phit;
      trace_row(trace, trace_cap, trace_len, row);
      if (norm_inf(n, F) <= abstol) { r.retcode = OR_RC_SUCCESS; r.iters = k; goto done; }
    }
    r.retcode = OR_RC_MAXITERS; r.iters = maxiters;
    goto done;
  }

  if (alg == OR_ALG_DOGLEG) {
    /* Sec. 2.2.2: quadratic model m(d) = 0.5||f + J d||^2, subproblem
     * min m(d) s.t. ||d|| <= Delta solved by Powell's dogleg, ratio
     * rho = (||f||^2 - ||f(u+d)||^2) / (||f||^2 - ||f + J d||^2), and a
     * three-regime radius update (expand / keep / shrink and reject). */
    double Delta = o.tr_delta0;
    int fresh = 1;
    double nN = 0.0, ng2 = 0.0, nJg2 = 0.0;
    for (k = 1; k <= maxiters; ++k) {
      if (fresh) {
        r.njev += 1;
        if (newton_direction(family, n, p, u, F, J, lu, piv, dN)) {
          r.retcode = OR_RC_SINGULAR; r.iters = k; goto done;
        }
        /* steepest-descent direction of the merit: g = J^T f */
        for (j = 0; j < n; ++j) {
          double s = 0.0;
          for (i = 0; i < n; ++i) s = s + J[i * n + j] * F[i];
          g[j] = s;
        }
        for (i = 0; i < n; ++i) {
          double s = 0.0;
          for (j = 0; j < n; ++j) s = s + J[i * n + j] * g[j];
          Jg[i] = s;
        }
        nN = sqrt(sumsq(n, dN));
        ng2 = sumsq(n, g);
        nJg2 = sumsq(n, Jg);
        fresh = 0;
      }
      double kind, tcauchy = NAN;
      double tcauchy_trace = nJg2 > 0.0 ? ng2 / nJg2 : INFINITY; /* trace only */
      if (nN <= Delta) {
        for (i = 0; i < n; ++i) step[i] = dN[i];
        kind = 0;
      } else if (ng2 == 0.0) {
        double s = Delta / nN;
        for (i = 0; i < n; ++i) step[i] = dN[i] * s;
        kind = 3;
      } else {
        /* unconstrained minimiser of the model along -g (Cauchy point) */
        tcauchy = ng2 / nJg2;
        for (i = 0; i < n; ++i) dC[i] = -tcauchy * g[i];
        double nC2 = sumsq(n, dC);
        double nC = sqrt(nC2);
        if (nC >= Delta) {
          double s = Delta / sqrt(ng2);
          for (i = 0; i < n; ++i) step[i] = -s * g[i];
          kind = 1;
        } else {
          /* dC + tau (dN - dC) on the sphere ||.|| = Delta */
          double d[OR_NMAX];
          for (i = 0; i < n; ++i) d[i] = dN[i] - dC[i];
          double qa = dot(n, d, d);
          double qb = 2.0 * dot(n, dC, d);
          double qc = nC2 - Delta * Delta;
          double disc = qb * qb - 4.0 * qa * qc;
          double sq = sqrt(disc);
          double tau = (qb <= 0.0) ? (-qb + sq) / (2.0 * qa) : (-2.0 * qc) / (qb + sq);
          for (i = 0; i < n; ++i) step[i] = dC[i] + tau * d[i];
          kind = 2;
        }
      }
      OR_NUDGE(n, step, k);
      for (i = 0; i < n; ++i) ut[i] = u[i] + step[i];
      or_residual(family, n, p, ut, Ft);
      r.nfev += 1;
      double phi = sumsq(n, F);
      double phit = sumsq(n, Ft);
      for (i = 0; i < n; ++i) {
        double s = 0.0;
        for (j = 0; j < n; ++j) s = s + J[i * n + j] * step[j];
        lin[i] = F[i] + s;
      }
      double pred = phi - sumsq(n, lin);
      double ared = phi - phit;
      double rho = (all_finite(n, Ft) && pred > 0.0) ? ared / pred : -INFINITY;
      double nstep = sqrt(sumsq(n, step));
      int accept;
      row_clear(row);
      row[OR_TR_K] = k; row[OR_TR_MERIT_BEFORE] = phi; row[OR_TR_ALPHA] = rho;
      row[OR_TR_DELTA] = Delta; row[OR_TR_STEP] = nstep; row[OR_TR_PRED] = pred;
      row[OR_TR_ARED] = ared; row[OR_TR_GNORM] = sqrt(ng2); row[OR_TR_CAUCHY] = tcauchy_trace;
      row[OR_TR_KIND] = kind; row[OR_TR_NEWTON_NORM] = nN;
      if (rho >= o.tr_eta2) {
        accept = 1;
        Delta = fmin(o.tr_expand * Delta, o.tr_delta_max);
      } else if (rho > o.tr_eta1) {
        accept = 1;
      } else {
        accept = 0;
        Delta = o.tr_shrink * nstep;
      }
      if (accept) {
        memcpy(u, ut, sizeof(double) * n);
        memcpy(F, Ft, sizeof(double) * n);
        fresh = 1;
      }
      row[OR_TR_ACCEPTED] = accept;
      row[OR_TR_FINF] = norm_inf(n, F); row[OR_TR_MERIT] = sumsq(n, F);
      trace_row(trace, trace_cap, trace_len, row);
      if (accept) {
        if (norm_inf(n, F) <= abstol) { r.retcode = OR_RC_SUCCESS; r.iters = k; goto done; }
      } else {
        double unorm = sqrt(sumsq(n, u));
        if (Delta < o.tr_collapse * fmax(1.0, unorm)) {
          r.retcode = OR_RC_TR_COLLAPSED; r.iters = k; goto done;
        }
      }
    }
    r.retcode = OR_RC_MAXITERS; r.iters = maxiters;
    goto done;
  }

  r.retcode = -1;
done:
  r.fnorm_inf = report_norm(n, F);
  memcpy(u_out, u, sizeof(double) * n);
  return r;
}

/* ------------------------------------------------------------------------ */
/* Batch driver: contiguous chunks of systems, one pthread per chunk.        */
/* ------------------------------------------------------------------------ */
typedef struct {
  int64_t lo, hi;
  const uint8_t *family, *n, *alg;
  const double* params; const int64_t* p_off;
  const double* u0; const int64_t* u_off;
  double abstol; int32_t maxiters; const or_opts* o;
  double* u_out; double* fnorm; int32_t *iters, *retcode, *nfev, *njev;
} chunk_args;

static void* run_chunk(void* arg) {
  chunk_args* c = (chunk_args*)arg;
  int64_t s;
  for (s = c->lo; s < c->hi; ++s) {
    int n = c->n[s];
    or_result r;
    if (or_nparams(c->family[s], n) < 0 ||
        c->p_off[s + 1] - c->p_off[s] != or_nparams(c->family[s], n)) {
      c->retcode[s] = 6; c->iters[s] = 0; c->fnorm[s] = NAN;
      if (c->nfev) c->nfev[s] = 0;
      if (c->njev) c->njev[s] = 0;
      continue;
    }
    r = or_solve_one(c->family[s], n, c->alg[s], c->params + c->p_off[s], c->u0 + c->u_off[s],
                     c->abstol, c->maxiters, c->o, c->u_out + c->u_off[s], NULL, 0, NULL);
    c->retcode[s] = r.retcode; c->iters[s] = r.iters; c->fnorm[s] = r.fnorm_inf;
    if (c->nfev) c->nfev[s] = r.nfev;
    if (c->njev) c->njev[s] = r.njev;
  }
  return NULL;
}

void or_solve_batch(int64_t M, const uint8_t* family, const uint8_t* n, const uint8_t* alg,
                    const double* params, const int64_t* p_off, const double* u0,
                    const int64_t* u_off, double abstol, int32_t maxiters, const or_opts* o,
                    double* u_out, double* fnorm, int32_t* iters, int32_t* retcode,
                    int32_t* nfev, int32_t* njev, int32_t nthreads) {
  int32_t t;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  chunk_args args[256];
  pthread_t th[256];
  for (t = 0; t < nthreads; ++t) {
    chunk_args* c = &args[t];
    c->lo = M * t / nthreads; c->hi = M * (t + 1) / nthreads;
    c->family = family; c->n = n; c->alg = alg; c->params = params; c->p_off = p_off;
    c->u0 = u0; c->u_off = u_off; c->abstol = abstol; c->maxiters = maxiters; c->o = o;
    c->u_out = u_out; c->fnorm = fnorm; c->iters = iters; c->retcode = retcode;
    c->nfev = nfev; c->njev = njev;
  }
  if (nthreads == 1) { run_chunk(&args[0]); return; }
  for (t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, run_chunk, &args[t]);
  for (t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
}
