/*
 * nls_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, single-threaded, FP64 CPU reference of the batched small-system
 * nonlinear solver (paper "NonlinearSolve.jl", arXiv 2403.16341).  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg load it.
 * It shares no source, header, table or helper with the HIP library: the
 * enums below are this file's own copies of the public numbering.
 *
 * Semantics (each routine cites the passage it follows):
 *   residual families ...... problem statement, Sec. 2 eq. (nonlinear-root-finding);
 *                            generalized Rosenbrock eq. (gen_rosenbrock_function);
 *                            workflow example of Sec. 3
 *   Jacobian ............... forward-mode dual numbers, one JVP per column, Sec. 2.4
 *   LU with partial pivots . small dense LU (Sec. 3.2, default linear solver), LAPACK
 *                            getrf pivot rule (first maximum in logical row order)
 *   NEWTON ................. Sec. 2.1 eq. (newton_descent), L-inf stopping test
 *   NEWTON_ARMIJO .......... Sec. 2.2.1 eq. (sufficient-decrease), backtracking
 *   DOGLEG ................. Sec. 2.2.2 eq. (tr_subproblem), ratio rho_k, Powell dogleg
 *   POTRA_PTAK ............. Sec. 2.1 multi-step scheme: two solves with one Jacobian
 *   POLY ................... Sec. 3.2 default poly-algorithm, first-order part
 *                            (Newton, then Newton with line search, then trust region)
 *   sensitivities .......... Sec. 2.3, implicit function theorem (tangent and adjoint)
 */
#ifndef NLS_ORACLE_H
#define NLS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* OR_FAM_SQUARE (F_i = u_i^2 - p_i, the worked example of Sec. 2.3) exists in
 * the oracle only, to pin its sensitivities against the paper's closed form */
enum { OR_FAM_CUBIC = 0, OR_FAM_TANH = 1, OR_FAM_ROSENBROCK = 2, OR_FAM_PAPER = 3, OR_FAM_SQUARE = 9 };
enum { OR_ALG_NEWTON = 0, OR_ALG_ARMIJO = 1, OR_ALG_DOGLEG = 2, OR_ALG_POLY = 3, OR_ALG_POTRA_PTAK = 4 };
enum {
  OR_RC_SUCCESS = 0, OR_RC_MAXITERS = 1, OR_RC_SINGULAR = 2, OR_RC_NONFINITE = 3,
  OR_RC_LINESEARCH_FAILED = 4, OR_RC_TR_COLLAPSED = 5
};

typedef struct {
  double armijo_c;          /* sufficient-decrease constant c1            */
  double armijo_rho;        /* backtracking factor in (0,1)                */
  int32_t armijo_max_halvings; /* trials = max_halvings + 1               */
  double tr_delta0;         /* initial trust radius                        */
  double tr_delta_max;      /* radius cap                                  */
  double tr_eta1;           /* accept threshold (rho > eta1)               */
  double tr_eta2;           /* expand threshold (rho >= eta2)              */
  double tr_expand;         /* expansion factor                            */
  double tr_shrink;         /* new radius = shrink * ||step||_2 on reject  */
  double tr_collapse;       /* collapse when radius < collapse*max(1,||u||)*/
} or_opts;

void or_default_opts(or_opts* o);

/* number of parameters of a family at size n (-1 if the pair is invalid) */
int or_nparams(int family, int n);

/* plain FP64 residual F(u;p) */
void or_residual(int family, int n, const double* p, const double* u, double* F);

/* value part of the dual-number residual (must equal or_residual bit for bit) */
void or_residual_dual_value(int family, int n, const double* p, const double* u, double* F);

/* Jacobian, row-major J[i*n+j] = dF_i/du_j, from n forward-mode JVPs */
void or_jacobian(int family, int n, const double* p, const double* u, double* J);

/* In-place LU with partial pivoting (getrf semantics), row-major.  piv[k] is the
 * row exchanged with row k at step k.  Returns 0, or k+1 if the pivot of step k
 * is zero or non-finite (the factorisation stops there). */
int or_lu(int n, double* a, int32_t* piv);

/* Solve (P^T L U) x = b in place using the factors of or_lu. */
void or_lu_solve(int n, const double* lu, const int32_t* piv, double* b);

/* Per-iteration trace row (OR_TRACE_FIELDS doubles per outer iteration). */
enum {
  OR_TR_K = 0,        /* outer iteration index k                               */
  OR_TR_FINF,         /* ||F||_inf of the current iterate after the iteration  */
  OR_TR_MERIT,        /* ||F||_2^2 of the current iterate after the iteration  */
  OR_TR_MERIT_BEFORE, /* ||F||_2^2 before the iteration                        */
  OR_TR_ALPHA,        /* Armijo: accepted alpha (0 if none); dogleg: rho       */
  OR_TR_DELTA,        /* dogleg: radius used for this trial                    */
  OR_TR_STEP,         /* ||step||_2 actually tried                             */
  OR_TR_PRED,         /* dogleg predicted reduction                            */
  OR_TR_ARED,         /* actual reduction (merit_before - merit_trial)         */
  OR_TR_GNORM,        /* dogleg ||J^T F||_2                                    */
  OR_TR_CAUCHY,       /* dogleg ||g||^2/||Jg||^2                               */
  OR_TR_KIND,         /* dogleg: 0 newton, 1 boundary steepest, 2 interpolated, 3 degenerate */
  OR_TR_ACCEPTED,     /* 1 accepted, 0 rejected                                */
  OR_TR_NEWTON_NORM,  /* ||delta_newton||_2                                    */
  OR_TRACE_FIELDS
};

typedef struct {
  int32_t retcode, iters, nfev, njev;
  double fnorm_inf;
} or_result;

/* Solve one system.  u_out receives the final iterate.  trace may be NULL
 * (POLY writes no trace).  POLY runs NEWTON, ARMIJO and DOGLEG in that order,
 * each from u0 with the full iteration budget, and stops at the first
 * SUCCESS; if none succeeds it returns the attempt with the smallest
 * ||F||_inf (the earliest on ties).  Its iters, nfev and njev are totals over
 * the attempts it ran. */
or_result or_solve_one(int family, int n, int alg, const double* p, const double* u0,
                       double abstol, int32_t maxiters, const or_opts* o, double* u_out,
                       double* trace, int32_t trace_cap, int32_t* trace_len);

/* Derivative of F with respect to the parameters, n x P row-major:
 * Jp[i*P+j] = dF_i/dtheta_j, from P forward-mode JVPs (seed theta_j + eps). */
void or_param_jacobian(int family, int n, const double* p, const double* u, double* Jp);

/* Sensitivities at a solution u* of F(u, theta) = 0 (Sec. 2.3, implicit
 * function theorem; J = dF/du at u* must be nonsingular; the minus sign is
 * the theorem's):
 *   or_tangent: du = -J^{-1} (dF/dtheta) v     (v: P values; du: n values)
 *   or_adjoint: lambda = J^{-T} w, grad = -(dF/dtheta)^T lambda
 *               (w: n values; lambda: n values; grad: P values)
 * Return 0, 2 (a zero or non-finite pivot in the LU) or 3 (a non-finite
 * input or Jacobian entry); on a nonzero return the outputs are NaN. */
int or_tangent(int family, int n, const double* p, const double* u, const double* v, double* du);
int or_adjoint(int family, int n, const double* p, const double* u, const double* w, double* lambda,
               double* grad);

/* Solve a batch; offsets are [M+1] prefix arrays.  nthreads >= 1 threads each
 * run or_solve_one over a contiguous chunk.  nfev/njev may be NULL. */
void or_solve_batch(int64_t M, const uint8_t* family, const uint8_t* n, const uint8_t* alg,
                    const double* params, const int64_t* p_off, const double* u0,
                    const int64_t* u_off, double abstol, int32_t maxiters, const or_opts* o,
                    double* u_out, double* fnorm, int32_t* iters, int32_t* retcode,
                    int32_t* nfev, int32_t* njev, int32_t nthreads);

#ifdef __cplusplus
}
#endif
#endif
