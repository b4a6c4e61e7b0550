/*
 * nls.h -- C ABI of the MI355X batched small-system nonlinear solver.
 *
 * Solves M independent dense systems F(u; p) = 0, u in R^n (1 <= n <= 64),
 * in one batch on one GPU, as in the problem statement of the paper
 * (arXiv 2403.16341, Sec. 2, eq. nonlinear-root-finding): per system a residual
 * family, fixed parameters p (theta) and an initial guess u0; an absolute
 * tolerance on ||F||_inf (Sec. 2.1 stopping test); an iteration cap (Sec. 4
 * uses 1000; here a per-batch value); and an algorithm (Sec. 3 workflow: the
 * algorithm is the second argument of solve).  Per system the library returns
 * the final iterate u, ||F(u)||_inf, the iteration count and a return code
 * (the solution object and its success flag, Sec. 3.3).
 *
 * Algorithms (Sec. 2.1 and 2.2): Newton-Raphson (eq. newton_descent),
 * Newton-Raphson with backtracking under the Armijo sufficient-decrease test
 * (eq. sufficient-decrease), and a trust region whose subproblem
 * (eq. tr_subproblem) is solved by Powell's dogleg.  Jacobians come from
 * forward-mode dual numbers (Sec. 2.4); each Newton system is solved by LU
 * with partial pivoting (Sec. 3.2, small dense default).
 *
 * Conventions for every entry point:
 *   - return value: NLS_OK (0), NLS_PENDING (1, nls_query only) or a negative
 *     NLS_E_* code.  Numerical outcomes are never API errors: they are the
 *     per-system return codes NLS_RC_*.
 *   - an API error is reported before any device work is enqueued and leaves
 *     every output buffer untouched; nls_last_error() then holds a message
 *     (and, for a bad system, its index).
 *   - "host" arrays are ordinary CPU memory; "payload" arrays live where
 *     nls_batch.mem_kind says (host memory, or device memory of the context's
 *     GPU, e.g. torch tensors' data_ptr()).
 *   - the library never retains a pointer to caller memory beyond the call,
 *     except device payload pointers, which it reads/writes until nls_query
 *     reports the ticket done, and the arrays of a server request (see the
 *     request server below), held until nls_server_poll reports it.
 */
#ifndef NLS_H
#define NLS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NLS_ABI_VERSION 1
#define NLS_NMAX 64

/* ---- status codes ------------------------------------------------------ */
#define NLS_OK 0
#define NLS_PENDING 1
#define NLS_E_INVALID (-1)  /* null pointer, bad size/id/option, bad offsets  */
#define NLS_E_NOMEM (-2)    /* request can never fit the memory budget        */
#define NLS_E_DEVICE (-3)   /* HIP error (message in nls_last_error)          */
#define NLS_E_NOTFOUND (-4) /* unknown or already-released ticket             */

/* ---- residual families (parameter packing per system, row-major A) -------
 * CUBIC       F_i = sum_j A_ij u_j + 0.1 u_i^3 - b_i       p = [A (n*n), b (n)]
 * TANH        F_i = sum_j A_ij tanh(u_j) + beta u_i - b_i  p = [A (n*n), b (n), beta]
 * ROSENBROCK  F_1 = 1 - u_1, F_i = 10 (u_i - u_{i-1}^2)     p = [] (n >= 2)
 *             (generalized Rosenbrock, Sec. 2.2.1 eq. gen_rosenbrock_function)
 * PAPER_EXAMPLE  F_1 = (u_1 + a)(u_2^3 - b) + c,
 *                F_2 = sin(u_2 exp(u_1) - 1)               p = [a, b, c] (n = 2)
 *             (the workflow example of Sec. 3)                                  */
#define NLS_FAMILY_CUBIC 0
#define NLS_FAMILY_TANH 1
#define NLS_FAMILY_ROSENBROCK 2
#define NLS_FAMILY_PAPER_EXAMPLE 3

/* ---- algorithms --------------------------------------------------------- */
#define NLS_ALG_NEWTON 0        /* Sec. 2.1                                  */
#define NLS_ALG_NEWTON_ARMIJO 1 /* Sec. 2.2.1, backtracking                  */
#define NLS_ALG_DOGLEG 2        /* Sec. 2.2.2, trust region + Powell dogleg  */
/* Sec. 3.2, first-order part of the default poly-algorithm: NEWTON, then
 * NEWTON_ARMIJO, then DOGLEG, each from u0 with the full maxiters, stopping at
 * the first SUCCESS; if none succeeds, the attempt with the smallest
 * ||F||_inf (the earliest on ties) is returned.  u, fnorm_inf and retcode
 * come from the returned attempt; iters, nfev and njev are totals over the
 * attempts run.  Served by nls_solve_batch and by the request server.       */
#define NLS_ALG_POLY 3
/* Sec. 2.1, multi-step scheme of Potra and Ptak: per iteration one Jacobian
 * J_k and two solves, J_k d1 = -F(u_k), y_k = u_k + d1, J_k d2 = -F(y_k),
 * u_{k+1} = y_k + d2 (local order three).  The stopping test applies to u_k;
 * a non-finite F(y_k) ends the system as NONFINITE with u = y_k.  Counters:
 * njev = iters, nfev = 2 iters + 1.                                         */
#define NLS_ALG_POTRA_PTAK 4

/* ---- precision forms ----------------------------------------------------
 * FP64       : everything in binary64.
 * FP32_INNER : Jacobian, LU factor/solve and the dogleg step algebra in
 *              binary32; residual, norms, acceptance tests and the update
 *              u += delta stay binary64 (Newton acts as iterative refinement). */
#define NLS_PREC_FP64 0
#define NLS_PREC_FP32_INNER 1

#define NLS_MEM_HOST 0
#define NLS_MEM_DEVICE 1

/* ---- per-system return codes ------------------------------------------- */
#define NLS_RC_SUCCESS 0           /* ||F(u)||_inf <= abstol                  */
#define NLS_RC_MAXITERS 1          /* iteration cap reached                   */
#define NLS_RC_SINGULAR 2          /* zero or non-finite LU pivot             */
#define NLS_RC_NONFINITE 3         /* non-finite residual (Newton / start)    */
#define NLS_RC_LINESEARCH_FAILED 4 /* no trial passed the Armijo test         */
#define NLS_RC_TR_COLLAPSED 5      /* trust radius below collapse threshold   */
/* NLS_RC_INVALID is never a numerical outcome of a validated system.  The
 * kernels produce it only as a safeguard that keeps every launch finite:
 * (a) trip guard -- a system still running after maxiters * (max_halvings +
 *     1) + 4 main-loop trips ends with RC_INVALID, iters = -1 - k and
 *     fnorm_inf = the trip count;
 * (b) group disagreement -- in the group mapping (n > 8, or n <= 8 mapped to
 *     groups), a lane whose copy of the group's state differed from the
 *     group leader's marks the system RC_INVALID with iters = -100000.
 * Neither is expected: the test suite asserts that no system ends with it. */
#define NLS_RC_INVALID 6           /* safeguard only (see above)              */

/* ---- context ------------------------------------------------------------ */
typedef struct nls_context nls_context;

#define NLS_CTX_THREADSAFE 1u /* serialise calls on one context with a mutex */
#define NLS_CTX_AUTOTUNE 2u   /* time the mappings of each (n <= 16, family,
                                 algorithm, precision) on first use -- one
                                 system per lane (n <= 8), per 8-lane group
                                 with two rows per lane, per 16-lane group --
                                 and keep the fastest; NLS_AUTOTUNE_CACHE
                                 names a file that persists the choices; the
                                 environment variable NLS_MAPPING=lane|group,
                                 read at nls_create, fixes the n <= 8 mapping
                                 instead, and NLS_GROUP_ROWS=1 makes one row
                                 per lane the group default                  */

typedef struct {
  int32_t device;            /* HIP device ordinal                            */
  uint32_t flags;            /* NLS_CTX_*                                     */
  uint64_t mem_budget_bytes; /* device bytes the library may hold; 0 = no cap */
  void* stream;              /* hipStream_t to enqueue on; NULL = own stream  */
} nls_context_desc;

/* Algorithm options; a NULL pointer selects the defaults in brackets.
 * Armijo (Sec. 2.2.1): trial steps alpha = rho^m, m = 0..max_halvings, accept
 *   the first with ||F(u + alpha d)||_2^2 <= (1 - 2 c alpha) ||F(u)||_2^2
 *   [c = 1e-4, rho = 0.5, max_halvings = 10].
 * Trust region (Sec. 2.2.2): rho >= eta2 accept and radius = min(expand *
 *   radius, delta_max); eta1 < rho < eta2 accept; otherwise reject and radius
 *   = shrink * ||step||_2, failing with TR_COLLAPSED once radius < collapse *
 *   max(1, ||u||_2) [delta0 = 1, delta_max = 1e8, eta1 = 1e-4, eta2 = 0.75,
 *   expand = 2, shrink = 0.25, collapse = 1e-14].                             */
typedef struct {
  double armijo_c;
  double armijo_rho;
  int32_t armijo_max_halvings;
  int32_t reserved0;
  double tr_delta0;
  double tr_delta_max;
  double tr_eta1;
  double tr_eta2;
  double tr_expand;
  double tr_shrink;
  double tr_collapse;
} nls_alg_options;

/* A batch of M systems.
 *   family/n/alg : host uint8[M] per-system descriptors, or NULL to give every
 *                  system family_all / n_all / alg_all.
 *   params       : payload float64, system s uses the family's P parameters at
 *                  params[p_offset[s] .. p_offset[s] + P); p_offset: host
 *                  int64[M+1], non-decreasing with p_offset[s+1] - p_offset[s]
 *                  >= P (gaps allowed), or NULL = systems packed back to back.
 *   u0           : payload float64, system s uses u0[u_offset[s] .. +n[s]);
 *                  u_offset: host int64[M+1] with spans >= n, or NULL =
 *                  prefix sums of n.  Result u uses the same offsets; entries
 *                  in gaps are left untouched (device) or copied from u0 (host).
 *   abstol >= 0, maxiters >= 0 (0 = test the start only).                     */
typedef struct {
  int64_t count;
  const uint8_t* family;
  const uint8_t* n;
  const uint8_t* alg;
  uint8_t family_all;
  uint8_t n_all;
  uint8_t alg_all;
  uint8_t precision;    /* NLS_PREC_*                                        */
  uint32_t mem_kind;    /* NLS_MEM_* for params, u0 and every result array  */
  int32_t maxiters;
  double abstol;
  const double* params;
  const int64_t* p_offset;
  const double* u0;
  const int64_t* u_offset;
  const nls_alg_options* opts;
} nls_batch;

/* Result arrays (payload memory, caller-owned, written only by the ticket's
 * work): u uses the same offsets as u0; the others are [M].  nfev (residual
 * evaluations) and njev (Jacobian factorisations) may be NULL.              */
typedef struct {
  double* u;
  double* fnorm_inf;
  int32_t* iters;
  int32_t* retcode;
  int32_t* nfev;
  int32_t* njev;
} nls_results;

typedef struct {
  int32_t done;        /* 1 once every result of the ticket is written       */
  int32_t status;      /* NLS_OK, or NLS_E_DEVICE if its work failed         */
  double gpu_ms;       /* device time between the ticket's first and last op */
  int64_t systems;     /* M                                                  */
} nls_ticket_info;

/* Create a context on a device.  d: non-NULL.  *out receives the handle.
 * Errors: NLS_E_INVALID (NULL, bad device ordinal), NLS_E_DEVICE.           */
int nls_create(const nls_context_desc* d, nls_context** out);

/* Destroy a context: waits for its outstanding tickets, frees everything it
 * owns (never the caller's buffers or stream).  NULL is a no-op.            */
int nls_destroy(nls_context* c);

/* Validate, then enqueue the solve of batch b writing r, on the context's
 * stream; returns at once with *ticket set (device payloads) or after the
 * inputs have been copied to the device (host payloads).  The ticket must be
 * released by a nls_query call that reports it done.
 * Errors: NLS_E_INVALID (see nls_validate), NLS_E_NOMEM (the batch's device
 * footprint exceeds mem_budget_bytes), NLS_E_DEVICE.                         */
int nls_solve_batch(nls_context* c, const nls_batch* b, const nls_results* r, uint64_t* ticket);

/* Poll (wait_ms = 0), wait up to wait_ms, or wait forever (wait_ms < 0) for
 * a ticket.  Returns NLS_PENDING while it runs; NLS_OK once done, filling
 * info (may be NULL) and releasing the ticket.  Errors: NLS_E_NOTFOUND.     */
int nls_query(nls_context* c, uint64_t ticket, int32_t wait_ms, nls_ticket_info* info);

/* Host-only validation of a batch (no device touched): NLS_OK or
 * NLS_E_INVALID with *first_bad (may be NULL) = index of the first bad
 * system, or -1 for a batch-level error.                                    */
int nls_validate(const nls_batch* b, int64_t* first_bad);

/* Message of the last error on this context (or of the last context-less
 * call on this thread when c is NULL).  Never NULL.                         */
const char* nls_last_error(const nls_context* c);

/* Kernel mapping the context uses for a combination: *lanes_per_system = 1
 * (one system per lane), 8 (one system per group of 8 lanes holding two rows
 * each: n <= 16, dense families, all algorithms but Potra-Ptak) or 16/32/64
 * (one system per group of that many lanes, one row each); 0 if the
 * combination has not been tuned yet under NLS_CTX_AUTOTUNE (which chooses
 * among these for n <= 16).  Errors: NLS_E_INVALID.                          */
int nls_get_mapping(const nls_context* c, int family, int n, int alg, int precision, int32_t* lanes_per_system);

/* ---- sensitivities at a solution (Sec. 2.3) ------------------------------
 * At a root u* of F(u, theta) = 0 whose Jacobian J = dF/du is nonsingular,
 * the implicit function theorem gives the derivative of u* in the parameters
 * theta as D = -J^{-1} dF/dtheta (the theorem's minus sign).  Per system:
 *   TANGENT : du = D v for a parameter direction v (one solve with J);
 *   ADJOINT : lambda = J^{-T} w and grad = w^T D = -(dF/dtheta)^T lambda,
 *             the gradient of w . u* in theta (one solve with J^T).
 * J is formed afresh at u*; dF/dtheta are the families' parameter
 * derivatives (the forward-mode tangents of their residuals). FP64 only.   */
#define NLS_SENS_TANGENT 0
#define NLS_SENS_ADJOINT 1

/* A batch of M solved systems.  family/n, params/p_offset and u/u_offset
 * follow nls_batch (u: the solutions, laid out like u0 there).
 *   seed : TANGENT: v, laid out like params (same p_offset);
 *          ADJOINT: w, laid out like u (same u_offset).                   */
typedef struct {
  int64_t count;
  const uint8_t* family;
  const uint8_t* n;
  uint8_t family_all;
  uint8_t n_all;
  uint8_t mode;         /* NLS_SENS_*                                        */
  uint8_t reserved;
  uint32_t mem_kind;    /* NLS_MEM_* for params, u, seed and every result    */
  const double* params;
  const int64_t* p_offset;
  const double* u;
  const int64_t* u_offset;
  const double* seed;
} nls_sens_batch;

/* Results (caller-owned; entries in offset gaps are left as they are):
 *   out    : TANGENT: du, laid out like u; ADJOINT: the gradient, laid out
 *            like params (may be NULL when no system has parameters)
 *   lambda : ADJOINT only, may be NULL: J^{-T} w, laid out like u
 *   status : [M] NLS_RC_SUCCESS, NLS_RC_SINGULAR (a zero or non-finite
 *            pivot in the LU of J) or NLS_RC_NONFINITE (u, params or J not
 *            finite); the system's outputs are NaN unless SUCCESS.           */
typedef struct {
  double* out;
  double* lambda;
  int32_t* status;
} nls_sens_results;

/* Validate, then enqueue the sensitivities of batch b writing r; tickets and
 * payload rules as in nls_solve_batch (host payloads: synchronous).
 * Errors: NLS_E_INVALID (bad mode, family/size, offsets or NULL arrays),
 * NLS_E_NOMEM, NLS_E_DEVICE.                                                 */
int nls_sensitivity_batch(nls_context* c, const nls_sens_batch* b, const nls_sens_results* r, uint64_t* ticket);

/* ---- solve without allocating ---------------------------------------------
 * For callers that cannot allocate device memory: code under HIP stream
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * kernels and results as nls_solve_batch, enqueued on `stream` (a
 * hipStream_t of the current device; NULL = the null stream) with no
 * context, no ticket and no allocation: completion is stream-ordered (the
 * caller synchronises the stream).  The kernels' scratch (work counters, and
 * for NLS_ALG_POLY the lists of unsolved systems and the outputs of the
 * chain's later stages) lives in one fixed device array of
 * NLS_NOALLOC_SCRATCH_BYTES that each device holds until the process ends.
 *   b : a uniform batch -- one family, size and algorithm for every system,
 *       packed back to back (family/n/alg NULL or all equal, offsets NULL or
 *       the packed ones) -- with mem_kind NLS_MEM_DEVICE; r likewise device.
 *   NLS_ALG_POLY batches hold at most NLS_NOALLOC_MAX_CHAIN_SYSTEMS systems
 *   and NLS_NOALLOC_MAX_CHAIN_UNKNOWNS unknowns; other algorithms have no
 *   size limit beyond nls_solve_batch's.
 * Every call on one device shares that device's scratch and leaves its
 * contents behind (the kernels clear what must start at zero): calls whose
 * work overlaps on one device race, so issue them on one stream or
 * serialise them.  Errors (nothing enqueued): NLS_E_INVALID (as
 * nls_validate, host memory, or a non-uniform batch), NLS_E_NOMEM (a POLY
 * batch beyond the limits), NLS_E_DEVICE; the message is in
 * nls_last_error(NULL).                                                     */
#define NLS_NOALLOC_MAX_CHAIN_SYSTEMS 65536
#define NLS_NOALLOC_MAX_CHAIN_UNKNOWNS 1048576
#define NLS_NOALLOC_SCRATCH_BYTES 10486272
int nls_solve_batch_noalloc(const nls_batch* b, const nls_results* r, void* stream);

/* Number of float64 parameters of a family at size n, or -1 if invalid.      */
int nls_nparams(int family, int n);

/* Default option values (see nls_alg_options).                              */
void nls_default_options(nls_alg_options* o);

/* NLS_ABI_VERSION of the loaded library.                                     */
int nls_abi_version(void);

/* ---- request server ------------------------------------------------------
 * Continuous batching of independent solve requests that arrive over time
 * (the many-independent-solves setting of Sec. 4, served as a stream).  A
 * scheduler thread owned by the server admits queued requests first come,
 * first served into a device arena of mem_budget_bytes (with a pinned host
 * mirror of the same size for the copies); requests admitted together that
 * share a kernel, tolerance, iteration cap and options run as one persistent
 * launch; launches go to the least-loaded of `streams` streams, so work
 * admitted while other work runs overlaps with it on the device.  A request
 * whose footprint does not fit waits (it blocks the requests behind it) until
 * completed requests release memory.  A system's result depends only on its
 * own inputs: it is the same whether its request ran alone or in a mix.
 *
 * Requests are host-memory batches (mem_kind = NLS_MEM_HOST) of one family,
 * size and algorithm.  The server reads the batch's arrays (params, u0,
 * p_offset, u_offset) when it admits the request and writes the result
 * arrays when the request completes: unlike nls_solve_batch, the caller keeps
 * every array of a submitted request alive and untouched until nls_server_poll
 * has reported the request.                                                  */
typedef struct nls_server nls_server;

typedef struct {
  int32_t device;            /* HIP device ordinal                            */
  int32_t streams;           /* concurrent streams, 1..16 (0 = 4)             */
  uint64_t mem_budget_bytes; /* device arena for admitted requests (> 0)      */
  int32_t max_inflight;      /* launches in flight at once, 1..4096 (0 = 256)  */
  int32_t max_admit;         /* requests admitted per scheduling step (0 = 256) */
} nls_server_desc;

typedef struct {
  uint64_t id;           /* as returned by nls_server_submit                   */
  int32_t status;        /* NLS_OK, or NLS_E_DEVICE if its launch failed       */
  int32_t merged;        /* requests that shared its launch (1 = alone)        */
  int64_t systems;       /* M                                                  */
  double t_submit_ms;    /* host clock stamps, ms since the server was created */
  double t_admit_ms;     /*   admitted: taken from the queue by a scheduling   */
                         /*   step (every request of a step has its stamp)     */
  double t_done_ms;      /*   results written to the caller's arrays           */
} nls_request_info;

typedef struct {
  int64_t queued;            /* submitted, not yet admitted                   */
  int64_t inflight_launches; /* launches enqueued, not yet complete           */
  int64_t completed;         /* requests reported or ready to report          */
  int64_t launches;          /* launches issued since creation                */
  uint64_t resident_bytes;   /* arena bytes held by admitted requests         */
  uint64_t peak_resident_bytes;
  uint64_t budget_bytes;     /* arena capacity (mem_budget_bytes, rounded)    */
} nls_server_stats;

/* Create a server: allocates the device arena and its pinned host mirror and
 * starts the scheduler thread and four host copy threads (a launch with more
 * than 4 MiB of inputs or results to copy between the callers' arrays and
 * the pinned mirror has the copies done there, in jobs of about 16 MiB, while
 * the scheduler goes on admitting and completing others; the environment
 * variables NLS_SERVE_INLINE_COPY_BYTES and NLS_SERVE_COPY_JOB_BYTES, read
 * here, change the two sizes).  Errors: NLS_E_INVALID (NULL, bad device or
 * field), NLS_E_NOMEM / NLS_E_DEVICE (allocation failed).                   */
int nls_server_create(const nls_server_desc* d, nls_server** out);

/* Queue one request (validated as by nls_validate, plus the rules above).
 * r: host result arrays (nfev/njev may be NULL).  *id receives its id.
 * Errors: NLS_E_INVALID, NLS_E_NOMEM (its footprint exceeds the arena).     */
int nls_server_submit(nls_server* s, const nls_batch* b, const nls_results* r, uint64_t* id);

/* Report completed requests: waits up to wait_ms (0 = poll, < 0 = until at
 * least one is ready or nothing is outstanding), then moves up to max_out
 * completed requests, oldest completion first, into out and sets *n_out.
 * A reported request is forgotten by the server.  Errors: NLS_E_INVALID.    */
int nls_server_poll(nls_server* s, int32_t wait_ms, nls_request_info* out, int32_t max_out, int32_t* n_out);

/* Counters of the server (a consistent snapshot).                           */
int nls_server_stats_get(nls_server* s, nls_server_stats* st);

/* Drain (every submitted request runs to completion and its results are
 * written), stop the scheduler and free everything.  NULL is a no-op.       */
int nls_server_destroy(nls_server* s);

#ifdef __cplusplus
}
#endif
#endif /* NLS_H */
