// nls_kernels.hpp -- device side of the batched small-system nonlinear solver
// for gfx950 (CDNA4, wave64).
//
// Two mappings of systems onto a wavefront:
//   * lane mapping  (n <= 8):  one system per lane; the parameters, the
//     iterate and the Jacobian live in VGPRs with compile-time indices; row
//     exchanges of partial pivoting are branch-free select networks.
//   * group mapping (n <= 64): one system per group of L = 16/32/64 lanes,
//     one row (and one component of every vector) per lane; the pivot search
//     is a butterfly arg-max over the group, the pivot row is broadcast
//     through LDS, and logical row positions replace physical row swaps.
//
// What is computed follows arXiv 2403.16341:
//   residual families .... Sec. 2 problem statement; generalized Rosenbrock
//                          (Sec. 2.2.1); workflow example (Sec. 3)
//   Jacobian ............. forward-mode dual numbers: column j is the tangent
//                          of F for the seed u_j + eps (Sec. 2.4)
//   LU with partial pivots small dense LU (Sec. 3.2); pivot = first maximum
//                          in current row order
//   NEWTON ............... Sec. 2.1, eq. newton_descent, L-inf stopping test
//   NEWTON_ARMIJO ........ Sec. 2.2.1, eq. sufficient-decrease, backtracking
//   DOGLEG ............... Sec. 2.2.2, eq. tr_subproblem, ratio rho_k, Powell
//                          dogleg, three-regime radius update
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nls_types.h"

namespace nls {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool finite64(double x) { return __builtin_isfinite(x); }
__device__ __forceinline__ bool finite32(float x) { return __builtin_isfinite(x); }
template <typename T> __device__ __forceinline__ bool fin(T x) { return __builtin_isfinite(x); }

// Wave-level ordering point for LDS traffic between lanes of one wavefront
// (every workgroup here is a single wave, so no s_barrier is needed).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// Dual numbers a + a' eps, eps^2 = 0 (Sec. 2.4).
// ---------------------------------------------------------------------------
template <typename T> struct Dual {
  T v, d;
};
template <typename T> __device__ __forceinline__ Dual<T> dseed(T v) { return {v, T(1)}; }
template <typename T> __device__ __forceinline__ Dual<T> dconst(T v) { return {v, T(0)}; }
template <typename T> __device__ __forceinline__ Dual<T> operator+(Dual<T> a, Dual<T> b) {
  return {a.v + b.v, a.d + b.d};
}
template <typename T> __device__ __forceinline__ Dual<T> operator-(Dual<T> a, Dual<T> b) {
  return {a.v - b.v, a.d - b.d};
}
// (a, a')(b, b') = (ab, a'b + ab')
template <typename T> __device__ __forceinline__ Dual<T> operator*(Dual<T> a, Dual<T> b) {
  return {a.v * b.v, a.d * b.v + a.v * b.d};
}
template <typename T> __device__ __forceinline__ Dual<T> operator*(T c, Dual<T> a) {
  return {c * a.v, c * a.d};
}
// tanh with its value already known (reused from the residual at the same point)
template <typename T> __device__ __forceinline__ Dual<T> dtanh_known(Dual<T> a, T t) {
  return {t, (T(1) - t * t) * a.d};
}
__device__ __forceinline__ Dual<double> dsin(Dual<double> a) { return {sin(a.v), cos(a.v) * a.d}; }
__device__ __forceinline__ Dual<double> dexp(Dual<double> a) {
  double e = exp(a.v);
  return {e, e * a.d};
}

// derivative of the elementwise term of each dense family, by a dual pass
// with seed 1 at x:  cubic: 0.1 x^3;  tanh: beta x
__device__ __forceinline__ double cubic_term_deriv(double x) {
  Dual<double> X = dseed(x);
  Dual<double> c = X * X * X;
  return (0.1 * c).d;
}

// ---------------------------------------------------------------------------
// Lane mapping: family residual / Jacobian with compile-time N.
// ---------------------------------------------------------------------------
template <int N, int FAM> struct LaneFam;

template <int N> struct LaneFam<N, FAM_CUBIC> {
  double A[N][N];
  double b[N];
  __device__ __forceinline__ void load_lds(const double* p) { load(p); }
  __device__ __forceinline__ void load(const double* __restrict__ p) {
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) A[i][j] = p[i * N + j];
#pragma unroll
    for (int i = 0; i < N; ++i) b[i] = p[N * N + i];
  }
  // F_i = sum_j A_ij u_j + 0.1 u_i^3 - b_i   (aux unused)
  __device__ __forceinline__ void residual(const double (&u)[N], double (&F)[N], double (&aux)[N]) const {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double s = A[i][0] * u[0];
#pragma unroll
      for (int j = 1; j < N; ++j) s = __builtin_fma(A[i][j], u[j], s);
      double cube = u[i] * u[i] * u[i];
      F[i] = (s + 0.1 * cube) - b[i];
      aux[i] = 0.0;
    }
  }
  // column j = tangent for seed e_j: A[:, j] from the linear part, plus the
  // dual derivative of 0.1 u_j^3 on the diagonal
  template <typename TI>
  __device__ __forceinline__ void jacobian(const double (&u)[N], const double (&)[N], TI (&J)[N][N]) const {
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) J[i][j] = (TI)(i == j ? A[i][i] + cubic_term_deriv(u[i]) : A[i][j]);
  }
};

template <int N> struct LaneFam<N, FAM_TANH> {
  double A[N][N];
  double b[N];
  double beta;
  __device__ __forceinline__ void load_lds(const double* p) { load(p); }
  __device__ __forceinline__ void load(const double* __restrict__ p) {
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) A[i][j] = p[i * N + j];
#pragma unroll
    for (int i = 0; i < N; ++i) b[i] = p[N * N + i];
    beta = p[N * N + N];
  }
  // F_i = sum_j A_ij tanh(u_j) + beta u_i - b_i;  aux_j = tanh(u_j)
  __device__ __forceinline__ void residual(const double (&u)[N], double (&F)[N], double (&aux)[N]) const {
#pragma unroll
    for (int j = 0; j < N; ++j) aux[j] = tanh(u[j]);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double s = A[i][0] * aux[0];
#pragma unroll
      for (int j = 1; j < N; ++j) s = __builtin_fma(A[i][j], aux[j], s);
      F[i] = (s + beta * u[i]) - b[i];
    }
  }
  // column j: A[:, j] * tanh'(u_j) (dual tanh, value reused from aux) + beta e_j
  template <typename TI>
  __device__ __forceinline__ void jacobian(const double (&u)[N], const double (&aux)[N], TI (&J)[N][N]) const {
    double dphi[N];
#pragma unroll
    for (int j = 0; j < N; ++j) dphi[j] = dtanh_known(dseed(u[j]), aux[j]).d;
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) {
        double v = A[i][j] * dphi[j];
        J[i][j] = (TI)(i == j ? v + beta : v);
      }
  }
};

template <int N> struct LaneFam<N, FAM_ROSENBROCK> {
  __device__ __forceinline__ void load_lds(const double*) {}
  __device__ __forceinline__ void load(const double* __restrict__) {}
  __device__ __forceinline__ void residual(const double (&u)[N], double (&F)[N], double (&aux)[N]) const {
    F[0] = 1.0 - u[0];
    aux[0] = 0.0;
#pragma unroll
    for (int i = 1; i < N; ++i) {
      F[i] = 10.0 * (u[i] - u[i - 1] * u[i - 1]);
      aux[i] = 0.0;
    }
  }
  template <typename TI>
  __device__ __forceinline__ void jacobian(const double (&u)[N], const double (&)[N], TI (&J)[N][N]) const {
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) J[i][j] = TI(0);
    J[0][0] = TI(-1);  // tangent of 1 - u_1 for seed e_1
#pragma unroll
    for (int i = 1; i < N; ++i) {
      // 10 (u_i - u_{i-1}^2) with seed on u_{i-1}, then with seed on u_i
      Dual<double> um = dseed(u[i - 1]);
      Dual<double> fm = 10.0 * (dconst(u[i]) - um * um);
      Dual<double> fi = 10.0 * (dseed(u[i]) - dconst(u[i - 1]) * dconst(u[i - 1]));
      J[i][i - 1] = (TI)fm.d;
      J[i][i] = (TI)fi.d;
    }
  }
};

template <int N> struct LaneFam<N, FAM_PAPER> {
  static_assert(N == 2, "the workflow example has two unknowns");
  double a, b, c;
  __device__ __forceinline__ void load_lds(const double* p) { load(p); }
  __device__ __forceinline__ void load(const double* __restrict__ p) {
    a = p[0];
    b = p[1];
    c = p[2];
  }
  // F_1 = (u_1 + a)(u_2^3 - b) + c,  F_2 = sin(u_2 exp(u_1) - 1)
  __device__ __forceinline__ void residual(const double (&u)[N], double (&F)[N], double (&aux)[N]) const {
    const double cube = u[1] * u[1] * u[1];
    F[0] = (u[0] + a) * (cube - b) + c;
    F[1] = sin(u[1] * exp(u[0]) - 1.0);
    aux[0] = aux[1] = 0.0;
  }
  // two JVPs with seeds e_1, e_2 through the same expression on duals
  template <typename TI>
  __device__ __forceinline__ void jacobian(const double (&u)[N], const double (&)[N], TI (&J)[N][N]) const {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const Dual<double> x0 = {u[0], j == 0 ? 1.0 : 0.0};
      const Dual<double> x1 = {u[1], j == 1 ? 1.0 : 0.0};
      const Dual<double> cube = x1 * x1 * x1;
      const Dual<double> f0 = (x0 + dconst(a)) * (cube - dconst(b)) + dconst(c);
      const Dual<double> f1 = dsin(x1 * dexp(x0) - dconst(1.0));
      J[0][j] = (TI)f0.d;
      J[1][j] = (TI)f1.d;
    }
  }
};

// ---------------------------------------------------------------------------
// Lane LU with partial pivoting, RHS carried along (forward substitution is
// applied while eliminating), then back substitution.  Returns false on a
// zero or non-finite pivot.  x holds the RHS on entry, the solution on exit.
// ---------------------------------------------------------------------------
template <int N, typename T>
__device__ __forceinline__ bool lane_lu_solve(T (&a)[N][N], T (&x)[N]) {
  bool ok = true;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    // first maximum of |a_ik|, i >= k, in current row order
    T best = __builtin_fabs(a[k][k]);
    int p = k;
#pragma unroll
    for (int i = k + 1; i < N; ++i) {
      T v = __builtin_fabs(a[i][k]);
      bool c = v > best;
      best = c ? v : best;
      p = c ? i : p;
    }
    // exchange rows k and p (columns k.. and the RHS) with selects; the whole
    // network is skipped when no lane of the wavefront needs an exchange
    if (__any(p != k)) {
#pragma unroll
      for (int i = k + 1; i < N; ++i) {
        const bool sel = (p == i);
#pragma unroll
        for (int j = k; j < N; ++j) {
          T t = a[k][j];
          a[k][j] = sel ? a[i][j] : t;
          a[i][j] = sel ? t : a[i][j];
        }
        T t = x[k];
        x[k] = sel ? x[i] : t;
        x[i] = sel ? t : x[i];
      }
    }
    const T piv = a[k][k];
    ok = ok && (piv != T(0)) && fin(piv);
    const T r = T(1) / piv;
    a[k][k] = r;  // the pivot is only needed as its reciprocal from here on
#pragma unroll
    for (int i = k + 1; i < N; ++i) {
      const T l = a[i][k] * r;
#pragma unroll
      for (int j = k + 1; j < N; ++j) a[i][j] = __builtin_fma(-l, a[k][j], a[i][j]);
      x[i] = __builtin_fma(-l, x[k], x[i]);
    }
  }
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    T s = x[i];
#pragma unroll
    for (int j = i + 1; j < N; ++j) s = __builtin_fma(-a[i][j], x[j], s);
    x[i] = s * a[i][i];
  }
  return ok;
}

template <int N> __device__ __forceinline__ bool all_finite(const double (&F)[N]) {
  bool ok = true;
#pragma unroll
  for (int i = 0; i < N; ++i) ok = ok && finite64(F[i]);
  return ok;
}
template <int N> __device__ __forceinline__ double norm_inf(const double (&F)[N]) {
  double m = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) m = fmax(m, __builtin_fabs(F[i]));
  return m;
}
template <int N, typename T> __device__ __forceinline__ T sumsq(const T (&x)[N]) {
  T s = x[0] * x[0];
#pragma unroll
  for (int i = 1; i < N; ++i) s = __builtin_fma(x[i], x[i], s);
  return s;
}

// ---------------------------------------------------------------------------
// Lane-mapping solver kernel: one system per lane, persistent wavefronts.
//
// Each wavefront walks the 64-system chunks blockIdx.x, blockIdx.x +
// gridDim.x, ...  A lane whose system finishes writes its results and takes
// the next system of the wavefront's current chunk (retire and refill), so a
// wavefront does not wait for its slowest lane.  Every trip of the main loop
// runs one phase-uniform step: a factorisation for the lanes that need a new
// direction, then one residual evaluation for every lane holding a trial
// point.  When the batch is uniform and packed, the parameters of the next
// chunk are copied into LDS with coalesced global->LDS loads as soon as the
// previous chunk has been handed out, so the copy overlaps the solve.
// ---------------------------------------------------------------------------
template <int N, int FAM> struct LaneParams {
  static constexpr int P = FAM == FAM_CUBIC ? N * N + N
                         : FAM == FAM_TANH ? N * N + N + 1
                         : FAM == FAM_PAPER ? 3 : 0;
};

enum : int { ST_IDLE = 0, ST_DIR = 1, ST_TRIAL = 2 };

// copy `bytes` (a multiple of 8) from global memory into LDS, 16 bytes per
// lane per instruction and a 4-byte-granule tail; asynchronous until the next
// s_waitcnt
__device__ __forceinline__ void stage_to_lds(const double* __restrict__ src, double* dst, int64_t bytes) {
  const int lane = threadIdx.x;
  const char* g = reinterpret_cast<const char*>(src);
  char* l = reinterpret_cast<char*>(dst);
  const int64_t full = bytes & ~int64_t(1023);
  for (int64_t off = 0; off < full; off += 1024) {
    __builtin_amdgcn_global_load_lds(g + off + lane * 16,
                                     (__attribute__((address_space(3))) void*)(l + off), 16, 0, 0);
  }
  // remainder (a multiple of 8 bytes): 4 bytes per lane per instruction
  for (int64_t off = full; off < bytes; off += 256) {
    if (off + lane * 4 < bytes)
      __builtin_amdgcn_global_load_lds(g + off + lane * 4,
                                       (__attribute__((address_space(3))) void*)(l + off), 4, 0, 0);
  }
}

template <int N, int FAM, int ALG, typename TI>
__global__ __launch_bounds__(64) void k_lane(const KArgs a) {
  constexpr int P = LaneParams<N, FAM>::P;
  constexpr int PS = P > 0 ? P : 1;
  __shared__ __attribute__((aligned(16))) double stage[64 * PS];

  const int lane = threadIdx.x;
  const bool staged = P > 0 && a.sys == nullptr && a.p_off == nullptr;
  const int64_t nchunks = (a.count + 63) / 64;
  const double tol = a.abstol;
  const int32_t maxit = a.maxiters;
  const double c2 = 2.0 * a.o.armijo_c;
  const double rho_bt = a.o.armijo_rho;
  const int32_t mh = a.o.armijo_max_halvings;
  const DoglegOpts o = a.o.dogleg();

  // chunk currently being handed out (wave-uniform)
  int64_t chunk = blockIdx.x;
  int buf_next = 0, buf_cnt = 0;
  bool buf_wait = false;
  if (chunk < nchunks) {
    buf_cnt = (int)min<int64_t>(64, a.count - chunk * 64);
    if (staged) {
      stage_to_lds(a.params + chunk * 64 * (int64_t)P, stage, (int64_t)buf_cnt * P * 8);
      buf_wait = true;
    }
  }

  // per-lane state
  int st = ST_IDLE;
  int64_t s = 0, uo = 0;
  int32_t k = 0, nf = 0, nj = 0, m = 0;
  double alpha = 1.0, phi0 = 0.0, Delta = o.delta0;
  LaneFam<N, FAM> fam;
  double u[N], F[N], aux[N], d[N];
  TI dN[N], g[N], dC[N], dd[N];
  TI nN = 0, ng2 = 0, nJg2 = 0, tC = 0, nC2 = 0, qa = 0, qb = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) { u[i] = F[i] = aux[i] = d[i] = 0.0; dN[i] = g[i] = dC[i] = dd[i] = TI(0); }

  auto finish = [&](int32_t rc, int32_t iters) {
#pragma unroll
    for (int i = 0; i < N; ++i) a.u_out[uo + i] = u[i];
    a.fnorm[s] = all_finite(F) ? norm_inf(F) : __builtin_inf();
    a.iters[s] = iters;
    a.retcode[s] = rc;
    if (a.nfev) a.nfev[s] = nf;
    if (a.njev) a.njev[s] = nj;
    st = ST_IDLE;
  };

  while (true) {
    // ---------------- retire / refill ----------------
    const bool more = chunk < nchunks;
    if (__any(st == ST_IDLE) && more) {
      if (buf_wait) {
        __builtin_amdgcn_s_waitcnt(0);
        wave_sync();
        buf_wait = false;
      }
      const unsigned long long idle = __ballot(st == ST_IDLE);
      const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(idle >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((unsigned)idle, 0u));
      const int take = min(__popcll(idle), buf_cnt - buf_next);
      const bool fresh = st == ST_IDLE && rank < take;
      if (fresh) {
        const int slot = buf_next + rank;
        const int64_t t = chunk * 64 + slot;
        s = a.sys ? (int64_t)a.sys[t] : t;
        uo = a.u_off ? a.u_off[s] : s * N;
        if (staged) fam.load_lds(stage + slot * P);
        else fam.load(a.params + (a.p_off ? a.p_off[s] : s * a.P));
#pragma unroll
        for (int i = 0; i < N; ++i) u[i] = a.u0[uo + i];
      }
      buf_next += take;
      if (buf_next == buf_cnt) {
        // chunk handed out: once every lane has read its slot, start copying
        // the next chunk into the same buffer
        __builtin_amdgcn_s_waitcnt(0);
        wave_sync();
        chunk += gridDim.x;
        buf_next = 0;
        buf_cnt = chunk < nchunks ? (int)min<int64_t>(64, a.count - chunk * 64) : 0;
        if (staged && chunk < nchunks) {
          stage_to_lds(a.params + chunk * 64 * (int64_t)P, stage, (int64_t)buf_cnt * P * 8);
          buf_wait = true;
        }
      }
      if (fresh) {
        fam.residual(u, F, aux);
        nf = 1;
        nj = 0;
        k = 0;
        Delta = o.delta0;
        st = ST_DIR;
        if (!all_finite(F)) finish(RC_NONFINITE, 0);
        else if (norm_inf(F) <= tol) finish(RC_SUCCESS, 0);
        else if (maxit == 0) finish(RC_MAXITERS, 0);
      }
    }
    if (__all(st == ST_IDLE) && chunk >= nchunks) break;

    // ---------------- direction (lanes that need one) ----------------
    if (ALG == ALG_DOGLEG && st != ST_IDLE) ++k;  // every trial is an iteration
    if (__any(st == ST_DIR)) {
      if (st == ST_DIR) {
        if (ALG != ALG_DOGLEG) ++k;
        TI J[N][N];
        fam.template jacobian<TI>(u, aux, J);
        ++nj;
        if (ALG != ALG_DOGLEG) {
          // J_k delta = -F(u_k)
          TI x[N];
#pragma unroll
          for (int i = 0; i < N; ++i) x[i] = (TI)(-F[i]);
          if (!lane_lu_solve<N, TI>(J, x)) {
            finish(RC_SINGULAR, k);
          } else {
#pragma unroll
            for (int i = 0; i < N; ++i) d[i] = (double)x[i];
            alpha = 1.0;
            m = 0;
            phi0 = sumsq<N, double>(F);
            st = ST_TRIAL;
          }
        } else {
          TI Ff[N];
#pragma unroll
          for (int i = 0; i < N; ++i) Ff[i] = (TI)F[i];
          // g = J^T F (steepest-descent direction of 0.5||F||^2), Jg = J g
          TI Jg[N];
#pragma unroll
          for (int j = 0; j < N; ++j) {
            TI sacc = J[0][j] * Ff[0];
#pragma unroll
            for (int i = 1; i < N; ++i) sacc = __builtin_fma(J[i][j], Ff[i], sacc);
            g[j] = sacc;
          }
#pragma unroll
          for (int i = 0; i < N; ++i) {
            TI sacc = J[i][0] * g[0];
#pragma unroll
            for (int j = 1; j < N; ++j) sacc = __builtin_fma(J[i][j], g[j], sacc);
            Jg[i] = sacc;
          }
#pragma unroll
          for (int i = 0; i < N; ++i) dN[i] = -Ff[i];
          if (!lane_lu_solve<N, TI>(J, dN)) {
            finish(RC_SINGULAR, k);
          } else {
            nN = __builtin_sqrt(sumsq<N, TI>(dN));
            ng2 = sumsq<N, TI>(g);
            nJg2 = sumsq<N, TI>(Jg);
            // the Cauchy point and the dogleg segment do not depend on the radius
            tC = ng2 / nJg2;
#pragma unroll
            for (int i = 0; i < N; ++i) dC[i] = -tC * g[i];
            nC2 = sumsq<N, TI>(dC);
#pragma unroll
            for (int i = 0; i < N; ++i) dd[i] = dN[i] - dC[i];
            qa = sumsq<N, TI>(dd);
            TI dcd = dC[0] * dd[0];
#pragma unroll
            for (int i = 1; i < N; ++i) dcd = __builtin_fma(dC[i], dd[i], dcd);
            qb = TI(2) * dcd;
            st = ST_TRIAL;
          }
        }
      }
    }

    // ---------------- trial point, residual, decision ----------------
    if (st == ST_TRIAL) {
      double ut[N], Ft[N], auxt[N];
      double step[N];
      double pred = 0.0, phi = 0.0;
      if (ALG == ALG_NEWTON) {
#pragma unroll
        for (int i = 0; i < N; ++i) ut[i] = u[i] + d[i];
      } else if (ALG == ALG_ARMIJO) {
#pragma unroll
        for (int i = 0; i < N; ++i) ut[i] = __builtin_fma(alpha, d[i], u[i]);
      } else {
        // dogleg step for the current radius (step algebra in TI)
        phi = sumsq<N, double>(F);
        const TI D = (TI)Delta;
        if ((double)nN <= Delta) {
#pragma unroll
          for (int i = 0; i < N; ++i) step[i] = (double)dN[i];
          pred = phi;  // F + J dN = 0
        } else if (ng2 == TI(0)) {
          const TI r = D / nN;
#pragma unroll
          for (int i = 0; i < N; ++i) step[i] = (double)(dN[i] * r);
          const double om = 1.0 - (double)r;
          pred = phi * (1.0 - om * om);  // F + J step = (1 - r) F
        } else if (__builtin_sqrt(nC2) >= D) {
          const TI sc = D / __builtin_sqrt(ng2);
#pragma unroll
          for (int i = 0; i < N; ++i) step[i] = (double)(-sc * g[i]);
          // ||F - sc Jg||^2 = phi - 2 sc ||g||^2 + sc^2 ||Jg||^2, as F.Jg = ||g||^2
          pred = (double)sc * (2.0 * (double)ng2 - (double)sc * (double)nJg2);
        } else {
          const TI qc = nC2 - D * D;
          const TI disc = qb * qb - TI(4) * qa * qc;
          const TI sq = __builtin_sqrt(disc);
          const TI tau = (qb <= TI(0)) ? (-qb + sq) / (TI(2) * qa) : (TI(-2) * qc) / (qb + sq);
#pragma unroll
          for (int i = 0; i < N; ++i) step[i] = (double)__builtin_fma(tau, dd[i], dC[i]);
          // F + J step = (1 - tau)(F - tC Jg), ||F - tC Jg||^2 = phi - tC ||g||^2
          const double om = 1.0 - (double)tau;
          pred = phi - om * om * (phi - (double)tC * (double)ng2);
        }
#pragma unroll
        for (int i = 0; i < N; ++i) ut[i] = u[i] + step[i];
      }
      fam.residual(ut, Ft, auxt);
      ++nf;
      if (ALG == ALG_NEWTON) {
#pragma unroll
        for (int i = 0; i < N; ++i) { u[i] = ut[i]; F[i] = Ft[i]; aux[i] = auxt[i]; }
        if (!all_finite(F)) finish(RC_NONFINITE, k);
        else if (norm_inf(F) <= tol) finish(RC_SUCCESS, k);
        else if (k >= maxit) finish(RC_MAXITERS, maxit);
        else st = ST_DIR;
      } else if (ALG == ALG_ARMIJO) {
        if (all_finite(Ft) && sumsq<N, double>(Ft) <= (1.0 - c2 * alpha) * phi0) {
#pragma unroll
          for (int i = 0; i < N; ++i) { u[i] = ut[i]; F[i] = Ft[i]; aux[i] = auxt[i]; }
          if (norm_inf(F) <= tol) finish(RC_SUCCESS, k);
          else if (k >= maxit) finish(RC_MAXITERS, maxit);
          else st = ST_DIR;
        } else {
          ++m;
          alpha *= rho_bt;
          if (m > mh) finish(RC_LINESEARCH_FAILED, k);
        }
      } else {
        const double ared = phi - sumsq<N, double>(Ft);
        const double rho = (all_finite(Ft) && pred > 0.0) ? ared / pred : -__builtin_inf();
        bool accept;
        if (rho >= o.eta2) {
          accept = true;
          Delta = fmin(o.expand * Delta, o.delta_max);
        } else if (rho > o.eta1) {
          accept = true;
        } else {
          accept = false;
          Delta = o.shrink * __builtin_sqrt(sumsq<N, double>(step));
        }
        if (accept) {
#pragma unroll
          for (int i = 0; i < N; ++i) { u[i] = ut[i]; F[i] = Ft[i]; aux[i] = auxt[i]; }
          if (norm_inf(F) <= tol) finish(RC_SUCCESS, k);
          else if (k >= maxit) finish(RC_MAXITERS, maxit);
          else st = ST_DIR;
        } else {
          const double un = __builtin_sqrt(sumsq<N, double>(u));
          if (Delta < o.collapse * fmax(1.0, un)) finish(RC_TR_COLLAPSED, k);
          else if (k >= maxit) finish(RC_MAXITERS, maxit);
        }
      }
    }
  }
}

}  // namespace nls

namespace nls {

// ---------------------------------------------------------------------------
// Group mapping: one system per group of L lanes (L = 16, 32 or 64), lane r
// owns row r of A and J and component r of every vector.  Sizes up to the
// bucket NB are handled with a runtime n <= NB: rows and columns n..NB-1 are
// zero and never take part in a pivot search.
// ---------------------------------------------------------------------------
template <int L, typename T> __device__ __forceinline__ T grp_sum(T v) {
#pragma unroll
  for (int m = 1; m < L; m <<= 1) v += __shfl_xor(v, m, L);
  return v;
}
template <int L, typename T> __device__ __forceinline__ T grp_max(T v) {
#pragma unroll
  for (int m = 1; m < L; m <<= 1) v = fmax(v, __shfl_xor(v, m, L));
  return v;
}
// true if pred holds on any lane of this lane's group
template <int L> __device__ __forceinline__ bool grp_any(bool pred) {
  const unsigned long long b = __ballot(pred);
  const int gi = threadIdx.x / L;
  const unsigned long long mask = (L == 64) ? ~0ull : (((1ull << L) - 1ull) << (gi * L));
  return (b & mask) != 0ull;
}

template <int NB, int L, typename TI> struct GroupShared {
  static constexpr int G = 64 / L;
  // per-component arrays are sized by the group width L so that every lane
  // (including lanes r >= n that own no row) has a slot of its own
  double x[G][L];        // evaluation point
  double aux[G][L];      // tanh of the evaluation point (tanh family)
  double dphi[G][L];     // dual derivative of the column map at the current u
  TI piv[G][NB + 2];     // pivot row of the current elimination step + RHS
  TI sol[G][L];          // solution of the triangular solves
  TI gv[G][L];           // g = J^T F
};
template <int NB, int L, typename TI> struct GroupSharedT {
  static constexpr int G = 64 / L;
  TI t[G][L][NB];        // products J_ij F_i for the column sums of J^T F
};

template <int NB, int FAM> struct RowFam;

template <int NB> struct RowFam<NB, FAM_CUBIC> {
  double A[NB];
  double b;
  __device__ __forceinline__ void load(const double* __restrict__ p, int n, int r, bool own) {
#pragma unroll
    for (int j = 0; j < NB; ++j) A[j] = (own && j < n) ? p[r * n + j] : 0.0;
    b = own ? p[n * n + r] : 0.0;
  }
  // F_r = sum_j A_rj x_j + 0.1 x_r^3 - b_r   (x read from LDS)
  template <int L, typename TI>
  __device__ __forceinline__ double residual(GroupShared<NB, L, TI>& sh, int gi, int r, bool own,
                                             double xr, double& auxr) const {
    sh.x[gi][r] = xr;
    wave_sync();
    double s = A[0] * sh.x[gi][0];
#pragma unroll
    for (int j = 1; j < NB; ++j) s = __builtin_fma(A[j], sh.x[gi][j], s);
    auxr = 0.0;
    wave_sync();
    return own ? (s + 0.1 * (xr * xr * xr)) - b : 0.0;
  }
  template <int L, typename TI>
  __device__ __forceinline__ void jacobian_row(GroupShared<NB, L, TI>& sh, int gi, int r, bool own,
                                               double ur, double, TI (&J)[NB]) const {
    const double diag = cubic_term_deriv(ur);
#pragma unroll
    for (int j = 0; j < NB; ++j) J[j] = (TI)((j == r && own) ? A[j] + diag : A[j]);
  }
};

template <int NB> struct RowFam<NB, FAM_TANH> {
  double A[NB];
  double b, beta;
  __device__ __forceinline__ void load(const double* __restrict__ p, int n, int r, bool own) {
#pragma unroll
    for (int j = 0; j < NB; ++j) A[j] = (own && j < n) ? p[r * n + j] : 0.0;
    b = own ? p[n * n + r] : 0.0;
    beta = p[n * n + n];
  }
  // F_r = sum_j A_rj tanh(x_j) + beta x_r - b_r; lane j computes tanh(x_j)
  template <int L, typename TI>
  __device__ __forceinline__ double residual(GroupShared<NB, L, TI>& sh, int gi, int r, bool own,
                                             double xr, double& auxr) const {
    auxr = own ? tanh(xr) : 0.0;
    sh.aux[gi][r] = auxr;
    wave_sync();
    double s = A[0] * sh.aux[gi][0];
#pragma unroll
    for (int j = 1; j < NB; ++j) s = __builtin_fma(A[j], sh.aux[gi][j], s);
    wave_sync();
    return own ? (s + beta * xr) - b : 0.0;
  }
  // J_rj = A_rj tanh'(u_j) + beta [r == j]; tanh'(u_j) from the dual tanh of lane j
  template <int L, typename TI>
  __device__ __forceinline__ void jacobian_row(GroupShared<NB, L, TI>& sh, int gi, int r, bool own,
                                               double ur, double auxr, TI (&J)[NB]) const {
    sh.dphi[gi][r] = own ? dtanh_known(dseed(ur), auxr).d : 0.0;
    wave_sync();
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const double v = A[j] * sh.dphi[gi][j];
      J[j] = (TI)((j == r && own) ? v + beta : v);
    }
    wave_sync();
  }
};

template <int NB> struct RowFam<NB, FAM_ROSENBROCK> {
  __device__ __forceinline__ void load(const double* __restrict__, int, int, bool) {}
  template <int L, typename TI>
  __device__ __forceinline__ double residual(GroupShared<NB, L, TI>& sh, int gi, int r, bool own,
                                             double xr, double& auxr) const {
    sh.x[gi][r] = xr;
    wave_sync();
    const double xm = (own && r > 0) ? sh.x[gi][r - 1] : 0.0;
    wave_sync();
    auxr = 0.0;
    if (!own) return 0.0;
    return r == 0 ? 1.0 - xr : 10.0 * (xr - xm * xm);
  }
  template <int L, typename TI>
  __device__ __forceinline__ void jacobian_row(GroupShared<NB, L, TI>& sh, int gi, int r, bool own,
                                               double ur, double, TI (&J)[NB]) const {
    sh.x[gi][r] = ur;
    wave_sync();
    const double um = (own && r > 0) ? sh.x[gi][r - 1] : 0.0;
    wave_sync();
    // 10 (u_r - u_{r-1}^2) with seeds on u_{r-1} and on u_r; 1 - u_0 for r = 0
    const Dual<double> dm = 10.0 * (dconst(ur) - dseed(um) * dseed(um));
    const Dual<double> dd = r == 0 ? dconst(1.0) - dseed(ur) : 10.0 * (dseed(ur) - dconst(um) * dconst(um));
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      double v = 0.0;
      v = (j == r) ? dd.d : v;
      v = (j == r - 1) ? dm.d : v;
      J[j] = (TI)(own ? v : 0.0);
    }
  }
};

// LU with partial pivoting of the group's rows (logical positions instead of
// row exchanges), RHS carried along, then back substitution.  On return the
// solution component r is in sh.sol[gi][r].  Returns false (group-uniform) on
// a zero or non-finite pivot.
template <int NB, int L, typename TI>
__device__ __forceinline__ bool group_lu_solve(GroupShared<NB, L, TI>& sh, int gi, int r, int n,
                                               TI (&J)[NB], TI rhs) {
  const bool own = r < n;
  int pos = own ? r : NB + 1 + r;  // logical row position; non-rows never pivot
  bool ok = true;
  TI myrd = TI(0);  // reciprocal of this row's pivot, once it has been the pivot row
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    if (k < n) {
      const TI v = J[k];
      const bool cand = pos >= k && pos < NB;
      // the row in position k wins every tie and keeps a NaN (-> singular);
      // other NaN rows never win: they rank below every number
      const bool nan_at_k = grp_any<L>(pos == k && v != v);
      TI key = cand ? (v != v ? TI(-1) : __builtin_fabs(v)) : TI(-2);
      int kp = pos;
#pragma unroll
      for (int m = 1; m < L; m <<= 1) {
        const TI ok_ = __shfl_xor(key, m, L);
        const int op = __shfl_xor(kp, m, L);
        const bool take = ok_ > key || (ok_ == key && op < kp);
        key = take ? ok_ : key;
        kp = take ? op : kp;
      }
      // the pivot row publishes columns k.. and its RHS
      if (pos == kp) {
#pragma unroll
        for (int j = k; j < NB; ++j) sh.piv[gi][j] = J[j];
        sh.piv[gi][NB] = rhs;
      }
      wave_sync();
      const TI pv = sh.piv[gi][k];
      ok = ok && !nan_at_k && pv != TI(0) && fin(pv);
      const TI rp = TI(1) / pv;
      // exchange of logical positions k <-> kp
      if (pos == kp) myrd = rp;
      if (pos == kp) pos = k;
      else if (pos == k) pos = kp;
      if (own && pos > k) {
        const TI l = J[k] * rp;
        J[k] = l;
#pragma unroll
        for (int j = k + 1; j < NB; ++j) J[j] = __builtin_fma(-l, sh.piv[gi][j], J[j]);
        rhs = __builtin_fma(-l, sh.piv[gi][NB], rhs);
      }
      wave_sync();
    }
  }
  // back substitution, column by column from the last
#pragma unroll
  for (int k = NB - 1; k >= 0; --k) {
    if (k < n) {
      if (pos == k) sh.sol[gi][k] = rhs * myrd;
      wave_sync();
      if (own && pos < k) rhs = __builtin_fma(-J[k], sh.sol[gi][k], rhs);
      wave_sync();
    }
  }
  return ok;
}

template <int NB, int L, int FAM, int ALG, typename TI>
__global__ __launch_bounds__(64) void k_group(const KArgs a) {
  constexpr int G = 64 / L;
  __shared__ GroupShared<NB, L, TI> sh;
  const int lane = threadIdx.x;
  const int gi = lane / L;
  const int r = lane % L;
  const int64_t t = (int64_t)blockIdx.x * G + gi;
  if (t >= a.count) return;  // whole group leaves together
  const int64_t s = a.sys ? (int64_t)a.sys[t] : t;
  const int n = a.nsys ? (int)a.nsys[s] : a.n;
  const bool own = r < n;
  const double* __restrict__ p = a.params + (a.p_off ? a.p_off[s] : s * a.P);
  const int64_t uo = a.u_off ? a.u_off[s] : s * (int64_t)n;

  RowFam<NB, FAM> fam;
  fam.load(p, n, r, own);
  double u = own ? a.u0[uo + r] : 0.0;
  double aux = 0.0;
  double F = fam.template residual<L, TI>(sh, gi, r, own, u, aux);

  int32_t rc = RC_MAXITERS, it = 0, nf = 1, nj = 0;
  const double tol = a.abstol;
  const int32_t maxit = a.maxiters;
  bool done = true;
  if (grp_any<L>(!finite64(F))) {
    rc = RC_NONFINITE;
  } else if (grp_max<L>(__builtin_fabs(F)) <= tol) {
    rc = RC_SUCCESS;
  } else {
    done = false;
  }

  if (!done && (ALG == ALG_NEWTON || ALG == ALG_ARMIJO)) {
    const double c2 = 2.0 * a.o.armijo_c;
    const double rho = a.o.armijo_rho;
    const int32_t mh = a.o.armijo_max_halvings;
    int k = 1;
    for (; k <= maxit; ++k) {
      TI J[NB];
      fam.template jacobian_row<L, TI>(sh, gi, r, own, u, aux, J);
      ++nj;
      if (!group_lu_solve<NB, L, TI>(sh, gi, r, n, J, (TI)(-F))) { rc = RC_SINGULAR; break; }
      const double d = own ? (double)sh.sol[gi][r] : 0.0;
      wave_sync();
      if (ALG == ALG_NEWTON) {
        u += d;
        F = fam.template residual<L, TI>(sh, gi, r, own, u, aux);
        ++nf;
        if (grp_any<L>(!finite64(F))) { rc = RC_NONFINITE; break; }
        if (grp_max<L>(__builtin_fabs(F)) <= tol) { rc = RC_SUCCESS; break; }
      } else {
        const double phi0 = grp_sum<L>(F * F);
        double alpha = 1.0;
        bool acc = false;
        double ut = u, Ft = F, auxt = aux;
        for (int m = 0; m <= mh; ++m) {
          ut = __builtin_fma(alpha, d, u);
          Ft = fam.template residual<L, TI>(sh, gi, r, own, ut, auxt);
          ++nf;
          const bool fin_t = !grp_any<L>(!finite64(Ft));
          const double phit = grp_sum<L>(Ft * Ft);
          if (fin_t && phit <= (1.0 - c2 * alpha) * phi0) { acc = true; break; }
          alpha *= rho;
        }
        if (!acc) { rc = RC_LINESEARCH_FAILED; break; }
        u = ut;
        F = Ft;
        aux = auxt;
        if (grp_max<L>(__builtin_fabs(F)) <= tol) { rc = RC_SUCCESS; break; }
      }
    }
    it = k > maxit ? maxit : k;
  }

  if (!done && ALG == ALG_DOGLEG) {
    __shared__ GroupSharedT<NB, L, TI> st;
    const DoglegOpts o = a.o.dogleg();
    double Delta = o.delta0;
    bool fresh = true;
    TI dN = 0, g = 0, dC = 0, dd = 0;
    TI nN = 0, ng2 = 0, nJg2 = 0, tC = 0, nC2 = 0, qa = 0, qb = 0;
    int k = 1;
    for (; k <= maxit; ++k) {
      if (fresh) {
        TI J[NB];
        fam.template jacobian_row<L, TI>(sh, gi, r, own, u, aux, J);
        const TI Ff = (TI)F;
        // g_j = sum_i J_ij F_i: row products through LDS, column sums in row order
#pragma unroll
        for (int j = 0; j < NB; ++j) st.t[gi][r][j] = J[j] * Ff;
        wave_sync();
        TI gs = TI(0);
        if (own) {
          gs = st.t[gi][0][r];
          for (int i = 1; i < n; ++i) gs += st.t[gi][i][r];
        }
        g = gs;
        sh.gv[gi][r] = own ? g : TI(0);
        wave_sync();
        TI jg = J[0] * sh.gv[gi][0];
#pragma unroll
        for (int j = 1; j < NB; ++j) jg = __builtin_fma(J[j], sh.gv[gi][j], jg);
        const TI Jg = own ? jg : TI(0);
        wave_sync();
        ++nj;
        if (!group_lu_solve<NB, L, TI>(sh, gi, r, n, J, -Ff)) { rc = RC_SINGULAR; break; }
        dN = own ? sh.sol[gi][r] : TI(0);
        wave_sync();
        nN = __builtin_sqrt(grp_sum<L>(dN * dN));
        ng2 = grp_sum<L>(g * g);
        nJg2 = grp_sum<L>(Jg * Jg);
        tC = ng2 / nJg2;
        dC = -tC * g;
        nC2 = grp_sum<L>(dC * dC);
        dd = dN - dC;
        qa = grp_sum<L>(dd * dd);
        qb = TI(2) * grp_sum<L>(dC * dd);
        fresh = false;
      }
      const double phi = grp_sum<L>(F * F);
      double step, pred;
      const TI D = (TI)Delta;
      if ((double)nN <= Delta) {
        step = (double)dN;
        pred = phi;
      } else if (ng2 == TI(0)) {
        const TI rr = D / nN;
        step = (double)(dN * rr);
        const double om = 1.0 - (double)rr;
        pred = phi * (1.0 - om * om);
      } else if (__builtin_sqrt(nC2) >= D) {
        const TI sc = D / __builtin_sqrt(ng2);
        step = (double)(-sc * g);
        pred = (double)sc * (2.0 * (double)ng2 - (double)sc * (double)nJg2);
      } else {
        const TI qc = nC2 - D * D;
        const TI disc = qb * qb - TI(4) * qa * qc;
        const TI sq = __builtin_sqrt(disc);
        const TI tau = (qb <= TI(0)) ? (-qb + sq) / (TI(2) * qa) : (TI(-2) * qc) / (qb + sq);
        step = (double)__builtin_fma(tau, dd, dC);
        const double om = 1.0 - (double)tau;
        pred = phi - om * om * (phi - (double)tC * (double)ng2);
      }
      if (!own) step = 0.0;
      const double ut = u + step;
      double auxt = 0.0;
      const double Ft = fam.template residual<L, TI>(sh, gi, r, own, ut, auxt);
      ++nf;
      const bool fin_t = !grp_any<L>(!finite64(Ft));
      const double ared = phi - grp_sum<L>(Ft * Ft);
      const double rho = (fin_t && pred > 0.0) ? ared / pred : -__builtin_inf();
      bool accept;
      if (rho >= o.eta2) {
        accept = true;
        Delta = fmin(o.expand * Delta, o.delta_max);
      } else if (rho > o.eta1) {
        accept = true;
      } else {
        accept = false;
        Delta = o.shrink * __builtin_sqrt(grp_sum<L>(step * step));
      }
      if (accept) {
        u = ut;
        F = Ft;
        aux = auxt;
        fresh = true;
        if (grp_max<L>(__builtin_fabs(F)) <= tol) { rc = RC_SUCCESS; break; }
      } else {
        const double un = __builtin_sqrt(grp_sum<L>(u * u));
        if (Delta < o.collapse * fmax(1.0, un)) { rc = RC_TR_COLLAPSED; break; }
      }
    }
    it = k > maxit ? maxit : k;
  }

  if (own) a.u_out[uo + r] = u;
  const bool finF = !grp_any<L>(!finite64(F));
  const double fn = grp_max<L>(__builtin_fabs(F));
  if (r == 0) {
    a.fnorm[s] = finF ? fn : __builtin_inf();
    a.iters[s] = it;
    a.retcode[s] = rc;
    if (a.nfev) a.nfev[s] = nf;
    if (a.njev) a.njev[s] = nj;
  }
}

}  // namespace nls
