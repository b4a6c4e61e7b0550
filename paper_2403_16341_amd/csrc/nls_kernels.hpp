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

#include <type_traits>

#include "nls_types.h"

namespace nls {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool finite64(double x) { return __builtin_isfinite(x); }
__device__ __forceinline__ bool finite32(float x) { return __builtin_isfinite(x); }
template <typename T> __device__ __forceinline__ bool fin(T x) { return __builtin_isfinite(x); }

// Multiply-add, square root and magnitude in the operands' own precision: the
// unsuffixed builtins take double, so a float operand would be widened,
// computed in FP64 and rounded twice.
__device__ __forceinline__ float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float sqrtt(float x) { return __builtin_sqrtf(x); }
__device__ __forceinline__ double sqrtt(double x) { return __builtin_sqrt(x); }
__device__ __forceinline__ float fabst(float x) { return __builtin_fabsf(x); }
__device__ __forceinline__ double fabst(double x) { return __builtin_fabs(x); }

// s_waitcnt operands (gfx9 encoding: vmcnt in bits 3:0 and 15:14, expcnt in
// 6:4, lgkmcnt in 11:8; a field at its maximum does not wait)
enum : int { WAITCNT_VM0 = 0x0F70, WAITCNT_LGKM0 = 0xC07F };

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
      for (int j = 1; j < N; ++j) s = fmat(A[i][j], u[j], s);
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
      for (int j = 1; j < N; ++j) s = fmat(A[i][j], aux[j], s);
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

// Reciprocal for pivots: the hardware estimate refined by Newton-Raphson
// (e = 1 - x r, r += r e; two steps in FP64, one in FP32) -- within an ulp or
// two of 1/x for every finite non-zero x whose reciprocal is a normal number.
// Zero and non-finite pivots never reach it (they end the factorisation).
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fmat(-x, r, 1.0);
  r = fmat(r, e, r);
  e = fmat(-x, r, 1.0);
  return fmat(r, e, r);
}
__device__ __forceinline__ float recip(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  float e = __builtin_fmaf(-x, r, 1.0f);
  return __builtin_fmaf(r, e, r);
}

// ---------------------------------------------------------------------------
// Lane LU with partial pivoting, RHS carried along (forward substitution is
// applied while eliminating), then back substitution.  Returns false on a
// zero or non-finite pivot.  x holds the RHS on entry, the solution on exit.
// With KEEP the factors stay for lane_lu_resolve: the multipliers below the
// diagonal, the pivot reciprocals on it, and the row exchanged at step k in
// pr[k].  Exchanges move columns k.. only, so the multiplier of column k
// stays in the position it was computed for, where the carried elimination
// of a second right-hand side meets it again.
// ---------------------------------------------------------------------------
template <int N, typename T, bool KEEP = false>
__device__ __forceinline__ bool lane_lu_solve(T (&a)[N][N], T (&x)[N], int* pr = nullptr) {
  bool ok = true;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    // Pivot: the first maximum of |a_ik|, i >= k, in current row order.  Row k
    // keeps the pivot unless some later |a_ik| is strictly larger than |a_kk|
    // (one compare per candidate); the full running-maximum search runs only
    // when that happens on some lane of the wavefront.
    const T dkk = fabst(a[k][k]);
    bool larger = false;
#pragma unroll
    for (int i = k + 1; i < N; ++i) larger = larger || (fabst(a[i][k]) > dkk);
    int p = k;
    if (__any(larger)) {
      __asm__ volatile("" ::: "memory");
      T best = dkk;
#pragma unroll
      for (int i = k + 1; i < N; ++i) {
        T v = fabst(a[i][k]);
        bool c = v > best;
        best = c ? v : best;
        p = c ? i : p;
      }
    }
    // exchange rows k and p (columns k.. and the RHS) with selects; the whole
    // network is skipped when no lane of the wavefront needs an exchange (the
    // empty asm keeps the compiler from turning the branch into selects)
    if constexpr (KEEP) pr[k] = p;
    if (__any(p != k)) {
      __asm__ volatile("" ::: "memory");
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
    const T r = recip(piv);
    a[k][k] = r;  // the pivot is only needed as its reciprocal from here on
#pragma unroll
    for (int i = k + 1; i < N; ++i) {
      const T l = a[i][k] * r;
      if constexpr (KEEP) a[i][k] = l;
#pragma unroll
      for (int j = k + 1; j < N; ++j) a[i][j] = fmat(-l, a[k][j], a[i][j]);
      x[i] = fmat(-l, x[k], x[i]);
    }
  }
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    T s = x[i];
#pragma unroll
    for (int j = i + 1; j < N; ++j) s = fmat(-a[i][j], x[j], s);
    x[i] = s * a[i][i];
  }
  return ok;
}

// Second right-hand side on the factors lane_lu_solve<KEEP> left: the same
// exchanges and eliminations in the same interleaved order as the carried
// right-hand side of the factorisation, then back substitution.
template <int N, typename T>
__device__ __forceinline__ void lane_lu_resolve(const T (&a)[N][N], const int (&pr)[N], T (&x)[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k) {
    if (__any(pr[k] != k)) {
      __asm__ volatile("" ::: "memory");
#pragma unroll
      for (int i = k + 1; i < N; ++i) {
        const bool sel = (pr[k] == i);
        T t = x[k];
        x[k] = sel ? x[i] : t;
        x[i] = sel ? t : x[i];
      }
    }
#pragma unroll
    for (int i = k + 1; i < N; ++i) x[i] = fmat(-a[i][k], x[k], x[i]);
  }
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    T s = x[i];
#pragma unroll
    for (int j = i + 1; j < N; ++j) s = fmat(-a[i][j], x[j], s);
    x[i] = s * a[i][i];
  }
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
  for (int i = 0; i < N; ++i) m = fmax(m, fabst(F[i]));
  return m;
}
template <int N, typename T> __device__ __forceinline__ T sumsq(const T (&x)[N]) {
  T s = x[0] * x[0];
#pragma unroll
  for (int i = 1; i < N; ++i) s = fmat(x[i], x[i], s);
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

// Most main-loop trips one system can take: every trip evaluates one trial
// point, and a system evaluates at most maxiters directions with at most
// max_halvings + 1 trial points each (one per trial for dogleg and Newton).
__device__ __forceinline__ int64_t trip_limit(int32_t maxit, int32_t mh) {
  return (int64_t)maxit * ((int64_t)(mh > 0 ? mh : 0) + 1) + 4;
}

// slots of a launch: count, or the device-side count when one is given
__device__ __forceinline__ int64_t launch_slots(const KArgs& a) {
  if (!a.count_dev) return a.count;
  const int64_t c = *a.count_dev;
  return c < a.count ? (c > 0 ? c : 0) : a.count;
}

// Chunk staging.  Lane l copies the P parameters and the N starting values of
// system l of the chunk from global memory into LDS "column" l: a region of
// K doubles is laid out as 16-byte granules (granule g of lane l at byte
// g * 1024 + l * 16) when K is even, else as 4-byte words (word w at
// w * 256 + l * 4), so that a lane later reads any slot's values without LDS
// bank conflicts.  The copies are asynchronous until the next s_waitcnt.
template <int K> struct StageRegion {
  static constexpr bool X4 = (K % 2) == 0;
  static constexpr int BYTES = K <= 0 ? 0 : (X4 ? (K / 2) * 1024 : 2 * K * 256);
};
template <int P, int N> struct StageLayout {
  static constexpr int U0_OFFSET = StageRegion<P>::BYTES;  // bytes
  static constexpr int BYTES = StageRegion<P>::BYTES + StageRegion<N>::BYTES;
  static constexpr int DOUBLES = BYTES / 8 > 0 ? BYTES / 8 : 1;
};

typedef __attribute__((address_space(3))) char lds_char;

template <int K>
__device__ __forceinline__ void stage_region(const double* __restrict__ src, lds_char* l) {
  const char* g = reinterpret_cast<const char*>(src);
  if (StageRegion<K>::X4) {
#pragma unroll
    for (int e = 0; e < K / 2; ++e)
      __builtin_amdgcn_global_load_lds(g + e * 16, (__attribute__((address_space(3))) void*)(l + e * 1024),
                                       16, 0, 0);
  } else {
#pragma unroll
    for (int w = 0; w < 2 * K; ++w)
      __builtin_amdgcn_global_load_lds(g + w * 4, (__attribute__((address_space(3))) void*)(l + w * 256),
                                       4, 0, 0);
  }
}

// stage systems first .. first+cnt-1 (lane l takes system first + l); `l` is
// the staging buffer as an LDS-space pointer
template <int P, int N>
__device__ __forceinline__ void stage_chunk(const double* __restrict__ params, const double* __restrict__ u0,
                                            int64_t first, lds_char* l, int cnt) {
  const int lane = threadIdx.x;
  if (lane >= cnt) return;
  stage_region<P>(params + (first + lane) * P, l);
  stage_region<N>(u0 + (first + lane) * N, l + StageLayout<P, N>::U0_OFFSET);
}

template <int K>
__device__ __forceinline__ void unstage_region(const char* l, int slot, double (&v)[K]) {
  if (StageRegion<K>::X4) {
    const double2* st2 = reinterpret_cast<const double2*>(l);
#pragma unroll
    for (int e = 0; e < K / 2; ++e) {
      const double2 x = st2[e * 64 + slot];
      v[2 * e] = x.x;
      v[2 * e + 1] = x.y;
    }
  } else {
    const uint32_t* st4 = reinterpret_cast<const uint32_t*>(l);
#pragma unroll
    for (int e = 0; e < K; ++e) {
      const uint32_t lo = st4[(2 * e) * 64 + slot];
      const uint32_t hi = st4[(2 * e + 1) * 64 + slot];
      v[e] = __hiloint2double((int)hi, (int)lo);
    }
  }
}

template <int N, int FAM, int ALG, typename TI>
__global__ __launch_bounds__(64) void k_lane(const KArgs a) {
  constexpr int P = LaneParams<N, FAM>::P;
  constexpr int PS = P > 0 ? P : 1;
  __shared__ __attribute__((aligned(16))) double stage[StageLayout<PS, N>::DOUBLES];
  lds_char* const stage_lds = (lds_char*)stage;

  const int lane = threadIdx.x;
  // staging needs packed systems and, for 16-byte granules, 16-byte aligned bases
  const bool staged = P > 0 && a.sys == nullptr && a.p_off == nullptr && a.u_off == nullptr &&
                      (!StageRegion<PS>::X4 || (reinterpret_cast<uintptr_t>(a.params) & 15) == 0) &&
                      (!StageRegion<N>::X4 || (reinterpret_cast<uintptr_t>(a.u0) & 15) == 0);
  const int64_t count = launch_slots(a);
  const int64_t nchunks = (count + 63) / 64;
  const double tol = a.abstol;
  const int32_t maxit = a.maxiters;
  const double c2 = 2.0 * a.o.armijo_c;
  const double rho_bt = a.o.armijo_rho;
  const int32_t mh = a.o.armijo_max_halvings;
  const DoglegOpts o = a.o.dogleg();
  const int64_t trip_cap = trip_limit(maxit, mh);

  // Chunk currently being handed out (wave-uniform).  Without a device-wide
  // counter: blockIdx.x, blockIdx.x + gridDim.x, ...  With one, the first
  // three quarters of each wavefront's fair share of chunks are assigned the
  // same way and only the rest come from the counter: dynamic assignment
  // still balances the end of the launch, while most hand-outs skip the
  // atomic's round trip (its result is needed at once).
  const int64_t nstatic = a.counter ? (nchunks / gridDim.x) * 3 / 4 : INT64_MAX;
  int64_t taken = 0;  // chunks this wavefront has taken
  auto next_chunk = [&]() -> int64_t {
    const int64_t t = taken++;
    if (t < nstatic) return (int64_t)blockIdx.x + t * gridDim.x;
    int64_t c = 0;
    if (lane == 0) c = (int64_t)atomicAdd(reinterpret_cast<unsigned long long*>(a.counter), 1ull);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)c);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)c >> 32));
    return nstatic * gridDim.x + (int64_t)(((uint64_t)hi << 32) | lo);
  };
  int64_t chunk = next_chunk();
  int buf_next = 0, buf_cnt = 0;
  if (chunk < nchunks) {
    buf_cnt = (int)min<int64_t>(64, count - chunk * 64);
    if (staged) stage_chunk<PS, N>(a.params, a.u0, chunk * 64, stage_lds, buf_cnt);
  }
  // The first copy completes before the loop.  Each later copy is issued in a
  // trip's refill and waited for in the middle of that trip, ahead of the
  // trip's result stores: a wait on the vector-memory counter cannot tell
  // loads from stores, so a wait at the next refill would also wait for the
  // stores just issued.  With no copy in flight at the loop head, the LDS
  // reads of the refill need no wait on the vector-memory counter.
  __builtin_amdgcn_s_waitcnt(WAITCNT_VM0);
  wave_sync();

  // per-lane state
  int st = ST_IDLE;
  int64_t s = 0, uo = 0;
  int64_t trips = 0;  // main-loop trips on the current system
  int32_t k = 0, nf = 0, nj = 0, m = 0;
  double alpha = 1.0, phi0 = 0.0, Delta = o.delta0;
  // ||F||_inf (+inf if F is not finite) and ||F||_2^2 of the current iterate,
  // kept so that F itself need not stay live across a factorisation
  double fcur = 0.0, phi = 0.0;
  LaneFam<N, FAM> fam;
  double u[N], F[N], aux[N], d[N];
  TI dN[N], g[N], dC[N], dd[N];
  TI nN = 0, ng2 = 0, nJg2 = 0, tC = 0, nC2 = 0, qa = 0, qb = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) { u[i] = F[i] = aux[i] = d[i] = 0.0; dN[i] = g[i] = dC[i] = dd[i] = TI(0); }

  auto finish = [&](int32_t rc, int32_t iters) {
#pragma unroll
    for (int i = 0; i < N; ++i) a.u_out[uo + i] = u[i];
    a.fnorm[s] = fcur;
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
      const unsigned long long idle = __ballot(st == ST_IDLE);
      const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(idle >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((unsigned)idle, 0u));
      const int take = min(__popcll(idle), buf_cnt - buf_next);
      const bool fresh = st == ST_IDLE && rank < take;
      if (fresh) {
        const int slot = buf_next + rank;
        const int64_t t = chunk * 64 + slot;
        if (staged) {
          // packed and uniform: no index lookups
          s = t;
          uo = t * N;
          double pv[PS];
          const char* l = reinterpret_cast<const char*>(stage);
          unstage_region<PS>(l, slot, pv);
          fam.load(pv);
          unstage_region<N>(l + StageLayout<PS, N>::U0_OFFSET, slot, u);
        } else {
          s = a.sys ? (int64_t)a.sys[t] : t;
          uo = a.u_off ? a.u_off[s] : s * N;
          fam.load(a.params + (a.p_off ? a.p_off[s] : s * a.P));
#pragma unroll
          for (int i = 0; i < N; ++i) u[i] = a.u0[uo + i];
          // complete here, so that the paths join with no load in flight
          __builtin_amdgcn_s_waitcnt(WAITCNT_VM0);
        }
      }
      buf_next += take;
      if (buf_next == buf_cnt) {
        // chunk handed out: once every lane's LDS reads have returned, start
        // copying the next chunk into the same buffer
        __builtin_amdgcn_s_waitcnt(WAITCNT_LGKM0);
        wave_sync();
        chunk = next_chunk();
        buf_next = 0;
        buf_cnt = chunk < nchunks ? (int)min<int64_t>(64, count - chunk * 64) : 0;
        if (staged && chunk < nchunks) stage_chunk<PS, N>(a.params, a.u0, chunk * 64, stage_lds, buf_cnt);
      }
      if (fresh) {
        fam.residual(u, F, aux);
        nf = 1;
        nj = 0;
        k = 0;
        trips = 0;
        Delta = o.delta0;
        st = ST_DIR;
        const bool fin0 = all_finite(F);
        fcur = fin0 ? norm_inf(F) : __builtin_inf();
        phi = sumsq<N, double>(F);
        if (!fin0) finish(RC_NONFINITE, 0);
        else if (fcur <= tol) finish(RC_SUCCESS, 0);
        else if (maxit == 0) finish(RC_MAXITERS, 0);
      }
    }
    // every lane idle and no chunk left: the rest of this trip does nothing,
    // and the loop ends after it (an exit here would join the loop's back
    // edge ahead of the trip's wait for the chunk copy)
    const bool quit = __all(st == ST_IDLE) && chunk >= nchunks;
    // no system needs more trips than trip_cap: past it, end the system as
    // invalid rather than loop (iters = -1 - k, fnorm = trips)
    if (st != ST_IDLE && ++trips > trip_cap) {
      fcur = (double)trips;
      finish(RC_INVALID, -1 - k);
    }

    // ---------------- direction (lanes that need one) ----------------
    if (ALG == ALG_DOGLEG && st != ST_IDLE) ++k;  // every trial is an iteration
    if (__any(st == ST_DIR)) {
      if (st == ST_DIR) {
        if (ALG != ALG_DOGLEG) ++k;
        TI J[N][N];
        fam.template jacobian<TI>(u, aux, J);
        ++nj;
        if constexpr (ALG == ALG_POTRA) {
          // J_k d1 = -F(u_k), y = u_k + d1; J_k d2 = -F(y) on the same factors;
          // the trial point below is y + d2
          TI x[N];
          int pr[N];
#pragma unroll
          for (int i = 0; i < N; ++i) x[i] = (TI)(-F[i]);
          if (!lane_lu_solve<N, TI, true>(J, x, pr)) {
            finish(RC_SINGULAR, k);
          } else {
            double Fy[N], auxy[N];
#pragma unroll
            for (int i = 0; i < N; ++i) u[i] = u[i] + (double)x[i];
            fam.residual(u, Fy, auxy);
            ++nf;
#pragma unroll
            for (int i = 0; i < N; ++i) { F[i] = Fy[i]; aux[i] = auxy[i]; }
            if (!all_finite(F)) {
              fcur = __builtin_inf();
              phi = sumsq<N, double>(F);
              finish(RC_NONFINITE, k);
            } else {
#pragma unroll
              for (int i = 0; i < N; ++i) x[i] = (TI)(-F[i]);
              lane_lu_resolve<N, TI>(J, pr, x);
#pragma unroll
              for (int i = 0; i < N; ++i) d[i] = (double)x[i];
              st = ST_TRIAL;
            }
          }
        } else if constexpr (ALG != ALG_DOGLEG) {
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
            phi0 = phi;
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
            for (int i = 1; i < N; ++i) sacc = fmat(J[i][j], Ff[i], sacc);
            g[j] = sacc;
          }
#pragma unroll
          for (int i = 0; i < N; ++i) {
            TI sacc = J[i][0] * g[0];
#pragma unroll
            for (int j = 1; j < N; ++j) sacc = fmat(J[i][j], g[j], sacc);
            Jg[i] = sacc;
          }
#pragma unroll
          for (int i = 0; i < N; ++i) dN[i] = -Ff[i];
          if (!lane_lu_solve<N, TI>(J, dN)) {
            finish(RC_SINGULAR, k);
          } else {
            nN = sqrtt(sumsq<N, TI>(dN));
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
            for (int i = 1; i < N; ++i) dcd = fmat(dC[i], dd[i], dcd);
            qb = TI(2) * dcd;
            st = ST_TRIAL;
          }
        }
      }
    }

    // the chunk copy issued in this trip's refill completes here (see above)
    __builtin_amdgcn_s_waitcnt(WAITCNT_VM0);
    wave_sync();

    // ---------------- trial point, residual, decision ----------------
    if (st == ST_TRIAL) {
      double ut[N], Ft[N], auxt[N];
      double step[N];
      double pred = 0.0;
      if (ALG == ALG_NEWTON || ALG == ALG_POTRA) {
#pragma unroll
        for (int i = 0; i < N; ++i) ut[i] = u[i] + d[i];
      } else if (ALG == ALG_ARMIJO) {
#pragma unroll
        for (int i = 0; i < N; ++i) ut[i] = fmat(alpha, d[i], u[i]);
      } else {
        // dogleg step for the current radius (step algebra in TI)
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
        } else if (sqrtt(nC2) >= D) {
          const TI sc = D / sqrtt(ng2);
#pragma unroll
          for (int i = 0; i < N; ++i) step[i] = (double)(-sc * g[i]);
          // ||F - sc Jg||^2 = phi - 2 sc ||g||^2 + sc^2 ||Jg||^2, as F.Jg = ||g||^2
          pred = (double)sc * (2.0 * (double)ng2 - (double)sc * (double)nJg2);
        } else {
          const TI qc = nC2 - D * D;
          const TI disc = qb * qb - TI(4) * qa * qc;
          const TI sq = sqrtt(disc);
          const TI tau = (qb <= TI(0)) ? (-qb + sq) / (TI(2) * qa) : (TI(-2) * qc) / (qb + sq);
#pragma unroll
          for (int i = 0; i < N; ++i) step[i] = (double)fmat(tau, dd[i], dC[i]);
          // F + J step = (1 - tau)(F - tC Jg), ||F - tC Jg||^2 = phi - tC ||g||^2
          const double om = 1.0 - (double)tau;
          pred = phi - om * om * (phi - (double)tC * (double)ng2);
        }
#pragma unroll
        for (int i = 0; i < N; ++i) ut[i] = u[i] + step[i];
      }
      fam.residual(ut, Ft, auxt);
      ++nf;
      if (ALG == ALG_NEWTON || ALG == ALG_POTRA) {
#pragma unroll
        for (int i = 0; i < N; ++i) { u[i] = ut[i]; F[i] = Ft[i]; aux[i] = auxt[i]; }
        const bool fin1 = all_finite(F);
        fcur = fin1 ? norm_inf(F) : __builtin_inf();
        phi = sumsq<N, double>(F);
        if (!fin1) finish(RC_NONFINITE, k);
        else if (fcur <= tol) finish(RC_SUCCESS, k);
        else if (k >= maxit) finish(RC_MAXITERS, maxit);
        else st = ST_DIR;
      } else if (ALG == ALG_ARMIJO) {
        const double phit = sumsq<N, double>(Ft);
        if (all_finite(Ft) && phit <= (1.0 - c2 * alpha) * phi0) {
#pragma unroll
          for (int i = 0; i < N; ++i) { u[i] = ut[i]; F[i] = Ft[i]; aux[i] = auxt[i]; }
          fcur = norm_inf(F);
          phi = phit;
          if (fcur <= tol) finish(RC_SUCCESS, k);
          else if (k >= maxit) finish(RC_MAXITERS, maxit);
          else st = ST_DIR;
        } else {
          ++m;
          alpha *= rho_bt;
          if (m > mh) finish(RC_LINESEARCH_FAILED, k);
        }
      } else {
        const double phit = sumsq<N, double>(Ft);
        const double ared = phi - phit;
        const double rho = (all_finite(Ft) && pred > 0.0) ? ared / pred : -__builtin_inf();
        bool accept;
        if (rho >= o.eta2) {
          accept = true;
          Delta = fmin(o.expand * Delta, o.delta_max);
        } else if (rho > o.eta1) {
          accept = true;
        } else {
          accept = false;
          Delta = o.shrink * sqrtt(sumsq<N, double>(step));
        }
        if (accept) {
#pragma unroll
          for (int i = 0; i < N; ++i) { u[i] = ut[i]; F[i] = Ft[i]; aux[i] = auxt[i]; }
          fcur = norm_inf(F);
          phi = phit;
          if (fcur <= tol) finish(RC_SUCCESS, k);
          else if (k >= maxit) finish(RC_MAXITERS, maxit);
          else st = ST_DIR;
        } else {
          const double un = sqrtt(sumsq<N, double>(u));
          if (Delta < o.collapse * fmax(1.0, un)) finish(RC_TR_COLLAPSED, k);
          else if (k >= maxit) finish(RC_MAXITERS, maxit);
        }
      }
    }
    if (quit) break;
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
// Partner value at butterfly level M of a group reduction.  Inside a row of
// 16 lanes the partners come from DPP lane moves (quad permutations for
// M = 1, 2; half-row and row mirrors for M = 4, 8), which pair every lane
// with one lane of the other half of its current block, as an exclusive-or
// butterfly does; across rows (M = 16, 32) from a backward permute.  Every
// combine below is symmetric, so all lanes of a group end with the same bits.
enum : int { DPP_QUAD_XOR1 = 0xB1, DPP_QUAD_XOR2 = 0x4E, DPP_ROW_MIRROR = 0x140, DPP_ROW_HALF_MIRROR = 0x141 };
template <int CTRL> __device__ __forceinline__ int dpp_move(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
template <int M, int L> __device__ __forceinline__ int grp_partner(int v) {
  if constexpr (M == 1) return dpp_move<DPP_QUAD_XOR1>(v);
  else if constexpr (M == 2) return dpp_move<DPP_QUAD_XOR2>(v);
  else if constexpr (M == 4) return dpp_move<DPP_ROW_HALF_MIRROR>(v);
  else if constexpr (M == 8) return dpp_move<DPP_ROW_MIRROR>(v);
  else return __shfl_xor(v, M, L);
}
template <int M, int L> __device__ __forceinline__ float grp_partner(float v) {
  return __int_as_float(grp_partner<M, L>(__float_as_int(v)));
}
template <int M, int L> __device__ __forceinline__ double grp_partner(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = grp_partner<M, L>((int)(b & 0xffffffffll));
  const int hi = grp_partner<M, L>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
// apply f(M) for the levels M = 1, 2, 4, ... < L in increasing order
template <int L, typename F> __device__ __forceinline__ void grp_levels(F&& f) {
  f(std::integral_constant<int, 1>{});
  f(std::integral_constant<int, 2>{});
  f(std::integral_constant<int, 4>{});
  if constexpr (L > 8) f(std::integral_constant<int, 8>{});
  if constexpr (L > 16) f(std::integral_constant<int, 16>{});
  if constexpr (L > 32) f(std::integral_constant<int, 32>{});
}
// Sum over the group.  The opaque copy makes v a rounded value before the
// first addition: without it the compiler may fuse that addition with the
// multiply that produced v (as in grp_sum(x * y)), and a fused
// x_i y_i + rnd(x_j y_j) is not symmetric in i and j -- the lanes of a group
// would end with sums that differ in the last bits, and decisions taken on
// them could split the group.
template <int L, typename T> __device__ __forceinline__ T grp_sum(T v) {
  __asm__ volatile("" : "+v"(v));
  grp_levels<L>([&](auto mc) { v += grp_partner<decltype(mc)::value, L>(v); });
  return v;
}
template <int L, typename T> __device__ __forceinline__ T grp_max(T v) {
  grp_levels<L>([&](auto mc) { v = fmax(v, grp_partner<decltype(mc)::value, L>(v)); });
  return v;
}
// true if pred holds on any lane of this lane's group
template <int L> __device__ __forceinline__ bool grp_any(bool pred) {
  const unsigned long long b = __ballot(pred);
  const int gi = threadIdx.x / L;
  const unsigned long long mask = (L == 64) ? ~0ull : (((1ull << L) - 1ull) << (gi * L));
  return (b & mask) != 0ull;
}

// Per-wavefront LDS of the group mapping.  A holds the coefficient matrix of
// each group's current system (dense families), rows padded to NB + 2
// doubles: 16-byte aligned rows whose stride spreads a group's row reads over
// distinct banks.
template <int NB, int L, typename TI> struct GroupShared {
  static constexpr int G = 64 / L;
  static constexpr int AS = NB + 2;  // row stride of A in doubles
  double x[G][L];        // evaluation point, or the column map at it (tanh)
  double fv[G][L];       // F at the current iterate (for J^T F)
  double dphi[G][L];     // dual derivative of the column map at the iterate
  TI piv[G][NB + 2];     // pivot row of the current elimination step + RHS
  // zeros: the pivot row seen by the rows a step leaves as they are (the
  // FP64 form of groups narrower than the wavefront)
  TI zrow[G][(L < 64 && sizeof(TI) == 8) ? NB : 1];
  int ppos[G];           // the pivot row's logical position
  TI sol[G][L];          // solution of the triangular solves
  TI gv[G][L];           // g = J^T F
};
template <int NB, int L, bool HAS_A> struct GroupA {
  static constexpr int G = 64 / L;
  double a[G][NB][NB + 2];
};
template <int NB, int L> struct GroupA<NB, L, false> {
  double a[1][1][2];
};

template <int NB, int FAM> struct RowFam;

// Copy the n x n matrix at p into the group's LDS rows (zero outside n x n):
// consecutive lanes read consecutive doubles of a row.
template <int NB, int L>
__device__ __forceinline__ void stage_matrix(double (&a)[NB][NB + 2], const double* __restrict__ p, int n, int r) {
  constexpr int E = (NB * NB) / L;
  if constexpr (NB < 40) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int idx = e * L + r;
      const int i = idx / NB, j = idx % NB;
      a[i][j] = (i < n && j < n) ? p[i * n + j] : 0.0;
    }
  } else {
    // Large buckets: loads in batches of eight, issued back to back before
    // any is used (a load per element behind its own branch waits for each in
    // turn); entries outside n x n read p[0] and are stored as zero.  (Measured
    // on the mixed batch, the smaller buckets run no faster this way.)
    constexpr int B = 8;
#pragma unroll
    for (int e0 = 0; e0 < E; e0 += B) {
      double v[B];
#pragma unroll
      for (int b = 0; b < B; ++b) {
        if (e0 + b < E) {
          const int idx = (e0 + b) * L + r;
          const int i = idx / NB, j = idx % NB;
          v[b] = p[(i < n && j < n) ? i * n + j : 0];
        }
      }
#pragma unroll
      for (int b = 0; b < B; ++b) {
        if (e0 + b < E) {
          const int idx = (e0 + b) * L + r;
          const int i = idx / NB, j = idx % NB;
          a[i][j] = (i < n && j < n) ? v[b] : 0.0;
        }
      }
    }
  }
}

// Row of the group's LDS matrix that lane r reads: its own row, or row 0 for
// the lanes past the bucket (r >= NB, only when the group is wider than the
// bucket), whose values are never used -- so no lane reads past the matrix.
template <int NB, int L> __device__ __forceinline__ int lds_row(int r) {
  if constexpr (L > NB) return r < NB ? r : 0;
  else return r;
}

// sum_j a_rj v_j over the NB columns of an LDS row (zeros beyond n), in column
// order, with 16-byte reads of both operands
template <int NB>
__device__ __forceinline__ double row_dot(const double* __restrict__ arow, const double* __restrict__ v) {
  const double2* a2 = reinterpret_cast<const double2*>(arow);
  const double2* v2 = reinterpret_cast<const double2*>(v);
  double2 a0 = a2[0], v0 = v2[0];
  double s = a0.x * v0.x;
  s = fmat(a0.y, v0.y, s);
#pragma unroll
  for (int h = 1; h < NB / 2; ++h) {
    const double2 ah = a2[h], vh = v2[h];
    s = fmat(ah.x, vh.x, s);
    s = fmat(ah.y, vh.y, s);
  }
  return s;
}

// sum_i a_ir w_i down column r (zeros beyond n), in row order
template <int NB>
__device__ __forceinline__ double col_dot(const double (&a)[NB][NB + 2], int r, const double* __restrict__ w) {
  double s = a[0][r] * w[0];
#pragma unroll
  for (int i = 1; i < NB; ++i) s = fmat(a[i][r], w[i], s);
  return s;
}

template <int NB> struct RowFam<NB, FAM_CUBIC> {
  static constexpr bool HAS_A = true;
  double b;
  template <int L>
  __device__ __forceinline__ void load(GroupA<NB, L, true>& A, int gi, const double* __restrict__ p, int n, int r,
                                       bool own) {
    stage_matrix<NB, L>(A.a[gi], p, n, r);
    b = own ? p[n * n + r] : 0.0;
  }
  // F_r = sum_j A_rj x_j + 0.1 x_r^3 - b_r
  template <int L, typename TI>
  __device__ __forceinline__ double residual(GroupShared<NB, L, TI>& sh, GroupA<NB, L, true>& A, int gi, int r,
                                             bool own, double xr, double& auxr) const {
    sh.x[gi][r] = own ? xr : 0.0;
    wave_sync();
    const double s = row_dot<NB>(A.a[gi][lds_row<NB, L>(r)], sh.x[gi]);
    auxr = 0.0;
    wave_sync();
    return own ? (s + 0.1 * (xr * xr * xr)) - b : 0.0;
  }
  // row r: A_rj, plus the dual derivative of 0.1 u_r^3 on the diagonal
  template <int L, typename TI>
  __device__ __forceinline__ void jacobian_row(GroupShared<NB, L, TI>& sh, GroupA<NB, L, true>& A, int gi, int r,
                                               bool own, double ur, double, TI (&J)[NB]) const {
    const double diag = cubic_term_deriv(ur);
    const double2* a2 = reinterpret_cast<const double2*>(A.a[gi][lds_row<NB, L>(r)]);
#pragma unroll
    for (int h = 0; h < NB / 2; ++h) {
      const double2 v = a2[h];
      J[2 * h] = (TI)((2 * h == r && own) ? v.x + diag : v.x);
      J[2 * h + 1] = (TI)((2 * h + 1 == r && own) ? v.y + diag : v.y);
    }
  }
  // (J^T F)_r = sum_i A_ir F_i + c'(u_r) F_r with J = A + diag(c'(u))
  template <int L, typename TI>
  __device__ __forceinline__ double jt_times(GroupShared<NB, L, TI>& sh, GroupA<NB, L, true>& A, int gi, int r,
                                             bool own, double ur, double, double Fr) const {
    sh.fv[gi][r] = own ? Fr : 0.0;
    wave_sync();
    const double s = own ? col_dot<NB>(A.a[gi], r, sh.fv[gi]) : 0.0;
    wave_sync();
    return own ? fmat(cubic_term_deriv(ur), Fr, s) : 0.0;
  }
};

template <int NB> struct RowFam<NB, FAM_TANH> {
  static constexpr bool HAS_A = true;
  double b, beta;
  template <int L>
  __device__ __forceinline__ void load(GroupA<NB, L, true>& A, int gi, const double* __restrict__ p, int n, int r,
                                       bool own) {
    stage_matrix<NB, L>(A.a[gi], p, n, r);
    b = own ? p[n * n + r] : 0.0;
    beta = p[n * n + n];
  }
  // F_r = sum_j A_rj tanh(x_j) + beta x_r - b_r; lane j computes tanh(x_j)
  template <int L, typename TI>
  __device__ __forceinline__ double residual(GroupShared<NB, L, TI>& sh, GroupA<NB, L, true>& A, int gi, int r,
                                             bool own, double xr, double& auxr) const {
    auxr = own ? tanh(xr) : 0.0;
    sh.x[gi][r] = auxr;
    wave_sync();
    const double s = row_dot<NB>(A.a[gi][lds_row<NB, L>(r)], sh.x[gi]);
    wave_sync();
    return own ? (s + beta * xr) - b : 0.0;
  }
  // J_rj = A_rj tanh'(u_j) + beta [r == j]; tanh'(u_j) from the dual tanh of lane j
  template <int L, typename TI>
  __device__ __forceinline__ void jacobian_row(GroupShared<NB, L, TI>& sh, GroupA<NB, L, true>& A, int gi, int r,
                                               bool own, double ur, double auxr, TI (&J)[NB]) const {
    sh.dphi[gi][r] = own ? dtanh_known(dseed(ur), auxr).d : 0.0;
    wave_sync();
    const double2* a2 = reinterpret_cast<const double2*>(A.a[gi][lds_row<NB, L>(r)]);
    const double2* d2 = reinterpret_cast<const double2*>(sh.dphi[gi]);
#pragma unroll
    for (int h = 0; h < NB / 2; ++h) {
      const double2 v = a2[h], dv = d2[h];
      const double v0 = v.x * dv.x, v1 = v.y * dv.y;
      J[2 * h] = (TI)((2 * h == r && own) ? v0 + beta : v0);
      J[2 * h + 1] = (TI)((2 * h + 1 == r && own) ? v1 + beta : v1);
    }
    wave_sync();
  }
  // (J^T F)_r = tanh'(u_r) sum_i A_ir F_i + beta F_r
  template <int L, typename TI>
  __device__ __forceinline__ double jt_times(GroupShared<NB, L, TI>& sh, GroupA<NB, L, true>& A, int gi, int r,
                                             bool own, double ur, double auxr, double Fr) const {
    sh.fv[gi][r] = own ? Fr : 0.0;
    wave_sync();
    const double s = own ? col_dot<NB>(A.a[gi], r, sh.fv[gi]) : 0.0;
    wave_sync();
    return own ? fmat(beta, Fr, dtanh_known(dseed(ur), auxr).d * s) : 0.0;
  }
};

template <int NB> struct RowFam<NB, FAM_ROSENBROCK> {
  static constexpr bool HAS_A = false;
  template <int L>
  __device__ __forceinline__ void load(GroupA<NB, L, false>&, int, const double* __restrict__, int, int, bool) {}
  template <int L, typename TI>
  __device__ __forceinline__ double residual(GroupShared<NB, L, TI>& sh, GroupA<NB, L, false>&, int gi, int r,
                                             bool own, double xr, double& auxr) const {
    sh.x[gi][r] = xr;
    wave_sync();
    const double xm = (own && r > 0) ? sh.x[gi][r - 1] : 0.0;
    wave_sync();
    auxr = 0.0;
    if (!own) return 0.0;
    return r == 0 ? 1.0 - xr : 10.0 * (xr - xm * xm);
  }
  // row r of the dual Jacobian: seeds on u_{r-1} and u_r (1 - u_0 for r = 0)
  __device__ __forceinline__ static void row_derivs(int r, double ur, double um, double& dm, double& dd) {
    dm = (10.0 * (dconst(ur) - dseed(um) * dseed(um))).d;
    dd = r == 0 ? (dconst(1.0) - dseed(ur)).d : (10.0 * (dseed(ur) - dconst(um) * dconst(um))).d;
  }
  template <int L, typename TI>
  __device__ __forceinline__ void jacobian_row(GroupShared<NB, L, TI>& sh, GroupA<NB, L, false>&, int gi, int r,
                                               bool own, double ur, double, TI (&J)[NB]) const {
    sh.x[gi][r] = ur;
    wave_sync();
    const double um = (own && r > 0) ? sh.x[gi][r - 1] : 0.0;
    wave_sync();
    double dm, dd;
    row_derivs(r, ur, um, dm, dd);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      double v = 0.0;
      v = (j == r) ? dd : v;
      v = (j == r - 1) ? dm : v;
      J[j] = (TI)(own ? v : 0.0);
    }
  }
  // (J^T F)_r = J_rr F_r + J_{r+1,r} F_{r+1}: lane r + 1 hands over its
  // sub-diagonal product
  template <int L, typename TI>
  __device__ __forceinline__ double jt_times(GroupShared<NB, L, TI>& sh, GroupA<NB, L, false>&, int gi, int r,
                                             bool own, double ur, double, double Fr) const {
    sh.x[gi][r] = ur;
    wave_sync();
    const double um = (own && r > 0) ? sh.x[gi][r - 1] : 0.0;
    wave_sync();
    double dm, dd;
    row_derivs(r, ur, um, dm, dd);
    sh.fv[gi][r] = (own && r > 0) ? dm * Fr : 0.0;  // J_{r,r-1} F_r, for lane r - 1
    wave_sync();
    const double below = (r + 1 < L) ? sh.fv[gi][r + 1] : 0.0;
    wave_sync();
    return own ? dd * Fr + below : 0.0;
  }
};

// Value of x on lane src for every lane of the wavefront (src wave-uniform):
// lane reads into scalar registers, no LDS round trip.
__device__ __forceinline__ double wave_bcast(double x, int src) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ float wave_bcast(float x, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), src));
}
// the one lane of the wavefront where pred holds (wave-uniform result)
__device__ __forceinline__ int wave_lane_of(bool pred) { return __builtin_ctzll(__ballot(pred)); }

// Back substitution over the kept factors, column by column from the last;
// on return component k of the solution is in sh.sol[gi][k].
// Lane of the wavefront holding the lowest bit of the ballot b that falls in
// this lane's group of L lanes (every group has one where this is used).
template <int L> __device__ __forceinline__ int group_lane_of(unsigned long long b, int gi) {
  const unsigned long long gbits = (L == 64) ? b : ((b >> (gi * L)) & ((1ull << L) - 1ull));
  return gi * L + (int)__builtin_ctzll(gbits | (1ull << (L == 64 ? 63 : L)));
}
__device__ __forceinline__ double lane_shfl(double v, int src) { return __shfl(v, src, 64); }
__device__ __forceinline__ float lane_shfl(float v, int src) { return __shfl(v, src, 64); }

template <int NB, int L, typename TI>
__device__ __forceinline__ void group_back_substitute(GroupShared<NB, L, TI>& sh, int gi, int r, int n,
                                                      const TI (&J)[NB], int pos, TI myrd, TI rhs) {
  const bool own = r < n;
  if constexpr (L == 64) {
    TI mine = TI(0);
#pragma unroll
    for (int k = NB - 1; k >= 0; --k) {
      if (k < n) {
        const TI xk = wave_bcast(rhs * myrd, wave_lane_of(pos == k));
        if (r == k) mine = xk;
        if (own && pos < k) rhs = fmat(-J[k], xk, rhs);
      }
    }
    if (own) sh.sol[gi][r] = mine;
    wave_sync();
  } else if constexpr (sizeof(TI) == 4) {
    // FP32: each solution component comes from the lane holding its position
    // by a lane permute (one per component) instead of an LDS round trip
    TI mine = TI(0);
#pragma unroll
    for (int k = NB - 1; k >= 0; --k) {
      if (k < n) {
        const TI xk = lane_shfl(rhs * myrd, group_lane_of<L>(__ballot(pos == k), gi));
        if (r == k) mine = xk;
        if (own && pos < k) rhs = fmat(-J[k], xk, rhs);
      }
    }
    if (own) sh.sol[gi][r] = mine;
    wave_sync();
  } else {
#pragma unroll
    for (int k = NB - 1; k >= 0; --k) {
      if (k < n) {
        if (pos == k) sh.sol[gi][k] = rhs * myrd;
        wave_sync();
        if (own && pos < k) rhs = fmat(-J[k], sh.sol[gi][k], rhs);
        wave_sync();
      }
    }
  }
}

// LU with partial pivoting of the group's rows (logical positions instead of
// row exchanges), RHS carried along, then back substitution.  When the group
// is the whole wavefront (L = 64) the pivot row and the solution components
// travel by lane reads instead of through LDS.  Both loops are
// unrolled fully (see the unroll threshold in the build), so every row index
// is a constant and the row stays in registers.  On return the solution component r is in
// sh.sol[gi][r].  Returns false (group-uniform) on a zero or non-finite pivot.
// With the factors kept (J holds this row's multipliers left of its final
// position and its row of U from there on; pos is that final position, myrd
// the reciprocal of its pivot), group_lu_resolve solves for another RHS.
template <int NB, int L, typename TI>
__device__ __forceinline__ bool group_lu_solve(GroupShared<NB, L, TI>& sh, int gi, int r, int n,
                                               TI (&J)[NB], TI rhs, int& pos, TI& myrd) {
  const bool own = r < n;
  pos = own ? r : NB + 1 + r;  // logical row position; non-rows never pivot
  bool ok = true;
  myrd = TI(0);  // reciprocal of this row's pivot, once it has been the pivot row
  if constexpr (L < 64 && sizeof(TI) == 8) {
    // (ordered before its first read by the first step's wave_sync)
    for (int j = r; j < NB; j += L) sh.zrow[gi][j] = TI(0);
  }
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    if (k < n) {
      const TI v = J[k];
      const bool cand = pos >= k && pos < NB;
      // the row in position k wins every tie and keeps a NaN (-> singular);
      // other NaN rows never win: they rank below every number
      const bool nan_at_k = grp_any<L>(pos == k && v != v);
      const TI key = cand ? (v != v ? TI(-1) : fabst(v)) : TI(-2);
      // the group's largest key, then the row holding it: usually one lane
      // does; on a tie the smallest position among them wins
      const TI mx = grp_max<L>(key);
      const bool top = key == mx;
      const unsigned long long tb = __ballot(top);
      const unsigned long long gm = (L == 64) ? ~0ull : (((1ull << L) - 1ull) << (gi * L));
      bool owner = top;
      if (__any(__popcll(tb & gm) > 1)) {
        int pk = top ? pos : 4 * NB;
        grp_levels<L>([&](auto mc) { pk = min(pk, grp_partner<decltype(mc)::value, L>(pk)); });
        owner = top && pos == pk;
      }
      if constexpr (L == 64) {
        // the pivot row's lane; its columns k.. and RHS are read lane to lane
        const int pl = wave_lane_of(owner);
        const int kp = __builtin_amdgcn_readlane(pos, pl);
        const TI pv = wave_bcast(J[k], pl);
        const TI prhs = wave_bcast(rhs, pl);
        ok = ok && !nan_at_k && pv != TI(0) && fin(pv);
        const TI rp = recip(pv);
        if (pos == kp) myrd = rp;
        if (pos == kp) pos = k;
        else if (pos == k) pos = kp;
        const bool upd = own && pos > k;
        const TI l = J[k] * rp;
        if (upd) J[k] = l;
#pragma unroll
        for (int j = k + 1; j < NB; ++j) {
          const TI pj = wave_bcast(J[j], pl);  // read before this step changes any row
          if (upd) J[j] = fmat(-l, pj, J[j]);
        }
        if (upd) rhs = fmat(-l, prhs, rhs);
      } else if constexpr (sizeof(TI) == 4) {
        // FP32: the pivot row's columns k.., RHS and position come from its
        // lane by lane permutes (one per 32-bit word), with no LDS round trip
        const int src = group_lane_of<L>(__ballot(owner), gi);
        const int kp = __shfl(pos, src, 64);
        const TI pv = lane_shfl(J[k], src);
        const TI prhs = lane_shfl(rhs, src);
        ok = ok && !nan_at_k && pv != TI(0) && fin(pv);
        const TI rp = recip(pv);
        if (pos == kp) myrd = rp;
        if (pos == kp) pos = k;
        else if (pos == k) pos = kp;
        const bool upd = own && pos > k;
        const TI l = J[k] * rp;
        if (upd) J[k] = l;
#pragma unroll
        for (int j = k + 1; j < NB; ++j) {
          const TI pj = lane_shfl(J[j], src);  // read before this step changes any row
          if (upd) J[j] = fmat(-l, pj, J[j]);
        }
        if (upd) rhs = fmat(-l, prhs, rhs);
      } else {
        // the pivot row publishes columns k.., its RHS and its position
        if (owner) {
#pragma unroll
          for (int j = k; j < NB; ++j) sh.piv[gi][j] = J[j];
          sh.piv[gi][NB] = rhs;
          sh.ppos[gi] = pos;
        }
        wave_sync();
        const int kp = sh.ppos[gi];
        const TI pv = sh.piv[gi][k];
        ok = ok && !nan_at_k && pv != TI(0) && fin(pv);
        const TI rp = recip(pv);
        // exchange of logical positions k <-> kp
        if (pos == kp) myrd = rp;
        if (pos == kp) pos = k;
        else if (pos == k) pos = kp;
        // every lane runs the update, so that the row stays in the same
        // registers through the step: rows below the pivot row with their
        // multiplier and the pivot row's entries, the others with a zero
        // multiplier and the group's zero row (x + (-0 * 0) is x exactly)
        const bool upd = own && pos > k;
        const TI l = upd ? J[k] * rp : TI(0);
        const TI* __restrict__ prow = upd ? &sh.piv[gi][0] : &sh.zrow[gi][0];
        if (upd) J[k] = l;
#pragma unroll
        for (int j = k + 1; j < NB; ++j) J[j] = fmat(-l, prow[j], J[j]);
        const TI er = fmat(-l, sh.piv[gi][NB], rhs);
        rhs = upd ? er : rhs;
        wave_sync();
      }
    }
  }
  group_back_substitute<NB, L, TI>(sh, gi, r, n, J, pos, myrd, rhs);
  return ok;
}
template <int NB, int L, typename TI>
__device__ __forceinline__ bool group_lu_solve(GroupShared<NB, L, TI>& sh, int gi, int r, int n,
                                               TI (&J)[NB], TI rhs) {
  int pos;
  TI myrd;
  return group_lu_solve<NB, L, TI>(sh, gi, r, n, J, rhs, pos, myrd);
}

// Another right-hand side on the factors group_lu_solve kept: step k's pivot
// row (final position k) publishes its updated RHS, the rows after it apply
// their multipliers; then the same back substitution.  Solution in sh.sol.
// (group_back_substitute is defined before group_lu_solve.)
template <int NB, int L, typename TI>
__device__ __forceinline__ void group_lu_resolve(GroupShared<NB, L, TI>& sh, int gi, int r, int n,
                                                 const TI (&J)[NB], int pos, TI myrd, TI rhs) {
  const bool own = r < n;
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    if (k < n) {
      if constexpr (L == 64) {
        const TI rk = wave_bcast(rhs, wave_lane_of(pos == k));
        if (own && pos > k) rhs = fmat(-J[k], rk, rhs);
      } else {
        if (pos == k) sh.piv[gi][NB] = rhs;
        wave_sync();
        if (own && pos > k) rhs = fmat(-J[k], sh.piv[gi][NB], rhs);
        wave_sync();
      }
    }
  }
  group_back_substitute<NB, L, TI>(sh, gi, r, n, J, pos, myrd, rhs);
}

// Persistent group-mapping kernel.  Each group of L lanes solves one system at
// a time and, when it finishes, takes the next system from a device-wide
// counter (a.counter, zeroed before the launch) or, without a counter, the
// next one of its static stride; the system's matrix is copied into the
// group's LDS rows when it is taken.  Every trip runs the factorisation for
// the groups that need a new direction, then one residual evaluation for
// every group holding a trial point; groups diverge freely, and all cross-lane
// traffic stays inside a group.
// Minimum resident wavefronts per SIMD asked of the compiler, for the kernels
// that need a few registers more than that many wavefronts can hold: they
// are held to it at the price of a small spill (measured faster each time).
template <int NB, int ALG> struct GroupMinWaves {
  static constexpr int value = (ALG == ALG_DOGLEG && NB == 16) ? 3
                               : (ALG != ALG_DOGLEG && NB == 24) ? 3
                               : (ALG == ALG_DOGLEG && (NB == 24 || NB == 32 || NB == 40)) ? 2
                               : (ALG != ALG_DOGLEG && (NB == 48 || NB == 56)) ? 2 : 1;
};

template <int NB, int L, int FAM, int ALG, typename TI>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(GroupMinWaves<NB, ALG>::value)))
void k_group(const KArgs a) {
  constexpr int G = 64 / L;
  constexpr bool HAS_A = RowFam<NB, FAM>::HAS_A;
  __shared__ __attribute__((aligned(16))) GroupShared<NB, L, TI> sh;
  __shared__ __attribute__((aligned(16))) GroupA<NB, L, HAS_A> sa;
  const int lane = threadIdx.x;
  const int gi = lane / L;
  const int r = lane % L;
  const double tol = a.abstol;
  const int32_t maxit = a.maxiters;
  const double c2 = 2.0 * a.o.armijo_c;
  const double rho_bt = a.o.armijo_rho;
  const int32_t mh = a.o.armijo_max_halvings;
  const DoglegOpts o = a.o.dogleg();
  const int64_t total_groups = (int64_t)gridDim.x * G;
  int64_t next_static = (int64_t)blockIdx.x * G + gi;
  const int64_t trip_cap = trip_limit(maxit, mh);
  const int64_t count = launch_slots(a);

  // per-group state (every lane of a group holds the same copy)
  int gst = ST_IDLE;
  int64_t trips = 0;  // main-loop trips on the current system
  bool split = false; // a lane's copy of the state disagreed with the leader's
  bool exhausted = false;
  int64_t s = 0, uo = 0;
  int n = 0;
  int32_t k = 0, nf = 0, nj = 0, m = 0;
  double alpha = 1.0, phi0 = 0.0, Delta = o.delta0, fcur = 0.0, phi = 0.0;
  TI nN = 0, ng2 = 0, nJg2 = 0, tC = 0, nC2 = 0, qa = 0, qb = 0;
  // per-lane components (row / component r)
  bool own = false;
  RowFam<NB, FAM> fam;
  double u = 0.0, F = 0.0, aux = 0.0, d = 0.0;
  TI dN = 0, g = 0, dC = 0, dd = 0;

  auto finish = [&](int32_t rc, int32_t iters) {
    if (own) a.u_out[uo + r] = u;
    if (r == 0) {
      a.fnorm[s] = fcur;
      a.iters[s] = split ? -100000 : iters;
      a.retcode[s] = split ? RC_INVALID : rc;
      if (a.nfev) a.nfev[s] = nf;
      if (a.njev) a.njev[s] = nj;
    }
    gst = ST_IDLE;
  };
  auto set_norms = [&]() {
    const bool fin_ = !grp_any<L>(!finite64(F));
    fcur = fin_ ? grp_max<L>(fabst(F)) : __builtin_inf();
    phi = grp_sum<L>(F * F);
    return fin_;
  };

  while (true) {
    // The group's state is uniform by construction (every decision is taken
    // on group reductions or LDS broadcasts); the leader's copy (lane 0 of
    // the group) is made authoritative at every trip, so that lanes can never
    // refill on their own without advancing the work counter.  A lane that
    // disagreed marks the system (retcode invalid, iters -100000).
    {
      const int lead_st = __shfl(gst, gi * L, 64);
      const int lead_ex = __shfl((int)exhausted, gi * L, 64);
      const bool disagree = grp_any<L>(gst != lead_st || (int)exhausted != lead_ex);
      if (disagree && lead_st == ST_IDLE) {
        // the leader has already ended system s and written its results while
        // other lanes had not: those lanes write their components now, and
        // the system is marked invalid before the group moves on
        if (own && gst != ST_IDLE) a.u_out[uo + r] = u;
        if (r == 0) {
          a.retcode[s] = RC_INVALID;
          a.iters[s] = -100000;
        }
      }
      split = split || disagree;
      gst = lead_st;
      exhausted = lead_ex != 0;
    }
    // ---------------- retire / refill (idle groups) ----------------
    if (gst == ST_IDLE && !exhausted) {
      split = false;
      int64_t t;
      if (a.counter) {
        int64_t mine = 0;
        if (r == 0) mine = (int64_t)atomicAdd(reinterpret_cast<unsigned long long*>(a.counter), 1ull);
        t = __shfl(mine, gi * L, 64);
      } else {
        t = next_static;
        next_static += total_groups;
      }
      if (t >= count) {
        exhausted = true;
      } else {
        s = a.sys ? (int64_t)a.sys[t] : t;
        n = a.nsys ? (int)a.nsys[s] : a.n;
        own = r < n;
        uo = a.u_off ? a.u_off[s] : s * (int64_t)n;
        fam.template load<L>(sa, gi, a.params + (a.p_off ? a.p_off[s] : s * a.P), n, r, own);
        u = own ? a.u0[uo + r] : 0.0;
        wave_sync();
        F = fam.template residual<L, TI>(sh, sa, gi, r, own, u, aux);
        nf = 1;
        nj = 0;
        k = 0;
        trips = 0;
        Delta = o.delta0;
        gst = ST_DIR;
        const bool fin0 = set_norms();
        if (!fin0) finish(RC_NONFINITE, 0);
        else if (fcur <= tol) finish(RC_SUCCESS, 0);
        else if (maxit == 0) finish(RC_MAXITERS, 0);
      }
    }
    if (!__any(!(gst == ST_IDLE && exhausted))) break;
    // no system needs more trips than trip_cap: past it, end the system as
    // invalid rather than loop (iters = -1 - k, fnorm = trips)
    if (gst != ST_IDLE && ++trips > trip_cap) {
      fcur = (double)trips;
      finish(RC_INVALID, -1 - k);
    }

    // ---------------- direction (groups that need one) ----------------
    if (ALG == ALG_DOGLEG && gst != ST_IDLE) ++k;  // every trial is an iteration
    if (gst == ST_DIR) {
      if (ALG != ALG_DOGLEG) ++k;
      TI J[NB];
      fam.template jacobian_row<L, TI>(sh, sa, gi, r, own, u, aux, J);
      ++nj;
      if constexpr (ALG == ALG_POTRA) {
        // J_k d1 = -F(u_k), y = u_k + d1; J_k d2 = -F(y) on the same factors;
        // the trial point below is y + d2
        int pos;
        TI myrd;
        if (!group_lu_solve<NB, L, TI>(sh, gi, r, n, J, (TI)(-F), pos, myrd)) {
          finish(RC_SINGULAR, k);
        } else {
          const double d1 = own ? (double)sh.sol[gi][r] : 0.0;
          wave_sync();
          u = u + d1;
          F = fam.template residual<L, TI>(sh, sa, gi, r, own, u, aux);
          ++nf;
          if (!set_norms()) {
            finish(RC_NONFINITE, k);
          } else {
            group_lu_resolve<NB, L, TI>(sh, gi, r, n, J, pos, myrd, (TI)(-F));
            d = own ? (double)sh.sol[gi][r] : 0.0;
            wave_sync();
            gst = ST_TRIAL;
          }
        }
      } else if constexpr (ALG != ALG_DOGLEG) {
        if (!group_lu_solve<NB, L, TI>(sh, gi, r, n, J, (TI)(-F))) {
          finish(RC_SINGULAR, k);
        } else {
          d = own ? (double)sh.sol[gi][r] : 0.0;
          wave_sync();
          alpha = 1.0;
          m = 0;
          phi0 = phi;
          gst = ST_TRIAL;
        }
      } else {
        const TI Ff = (TI)F;
        // g = J^T F (steepest-descent direction of 0.5 ||F||^2) and J g
        g = (TI)fam.template jt_times<L, TI>(sh, sa, gi, r, own, u, aux, F);
        sh.gv[gi][r] = own ? g : TI(0);
        wave_sync();
        TI jg = J[0] * sh.gv[gi][0];
#pragma unroll
        for (int j = 1; j < NB; ++j) jg = fmat(J[j], sh.gv[gi][j], jg);
        const TI Jg = own ? jg : TI(0);
        wave_sync();
        if (!group_lu_solve<NB, L, TI>(sh, gi, r, n, J, -Ff)) {
          finish(RC_SINGULAR, k);
        } else {
          dN = own ? sh.sol[gi][r] : TI(0);
          wave_sync();
          nN = sqrtt(grp_sum<L>(dN * dN));
          ng2 = grp_sum<L>(g * g);
          nJg2 = grp_sum<L>(Jg * Jg);
          tC = ng2 / nJg2;
          dC = -tC * g;
          nC2 = grp_sum<L>(dC * dC);
          dd = dN - dC;
          qa = grp_sum<L>(dd * dd);
          qb = TI(2) * grp_sum<L>(dC * dd);
          gst = ST_TRIAL;
        }
      }
    }

    // ---------------- trial point, residual, decision ----------------
    if (gst == ST_TRIAL) {
      double ut, step = 0.0, pred = 0.0;
      if (ALG == ALG_NEWTON || ALG == ALG_POTRA) {
        ut = u + d;
      } else if (ALG == ALG_ARMIJO) {
        ut = fmat(alpha, d, u);
      } else {
        const TI D = (TI)Delta;
        if ((double)nN <= Delta) {
          step = (double)dN;
          pred = phi;
        } else if (ng2 == TI(0)) {
          const TI rr = D / nN;
          step = (double)(dN * rr);
          const double om = 1.0 - (double)rr;
          pred = phi * (1.0 - om * om);
        } else if (sqrtt(nC2) >= D) {
          const TI sc = D / sqrtt(ng2);
          step = (double)(-sc * g);
          pred = (double)sc * (2.0 * (double)ng2 - (double)sc * (double)nJg2);
        } else {
          const TI qc = nC2 - D * D;
          const TI disc = qb * qb - TI(4) * qa * qc;
          const TI sq = sqrtt(disc);
          const TI tau = (qb <= TI(0)) ? (-qb + sq) / (TI(2) * qa) : (TI(-2) * qc) / (qb + sq);
          step = (double)fmat(tau, dd, dC);
          const double om = 1.0 - (double)tau;
          pred = phi - om * om * (phi - (double)tC * (double)ng2);
        }
        if (!own) step = 0.0;
        ut = u + step;
      }
      double auxt = 0.0;
      const double Ft = fam.template residual<L, TI>(sh, sa, gi, r, own, ut, auxt);
      ++nf;
      const bool fin_t = !grp_any<L>(!finite64(Ft));
      const double phit = grp_sum<L>(Ft * Ft);
      if (ALG == ALG_NEWTON || ALG == ALG_POTRA) {
        u = ut;
        F = Ft;
        aux = auxt;
        const bool fin1 = set_norms();
        if (!fin1) finish(RC_NONFINITE, k);
        else if (fcur <= tol) finish(RC_SUCCESS, k);
        else if (k >= maxit) finish(RC_MAXITERS, maxit);
        else gst = ST_DIR;
      } else if (ALG == ALG_ARMIJO) {
        if (fin_t && phit <= (1.0 - c2 * alpha) * phi0) {
          u = ut;
          F = Ft;
          aux = auxt;
          set_norms();
          if (fcur <= tol) finish(RC_SUCCESS, k);
          else if (k >= maxit) finish(RC_MAXITERS, maxit);
          else gst = ST_DIR;
        } else {
          ++m;
          alpha *= rho_bt;
          if (m > mh) finish(RC_LINESEARCH_FAILED, k);
        }
      } else {
        const double ared = phi - phit;
        const double rho = (fin_t && pred > 0.0) ? ared / pred : -__builtin_inf();
        bool accept;
        if (rho >= o.eta2) {
          accept = true;
          Delta = fmin(o.expand * Delta, o.delta_max);
        } else if (rho > o.eta1) {
          accept = true;
        } else {
          accept = false;
          Delta = o.shrink * sqrtt(grp_sum<L>(step * step));
        }
        if (accept) {
          u = ut;
          F = Ft;
          aux = auxt;
          set_norms();
          if (fcur <= tol) finish(RC_SUCCESS, k);
          else if (k >= maxit) finish(RC_MAXITERS, maxit);
          else gst = ST_DIR;
        } else {
          const double un = sqrtt(grp_sum<L>(u * u));
          if (Delta < o.collapse * fmax(1.0, un)) finish(RC_TR_COLLAPSED, k);
          else if (k >= maxit) finish(RC_MAXITERS, maxit);
        }
      }
    }
  }
}

}  // namespace nls
