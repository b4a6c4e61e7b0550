// nls_mgroup.hpp -- group mapping with several rows per lane.
//
// One system per group of L lanes with R = NB / L rows per lane: lane q of a
// group holds rows i = r L + q (r < R) of the coefficient matrix and of the
// Jacobian in registers, and the matching entries of every vector.  The
// per-step work of the factorisation that does not grow with the rows -- the
// arg-max over the group, the pivot row's publication, the reciprocal -- is
// then shared by R times more systems per wavefront than with one row per
// lane (64 / L systems per wavefront), which is where the one-row group
// kernels spend most of their instructions.
//
// The arithmetic is the one-row group kernels' (nls_kernels.hpp, k_group):
// residuals and Jacobian rows of the dense families, LU with partial
// pivoting on logical row positions (first maximum in current row order,
// Sec. 3.2 small dense LU), Newton (Sec. 2.1, eq. newton_descent), Armijo
// backtracking (Sec. 2.2.1, eq. sufficient-decrease) and the Powell dogleg
// trust region (Sec. 2.2.2, eq. tr_subproblem, ratio rho_k, three-regime
// radius update); group sums are taken per lane over its rows first, then
// over the group's lanes by a symmetric butterfly, so every lane of a group
// holds the same bits and takes the same decisions.
#pragma once

#include "nls_kernels.hpp"

namespace nls {

template <int NB, int L> struct MGeom {
  static constexpr int R = NB / L;  // rows per lane
  static constexpr int G = 64 / L;  // systems per wavefront
  static_assert(R * L == NB && (L == 8 || L == 16 || L == 32), "bucket = rows per lane x group width");
};

// Strides: the groups of a wavefront read their own copies of these arrays at
// the same offsets, so each group's row is padded to NB + 2 doubles (144 B for
// NB = 16): the eight groups then fall on disjoint LDS banks.  The per-lane
// column sums of a group are rows of NB + 2 doubles (eight lanes writing 16 B
// each cover all banks) and each group's block is padded by 8 doubles more,
// so that two groups reading them together also fall on distinct banks.
template <int NB, int L, typename TI> struct MShared {
  static constexpr int G = 64 / L;
  static constexpr int RS = NB + 2;          // row stride of the per-group arrays
  static constexpr int CS_ROW = NB + 2;      // per-lane row of the column sums
  static constexpr int CS_GRP = L * CS_ROW + 8;
  double x[G][RS];      // evaluation point (cubic) or its column map tanh(x) (tanh)
  double dphi[G][RS];   // dual derivative of the column map at the iterate (tanh)
  // per-lane column sums sum_r A_{r L + q, j} F_{r L + q}; during an FP64
  // factorisation, each lane's candidate pivot row (a slot of NB + 2 per lane)
  double cs[G][CS_GRP];
  TI sol[G][RS];        // solution of the triangular solves
  TI gv[G][RS];         // g = J^T F
  TI jg[G][RS];         // J g
};

// group sum / max / any of per-row values (this lane's rows first, in row
// order, then the butterfly over the group's lanes)
template <int L, int R, typename T> __device__ __forceinline__ T mg_sum(const T (&v)[R]) {
  T s = v[0];
#pragma unroll
  for (int r = 1; r < R; ++r) s = s + v[r];
  return grp_sum<L>(s);
}
template <int L, int R, typename T> __device__ __forceinline__ T mg_max(const T (&v)[R]) {
  T s = v[0];
#pragma unroll
  for (int r = 1; r < R; ++r) s = fmax(s, v[r]);
  return grp_max<L>(s);
}
template <int L, int R> __device__ __forceinline__ bool mg_any(const bool (&v)[R]) {
  bool s = v[0];
#pragma unroll
  for (int r = 1; r < R; ++r) s = s || v[r];
  return grp_any<L>(s);
}

// Dense families with this lane's rows of A in registers.
template <int NB, int L, int FAM> struct MRows;

template <int NB, int L> struct MRowsBase {
  static constexpr int R = MGeom<NB, L>::R;
  double A[R][NB];
  double b[R];
  // rows r L + q of the n x n matrix at p (zero outside n x n), b from p[n n ..]
  __device__ __forceinline__ void load_rows(const double* __restrict__ p, int n, int q) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = r * L + q;
      const bool own = i < n;
#pragma unroll
      for (int j = 0; j < NB; ++j) A[r][j] = (own && j < n) ? p[i * n + j] : 0.0;
      b[r] = own ? p[n * n + i] : 0.0;
    }
  }
  // sum_j A_rj v_j over the NB columns (zeros beyond n), in column order, v in LDS
  __device__ __forceinline__ double row_dot(int r, const double* __restrict__ v) const {
    const double2* v2 = reinterpret_cast<const double2*>(v);
    double2 v0 = v2[0];
    double s = A[r][0] * v0.x;
    s = fmat(A[r][1], v0.y, s);
#pragma unroll
    for (int h = 1; h < NB / 2; ++h) {
      const double2 vh = v2[h];
      s = fmat(A[r][2 * h], vh.x, s);
      s = fmat(A[r][2 * h + 1], vh.y, s);
    }
    return s;
  }
  // column sums of A weighted by this lane's F entries, published to the
  // group; returns (sum_i A_ij F_i) for this lane's columns j = r L + q
  template <typename TI>
  __device__ __forceinline__ void col_sums(MShared<NB, L, TI>& sh, int gi, int q, const double (&F)[R],
                                           double (&out)[R]) const {
#pragma unroll
    for (int j = 0; j < NB; j += 2) {
      double c0 = A[0][j] * F[0], c1 = A[0][j + 1] * F[0];
#pragma unroll
      for (int r = 1; r < R; ++r) {
        c0 = fmat(A[r][j], F[r], c0);
        c1 = fmat(A[r][j + 1], F[r], c1);
      }
      *reinterpret_cast<double2*>(&sh.cs[gi][q * MShared<NB, L, TI>::CS_ROW + j]) = double2{c0, c1};
    }
    wave_sync();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int j = r * L + q;
      double s = sh.cs[gi][j];
#pragma unroll
      for (int l = 1; l < L; ++l) s = s + sh.cs[gi][l * MShared<NB, L, TI>::CS_ROW + j];
      out[r] = s;
    }
    wave_sync();
  }
};

template <int NB, int L> struct MRows<NB, L, FAM_CUBIC> : MRowsBase<NB, L> {
  using Base = MRowsBase<NB, L>;
  static constexpr int R = Base::R;
  __device__ __forceinline__ void load(const double* __restrict__ p, int n, int q) { Base::load_rows(p, n, q); }
  // F_i = sum_j A_ij x_j + 0.1 x_i^3 - b_i for this lane's rows
  template <typename TI>
  __device__ __forceinline__ void residual(MShared<NB, L, TI>& sh, int gi, int q, int n, const double (&x)[R],
                                           double (&F)[R], double (&aux)[R]) const {
#pragma unroll
    for (int r = 0; r < R; ++r) sh.x[gi][r * L + q] = (r * L + q < n) ? x[r] : 0.0;
    wave_sync();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double s = Base::row_dot(r, sh.x[gi]);
      F[r] = (r * L + q < n) ? (s + 0.1 * (x[r] * x[r] * x[r])) - Base::b[r] : 0.0;
      aux[r] = 0.0;
    }
    wave_sync();
  }
  // row i of J: A_ij, plus the dual derivative of 0.1 u_i^3 on the diagonal
  template <typename TI>
  __device__ __forceinline__ void jacobian(MShared<NB, L, TI>&, int, int q, int n, const double (&u)[R],
                                           const double (&)[R], TI (&J)[R][NB]) const {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = r * L + q;
      const double dg = (i < n) ? cubic_term_deriv(u[r]) : 0.0;
#pragma unroll
      for (int j = 0; j < NB; ++j) J[r][j] = (TI)(j == i ? Base::A[r][j] + dg : Base::A[r][j]);
    }
  }
  // (J^T F)_j = sum_i A_ij F_i + c'(u_j) F_j
  template <typename TI>
  __device__ __forceinline__ void jt_times(MShared<NB, L, TI>& sh, int gi, int q, int n, const double (&u)[R],
                                           const double (&)[R], const double (&F)[R], double (&g)[R]) const {
    double cs[R];
    Base::col_sums(sh, gi, q, F, cs);
#pragma unroll
    for (int r = 0; r < R; ++r) g[r] = (r * L + q < n) ? fmat(cubic_term_deriv(u[r]), F[r], cs[r]) : 0.0;
  }
};

template <int NB, int L> struct MRows<NB, L, FAM_TANH> : MRowsBase<NB, L> {
  using Base = MRowsBase<NB, L>;
  static constexpr int R = Base::R;
  double beta;
  __device__ __forceinline__ void load(const double* __restrict__ p, int n, int q) {
    Base::load_rows(p, n, q);
    beta = p[n * n + n];
  }
  // F_i = sum_j A_ij tanh(x_j) + beta x_i - b_i; aux = tanh of this lane's entries
  template <typename TI>
  __device__ __forceinline__ void residual(MShared<NB, L, TI>& sh, int gi, int q, int n, const double (&x)[R],
                                           double (&F)[R], double (&aux)[R]) const {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      aux[r] = (r * L + q < n) ? tanh(x[r]) : 0.0;
      sh.x[gi][r * L + q] = aux[r];
    }
    wave_sync();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double s = Base::row_dot(r, sh.x[gi]);
      F[r] = (r * L + q < n) ? (s + beta * x[r]) - Base::b[r] : 0.0;
    }
    wave_sync();
  }
  // J_ij = A_ij tanh'(u_j) + beta [i == j]; tanh'(u_j) from the dual tanh of
  // the lane holding entry j
  template <typename TI>
  __device__ __forceinline__ void jacobian(MShared<NB, L, TI>& sh, int gi, int q, int n, const double (&u)[R],
                                           const double (&aux)[R], TI (&J)[R][NB]) const {
#pragma unroll
    for (int r = 0; r < R; ++r) sh.dphi[gi][r * L + q] = (r * L + q < n) ? dtanh_known(dseed(u[r]), aux[r]).d : 0.0;
    wave_sync();
    const double2* d2 = reinterpret_cast<const double2*>(sh.dphi[gi]);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = r * L + q;
      const bool own = i < n;
#pragma unroll
      for (int h = 0; h < NB / 2; ++h) {
        const double2 dv = d2[h];
        const double v0 = Base::A[r][2 * h] * dv.x, v1 = Base::A[r][2 * h + 1] * dv.y;
        J[r][2 * h] = (TI)((2 * h == i && own) ? v0 + beta : v0);
        J[r][2 * h + 1] = (TI)((2 * h + 1 == i && own) ? v1 + beta : v1);
      }
    }
    wave_sync();
  }
  // (J^T F)_j = tanh'(u_j) sum_i A_ij F_i + beta F_j
  template <typename TI>
  __device__ __forceinline__ void jt_times(MShared<NB, L, TI>& sh, int gi, int q, int n, const double (&u)[R],
                                           const double (&aux)[R], const double (&F)[R], double (&g)[R]) const {
    double cs[R];
    Base::col_sums(sh, gi, q, F, cs);
#pragma unroll
    for (int r = 0; r < R; ++r)
      g[r] = (r * L + q < n) ? fmat(beta, F[r], dtanh_known(dseed(u[r]), aux[r]).d * cs[r]) : 0.0;
  }
};

// f(integral_constant<int, i>) for i = B .. E-1: loop bodies with compile-time
// indices, so that every nested loop has constant bounds and unrolls fully
template <int B, int E, typename F> __device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// LU with partial pivoting of the group's rows (logical positions instead of
// row exchanges), RHS carried along, then back substitution.  Each lane takes
// the first maximum among its own candidate rows (by position), the group's
// butterfly combines those.  On return entry r L + q of the solution is in
// x[r] (and the whole solution in sh.sol).  Returns false (group-uniform) on a
// zero or non-finite pivot.
template <int NB, int L, typename TI>
__device__ __forceinline__ bool mg_lu_solve(MShared<NB, L, TI>& sh, int gi, int q, int n,
                                            TI (&J)[MGeom<NB, L>::R][NB], TI (&x)[MGeom<NB, L>::R]) {
  constexpr int R = MGeom<NB, L>::R;
  int pos[R];
  TI rd[R];
  bool own[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = r * L + q;
    own[r] = i < n;
    pos[r] = own[r] ? i : NB + 1 + i;  // non-rows never pivot
    rd[r] = TI(0);
  }
  bool ok = true;
  static_for<0, NB>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    if (k < n) {
      bool nan_k = false;
      TI key = TI(-3);
      int kp = 4 * NB;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const TI v = J[r][k];
        nan_k = nan_k || (pos[r] == k && v != v);
        const bool cand = pos[r] >= k && pos[r] < NB;
        // NaN rows rank below every number, non-candidates below those
        const TI kr = cand ? (v != v ? TI(-1) : fabst(v)) : TI(-2);
        const bool take = kr > key || (kr == key && pos[r] < kp);
        key = take ? kr : key;
        kp = take ? pos[r] : kp;
      }
      if constexpr (sizeof(TI) == 8) {
        // every lane writes its candidate row (the local best) and RHS to a
        // slot of its own while the group search runs; the owner's slot is
        // read below (the column-sum area is free during the factorisation)
        int rs = 0;
#pragma unroll
        for (int r = 1; r < R; ++r) rs = pos[r] == kp ? r : rs;
        static_assert(sizeof(sh.cs) >= 64 * (NB + 2) * sizeof(TI), "a slot per lane in the column-sum area");
        TI* slot = reinterpret_cast<TI*>(&sh.cs[0][0]) + threadIdx.x * (NB + 2);
#pragma unroll
        for (int j = k + 1; j < NB; ++j) {
          TI v = J[0][j];
#pragma unroll
          for (int r = 1; r < R; ++r) v = rs == r ? J[r][j] : v;
          slot[j] = v;
        }
        TI v = x[0];
#pragma unroll
        for (int r = 1; r < R; ++r) v = rs == r ? x[r] : v;
        slot[NB] = v;
      }
      nan_k = grp_any<L>(nan_k);
      // The group's largest key, then the lane holding it.  Usually one lane
      // does: it publishes its row and position.  When several hold the
      // largest key (a tie), the smallest position among them wins.
      const TI mx = grp_max<L>(key);
      const bool top = key == mx;
      const unsigned long long tb = __ballot(top);
      const unsigned long long gm = (L == 64) ? ~0ull : (((1ull << L) - 1ull) << (gi * L));
      const bool tie = __popcll(tb & gm) > 1;
      bool owner = top;
      if (__any(tie)) {
        int pk = top ? kp : 4 * NB;
        grp_levels<L>([&](auto mc) { pk = min(pk, grp_partner<decltype(mc)::value, L>(pk)); });
        owner = top && kp == pk;
      }
      if constexpr (sizeof(TI) == 4) {
        // The pivot row, its right-hand side and its position come straight from
        // the lane that holds them (a lane permute from the group's owner lane,
        // no round trip through LDS): every lane picks its candidate row by
        // selects, and the group reads the owner's.
        const int src = group_lane_of<L>(__ballot(owner), gi);
        int rsel = 0;
#pragma unroll
        for (int r = 1; r < R; ++r) rsel = pos[r] == kp ? r : rsel;
        kp = __shfl(kp, src, 64);
        auto cand = [&](int j) {
          TI v = J[0][j];
#pragma unroll
          for (int r = 1; r < R; ++r) v = rsel == r ? J[r][j] : v;
          return v;
        };
        const TI pv = lane_shfl(cand(k), src);
        ok = ok && !nan_k && pv != TI(0) && fin(pv);
        const TI rp = recip(pv);
        TI l[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          // exchange of logical positions k <-> kp
          if (pos[r] == kp) {
            rd[r] = rp;
            pos[r] = k;
          } else if (pos[r] == k) {
            pos[r] = kp;
          }
          const bool upd = own[r] && pos[r] > k;
          l[r] = upd ? J[r][k] * rp : TI(0);
          if (upd) J[r][k] = l[r];
        }
#pragma unroll
        for (int j = k + 1; j < NB; ++j) {
          const TI pj = lane_shfl(cand(j), src);
#pragma unroll
          for (int r = 0; r < R; ++r)
            if (own[r] && pos[r] > k) J[r][j] = fmat(-l[r], pj, J[r][j]);
        }
        {
          TI xv = x[0];
#pragma unroll
          for (int r = 1; r < R; ++r) xv = rsel == r ? x[r] : xv;
          const TI px = lane_shfl(xv, src);
#pragma unroll
          for (int r = 0; r < R; ++r)
            if (own[r] && pos[r] > k) x[r] = fmat(-l[r], px, x[r]);
        }
      } else {
        // The pivot and its position come from the owner lane by a lane
        // permute, so that the reciprocal can start at once; the rest of the
        // pivot row and its RHS are published through LDS (the lane holding
        // the row picks it by selects, so the rows stay in registers).
        int rsel = 0;
#pragma unroll
        for (int r = 1; r < R; ++r) rsel = pos[r] == kp ? r : rsel;
        TI pl = J[0][k];
#pragma unroll
        for (int r = 1; r < R; ++r) pl = rsel == r ? J[r][k] : pl;
        const int src = group_lane_of<L>(__ballot(owner), gi);
        const TI pv = lane_shfl(pl, src);
        kp = __shfl(kp, src, 64);
        const TI* prow = reinterpret_cast<const TI*>(&sh.cs[0][0]) + src * (NB + 2);
        wave_sync();
        ok = ok && !nan_k && pv != TI(0) && fin(pv);
        const TI rp = recip(pv);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          // exchange of logical positions k <-> kp
          if (pos[r] == kp) {
            rd[r] = rp;
            pos[r] = k;
          } else if (pos[r] == k) {
            pos[r] = kp;
          }
          if (own[r] && pos[r] > k) {
            const TI l = J[r][k] * rp;
            J[r][k] = l;
#pragma unroll
            for (int j = k + 1; j < NB; ++j) J[r][j] = fmat(-l, prow[j], J[r][j]);
            x[r] = fmat(-l, prow[NB], x[r]);
          }
        }
        wave_sync();
      }
    }
  });
  if constexpr (sizeof(TI) == 4) {
    // back substitution, column by column from the last: the lane holding
    // logical position k computes x_k, the group takes it by a lane permute, and
    // the owner also stores it for the gather below
    static_for<0, NB>([&](auto kc) {
      constexpr int k = NB - 1 - decltype(kc)::value;
      if (k < n) {
        bool has = false;
        TI xl = TI(0);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const bool h = pos[r] == k;
          xl = h ? x[r] * rd[r] : xl;
          has = has || h;
        }
        const TI xk = lane_shfl(xl, group_lane_of<L>(__ballot(has), gi));
        if (has) sh.sol[gi][k] = xk;
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (own[r] && pos[r] < k) x[r] = fmat(-J[r][k], xk, x[r]);
      }
    });
    wave_sync();
  } else {
    // back substitution, column by column from the last
    static_for<0, NB>([&](auto kc) {
      constexpr int k = NB - 1 - decltype(kc)::value;
      if (k < n) {
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (pos[r] == k) sh.sol[gi][k] = x[r] * rd[r];
        wave_sync();
        const TI xk = sh.sol[gi][k];
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (own[r] && pos[r] < k) x[r] = fmat(-J[r][k], xk, x[r]);
        wave_sync();
      }
    });
  }
#pragma unroll
  for (int r = 0; r < R; ++r) x[r] = own[r] ? sh.sol[gi][r * L + q] : TI(0);
  wave_sync();
  return ok;
}

// Persistent multi-row group kernel (Newton, Newton + Armijo, dogleg; dense
// families).  Each group of L lanes solves one system at a time and takes the
// next from the device-wide counter when it finishes; every trip runs the
// factorisation for the groups that need a new direction, then one residual
// evaluation for every group holding a trial point.  The group leader's state
// is authoritative at every trip (a lane that disagreed marks its system
// invalid), and every system has a trip guard, as in k_group.
template <int NB, int L, int FAM, int ALG, typename TI>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
void k_mgroup(const KArgs a) {
  static_assert(ALG == ALG_NEWTON || ALG == ALG_ARMIJO || ALG == ALG_DOGLEG, "multi-row groups: no Potra-Ptak");
  static_assert(FAM == FAM_CUBIC || FAM == FAM_TANH, "multi-row groups: dense families");
  constexpr int R = MGeom<NB, L>::R;
  constexpr int G = MGeom<NB, L>::G;
  __shared__ __attribute__((aligned(16))) MShared<NB, L, TI> sh;
  const int lane = threadIdx.x;
  const int gi = lane / L;
  const int q = lane % L;
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
  int64_t trips = 0;
  bool split = false;
  bool exhausted = false;
  int64_t s = 0, uo = 0;
  int n = 0;
  int32_t k = 0, nf = 0, nj = 0, m = 0;
  double alpha = 1.0, phi0 = 0.0, Delta = o.delta0, fcur = 0.0, phi = 0.0;
  TI nN = 0, ng2 = 0, nJg2 = 0, tC = 0, nC2 = 0, qa = 0, qb = 0;
  // this lane's entries r L + q of every vector
  MRows<NB, L, FAM> fam;
  double u[R], F[R], aux[R], d[R];
  TI dN[R], g[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    u[r] = F[r] = aux[r] = d[r] = 0.0;
    dN[r] = g[r] = TI(0);
  }
  auto own = [&](int r) { return r * L + q < n; };

  auto finish = [&](int32_t rc, int32_t iters) {
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (own(r)) a.u_out[uo + r * L + q] = u[r];
    if (q == 0) {
      a.fnorm[s] = fcur;
      a.iters[s] = split ? -100000 : iters;
      a.retcode[s] = split ? RC_INVALID : rc;
      if (a.nfev) a.nfev[s] = nf;
      if (a.njev) a.njev[s] = nj;
    }
    gst = ST_IDLE;
  };
  auto set_norms = [&](const double (&Fv)[R], double& finf, double& f2) {
    bool bad[R];
    double av[R], sq[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      bad[r] = !finite64(Fv[r]);
      av[r] = fabst(Fv[r]);
      sq[r] = Fv[r] * Fv[r];
    }
    const bool fin_ = !mg_any<L, R>(bad);
    finf = fin_ ? mg_max<L, R>(av) : __builtin_inf();
    f2 = mg_sum<L, R>(sq);
    return fin_;
  };

  while (true) {
    {
      const int lead_st = __shfl(gst, gi * L, 64);
      const int lead_ex = __shfl((int)exhausted, gi * L, 64);
      const bool disagree = grp_any<L>(gst != lead_st || (int)exhausted != lead_ex);
      if (disagree && lead_st == ST_IDLE) {
        // the leader has already ended system s: the other lanes write their
        // entries, and the system is marked invalid before the group moves on
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (own(r) && gst != ST_IDLE) a.u_out[uo + r * L + q] = u[r];
        if (q == 0) {
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
        if (q == 0) mine = (int64_t)atomicAdd(reinterpret_cast<unsigned long long*>(a.counter), 1ull);
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
        uo = a.u_off ? a.u_off[s] : s * (int64_t)n;
        fam.load(a.params + (a.p_off ? a.p_off[s] : s * a.P), n, q);
#pragma unroll
        for (int r = 0; r < R; ++r) u[r] = own(r) ? a.u0[uo + r * L + q] : 0.0;
        fam.residual(sh, gi, q, n, u, F, aux);
        nf = 1;
        nj = 0;
        k = 0;
        trips = 0;
        Delta = o.delta0;
        gst = ST_DIR;
        const bool fin0 = set_norms(F, fcur, phi);
        if (!fin0) finish(RC_NONFINITE, 0);
        else if (fcur <= tol) finish(RC_SUCCESS, 0);
        else if (maxit == 0) finish(RC_MAXITERS, 0);
      }
    }
    if (!__any(!(gst == ST_IDLE && exhausted))) break;
    if (gst != ST_IDLE && ++trips > trip_cap) {
      fcur = (double)trips;
      finish(RC_INVALID, -1 - k);
    }

    // ---------------- direction (groups that need one) ----------------
    if (ALG == ALG_DOGLEG && gst != ST_IDLE) ++k;  // every trial is an iteration
    if (gst == ST_DIR) {
      if (ALG != ALG_DOGLEG) ++k;
      TI J[R][NB];
      fam.jacobian(sh, gi, q, n, u, aux, J);
      ++nj;
      if constexpr (ALG != ALG_DOGLEG) {
        TI x[R];
#pragma unroll
        for (int r = 0; r < R; ++r) x[r] = (TI)(-F[r]);
        if (!mg_lu_solve<NB, L, TI>(sh, gi, q, n, J, x)) {
          finish(RC_SINGULAR, k);
        } else {
#pragma unroll
          for (int r = 0; r < R; ++r) d[r] = (double)x[r];
          alpha = 1.0;
          m = 0;
          phi0 = phi;
          gst = ST_TRIAL;
        }
      } else {
        // g = J^T F (steepest-descent direction of 0.5 ||F||^2) and J g; both
        // wait in LDS while the factorisation holds the registers
        double gd[R];
        fam.jt_times(sh, gi, q, n, u, aux, F, gd);
#pragma unroll
        for (int r = 0; r < R; ++r) sh.gv[gi][r * L + q] = own(r) ? (TI)gd[r] : TI(0);
        wave_sync();
#pragma unroll
        for (int r = 0; r < R; ++r) {
          TI acc = J[r][0] * sh.gv[gi][0];
#pragma unroll
          for (int j = 1; j < NB; ++j) acc = fmat(J[r][j], sh.gv[gi][j], acc);
          sh.jg[gi][r * L + q] = own(r) ? acc : TI(0);
        }
        wave_sync();
        TI x[R];
#pragma unroll
        for (int r = 0; r < R; ++r) x[r] = (TI)(-F[r]);
        if (!mg_lu_solve<NB, L, TI>(sh, gi, q, n, J, x)) {
          finish(RC_SINGULAR, k);
        } else {
          TI sN[R], sg[R], sJg[R];
#pragma unroll
          for (int r = 0; r < R; ++r) {
            dN[r] = x[r];
            g[r] = sh.gv[gi][r * L + q];
            const TI jg = sh.jg[gi][r * L + q];
            sN[r] = dN[r] * dN[r];
            sg[r] = g[r] * g[r];
            sJg[r] = jg * jg;
          }
          wave_sync();
          nN = sqrtt(mg_sum<L, R>(sN));
          ng2 = mg_sum<L, R>(sg);
          nJg2 = mg_sum<L, R>(sJg);
          tC = ng2 / nJg2;
          // Cauchy point dC = -tC g and d = dN - dC (recomputed where used)
          TI sC[R], sd[R], sx[R];
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const TI dc = -tC * g[r];
            const TI dv = dN[r] - dc;
            sC[r] = dc * dc;
            sd[r] = dv * dv;
            sx[r] = dc * dv;
          }
          nC2 = mg_sum<L, R>(sC);
          qa = mg_sum<L, R>(sd);
          qb = TI(2) * mg_sum<L, R>(sx);
          gst = ST_TRIAL;
        }
      }
    }

    // ---------------- trial point, residual, decision ----------------
    if (gst == ST_TRIAL) {
      double ut[R], step[R], pred = 0.0;
      if (ALG == ALG_NEWTON) {
#pragma unroll
        for (int r = 0; r < R; ++r) ut[r] = u[r] + d[r];
      } else if (ALG == ALG_ARMIJO) {
#pragma unroll
        for (int r = 0; r < R; ++r) ut[r] = fmat(alpha, d[r], u[r]);
      } else {
        const TI D = (TI)Delta;
        if ((double)nN <= Delta) {
#pragma unroll
          for (int r = 0; r < R; ++r) step[r] = (double)dN[r];
          pred = phi;
        } else if (ng2 == TI(0)) {
          const TI rr = D / nN;
#pragma unroll
          for (int r = 0; r < R; ++r) step[r] = (double)(dN[r] * rr);
          const double om = 1.0 - (double)rr;
          pred = phi * (1.0 - om * om);
        } else if (sqrtt(nC2) >= D) {
          const TI sc = D / sqrtt(ng2);
#pragma unroll
          for (int r = 0; r < R; ++r) step[r] = (double)(-sc * g[r]);
          pred = (double)sc * (2.0 * (double)ng2 - (double)sc * (double)nJg2);
        } else {
          const TI qc = nC2 - D * D;
          const TI disc = qb * qb - TI(4) * qa * qc;
          const TI sq = sqrtt(disc);
          const TI tau = (qb <= TI(0)) ? (-qb + sq) / (TI(2) * qa) : (TI(-2) * qc) / (qb + sq);
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const TI dc = -tC * g[r];
            step[r] = (double)fmat(tau, dN[r] - dc, dc);
          }
          const double om = 1.0 - (double)tau;
          pred = phi - om * om * (phi - (double)tC * (double)ng2);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (!own(r)) step[r] = 0.0;
          ut[r] = u[r] + step[r];
        }
      }
      double Ft[R], auxt[R];
      fam.residual(sh, gi, q, n, ut, Ft, auxt);
      ++nf;
      double ft, phit;
      const bool fin_t = set_norms(Ft, ft, phit);
      if (ALG == ALG_NEWTON) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          u[r] = ut[r];
          F[r] = Ft[r];
          aux[r] = auxt[r];
        }
        fcur = ft;
        phi = phit;
        if (!fin_t) finish(RC_NONFINITE, k);
        else if (fcur <= tol) finish(RC_SUCCESS, k);
        else if (k >= maxit) finish(RC_MAXITERS, maxit);
        else gst = ST_DIR;
      } else if (ALG == ALG_ARMIJO) {
        if (fin_t && phit <= (1.0 - c2 * alpha) * phi0) {
#pragma unroll
          for (int r = 0; r < R; ++r) {
            u[r] = ut[r];
            F[r] = Ft[r];
            aux[r] = auxt[r];
          }
          fcur = ft;
          phi = phit;
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
          double s2[R];
#pragma unroll
          for (int r = 0; r < R; ++r) s2[r] = step[r] * step[r];
          Delta = o.shrink * sqrtt(mg_sum<L, R>(s2));
        }
        if (accept) {
#pragma unroll
          for (int r = 0; r < R; ++r) {
            u[r] = ut[r];
            F[r] = Ft[r];
            aux[r] = auxt[r];
          }
          fcur = ft;
          phi = phit;
          if (fcur <= tol) finish(RC_SUCCESS, k);
          else if (k >= maxit) finish(RC_MAXITERS, maxit);
          else gst = ST_DIR;
        } else {
          double u2[R];
#pragma unroll
          for (int r = 0; r < R; ++r) u2[r] = u[r] * u[r];
          const double un = sqrtt(mg_sum<L, R>(u2));
          if (Delta < o.collapse * fmax(1.0, un)) finish(RC_TR_COLLAPSED, k);
          else if (k >= maxit) finish(RC_MAXITERS, maxit);
        }
      }
    }
  }
}

}  // namespace nls
