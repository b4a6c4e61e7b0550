// nls_sens.hip -- sensitivities at a solution (Sec. 2.3).  At a root u* of
// F(u, theta) = 0 with J = dF/du nonsingular, the implicit function theorem
// gives the derivative of u* in theta as D = -J^{-1} dF/dtheta.  Tangent form:
// du = D v for a parameter direction v.  Adjoint form: lambda = J^{-T} w and
// the gradient of w^T u* in theta, -(dF/dtheta)^T lambda, from one solve.
//
// One system per group of L lanes (L = 16, 32 or 64; several groups per
// wavefront).  Lane r holds row r of J (tangent form) or of J^T (adjoint
// form) in registers and factorises it with the group LU of the solver
// kernels (partial pivoting, first maximum in row order as LAPACK's getrf,
// pivot search by butterfly over the group, pivot row broadcast through LDS),
// the right-hand side carried along.  The parameter derivatives are the
// families' forward-mode derivatives written out per row.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nls_kernels.hpp"
#include "nls_launch.h"

namespace nls {
namespace {

template <int NB> struct SensWidth {
  static constexpr int L = NB <= 16 ? 16 : (NB <= 32 ? 32 : 64);
  // wavefronts per SIMD the kernel is compiled for: four up to NB = 24 (no
  // spill at 128 registers), else the compiler's choice
  static constexpr int W = NB <= 24 ? 4 : 1;
};

template <int NB, int L, int FAM, int MODE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(SensWidth<NB>::W))) void k_sens(const SensArgs a) {
  constexpr int G = 64 / L;
  __shared__ __attribute__((aligned(16))) GroupShared<NB, L, double> sh;
  __shared__ double xs[G][NB];  // u
  __shared__ double ts[G][NB];  // tanh(u) (tanh family)
  const int lane = threadIdx.x;
  const int gi = lane / L;
  const int r = lane % L;
  const bool row = r < NB;

  for (int64_t base = (int64_t)blockIdx.x * G; base < a.count; base += (int64_t)gridDim.x * G) {
    const int64_t t = base + gi;
    const bool live = t < a.count;
    int64_t s = 0;
    int n = 0;
    if (live) {
      s = a.sys ? (int64_t)a.sys[t] : t;
      n = a.nsys ? (int)a.nsys[s] : a.n;
    }
    const bool own = live && r < n;
    const int64_t P = a.nsys ? (int64_t)(FAM == FAM_CUBIC ? n * n + n : (FAM == FAM_TANH ? n * n + n + 1 : (FAM == FAM_PAPER ? 3 : 0))) : a.P;
    const int64_t uo = a.u_off ? a.u_off[s] : s * (int64_t)n;
    const int64_t po = a.p_off ? a.p_off[s] : s * P;
    const double* __restrict__ p = a.params + po;

    // ---- this lane's parameters and u, loaded up front with no branch: u
    // first, so that tanh(u) needs only its own load while the rest are in
    // flight.  Lanes without a row (and groups past the end) load a clamped
    // valid entry and drop the value; indices past n are clamped the same way.
    const int ne = live ? n : 1;
    const int re = r < ne ? r : ne - 1;
    const double ul = a.u[uo + re];
    double pa[NB];
    double beta = 0.0, br = 0.0, wr = 0.0;
    if constexpr (FAM == FAM_CUBIC || FAM == FAM_TANH) {
      if constexpr (MODE == SENS_ADJOINT) wr = a.seed[uo + re];
      br = p[ne * ne + re];
      if constexpr (FAM == FAM_TANH) beta = p[ne * ne + ne];
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        const int cc = c < ne ? c : ne - 1;
        pa[c] = MODE == SENS_TANGENT ? p[re * ne + cc] : p[cc * ne + re];
      }
    }

    const double u = own ? ul : 0.0;
    const double tu = (FAM == FAM_TANH && own) ? tanh(u) : 0.0;
    if (row) {
      xs[gi][r] = u;
      ts[gi][r] = tu;
    }
    wave_sync();
    bool bad = own && !finite64(u);

    // ---- this lane's row of J (tangent) or of J^T (adjoint), in registers ----
    // entry (i, j) of J is dF_i/du_j, the forward-mode tangent of F_i for the
    // seed u_j + eps; the adjoint form takes column r of J as its row r
    double mrow[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      double v = 0.0;
      if (own && c < n) {
        const int i = MODE == SENS_TANGENT ? r : c;  // row of J
        const int j = MODE == SENS_TANGENT ? c : r;  // column of J
        if constexpr (FAM == FAM_CUBIC) {
          const double aij = pa[c];
          bad |= !finite64(aij);
          // (the diagonal entry is the lane's own: its u is in a register)
          v = i == j ? aij + cubic_term_deriv(u) : aij;
        } else if constexpr (FAM == FAM_TANH) {
          const double aij = pa[c];
          bad |= !finite64(aij);
          // adjoint: column j = r is the lane's own, tanh'(u_r) from registers
          const double w = aij * (MODE == SENS_ADJOINT ? dtanh_known(dseed(u), tu).d
                                                       : dtanh_known(dseed(xs[gi][j]), ts[gi][j]).d);
          v = i == j ? w + beta : w;
        } else if constexpr (FAM == FAM_ROSENBROCK) {
          if (i == 0) {
            v = j == 0 ? -1.0 : 0.0;
          } else if (j == i - 1) {
            const Dual<double> um = dseed(xs[gi][i - 1]);
            v = (10.0 * (dconst(xs[gi][i]) - um * um)).d;
          } else if (j == i) {
            v = (10.0 * (dseed(xs[gi][i]) - dconst(xs[gi][i - 1]) * dconst(xs[gi][i - 1]))).d;
          }
        } else {  // the workflow example, n = 2
          const Dual<double> x0 = {xs[gi][0], j == 0 ? 1.0 : 0.0};
          const Dual<double> x1 = {xs[gi][1], j == 1 ? 1.0 : 0.0};
          if (i == 0) {
            const Dual<double> cube = x1 * x1 * x1;
            v = ((x0 + dconst(p[0])) * (cube - dconst(p[1])) + dconst(p[2])).d;
          } else {
            v = dsin(x1 * dexp(x0) - dconst(1.0)).d;
          }
        }
        bad |= !finite64(v);
      }
      mrow[c] = v;
    }
    double rhs = 0.0;
    if (own) {
      if constexpr (MODE == SENS_ADJOINT) {
        if constexpr (FAM == FAM_CUBIC || FAM == FAM_TANH) rhs = wr;
        else rhs = a.seed[uo + r];
      } else {
        // -(dF_r/dtheta) . v, the parameter derivatives of row r
        const double* __restrict__ v = a.seed + po;
        double sdot = 0.0;
        if constexpr (FAM == FAM_CUBIC || FAM == FAM_TANH) {
          // the direction's row r, loaded up front as the parameters above
          double vr[NB];
#pragma unroll
          for (int j = 0; j < NB; ++j) vr[j] = v[r * n + (j < n ? j : n - 1)];
          const double vb = v[n * n + r];
          if constexpr (FAM == FAM_CUBIC) {
#pragma unroll
            for (int j = 0; j < NB; ++j)
              if (j < n) sdot = fmat(vr[j], xs[gi][j], sdot);
            sdot = sdot - vb;
          } else {
            const double vbeta = v[n * n + n];
#pragma unroll
            for (int j = 0; j < NB; ++j)
              if (j < n) sdot = fmat(vr[j], ts[gi][j], sdot);
            sdot = (sdot - vb) + vbeta * u;
          }
        } else if constexpr (FAM == FAM_PAPER) {
          if (r == 0) {
            const double u1 = xs[gi][1];
            sdot = (u1 * u1 * u1 - p[1]) * v[0] - (u + p[0]) * v[1] + v[2];
          }
        }
        rhs = -sdot;
      }
      if constexpr (FAM == FAM_CUBIC || FAM == FAM_TANH) bad |= !finite64(br);
      if constexpr (FAM == FAM_TANH) bad |= !finite64(beta);
      if constexpr (FAM == FAM_PAPER) bad |= r == 0 && !(finite64(p[0]) && finite64(p[1]) && finite64(p[2]));
    }
    bad = grp_any<L>(bad);

    // ---- LU with partial pivoting (first maximum in row order) and the
    // triangular solves, the rows staying in registers ----
    const bool ok = group_lu_solve<NB, L, double>(sh, gi, r, n, mrow, rhs);
    const int32_t st = bad ? RC_NONFINITE : (ok ? RC_SUCCESS : RC_SINGULAR);
    const double nan = __builtin_nan("");
    const double x = (own && st == RC_SUCCESS) ? sh.sol[gi][r] : nan;

    // ---- outputs ----
    if constexpr (MODE == SENS_TANGENT) {
      if (own) a.out[uo + r] = x;
    } else {
      if (own && a.lambda) a.lambda[uo + r] = x;
      double* __restrict__ g = a.out + po;
      if constexpr (FAM == FAM_CUBIC || FAM == FAM_TANH) {
        // dF_k/dA_kj = u_j (cubic) or tanh(u_j) (tanh): lane j writes column j
        const double phi = FAM == FAM_CUBIC ? u : tu;
        if (own) {
          for (int k = 0; k < n; ++k) {
            const double lk = st == RC_SUCCESS ? sh.sol[gi][k] : nan;
            g[k * n + r] = -(lk * phi);
          }
          g[n * n + r] = x;  // dF_r/db_r = -1
        }
        if constexpr (FAM == FAM_TANH) {
          const double sb = grp_sum<L>(own ? x * u : 0.0);  // dF_i/dbeta = u_i
          if (own && r == 0) g[n * n + n] = -sb;
        }
      } else if constexpr (FAM == FAM_PAPER) {
        if (own && r == 0) {
          const double u1 = xs[gi][1];
          g[0] = -(x * (u1 * u1 * u1 - p[1]));
          g[1] = -(x * -(u + p[0]));
          g[2] = -x;
        }
      }
    }
    if (live && r == 0) a.status[s] = st;
    wave_sync();
  }
}

template <typename K>
int sens_waves(K kernel) {
  int dev = 0, per_cu = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1024;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64, 0) != hipSuccess || per_cu < 1) per_cu = 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
  return per_cu * cus;
}

template <int NB, int FAM, int MODE>
int sens_go(const SensArgs& a, hipStream_t st) {
  if (a.count <= 0) return 0;
  constexpr int L = SensWidth<NB>::L;
  constexpr int G = 64 / L;
  static const int waves = sens_waves(k_sens<NB, L, FAM, MODE>);
  const int64_t need = (a.count + G - 1) / G;
  const unsigned blocks = (unsigned)(need < waves ? need : waves);
  hipLaunchKernelGGL((k_sens<NB, L, FAM, MODE>), dim3(blocks), dim3(64), 0, st, a);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : -(int)e;
}

template <int NB, int FAM>
int sens_mode(int mode, const SensArgs& a, hipStream_t st) {
  return mode == SENS_TANGENT ? sens_go<NB, FAM, SENS_TANGENT>(a, st) : sens_go<NB, FAM, SENS_ADJOINT>(a, st);
}

template <int NB>
int sens_fam(int fam, int mode, const SensArgs& a, hipStream_t st) {
  switch (fam) {
    case FAM_CUBIC: return sens_mode<NB, FAM_CUBIC>(mode, a, st);
    case FAM_TANH: return sens_mode<NB, FAM_TANH>(mode, a, st);
    case FAM_ROSENBROCK: return sens_mode<NB, FAM_ROSENBROCK>(mode, a, st);
    case FAM_PAPER:
      if constexpr (NB == 8) return sens_mode<NB, FAM_PAPER>(mode, a, st);
      return 1;
  }
  return 1;
}

}  // namespace

int launch_sens(int nb, int fam, int mode, const SensArgs& a, hipStream_t st) {
  switch (nb) {
    case 8: return sens_fam<8>(fam, mode, a, st);
    case 16: return sens_fam<16>(fam, mode, a, st);
    case 24: return sens_fam<24>(fam, mode, a, st);
    case 32: return sens_fam<32>(fam, mode, a, st);
    case 40: return sens_fam<40>(fam, mode, a, st);
    case 48: return sens_fam<48>(fam, mode, a, st);
    case 56: return sens_fam<56>(fam, mode, a, st);
    case 64: return sens_fam<64>(fam, mode, a, st);
  }
  return 1;
}

}  // namespace nls
