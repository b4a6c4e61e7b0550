// nls_sens.hip -- sensitivities at a solution (Sec. 2.3).  At a root u* of
// F(u, theta) = 0 with J = dF/du nonsingular, the implicit function theorem
// gives the derivative of u* in theta as D = -J^{-1} dF/dtheta.  Tangent form:
// du = D v for a parameter direction v.  Adjoint form: lambda = J^{-T} w and
// the gradient of w^T u* in theta, -(dF/dtheta)^T lambda, from one solve.
//
// One system per group of L lanes (L = 16, 32 or 64; several groups per
// wavefront).  Lane r owns row r of the NB x NB matrix -- J for the tangent
// form, J^T for the adjoint form -- padded with an identity block past n and
// staged in LDS; Gaussian elimination with partial pivoting (first maximum in
// row order, as LAPACK's getrf) runs on it with the right-hand side in
// registers, then back substitution.  The parameter derivatives are the
// families' forward-mode derivatives written out per row.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nls_kernels.hpp"
#include "nls_launch.h"

namespace nls {
namespace {

template <int NB> struct SensWidth {
  static constexpr int L = NB <= 16 ? 16 : (NB <= 32 ? 32 : 64);
};

template <int NB, int L, int FAM, int MODE>
__global__ __launch_bounds__(64) void k_sens(const SensArgs a) {
  constexpr int G = 64 / L;
  constexpr int LD = NB + 1;  // padded row stride (doubles)
  __shared__ double m[G][NB][LD];
  __shared__ double xs[G][NB];  // u
  __shared__ double ts[G][NB];  // tanh(u) (tanh family)
  const int lane = threadIdx.x;
  const int gi = lane / L;
  const int r = lane % L;
  const bool row = r < NB;  // the lane owns a row of the padded matrix
  const int src0 = gi * L;  // lane 0 of the group

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

    const double u = own ? a.u[uo + r] : 0.0;
    const double tu = (FAM == FAM_TANH && own) ? tanh(u) : 0.0;
    if (row) {
      xs[gi][r] = u;
      ts[gi][r] = tu;
    }
    wave_sync();
    bool bad = own && !finite64(u);

    // ---- row r of J (identity past n) and the right-hand side ----
    double rhs = 0.0;
    if (row) {
      for (int j = 0; j < NB; ++j) {
        double v = (j == r) ? 1.0 : 0.0;
        if (own) {
          v = 0.0;
          if (j < n) {
            if constexpr (FAM == FAM_CUBIC) {
              const double aij = p[r * n + j];
              bad |= !finite64(aij);
              v = j == r ? aij + cubic_term_deriv(u) : aij;
            } else if constexpr (FAM == FAM_TANH) {
              const double aij = p[r * n + j];
              bad |= !finite64(aij);
              const double dphi = dtanh_known(dseed(xs[gi][j]), ts[gi][j]).d;
              const double w = aij * dphi;
              v = j == r ? w + p[n * n + n] : w;
            } else if constexpr (FAM == FAM_ROSENBROCK) {
              if (r == 0) {
                v = j == 0 ? -1.0 : 0.0;
              } else if (j == r - 1) {
                const Dual<double> um = dseed(xs[gi][r - 1]);
                v = (10.0 * (dconst(u) - um * um)).d;
              } else if (j == r) {
                v = (10.0 * (dseed(u) - dconst(xs[gi][r - 1]) * dconst(xs[gi][r - 1]))).d;
              }
            } else {  // the workflow example, n = 2
              const Dual<double> x0 = {xs[gi][0], j == 0 ? 1.0 : 0.0};
              const Dual<double> x1 = {xs[gi][1], j == 1 ? 1.0 : 0.0};
              if (r == 0) {
                const Dual<double> cube = x1 * x1 * x1;
                v = ((x0 + dconst(p[0])) * (cube - dconst(p[1])) + dconst(p[2])).d;
              } else {
                v = dsin(x1 * dexp(x0) - dconst(1.0)).d;
              }
            }
            bad |= !finite64(v);
          }
        }
        if constexpr (MODE == SENS_TANGENT) m[gi][r][j] = v;
        else m[gi][j][r] = v;
      }
    }
    if (own) {
      if constexpr (MODE == SENS_ADJOINT) {
        rhs = a.seed[uo + r];
      } else {
        // -(dF_r/dtheta) . v, the parameter derivatives of row r
        const double* __restrict__ v = a.seed + po;
        double sdot = 0.0;
        if constexpr (FAM == FAM_CUBIC) {
          for (int j = 0; j < n; ++j) sdot = __builtin_fma(v[r * n + j], xs[gi][j], sdot);
          sdot = sdot - v[n * n + r];
        } else if constexpr (FAM == FAM_TANH) {
          for (int j = 0; j < n; ++j) sdot = __builtin_fma(v[r * n + j], ts[gi][j], sdot);
          sdot = (sdot - v[n * n + r]) + v[n * n + n] * u;
        } else if constexpr (FAM == FAM_PAPER) {
          if (r == 0) {
            const double u1 = xs[gi][1];
            sdot = (u1 * u1 * u1 - p[1]) * v[0] - (u + p[0]) * v[1] + v[2];
          }
        }
        rhs = -sdot;
      }
      if constexpr (FAM == FAM_CUBIC || FAM == FAM_TANH) bad |= !finite64(p[n * n + r]);
      if constexpr (FAM == FAM_TANH) bad |= !finite64(p[n * n + n]);
      if constexpr (FAM == FAM_PAPER) bad |= r == 0 && !(finite64(p[0]) && finite64(p[1]) && finite64(p[2]));
    }
    bad = grp_any<L>(bad);
    wave_sync();

    // ---- elimination with partial pivoting ----
    bool sing = false;
    for (int k = 0; k < NB; ++k) {
      double cand = -1.0;
      if (row && r >= k) {
        const double c = __builtin_fabs(m[gi][r][k]);
        cand = c == c ? c : -1.0;  // a NaN never wins the search
      }
      int idx = r;
      grp_levels<L>([&](auto mc) {
        constexpr int M = decltype(mc)::value;
        const double oc = grp_partner<M, L>(cand);
        const int oi = grp_partner<M, L>(idx);
        if (oc > cand || (oc == cand && oi < idx)) {
          cand = oc;
          idx = oi;
        }
      });
      const int piv = idx;
      const double pk = m[gi][piv][k];
      sing = sing || !(pk != 0.0 && finite64(pk));
      const double r_k = __shfl(rhs, src0 + k, 64);
      const double r_p = __shfl(rhs, src0 + piv, 64);
      if (piv != k) {
        if (row) {
          const double x = m[gi][k][r];
          m[gi][k][r] = m[gi][piv][r];
          m[gi][piv][r] = x;
        }
        if (r == k) rhs = r_p;
        else if (r == piv) rhs = r_k;
      }
      wave_sync();
      const double rk = __shfl(rhs, src0 + k, 64);
      if (row && r > k) {
        const double l = m[gi][r][k] / pk;
        for (int j = k + 1; j < NB; ++j) m[gi][r][j] = m[gi][r][j] - l * m[gi][k][j];
        rhs = rhs - l * rk;
      }
      wave_sync();
    }
    // ---- back substitution: lane r ends with component r ----
    for (int i = NB - 1; i >= 0; --i) {
      if (r == i) rhs = rhs / m[gi][i][i];
      const double xi = __shfl(rhs, src0 + i, 64);
      if (row && r < i) rhs = rhs - m[gi][r][i] * xi;
    }
    const int32_t st = bad ? RC_NONFINITE : (sing ? RC_SINGULAR : RC_SUCCESS);
    const double x = st == RC_SUCCESS ? rhs : __builtin_nan("");

    // ---- outputs ----
    if constexpr (MODE == SENS_TANGENT) {
      if (own) a.out[uo + r] = x;
    } else {
      if (own && a.lambda) a.lambda[uo + r] = x;
      double* __restrict__ g = a.out + po;
      if constexpr (FAM == FAM_CUBIC || FAM == FAM_TANH) {
        // dF_k/dA_kj = u_j (cubic) or tanh(u_j) (tanh): lane j writes column j
        const double phi = FAM == FAM_CUBIC ? u : tu;
        for (int k = 0; k < NB; ++k) {
          const double lk = __shfl(x, src0 + k, 64);
          if (own && k < n) g[k * n + r] = -(lk * phi);
        }
        if (own) g[n * n + r] = x;  // dF_r/db_r = -1
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
