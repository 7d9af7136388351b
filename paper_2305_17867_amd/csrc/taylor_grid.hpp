// FP64 derivatives of G at one point by Taylor-coefficient recurrences, computed cooperatively
// by the threads of a workgroup (Sec. 4.4: recurrences in the style of eq. deriv_laplace_3d).
// With a_k = G^(k)(x0)/k! and n = |k|:
//   G = r^nu (Laplace nu = -1, biharmonic nu = 1):
//     n r0^2 a_k = -(2n - 2 - nu) S1(a) - (n - 2 - nu) S2(a)
//   G = psi/r, psi = exp(-s r) (Yukawa s = lam, Helmholtz s = -i k), b = coefficients of psi:
//     n r0^2 a_k = -(2n - 1) S1(a) - (n - 1) S2(a) - s (S1(b) + S2(b)),
//     n b_k = -s (S1(a) + S2(a)),
//   S1(a) = sum_j x0_j a_{k - e_j},  S2(a) = sum_j a_{k - 2 e_j}.
// Order n only reads orders n-1 and n-2, and only lower or equal m_z, so the slab m_z < Sz is
// closed under the recurrence; a three-order ring in LDS holds what the next order reads.  The
// recurrences run at the point in units of h (x0 = d / h, with s h in place of s), which gives
// the scaled derivatives of Sec. 4.1.1 directly:  G^(m)(d) h^|m| = h^(-1) G~^(m)(x0)  (h^(+1)
// for the biharmonic kernel).
#pragma once

#include "../../include/fmm.h"
#include "device_util.hpp"

namespace fmm {

constexpr int kTaylorMaxS = 2 * FMM_MAX_ORDER + 1;  // grid side for |m| <= 2 FMM_MAX_ORDER
constexpr int kTaylorMaxZ = 7;                       // m_z < 7: 2 (c - 1) + 1 for c <= 4

struct TaylorFact {
  double v[2 * FMM_MAX_ORDER + 1];
  constexpr TaylorFact() : v() {
    v[0] = 1.0;
    for (int i = 1; i <= 2 * FMM_MAX_ORDER; ++i) v[i] = v[i - 1] * i;
  }
};

// The ring of the recurrence (LDS): ra[order % 3][m_z][m_x] (m_y = order - m_z - m_x), rb the
// same for psi.
template <bool CPLX>
struct TaylorRing {
  using T = typename Val<double, CPLX>::T;
  T ra[3][kTaylorMaxZ][kTaylorMaxS];
  T rb[3][kTaylorMaxZ][kTaylorMaxS];
};

// out[(m_z S + m_x) S + m_y] = G^(m)(h x0) h^|m| for |m| <= P2, m_z < Sz (entries with
// |m| > P2 are not written).  out may be global or LDS memory.  Every thread of the workgroup
// must call it (it synchronises after each order).
template <bool CPLX, typename OutT>
__device__ inline void taylor_grid(int kernel, double param, const double (&x0)[3], double h, int P2, int S, int Sz,
                                   OutT* out, TaylorRing<CPLX>& ring) {
  using T = typename Val<double, CPLX>::T;
  const double r02 = x0[0] * x0[0] + x0[1] * x0[1] + x0[2] * x0[2];
  const double r0 = sqrt(r02);
  T s{};  // s h: Yukawa lam h, Helmholtz -i k h
  if (kernel == FMM_YUKAWA) s = T(param * h);
  if constexpr (CPLX) {
    if (kernel == FMM_HELMHOLTZ) s = T(0.0, -param * h);
  }
  const bool expo = kernel == FMM_YUKAWA || kernel == FMM_HELMHOLTZ;
  const double nu = kernel == FMM_BIHARMONIC ? 1.0 : -1.0;
  const double norm = kernel == FMM_BIHARMONIC ? h : 1.0 / (4.0 * M_PI * h);
  auto A = [&](int n, int mx, int my, int mz) -> T {
    if (mx < 0 || my < 0 || mz < 0 || n < 0) return T(0.0);
    return ring.ra[n % 3][mz][mx];
  };
  auto B = [&](int n, int mx, int my, int mz) -> T {
    if (mx < 0 || my < 0 || mz < 0 || n < 0) return T(0.0);
    return ring.rb[n % 3][mz][mx];
  };
  for (int n = 0; n <= P2; ++n) {
    const int zmax = n < Sz - 1 ? n : Sz - 1;
    const int cnt = (zmax + 1) * (n + 1);  // (mz, mx) pairs, mx <= n - mz
    for (int k = threadIdx.x; k < cnt; k += blockDim.x) {
      const int mz = k / (n + 1), mx = k % (n + 1);
      if (mx > n - mz) continue;
      const int my = n - mz - mx;
      T av, bv;
      if (n == 0) {
        if (kernel == FMM_LAPLACE) {
          av = T(1.0 / r0);
        } else if (kernel == FMM_BIHARMONIC) {
          av = T(r0);
        } else {
          if constexpr (CPLX) {
            // exp(-s r0) with s = -i k h: exp(i k h r0)
            double ph = param * h * r0;
            bv = T(cos(ph), sin(ph));
          } else {
            bv = T(exp(-param * h * r0));
          }
          av = (1.0 / r0) * bv;
        }
      } else {
        // S1, S2 over the three axes
        T s1a = x0[0] * A(n - 1, mx - 1, my, mz) + x0[1] * A(n - 1, mx, my - 1, mz) +
                x0[2] * A(n - 1, mx, my, mz - 1);
        T s2a = A(n - 2, mx - 2, my, mz) + A(n - 2, mx, my - 2, mz) + A(n - 2, mx, my, mz - 2);
        const double dn = (double)n;
        if (!expo) {
          av = (-1.0 / (dn * r02)) * ((2.0 * dn - 2.0 - nu) * s1a + (dn - 2.0 - nu) * s2a);
        } else {
          T s1b = x0[0] * B(n - 1, mx - 1, my, mz) + x0[1] * B(n - 1, mx, my - 1, mz) +
                  x0[2] * B(n - 1, mx, my, mz - 1);
          T s2b = B(n - 2, mx - 2, my, mz) + B(n - 2, mx, my - 2, mz) + B(n - 2, mx, my, mz - 2);
          av = (-1.0 / (dn * r02)) * ((2.0 * dn - 1.0) * s1a + (dn - 1.0) * s2a + s * (s1b + s2b));
          bv = (-1.0 / dn) * (s * (s1a + s2a));
        }
      }
      ring.ra[n % 3][mz][mx] = av;
      if (expo) ring.rb[n % 3][mz][mx] = bv;
      constexpr TaylorFact F{};
      const double f = F.v[mx] * F.v[my] * F.v[mz] * norm;
      out[(mz * S + mx) * S + my] = f * av;
    }
    __syncthreads();
  }
}

}  // namespace fmm
