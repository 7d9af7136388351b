// FP64 derivative tables for the compressed M2L (Sec. 4.1: the derivatives G^(i+q) at the
// translation vector, |i + q| <= 2p, (i + q)_z <= 2(c - 1), precomputed per offset).
//
// Method: Taylor-coefficient recurrences in the style of the paper's Laplace recurrence
// (eq. deriv_laplace_3d).  With a_k = G^(k)(x0)/k! and n = |k|:
//   G = r^nu (Laplace nu = -1, biharmonic nu = 1):
//     n r0^2 a_k = -(2n - 2 - nu) S1(a) - (n - 2 - nu) S2(a)
//   G = psi/r, psi = exp(-s r) (Yukawa s = lam, Helmholtz s = -i k), b = coefficients of psi:
//     n r0^2 a_k = -(2n - 1) S1(a) - (n - 1) S2(a) - s (S1(b) + S2(b)),
//     n b_k = -s (S1(a) + S2(a)),
//   S1(a) = sum_j x0_j a_{k - e_j},  S2(a) = sum_j a_{k - 2 e_j}.
// Order n only reads orders n-1 and n-2, so a workgroup computes one table order by order
// with a three-order ring in LDS.  The recurrences are run at the offset in units of h
// (x0 = d / h, with s h in place of s), which gives the scaled table of Sec. 4.1.1
// directly:  G^(m)(d) h^|m| = h^(-1) G~^(m)(x0)  (h^(+1) for the biharmonic kernel).
#include "../../include/fmm.h"
#include "common.hpp"
#include "device_util.hpp"
#include "kernels.hpp"

namespace fmm {

namespace {

constexpr int kTabThreads = 256;
constexpr int kMaxS = 2 * FMM_MAX_ORDER + 1;

struct Fact {
  double v[2 * FMM_MAX_ORDER + 1];
  constexpr Fact() : v() {
    v[0] = 1.0;
    for (int i = 1; i <= 2 * FMM_MAX_ORDER; ++i) v[i] = v[i - 1] * i;
  }
};

template <bool CPLX>
__global__ __launch_bounds__(kTabThreads) void tables_kernel(TableArgs a) {
  using T = typename Val<double, CPLX>::T;
  const int64_t tb = blockIdx.x;
  if (tb >= a.n) return;
  const int S = a.S, Sz = a.Sz, P2 = a.p2;
  const double x0[3] = {a.offset[tb * 3 + 0], a.offset[tb * 3 + 1], a.offset[tb * 3 + 2]};
  const double h = a.h[tb];
  const double r02 = x0[0] * x0[0] + x0[1] * x0[1] + x0[2] * x0[2];
  const double r0 = sqrt(r02);
  // s * h: Yukawa lam h, Helmholtz -i k h
  T s{};
  if (a.kernel == FMM_YUKAWA) s = T(a.param * h);
  if constexpr (CPLX) {
    if (a.kernel == FMM_HELMHOLTZ) s = T(0.0, -a.param * h);
  }
  const bool expo = a.kernel == FMM_YUKAWA || a.kernel == FMM_HELMHOLTZ;
  const double nu = a.kernel == FMM_BIHARMONIC ? 1.0 : -1.0;
  const double norm = a.kernel == FMM_BIHARMONIC ? h : 1.0 / (4.0 * M_PI * h);

  // ring[order % 3][mz][mx] (my = order - mz - mx)
  __shared__ T ra[3][7][kMaxS];
  __shared__ T rb[3][7][kMaxS];

  T* out = reinterpret_cast<T*>(a.out) + tb * (int64_t)(Sz * S * S);
  // entries with |m| > 2p: zero
  for (int k = threadIdx.x; k < Sz * S * S; k += blockDim.x) {
    int mz = k / (S * S), rem = k % (S * S), mx = rem / S, my = rem % S;
    if (mx + my + mz > P2) out[k] = T(0.0);
  }

  auto A = [&](int n, int mx, int my, int mz) -> T {
    if (mx < 0 || my < 0 || mz < 0 || n < 0) return T(0.0);
    return ra[n % 3][mz][mx];
  };
  auto B = [&](int n, int mx, int my, int mz) -> T {
    if (mx < 0 || my < 0 || mz < 0 || n < 0) return T(0.0);
    return rb[n % 3][mz][mx];
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
        if (a.kernel == FMM_LAPLACE) {
          av = T(1.0 / r0);
        } else if (a.kernel == FMM_BIHARMONIC) {
          av = T(r0);
        } else {
          if constexpr (CPLX) {
            // exp(-s r0) with s = -i k h: exp(i k h r0)
            double ph = a.param * h * r0;
            bv = T(cos(ph), sin(ph));
          } else {
            bv = T(exp(-a.param * h * r0));
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
      ra[n % 3][mz][mx] = av;
      if (expo) rb[n % 3][mz][mx] = bv;
      constexpr Fact F{};
      const double f = F.v[mx] * F.v[my] * F.v[mz] * norm;
      out[(mz * S + mx) * S + my] = f * av;
    }
    __syncthreads();
  }
}

}  // namespace

int launch_tables(const TableArgs& a, bool cplx, hipStream_t s) {
  if (a.n == 0) return FMM_OK;
  if (cplx)
    hipLaunchKernelGGL(tables_kernel<true>, dim3((unsigned)a.n), dim3(kTabThreads), 0, s, a);
  else
    hipLaunchKernelGGL(tables_kernel<false>, dim3((unsigned)a.n), dim3(kTabThreads), 0, s, a);
  FMM_HIP_CHECK(hipGetLastError());
  return FMM_OK;
}

}  // namespace fmm
