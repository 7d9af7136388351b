// Compressed L2P (Sec. 3.3, eq. compressed-local-form): per box, decompress the scaled
// local theta~ (forward substitution over the PDE recursion, Thm. mult_decompression,
// levels of m_z ascending), multiply by 1/i!, and add
//   phi(x) = sum_{i in M(p)} L~_i / i! X^i,    X = (x - c) / h,
// to every target of the box.  One workgroup per box; the coefficients live in LDS and are
// read as wave-wide broadcasts; each thread evaluates a nested Horner scheme.
#pragma once

#include "../../include/fmm.h"
#include "common.hpp"
#include "device_util.hpp"
#include "kernels.hpp"

namespace fmm {

namespace detail_l2p {

constexpr int kThreads = 256;

struct InvFact {
  double v[FMM_MAX_ORDER + 1];
  constexpr InvFact() : v() {
    double f = 1.0;
    for (int i = 0; i <= FMM_MAX_ORDER; ++i) {
      if (i > 0) f *= i;
      v[i] = 1.0 / f;
    }
  }
};

template <int P, bool CPLX>
__device__ inline void decompress_lds(double* L, const RecArgs& rec, int c, double h) {
  double cf[kMaxRecTerms];
  for (int t = 0; t < rec.n; ++t) {
    double f = rec.coef[t];
    for (int e = 0; e < rec.hpow[t]; ++e) f *= h;
    cf[t] = f;
  }
  for (int z = c; z <= P; ++z) {
    const int cnt = tri(P - z);
    for (int k = threadIdx.x; k < cnt; k += blockDim.x) {
      int x = 0, rem = k;
      while (rem > P - z - x) {
        rem -= P - z - x + 1;
        ++x;
      }
      const int y = rem;
      double sr = 0.0, si = 0.0;
      for (int t = 0; t < rec.n; ++t) {
        const int nx = x + rec.dx[t], ny = y + rec.dy[t], nz = z + rec.dz[t];
        const int n = full_index(P, nx, ny, nz);
        if constexpr (CPLX) {
          sr += cf[t] * L[2 * n];
          si += cf[t] * L[2 * n + 1];
        } else {
          sr += cf[t] * L[n];
        }
      }
      const int m = full_index(P, x, y, z);
      if constexpr (CPLX) {
        L[2 * m] = sr;
        L[2 * m + 1] = si;
      } else {
        L[m] = sr;
      }
    }
    __syncthreads();
  }
}

template <int P, typename R, bool CPLX>
__global__ __launch_bounds__(kThreads) void l2p_kernel(L2PArgs a) {
  constexpr int NP = nfull(P);
  constexpr int W = CPLX ? 2 : 1;
  __shared__ double Ld[NP * W];
  __shared__ R Lc[NP * W];
  const int64_t b = blockIdx.x;
  int lev = a.level[b];
  lev = lev < 0 ? 0 : (lev >= a.n_levels ? a.n_levels - 1 : lev);
  const double h = a.level_h[lev];
  const int nc = a.nc;
  const R* loc = reinterpret_cast<const R*>(a.local) + b * (int64_t)nc * W;
  for (int k = threadIdx.x; k < nc * W; k += blockDim.x) Ld[k] = (double)loc[k];
  __syncthreads();
  decompress_lds<P, CPLX>(Ld, a.rec, a.c, h);
  for (int k = threadIdx.x; k < NP; k += blockDim.x) {
    // recover (x, y, z) of full index k
    int z = 0;
    while (nfull(P) - nfull(P - z - 1) <= k) ++z;
    int rem = k - (nfull(P) - nfull(P - z));
    int x = 0;
    while (rem > P - z - x) {
      rem -= P - z - x + 1;
      ++x;
    }
    const int y = rem;
    constexpr InvFact IF{};
    const double f = IF.v[x] * IF.v[y] * IF.v[z];
    for (int u = 0; u < W; ++u) Lc[k * W + u] = (R)(Ld[k * W + u] * f);
  }
  __syncthreads();
  const double cen[3] = {a.center[3 * b], a.center[3 * b + 1], a.center[3 * b + 2]};
  int64_t lo = a.range[2 * b], hi = a.range[2 * b + 1];
  lo = lo < 0 ? 0 : (lo > a.n_pts ? a.n_pts : lo);
  hi = hi < lo ? lo : (hi > a.n_pts ? a.n_pts : hi);
  const R* xyz = reinterpret_cast<const R*>(a.xyz);
  const R cx = (R)cen[0], cy = (R)cen[1], cz = (R)cen[2], ih = (R)(1.0 / h);
  for (int64_t s = lo + threadIdx.x; s < hi; s += blockDim.x) {
    const R X = (xyz[3 * s + 0] - cx) * ih;
    const R Y = (xyz[3 * s + 1] - cy) * ih;
    const R Z = (xyz[3 * s + 2] - cz) * ih;
    R pr = R(0), pi = R(0);
#pragma unroll
    for (int z = P; z >= 0; --z) {
      R qr = R(0), qi = R(0);
#pragma unroll
      for (int x = P - z; x >= 0; --x) {
        R rr = R(0), ri = R(0);
#pragma unroll
        for (int y = P - z - x; y >= 0; --y) {
          const int k = full_index(P, x, y, z);
          rr = rr * Y + Lc[k * W];
          if constexpr (CPLX) ri = ri * Y + Lc[k * W + 1];
        }
        qr = qr * X + rr;
        if constexpr (CPLX) qi = qi * X + ri;
      }
      pr = pr * Z + qr;
      if constexpr (CPLX) pi = pi * Z + qi;
    }
    R* pot = reinterpret_cast<R*>(a.pot);
    if constexpr (CPLX) {
      pot[2 * s] += pr;
      pot[2 * s + 1] += pi;
    } else {
      pot[s] += pr;
    }
  }
}

template <int P>
int launch_l2p_p(const L2PArgs& a, int dtype, hipStream_t s) {
  dim3 g((unsigned)a.n_box), t(kThreads);
  switch (dtype) {
    case FMM_F64: hipLaunchKernelGGL((l2p_kernel<P, double, false>), g, t, 0, s, a); break;
    case FMM_F32: hipLaunchKernelGGL((l2p_kernel<P, float, false>), g, t, 0, s, a); break;
    case FMM_C128: hipLaunchKernelGGL((l2p_kernel<P, double, true>), g, t, 0, s, a); break;
    case FMM_C64: hipLaunchKernelGGL((l2p_kernel<P, float, true>), g, t, 0, s, a); break;
    default: return fail(FMM_EINVAL, "dtype");
  }
  FMM_HIP_CHECK(hipGetLastError());
  return FMM_OK;
}

}  // namespace detail_l2p

#define FMM_INSTANTIATE_L2P(P) \
  int launch_l2p_order_##P(const L2PArgs& a, int dtype, hipStream_t s) { \
    return detail_l2p::launch_l2p_p<P>(a, dtype, s); \
  }

}  // namespace fmm
