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

// Nested Horner evaluation of sum_{|m| <= Q} C[full_index(Q, m)] X^m.
template <int Q, typename R>
__device__ inline R horner(const R* C, int W, int u, R X, R Y, R Z) {
  R pz = R(0);
#pragma unroll
  for (int z = Q; z >= 0; --z) {
    R qx = R(0);
#pragma unroll
    for (int x = Q - z; x >= 0; --x) {
      R ry = R(0);
#pragma unroll
      for (int y = Q - z - x; y >= 0; --y) ry = ry * Y + C[full_index(Q, x, y, z) * W + u];
      qx = qx * X + ry;
    }
    pz = pz * Z + qx;
  }
  return pz;
}

template <int P, typename R, bool CPLX, bool GRAD>
__global__ __launch_bounds__(kThreads) void l2p_kernel(L2PArgs a) {
  constexpr int NP = nfull(P);
  constexpr int NG = GRAD ? nfull(P - 1) : 0;
  constexpr int W = CPLX ? 2 : 1;
  __shared__ double Ld[NP * W];
  __shared__ R Lc[NP * W];
  __shared__ R Lg[3][(NG > 0 ? NG : 1) * W];
  const int64_t b = blockIdx.x;
  int lev = a.level[b];
  lev = lev < 0 ? 0 : (lev >= a.n_levels ? a.n_levels - 1 : lev);
  const double h = a.level_h[lev];
  const int nc = a.nc;
  const R* loc = reinterpret_cast<const R*>(a.local) + b * (int64_t)nc * W;
  for (int k = threadIdx.x; k < nc * W; k += blockDim.x) Ld[k] = (double)loc[k];
  __syncthreads();
  decompress_lds<P, CPLX>(Ld, a.rec, a.c, h);
  constexpr InvFact IF{};
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
    const double f = IF.v[x] * IF.v[y] * IF.v[z];
    for (int u = 0; u < W; ++u) Lc[k * W + u] = (R)(Ld[k * W + u] * f);
    if constexpr (GRAD) {
      // d/dX_k of L_m X^m / m!: coefficient of X^(m - e_k) is L_m / (m - e_k)!
      const int mm[3] = {x, y, z};
      for (int ax = 0; ax < 3; ++ax) {
        if (mm[ax] == 0) continue;
        int d[3] = {x, y, z};
        d[ax] -= 1;
        const int g = full_index(P - 1, d[0], d[1], d[2]);
        const double fg = IF.v[d[0]] * IF.v[d[1]] * IF.v[d[2]];
        for (int u = 0; u < W; ++u) Lg[ax][g * W + u] = (R)(Ld[k * W + u] * fg);
      }
    }
  }
  __syncthreads();
  const double cen[3] = {a.center[3 * b], a.center[3 * b + 1], a.center[3 * b + 2]};
  int64_t lo = a.range[2 * b], hi = a.range[2 * b + 1];
  lo = lo < 0 ? 0 : (lo > a.n_pts ? a.n_pts : lo);
  hi = hi < lo ? lo : (hi > a.n_pts ? a.n_pts : hi);
  const R* xyz = reinterpret_cast<const R*>(a.xyz);
  const R cx = (R)cen[0], cy = (R)cen[1], cz = (R)cen[2], ih = (R)(a.xsign / h);
  for (int64_t s = lo + threadIdx.x; s < hi; s += blockDim.x) {
    const R X = (xyz[3 * s + 0] - cx) * ih;
    const R Y = (xyz[3 * s + 1] - cy) * ih;
    const R Z = (xyz[3 * s + 2] - cz) * ih;
    if (a.pot) {
      R* pot = reinterpret_cast<R*>(a.pot);
      pot[s * W] += horner<P, R>(Lc, W, 0, X, Y, Z);
      if constexpr (CPLX) pot[2 * s + 1] += horner<P, R>(Lc, W, 1, X, Y, Z);
    }
    if constexpr (GRAD && P > 0 && !CPLX) {
      const R sc = a.gscale ? reinterpret_cast<const R*>(a.gscale)[s] : R(1);
      R* g = reinterpret_cast<R*>(a.grad);
      g[3 * s + 0] += sc * ih * horner<P - 1, R>(Lg[0], 1, 0, X, Y, Z);
      g[3 * s + 1] += sc * ih * horner<P - 1, R>(Lg[1], 1, 0, X, Y, Z);
      g[3 * s + 2] += sc * ih * horner<P - 1, R>(Lg[2], 1, 0, X, Y, Z);
    }
  }
}

template <int P>
int launch_l2p_p(const L2PArgs& a, int dtype, hipStream_t s) {
  dim3 g((unsigned)a.n_box), t(kThreads);
  const bool grad = a.grad != nullptr;
  switch (dtype) {
    case FMM_F64:
      if (grad) hipLaunchKernelGGL((l2p_kernel<P, double, false, true>), g, t, 0, s, a);
      else hipLaunchKernelGGL((l2p_kernel<P, double, false, false>), g, t, 0, s, a);
      break;
    case FMM_F32:
      if (grad) hipLaunchKernelGGL((l2p_kernel<P, float, false, true>), g, t, 0, s, a);
      else hipLaunchKernelGGL((l2p_kernel<P, float, false, false>), g, t, 0, s, a);
      break;
    case FMM_C128: hipLaunchKernelGGL((l2p_kernel<P, double, true, false>), g, t, 0, s, a); break;
    case FMM_C64: hipLaunchKernelGGL((l2p_kernel<P, float, true, false>), g, t, 0, s, a); break;
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
