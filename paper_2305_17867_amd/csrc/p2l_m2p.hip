// Compressed P2L (Sec. 3.2, eq. stored_local_coeffs) and compressed M2P (Sec. 3.5, eq.
// multipole_eval_beta): both need the derivatives of G on the kept set J only, at one point per
// source (P2L) or target (M2P).  A workgroup of one wavefront evaluates them for one point with
// the recurrences of taylor_grid.hpp into an LDS grid (orders <= p, m_z < c: the slab that J
// occupies) and contracts at once:
//   M2P  phi(x) += sum_s sum_{q in J} beta~_s[q] G^(q)(x - c_s) h_s^|q|   (one workgroup owns a
//        set of targets of a box and adds over the boxes of its list in list order)
//   P2L  theta~_t[j] += sum_s sum_{y in s} w(y) G^(j)(c_t - y) h_t^|j|   (one workgroup per
//        target box: the sums over all sources in a fixed order, one coefficient per lane)
// Scaled form of Sec. 4.1.1 (t = 1/h of the expansion's own box).  Deterministic.
// Real Laplace expansions up to order 8 take a faster path (one point per lane, derivatives in
// registers by the recurrence of eq. deriv_laplace_3d), further below.
#include "../../include/fmm.h"
#include "common.hpp"
#include "device_util.hpp"
#include "kernels.hpp"
#include "taylor_grid.hpp"

namespace fmm {

namespace {

constexpr int kPEThreads = 64;
constexpr int kPEMaxGrid = 4 * (FMM_MAX_ORDER + 1) * (FMM_MAX_ORDER + 1);  // m_z < 4, side p + 1
constexpr int kPEMaxPerLane = 8;  // kept coefficients per lane in P2L (Nc <= 512)

__device__ inline int grid_pos(int32_t packed, int S) {
  const int x = packed & 255, y = (packed >> 8) & 255, z = packed >> 16;
  return (z * S + x) * S + y;
}

__device__ inline int clamp_level(const PointExpArgs& a, int b) {
  int lev = a.level[b];
  return lev < 0 ? 0 : (lev >= a.n_levels ? a.n_levels - 1 : lev);
}

__device__ inline void clamp_range(const PointExpArgs& a, int b, int64_t& lo, int64_t& hi) {
  lo = a.range[2 * b];
  hi = a.range[2 * b + 1];
  lo = lo < 0 ? 0 : (lo > a.n_pts ? a.n_pts : lo);
  hi = hi < lo ? lo : (hi > a.n_pts ? a.n_pts : hi);
}

__device__ inline void list_bounds(const PointExpArgs& a, int64_t k, int& l0, int& l1) {
  l0 = a.list_ptr[k];
  l1 = a.list_ptr[k + 1];
  l0 = l0 < 0 ? 0 : (l0 > a.n_list ? (int)a.n_list : l0);
  l1 = l1 < l0 ? l0 : (l1 > a.n_list ? (int)a.n_list : l1);
}

// workgroup (k, y): targets y, y + gridDim.y, ... of box tbox[k]
template <typename R, bool CPLX>
__global__ __launch_bounds__(kPEThreads) void m2p_kernel(PointExpArgs a) {
  using T = typename Val<double, CPLX>::T;
  constexpr int W = CPLX ? 2 : 1;
  __shared__ TaylorRing<CPLX> ring;
  __shared__ T grid[kPEMaxGrid];
  const int64_t k = blockIdx.x;
  const int t = a.tbox[k];
  if (t < 0 || t >= a.n_box) return;  // uniform
  int64_t lo, hi;
  clamp_range(a, t, lo, hi);
  int l0, l1;
  list_bounds(a, k, l0, l1);
  const int S = a.p + 1;
  const R* xyz = reinterpret_cast<const R*>(a.xyz);
  const R* mp = reinterpret_cast<const R*>(a.mpole);
  for (int64_t i = lo + blockIdx.y; i < hi; i += gridDim.y) {
    const double x[3] = {(double)xyz[3 * i], (double)xyz[3 * i + 1], (double)xyz[3 * i + 2]};
    double sr = 0.0, si = 0.0;
    for (int e = l0; e < l1; ++e) {
      const int s = a.list[e];
      if (s < 0 || s >= a.n_box) continue;  // uniform
      const double h = a.level_h[clamp_level(a, s)];
      const double x0[3] = {(x[0] - a.center[3 * s]) / h, (x[1] - a.center[3 * s + 1]) / h,
                            (x[2] - a.center[3 * s + 2]) / h};
      taylor_grid<CPLX>(a.kernel, a.param, x0, h, a.p, S, a.c, grid, ring);
      const R* beta = mp + (int64_t)s * a.nc * W;
      for (int q = threadIdx.x; q < a.nc; q += kPEThreads) {
        const T g = grid[grid_pos(a.jxyz[q], S)];
        if constexpr (CPLX) {
          const double br = beta[2 * q], bi = beta[2 * q + 1];
          sr += g.re * br - g.im * bi;
          si += g.re * bi + g.im * br;
        } else {
          sr += g * (double)beta[q];
        }
      }
      __syncthreads();  // the grid is rewritten for the next box
    }
    // sum over the wavefront in a fixed order
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
      sr += __shfl_xor(sr, m, 64);
      if constexpr (CPLX) si += __shfl_xor(si, m, 64);
    }
    if (threadIdx.x == 0) {
      R* pot = reinterpret_cast<R*>(a.out);
      pot[W * i] = (R)((double)pot[W * i] + sr);
      if constexpr (CPLX) pot[2 * i + 1] = (R)((double)pot[2 * i + 1] + si);
    }
  }
}

// one workgroup per target box; lane l keeps the kept coefficients l, l + 64, ...
template <typename R, bool CPLX>
__global__ __launch_bounds__(kPEThreads) void p2l_kernel(PointExpArgs a) {
  using T = typename Val<double, CPLX>::T;
  constexpr int W = CPLX ? 2 : 1;
  __shared__ TaylorRing<CPLX> ring;
  __shared__ T grid[kPEMaxGrid];
  const int64_t k = blockIdx.x;
  const int t = a.tbox[k];
  if (t < 0 || t >= a.n_box) return;  // uniform
  int l0, l1;
  list_bounds(a, k, l0, l1);
  const int S = a.p + 1;
  const double h = a.level_h[clamp_level(a, t)];
  const double c[3] = {a.center[3 * t], a.center[3 * t + 1], a.center[3 * t + 2]};
  const R* xyz = reinterpret_cast<const R*>(a.xyz);
  const R* wv = reinterpret_cast<const R*>(a.w);
  double acc[kPEMaxPerLane][W];
  int pos[kPEMaxPerLane];
#pragma unroll
  for (int j = 0; j < kPEMaxPerLane; ++j) {
    const int q = threadIdx.x + j * kPEThreads;
    pos[j] = q < a.nc ? grid_pos(a.jxyz[q], S) : 0;
#pragma unroll
    for (int u = 0; u < W; ++u) acc[j][u] = 0.0;
  }
  for (int e = l0; e < l1; ++e) {
    const int s = a.list[e];
    if (s < 0 || s >= a.n_box) continue;  // uniform
    int64_t lo, hi;
    clamp_range(a, s, lo, hi);
    for (int64_t i = lo; i < hi; ++i) {
      const double x0[3] = {(c[0] - (double)xyz[3 * i]) / h, (c[1] - (double)xyz[3 * i + 1]) / h,
                            (c[2] - (double)xyz[3 * i + 2]) / h};
      taylor_grid<CPLX>(a.kernel, a.param, x0, h, a.p, S, a.c, grid, ring);
      const double wr = (double)wv[W * i], wi = CPLX ? (double)wv[W * i + 1] : 0.0;
#pragma unroll
      for (int j = 0; j < kPEMaxPerLane; ++j) {
        if (threadIdx.x + j * kPEThreads >= a.nc) break;
        const T g = grid[pos[j]];
        if constexpr (CPLX) {
          acc[j][0] += g.re * wr - g.im * wi;
          acc[j][1] += g.re * wi + g.im * wr;
        } else {
          acc[j][0] += g * wr;
        }
      }
      __syncthreads();  // the grid is rewritten for the next point
    }
  }
  R* loc = reinterpret_cast<R*>(a.out) + (int64_t)t * a.nc * W;
#pragma unroll
  for (int j = 0; j < kPEMaxPerLane; ++j) {
    const int q = threadIdx.x + j * kPEThreads;
    if (q >= a.nc) break;
#pragma unroll
    for (int u = 0; u < W; ++u) loc[W * q + u] = (R)((double)loc[W * q + u] + acc[j][u]);
  }
}

// ----------------------------------------------------------------------------- Laplace, p <= 8
//
// For the Laplace kernel the kept derivatives at one point are computed by one lane, in
// registers, with the recurrence of eq. deriv_laplace_3d for g = 1/r at the scaled offset X:
//   r^2 g(n,m,l) = -(2n-1) x g(n-1,m,l) - (n-1)^2 g(n-2,m,l) - 2m y g(n,m-1,l) - m(m-1) g(n,m-2,l)
//                  - 2l z g(n,m,l-1) - l(l-1) g(n,m,l-2)                             (n >= 1),
// with x and y exchanged for n = 0 (m >= 1) and the pure z recurrence for n = m = 0.  Every
// term it reads lies in the kept slab l < 2 itself, so the slab is all the lane holds.  In the
// scaled form G^(q)(h X) h^|q| = g^(q)(X) / (4 pi h).

constexpr int kLapMaxP = 8;

__host__ __device__ constexpr int lap_nkept(int P) { return (P + 1) * (P + 2) / 2 + P * (P + 1) / 2; }

// position of (x, y, z), z < 2, in the kept order (m_z, then m_x, then m_y fastest)
__host__ __device__ constexpr int lap_pos(int P, int x, int y, int z) {
  const int Q = P - z;  // order bound of the slab
  const int off = z == 0 ? 0 : (P + 1) * (P + 2) / 2;
  return off + x * (Q + 1) - x * (x - 1) / 2 + y;
}

template <int P>
__device__ __forceinline__ void lap_kept_derivs(double X, double Y, double Z, double (&g)[lap_nkept(P)]) {
  const double r2 = X * X + Y * Y + Z * Z, ir2 = 1.0 / r2;
#pragma unroll
  for (int l = 0; l < 2 && l <= P; ++l)
#pragma unroll
    for (int n = 0; n <= P - l; ++n)
#pragma unroll
      for (int m = 0; m <= P - l - n; ++m) {
        const int k = lap_pos(P, n, m, l);
        if (n == 0 && m == 0 && l == 0) {
          g[k] = sqrt(ir2);
        } else if (n >= 1) {
          double v = -(2.0 * n - 1.0) * X * g[lap_pos(P, n - 1, m, l)];
          if (n >= 2) v -= (double)((n - 1) * (n - 1)) * g[lap_pos(P, n - 2, m, l)];
          if (m >= 1) v -= 2.0 * m * Y * g[lap_pos(P, n, m - 1, l)];
          if (m >= 2) v -= (double)(m * (m - 1)) * g[lap_pos(P, n, m - 2, l)];
          if (l >= 1) v -= 2.0 * l * Z * g[lap_pos(P, n, m, l - 1)];
          g[k] = v * ir2;
        } else if (m >= 1) {
          double v = -(2.0 * m - 1.0) * Y * g[lap_pos(P, 0, m - 1, l)];
          if (m >= 2) v -= (double)((m - 1) * (m - 1)) * g[lap_pos(P, 0, m - 2, l)];
          if (l >= 1) v -= 2.0 * l * Z * g[lap_pos(P, 0, m, l - 1)];
          g[k] = v * ir2;
        } else {  // n = m = 0, l = 1
          g[k] = -Z * g[lap_pos(P, 0, 0, 0)] * ir2;
        }
      }
}

constexpr double kInv4Pi = 0.07957747154594767;  // 1 / (4 pi)

// M2P: workgroup (k, y) takes the chunks y, y + gridDim.y, ... of 64 targets of box tbox[k];
// lane = target; the list box's multipole is the same for every lane.
template <int P, typename R>
__global__ __launch_bounds__(kPEThreads) void m2p_laplace_kernel(PointExpArgs a) {
  constexpr int NC = lap_nkept(P);
  const int64_t k = blockIdx.x;
  const int t = a.tbox[k];
  if (t < 0 || t >= a.n_box) return;  // uniform
  int64_t lo, hi;
  clamp_range(a, t, lo, hi);
  int l0, l1;
  list_bounds(a, k, l0, l1);
  const R* xyz = reinterpret_cast<const R*>(a.xyz);
  const R* mp = reinterpret_cast<const R*>(a.mpole);
  for (int64_t c0 = lo + (int64_t)blockIdx.y * kPEThreads; c0 < hi; c0 += (int64_t)gridDim.y * kPEThreads) {
    const int64_t i = c0 + threadIdx.x;
    const bool ok = i < hi;
    const double x = ok ? (double)xyz[3 * i] : 0.0, y = ok ? (double)xyz[3 * i + 1] : 0.0,
                 z = ok ? (double)xyz[3 * i + 2] : 0.0;
    double phi = 0.0;
    for (int e = l0; e < l1; ++e) {
      const int s = a.list[e];
      if (s < 0 || s >= a.n_box) continue;  // uniform
      const double ih = 1.0 / a.level_h[clamp_level(a, s)];
      double g[NC];
      lap_kept_derivs<P>((x - a.center[3 * s]) * ih, (y - a.center[3 * s + 1]) * ih, (z - a.center[3 * s + 2]) * ih, g);
      const R* beta = mp + (int64_t)s * NC;
      double sum = 0.0;
#pragma unroll
      for (int q = 0; q < NC; ++q) sum = fma((double)beta[q], g[q], sum);
      phi = fma(sum, ih, phi);
    }
    if (ok) {
      R* pot = reinterpret_cast<R*>(a.out);
      pot[i] = (R)((double)pot[i] + phi * kInv4Pi);
    }
  }
}

// P2L: one wavefront per target box; lane = source point, 64 at a time; each chunk's weighted
// derivatives go through an LDS transpose so that lane l sums coefficients l and l + 64 over
// the chunk in lane order (deterministic).
template <int P, typename R>
__global__ __launch_bounds__(kPEThreads) void p2l_laplace_kernel(PointExpArgs a) {
  constexpr int NC = lap_nkept(P);
  constexpr int NJ = (NC + kPEThreads - 1) / kPEThreads;  // coefficients per lane
  __shared__ double tr[NC][kPEThreads + 1];
  const int64_t k = blockIdx.x;
  const int t = a.tbox[k];
  if (t < 0 || t >= a.n_box) return;  // uniform
  int l0, l1;
  list_bounds(a, k, l0, l1);
  const double ih = 1.0 / a.level_h[clamp_level(a, t)];
  const double c[3] = {a.center[3 * t], a.center[3 * t + 1], a.center[3 * t + 2]};
  const R* xyz = reinterpret_cast<const R*>(a.xyz);
  const R* wv = reinterpret_cast<const R*>(a.w);
  const int lane = threadIdx.x;
  double acc[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) acc[j] = 0.0;
  for (int e = l0; e < l1; ++e) {
    const int s = a.list[e];
    if (s < 0 || s >= a.n_box) continue;  // uniform
    int64_t lo, hi;
    clamp_range(a, s, lo, hi);
    for (int64_t c0 = lo; c0 < hi; c0 += kPEThreads) {  // uniform
      const int64_t i = c0 + lane;
      const bool ok = i < hi;
      double g[NC];
      lap_kept_derivs<P>(ok ? (c[0] - (double)xyz[3 * i]) * ih : 1.0, ok ? (c[1] - (double)xyz[3 * i + 1]) * ih : 0.0,
                         ok ? (c[2] - (double)xyz[3 * i + 2]) * ih : 0.0, g);
      const double wi = ok ? (double)wv[i] : 0.0;
#pragma unroll
      for (int q = 0; q < NC; ++q) tr[q][lane] = wi * g[q];
      __syncthreads();
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int q = lane + j * kPEThreads;
        if (q < NC) {
          double v = acc[j];
          for (int u = 0; u < kPEThreads; ++u) v += tr[q][u];
          acc[j] = v;
        }
      }
      __syncthreads();
    }
  }
  R* loc = reinterpret_cast<R*>(a.out) + (int64_t)t * NC;
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int q = lane + j * kPEThreads;
    if (q < NC) loc[q] = (R)((double)loc[q] + acc[j] * ih * kInv4Pi);
  }
}

template <typename R, int P>
int launch_laplace_p(const PointExpArgs& a, bool m2p, hipStream_t s) {
  if constexpr (P > kLapMaxP) {
    return fail(FMM_EUNSUPPORTED, "order");
  } else {
    if (a.p != P) return launch_laplace_p<R, P + 1>(a, m2p, s);
    if (m2p)
      hipLaunchKernelGGL((m2p_laplace_kernel<P, R>), dim3((unsigned)a.n_tbox, 2), dim3(kPEThreads), 0, s, a);
    else
      hipLaunchKernelGGL((p2l_laplace_kernel<P, R>), dim3((unsigned)a.n_tbox), dim3(kPEThreads), 0, s, a);
    FMM_HIP_CHECK(hipGetLastError());
    return FMM_OK;
  }
}

template <typename R, bool CPLX>
int launch_pe(const PointExpArgs& a, bool m2p, hipStream_t s) {
  if (a.n_tbox == 0) return FMM_OK;
  if constexpr (!CPLX) {
    if (a.kernel == FMM_LAPLACE && a.p <= kLapMaxP) return launch_laplace_p<R, 0>(a, m2p, s);
  }
  if (m2p) {
    // parallel workgroups per target box: enough that a box of 64 points has one per point
    hipLaunchKernelGGL((m2p_kernel<R, CPLX>), dim3((unsigned)a.n_tbox, 64), dim3(kPEThreads), 0, s, a);
  } else {
    hipLaunchKernelGGL((p2l_kernel<R, CPLX>), dim3((unsigned)a.n_tbox), dim3(kPEThreads), 0, s, a);
  }
  FMM_HIP_CHECK(hipGetLastError());
  return FMM_OK;
}

int launch_pe_dtype(const PointExpArgs& a, int dtype, bool m2p, hipStream_t s) {
  FMM_REQUIRE(a.nc <= kPEThreads * kPEMaxPerLane, FMM_EUNSUPPORTED, "P2L: more kept coefficients than instantiated");
  FMM_REQUIRE((a.p + 1) * (a.p + 1) * a.c <= kPEMaxGrid, FMM_EUNSUPPORTED, "P2L / M2P: order too high");
  switch (dtype) {
    case FMM_F64: return launch_pe<double, false>(a, m2p, s);
    case FMM_F32: return launch_pe<float, false>(a, m2p, s);
    case FMM_C128: return launch_pe<double, true>(a, m2p, s);
    case FMM_C64: return launch_pe<float, true>(a, m2p, s);
    default: return fail(FMM_EINVAL, "dtype");
  }
}

}  // namespace

int launch_m2p(const PointExpArgs& a, int dtype, hipStream_t s) { return launch_pe_dtype(a, dtype, true, s); }
int launch_p2l(const PointExpArgs& a, int dtype, hipStream_t s) { return launch_pe_dtype(a, dtype, false, s); }

}  // namespace fmm
