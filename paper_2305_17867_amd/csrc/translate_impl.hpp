// Compressed multipole-to-multipole and local-to-local translations (Secs. 4.2, 4.3).
//
// M2M (eq. define_psi): psi = M^T T E beta.  The child's kept coefficients are embedded in
// the full set with zeros elsewhere (E), translated by h = c_parent - c_child with the
// binomial formula of eq. mpole_translated_full_coeffs (T), summed over the children and
// compressed once at the parent (M^T, Thm. mult_decompression; linear, so one compression
// serves all eight children).
//
// L2L (eq. l2l-expr, derivative form): the parent's local is decompressed (M), translated
// by h = c_child - c_parent and the kept entries are added to the child's local.
//
// Transposes (for gradients): in the scaled form below, M2M^T is the L2L computation with the
// translation vector reversed (read at the parent, added at the child), and L2L^T is the M2M
// computation with the translation vector reversed, added to the parent instead of
// overwriting it (TransArgs::transpose).
//
// Both translations are separable, one axis at a time (the nested partial sums of the proof
// of the O(p^d) translation theorems): since the compressed coefficients have m_z < c, every
// pass except the one along z touches only the kept prefix of the full order, and the z pass
// has at most c terms per output (M2M) or only outputs with m_z < c (L2L).
//
// Scaled form (level box size h_l): beta~_q = beta_q / h^|q|, theta~_i = theta_i h^|i|.
// With delta = h / h_parent and r = h_child / h_parent the translated scaled coefficients are
//   M2M  sigma~_q = sum_{i <= q} delta^(q - i) / (q - i)!  r^|i| beta~_i,
//   L2L  theta~_i = r^|i| sum_{q >= i} delta^(q - i) / (q - i)!  L~_q,
// and the compression / decompression use the parent's box size.
//
// One workgroup per parent box, one wavefront per child (up to eight at once); the
// coefficients are kept in double in LDS.
#pragma once

#include "../../include/fmm.h"
#include "common.hpp"
#include "device_util.hpp"
#include "kernels.hpp"
#include "l2p_impl.hpp"
#include "p2m_impl.hpp"

namespace fmm {

namespace detail_trans {

// (x, y, z) of every full index of M(P) in the internal order (m_z, m_x, m_y).
template <int P>
struct Xyz {
  unsigned char x[nfull(P)], y[nfull(P)], z[nfull(P)];
  constexpr Xyz() : x(), y(), z() {
    int k = 0;
    for (int mz = 0; mz <= P; ++mz)
      for (int mx = 0; mx <= P - mz; ++mx)
        for (int my = 0; my <= P - mz - mx; ++my) {
          x[k] = (unsigned char)mx;
          y[k] = (unsigned char)my;
          z[k] = (unsigned char)mz;
          ++k;
        }
  }
};

template <int P>
__device__ constexpr Xyz<P> kXyz{};

__device__ inline int clamp_level(const TransArgs& a, int64_t box) {
  int l = a.level[box];
  return l < 0 ? 0 : (l >= a.n_levels ? a.n_levels - 1 : l);
}

// sh[ax][k] = delta_ax^k / k! for k = 0..P, rp[k] = r^k (lanes 0..3 of the wavefront).
template <int P>
__device__ inline void shift_factors(int lane, const double (&delta)[3], double r, double (&sh)[3][P + 1],
                                     double (&rp)[P + 1]) {
  if (lane < 3) {
    double v = 1.0;
    sh[lane][0] = 1.0;
    for (int k = 1; k <= P; ++k) {
      v *= delta[lane] / k;
      sh[lane][k] = v;
    }
  } else if (lane == 3) {
    double v = 1.0;
    rp[0] = 1.0;
    for (int k = 1; k <= P; ++k) {
      v *= r;
      rp[k] = v;
    }
  }
}

// Children translated at once, one wavefront each: as many as the per-child LDS buffers
// (two full coefficient sets in double) allow beside the parent's own set within 60 KB.
__host__ __device__ constexpr int kids_at_once(int p, bool cplx) {
  const int set = nfull(p) * (cplx ? 2 : 1) * 8;
  const int budget = 60 * 1024 - set;
  return 16 * set <= budget ? 8 : 8 * set <= budget ? 4 : 4 * set <= budget ? 2 : 1;
}

template <int P, typename R, bool CPLX>
__global__ __launch_bounds__(64 * kids_at_once(P, CPLX)) void m2m_kernel(TransArgs a) {
  constexpr int NP = nfull(P);
  constexpr int W = CPLX ? 2 : 1;
  constexpr int NK = kids_at_once(P, CPLX);
  constexpr int NT = 64 * NK;
  __shared__ double sig[NP * W];  // translated moments summed over the children (full set)
  __shared__ double buf[NK][2][NP * W];
  __shared__ double sh[NK][3][P + 1], rp[NK][P + 1];
  __shared__ int ok[NK];
  const int pb = a.parent[blockIdx.x];
  if (pb < 0 || pb >= a.n_box) return;  // uniform
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const double hp = a.level_h[clamp_level(a, pb)];
  const int nc = a.nc, c = a.c;
  for (int k = threadIdx.x; k < NP * W; k += NT) sig[k] = 0.0;
  const R* in = reinterpret_cast<const R*>(a.coef);
  for (int g = 0; g < 8; g += NK) {
    // wavefront `wave` translates child g + wave (uniform within the wavefront)
    const int cb = a.child[8 * (int64_t)blockIdx.x + g + wave];
    const bool have = cb >= 0 && cb < a.n_box;
    double* b0 = buf[wave][0];
    double* b1 = buf[wave][1];
    __syncthreads();  // the previous group is done with buf, sh and ok
    if (lane == 0) ok[wave] = have;
    if (have) {
      const double hc = a.level_h[clamp_level(a, cb)];
      const double sg = a.transpose ? -1.0 : 1.0;  // c_parent - c_child, or reversed
      const double delta[3] = {sg * (a.center[3 * pb] - a.center[3 * cb]) / hp,
                               sg * (a.center[3 * pb + 1] - a.center[3 * cb + 1]) / hp,
                               sg * (a.center[3 * pb + 2] - a.center[3 * cb + 2]) / hp};
      shift_factors<P>(lane, delta, hc / hp, sh[wave], rp[wave]);
    }
    __syncthreads();
    if (have) {  // E and the child-to-parent scaling r^|i|: the kept set is the prefix [0, nc)
      for (int k = lane; k < nc; k += 64) {
        const double f = rp[wave][kXyz<P>.x[k] + kXyz<P>.y[k] + kXyz<P>.z[k]];
#pragma unroll
        for (int u = 0; u < W; ++u) b0[k * W + u] = f * (double)in[(int64_t)cb * nc * W + k * W + u];
      }
    }
    __syncthreads();
    if (have) {  // along x: b1(e1, y, z) = sum_{s <= e1} delta_x^(e1 - s) / (e1 - s)! b0(s, y, z), z < c
      for (int k = lane; k < nc; k += 64) {
        const int x = kXyz<P>.x[k], y = kXyz<P>.y[k], z = kXyz<P>.z[k];
        double acc[W] = {};
        for (int s = 0; s <= x; ++s) {
          const int n = full_index(P, s, y, z);
#pragma unroll
          for (int u = 0; u < W; ++u) acc[u] += sh[wave][0][x - s] * b0[n * W + u];
        }
#pragma unroll
        for (int u = 0; u < W; ++u) b1[k * W + u] = acc[u];
      }
    }
    __syncthreads();
    if (have) {  // along y
      for (int k = lane; k < nc; k += 64) {
        const int x = kXyz<P>.x[k], y = kXyz<P>.y[k], z = kXyz<P>.z[k];
        double acc[W] = {};
        for (int s = 0; s <= y; ++s) {
          const int n = full_index(P, x, s, z);
#pragma unroll
          for (int u = 0; u < W; ++u) acc[u] += sh[wave][1][y - s] * b1[n * W + u];
        }
#pragma unroll
        for (int u = 0; u < W; ++u) b0[k * W + u] = acc[u];
      }
    }
    __syncthreads();
    if (have) {  // along z, into every entry of the full set (sources only at z < c)
      for (int k = lane; k < NP; k += 64) {
        const int x = kXyz<P>.x[k], y = kXyz<P>.y[k], z = kXyz<P>.z[k];
        const int smax = z < c - 1 ? z : c - 1;
        double acc[W] = {};
        for (int s = 0; s <= smax; ++s) {
          const int n = full_index(P, x, y, s);
#pragma unroll
          for (int u = 0; u < W; ++u) acc[u] += sh[wave][2][z - s] * b0[n * W + u];
        }
#pragma unroll
        for (int u = 0; u < W; ++u) b1[k * W + u] = acc[u];
      }
    }
    __syncthreads();
    // the children's contributions are added in child order
    for (int k = threadIdx.x; k < NP * W; k += NT) {
      double v = sig[k];
#pragma unroll
      for (int w = 0; w < NK; ++w)
        if (ok[w]) v += buf[w][1][k];
      sig[k] = v;
    }
  }
  __syncthreads();
  detail_p2m::compress_lds<P, CPLX>(sig, a.rec, c, hp);
  R* out = reinterpret_cast<R*>(a.coef) + (int64_t)pb * nc * W;
  if (a.transpose) {
    for (int k = threadIdx.x; k < nc * W; k += NT) out[k] += (R)sig[k];
  } else {
    for (int k = threadIdx.x; k < nc * W; k += NT) out[k] = (R)sig[k];
  }
}

template <int P, typename R, bool CPLX>
__global__ __launch_bounds__(64 * kids_at_once(P, CPLX)) void l2l_kernel(TransArgs a) {
  constexpr int NP = nfull(P);
  constexpr int W = CPLX ? 2 : 1;
  constexpr int NK = kids_at_once(P, CPLX);
  constexpr int NT = 64 * NK;
  __shared__ double L[NP * W];  // the parent's decompressed local (full set)
  __shared__ double buf[NK][2][NP * W];
  __shared__ double sh[NK][3][P + 1], rp[NK][P + 1];
  const int pb = a.parent[blockIdx.x];
  if (pb < 0 || pb >= a.n_box) return;  // uniform
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const double hp = a.level_h[clamp_level(a, pb)];
  const int nc = a.nc, c = a.c;
  R* coef = reinterpret_cast<R*>(a.coef);
  for (int k = threadIdx.x; k < nc * W; k += NT) L[k] = (double)coef[(int64_t)pb * nc * W + k];
  __syncthreads();
  detail_l2p::decompress_lds<P, CPLX>(L, a.rec, c, hp);
  for (int g = 0; g < 8; g += NK) {
    const int cb = a.child[8 * (int64_t)blockIdx.x + g + wave];
    const bool have = cb >= 0 && cb < a.n_box;
    double* b0 = buf[wave][0];
    double* b1 = buf[wave][1];
    __syncthreads();  // the previous group is done with buf and sh
    if (have) {
      const double hc = a.level_h[clamp_level(a, cb)];
      const double sg = a.transpose ? -1.0 : 1.0;  // c_child - c_parent, or reversed
      const double delta[3] = {sg * (a.center[3 * cb] - a.center[3 * pb]) / hp,
                               sg * (a.center[3 * cb + 1] - a.center[3 * pb + 1]) / hp,
                               sg * (a.center[3 * cb + 2] - a.center[3 * pb + 2]) / hp};
      shift_factors<P>(lane, delta, hc / hp, sh[wave], rp[wave]);
    }
    __syncthreads();
    if (have) {  // along z, only the outputs with z < c (the kept prefix):
                 //   b0(x, y, e3) = sum_{s >= e3} delta_z^(s - e3) / (s - e3)! L(x, y, s)
      for (int k = lane; k < nc; k += 64) {
        const int x = kXyz<P>.x[k], y = kXyz<P>.y[k], z = kXyz<P>.z[k];
        double acc[W] = {};
        for (int s = z; s <= P - x - y; ++s) {
          const int n = full_index(P, x, y, s);
#pragma unroll
          for (int u = 0; u < W; ++u) acc[u] += sh[wave][2][s - z] * L[n * W + u];
        }
#pragma unroll
        for (int u = 0; u < W; ++u) b0[k * W + u] = acc[u];
      }
    }
    __syncthreads();
    if (have) {  // along y
      for (int k = lane; k < nc; k += 64) {
        const int x = kXyz<P>.x[k], y = kXyz<P>.y[k], z = kXyz<P>.z[k];
        double acc[W] = {};
        for (int s = y; s <= P - x - z; ++s) {
          const int n = full_index(P, x, s, z);
#pragma unroll
          for (int u = 0; u < W; ++u) acc[u] += sh[wave][1][s - y] * b0[n * W + u];
        }
#pragma unroll
        for (int u = 0; u < W; ++u) b1[k * W + u] = acc[u];
      }
    }
    __syncthreads();
    if (have) {  // along x, then the parent-to-child scaling r^|i|, added to the child's local
      R* out = coef + (int64_t)cb * nc * W;
      for (int k = lane; k < nc; k += 64) {
        const int x = kXyz<P>.x[k], y = kXyz<P>.y[k], z = kXyz<P>.z[k];
        double acc[W] = {};
        for (int s = x; s <= P - y - z; ++s) {
          const int n = full_index(P, s, y, z);
#pragma unroll
          for (int u = 0; u < W; ++u) acc[u] += sh[wave][0][s - x] * b1[n * W + u];
        }
        const double f = rp[wave][x + y + z];
#pragma unroll
        for (int u = 0; u < W; ++u) out[k * W + u] += (R)(f * acc[u]);
      }
    }
  }
}

template <int P>
int launch_trans_p(const TransArgs& a, int dtype, bool l2l, hipStream_t s) {
  const dim3 g((unsigned)a.n_parent);
  switch (dtype) {
    case FMM_F64:
      if (l2l) hipLaunchKernelGGL((l2l_kernel<P, double, false>), g, dim3(64 * kids_at_once(P, false)), 0, s, a);
      else hipLaunchKernelGGL((m2m_kernel<P, double, false>), g, dim3(64 * kids_at_once(P, false)), 0, s, a);
      break;
    case FMM_F32:
      if (l2l) hipLaunchKernelGGL((l2l_kernel<P, float, false>), g, dim3(64 * kids_at_once(P, false)), 0, s, a);
      else hipLaunchKernelGGL((m2m_kernel<P, float, false>), g, dim3(64 * kids_at_once(P, false)), 0, s, a);
      break;
    case FMM_C128:
      if (l2l) hipLaunchKernelGGL((l2l_kernel<P, double, true>), g, dim3(64 * kids_at_once(P, true)), 0, s, a);
      else hipLaunchKernelGGL((m2m_kernel<P, double, true>), g, dim3(64 * kids_at_once(P, true)), 0, s, a);
      break;
    case FMM_C64:
      if (l2l) hipLaunchKernelGGL((l2l_kernel<P, float, true>), g, dim3(64 * kids_at_once(P, true)), 0, s, a);
      else hipLaunchKernelGGL((m2m_kernel<P, float, true>), g, dim3(64 * kids_at_once(P, true)), 0, s, a);
      break;
    default: return fail(FMM_EINVAL, "dtype");
  }
  FMM_HIP_CHECK(hipGetLastError());
  return FMM_OK;
}

}  // namespace detail_trans

#define FMM_INSTANTIATE_TRANS(P) \
  int launch_trans_order_##P(const TransArgs& a, int dtype, bool l2l, hipStream_t s) { \
    return detail_trans::launch_trans_p<P>(a, dtype, l2l, s); \
  }

}  // namespace fmm
