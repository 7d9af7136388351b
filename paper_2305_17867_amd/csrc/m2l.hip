// Batched compressed M2L (Sec. 4.1, eq. m2l_toeplitz) on the matrix cores of gfx950.
//
//   theta~_t[i] += sum over pairs (t, s):  sum_{q in J} T~_o[i, q] beta~_s[q],
//   T~_o[i, q] = G^(i+q)(d_o) h^|i+q|  (scaled form, Sec. 4.1.1), i, q in J.
//
// The host groups pairs by translation offset o and tiles the target boxes in groups of 16
// (same level and child parity, so that they share almost all offsets).  A tile's entry e is
// one offset o together with the source box of each of the 16 targets at that offset.  For an
// entry the work is the dense product
//   Theta[:, 0:16] += T~_o[J, J] * B,   B[:, col] = beta~ of the source of target col,
// a 16-column GEMM on v_mfma 16x16x4: rows of T~ (i) are split into 16-row tiles, one per
// wavefront; the K loop runs over q in steps of 4.  T~_o is never expanded: because
// T~_o[i, q] depends on i + q only, it is read from the compact derivative grid
// tab[(m_z, m_x, m_y)] staged in LDS at address base(i) + base(q), with
// base(m) = (m_z S + m_x) S + m_y, S = 2p + 1.
//
// Accumulation: FP64 dtypes accumulate in FP64 matrix-core registers.  FP32 dtypes run each
// entry (offset group) as an FP32 product with FP32 accumulation and add the entry's partial
// into FP64 registers, so the sum over the (up to 189 per level) offset groups is FP64.
// Complex dtypes use four real products per K step.  Every output coefficient is owned by
// one workgroup; a tile split over several workgroups writes FP64 partials to scratch and the
// last workgroup to finish (atomic counter) adds them in part order, so results are
// bit-reproducible.
#include "../../include/fmm.h"
#include "common.hpp"
#include "device_util.hpp"
#include "kernels.hpp"

namespace fmm {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename R>
struct MF;
// Operand layouts (both dtypes): lane l supplies A[l & 15][l >> 4] and B[l >> 4][l & 15].
// Result layouts differ: register v of lane l holds C[row(l >> 4, v)][l & 15] with
//   f64 16x16x4: row = 4 v + (l >> 4);   f32 16x16x4: row = 4 (l >> 4) + v.
template <>
struct MF<double> {
  using V = d4;
  static __device__ inline V mma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int kq, int v) { return 4 * v + kq; }
};
template <>
struct MF<float> {
  using V = f4;
  static __device__ inline V mma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int kq, int v) { return 4 * kq + v; }
};

// RT: row tiles per wavefront (1 or 2).
template <typename R, bool CPLX, int RT>
__global__ __launch_bounds__(1024) void m2l_kernel(M2LArgs a) {
  using V = typename MF<R>::V;
  constexpr int CW = CPLX ? 2 : 1;
  extern __shared__ __align__(16) char smem_raw[];
  R* tre = reinterpret_cast<R*>(smem_raw);
  R* tim = tre + a.ts;  // used when CPLX
  int* sb = reinterpret_cast<int*>(tre + (int64_t)a.ts * CW);
  __shared__ int s_last;

  const M2LItem it = a.items[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, W = blockDim.x >> 6;
  const int nc = a.nc, ncp = a.nc_pad;
  const int rtiles = ncp >> 4;
  const int col = lane & 15;  // B column / C column / A row within the tile
  const int kq = lane >> 4;   // k within the 4-deep MFMA step
  for (int k = tid; k < nc; k += blockDim.x) sb[k] = a.jbase[k];

  double acc[RT][CW][4];
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int u = 0; u < CW; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[r][u][v] = 0.0;

  const R* mp = reinterpret_cast<const R*>(a.mpole);
  const R* tabg = reinterpret_cast<const R*>(a.tab);
  const int k4 = (nc + 3) >> 2;

  for (int e = it.e0; e < it.e1; ++e) {
    __syncthreads();
    const int tabid = a.entry_tab[e];
    const R* src_tab = tabg + (int64_t)tabid * a.ts * CW;
    for (int k = tid; k < a.ts * CW; k += blockDim.x) tre[k] = src_tab[k];
    __syncthreads();
    const int src = a.entry_src[e * 16 + col];
    const R* bsrc = mp + (int64_t)(src < 0 ? 0 : src) * nc * CW;
    int ib[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      const int i = (wave + r * W) * 16 + col;
      ib[r] = (i < nc) ? sb[i] : -1;
    }
    V part[RT][CW];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int u = 0; u < CW; ++u) part[r][u] = V{};
    for (int ks = 0; ks < k4; ++ks) {
      const int q = ks * 4 + kq;
      const bool qok = q < nc;
      const int qb = qok ? sb[q] : 0;
      R br = R(0), bi = R(0);
      if (qok && src >= 0) {
        br = bsrc[q * CW];
        if constexpr (CPLX) bi = bsrc[q * CW + 1];
      }
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        if (wave + r * W >= rtiles) continue;
        const bool ok = qok && ib[r] >= 0;
        const R ar = ok ? tre[ib[r] + qb] : R(0);
        if constexpr (CPLX) {
          const R ai = ok ? tim[ib[r] + qb] : R(0);
          part[r][0] = MF<R>::mma(ar, br, part[r][0]);
          part[r][0] = MF<R>::mma(-ai, bi, part[r][0]);
          part[r][1] = MF<R>::mma(ar, bi, part[r][1]);
          part[r][1] = MF<R>::mma(ai, br, part[r][1]);
        } else {
          part[r][0] = MF<R>::mma(ar, br, part[r][0]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int u = 0; u < CW; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[r][u][v] += (double)part[r][u][v];
  }

  // result rows of this lane: MF<R>::row(kq, v), column col
  const int nparts = a.tile_nparts[it.tile];
  const int* tg = a.tile_tgt + it.tile * 16;
  if (nparts == 1) {
    const int t = tg[col];
    if (t >= 0) {
      R* out = reinterpret_cast<R*>(a.local) + (int64_t)t * nc * CW;
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        const int rt = wave + r * W;
        if (rt >= rtiles) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = rt * 16 + MF<R>::row(kq, v);
          if (i < nc) {
#pragma unroll
            for (int u = 0; u < CW; ++u) out[i * CW + u] = (R)((double)out[i * CW + u] + acc[r][u][v]);
          }
        }
      }
    }
    return;
  }
  // split tile: FP64 partial to scratch, last workgroup reduces in part order
  double* mine = a.scratch + (int64_t)blockIdx.x * 16 * ncp * CW;
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int rt = wave + r * W;
    if (rt >= rtiles) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = rt * 16 + MF<R>::row(kq, v);
#pragma unroll
      for (int u = 0; u < CW; ++u) mine[(col * ncp + i) * CW + u] = acc[r][u][v];
    }
  }
  __threadfence();
  __syncthreads();
  if (tid == 0) {
    const int old = atomicAdd(a.counter + it.tile, 1);
    s_last = (old == nparts - 1);
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  const int item0 = a.tile_item0[it.tile];
  for (int k = tid; k < 16 * nc; k += blockDim.x) {
    const int c = k / nc, i = k % nc;
    const int t = tg[c];
    if (t < 0) continue;
    double sr = 0.0, si = 0.0;
    for (int pt = 0; pt < nparts; ++pt) {
      const double* ps = a.scratch + (int64_t)(item0 + pt) * 16 * ncp * CW;
      sr += ps[(c * ncp + i) * CW];
      if constexpr (CPLX) si += ps[(c * ncp + i) * CW + 1];
    }
    R* out = reinterpret_cast<R*>(a.local) + (int64_t)t * nc * CW;
    out[i * CW] = (R)((double)out[i * CW] + sr);
    if constexpr (CPLX) out[i * CW + 1] = (R)((double)out[i * CW + 1] + si);
  }
  if (tid == 0) atomicExch(a.counter + it.tile, 0);
}

template <typename R, bool CPLX>
int launch_typed(const M2LArgs& a, int rt, int waves, hipStream_t s) {
  const size_t lds = (size_t)a.ts * sizeof(R) * (CPLX ? 2 : 1) + (size_t)a.nc * sizeof(int);
  dim3 g((unsigned)a.n_items), t((unsigned)(waves * 64));
  if (rt == 1)
    hipLaunchKernelGGL((m2l_kernel<R, CPLX, 1>), g, t, lds, s, a);
  else if (rt == 2)
    hipLaunchKernelGGL((m2l_kernel<R, CPLX, 2>), g, t, lds, s, a);
  else
    return fail(FMM_EUNSUPPORTED, "rows per wave must be 1 or 2");
  FMM_HIP_CHECK(hipGetLastError());
  return FMM_OK;
}

__global__ void convert_f32_kernel(const double* src, float* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

// Derivative tables [n][ts] (complex interleaved) -> M2L layout [n][CW][ts] (planar) in R.
template <typename R, bool CPLX>
__global__ void m2l_table_layout_kernel(const double* src, R* dst, int64_t n, int ts) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * ts) return;
  const int64_t tb = i / ts, k = i % ts;
  if constexpr (CPLX) {
    dst[(tb * 2 + 0) * ts + k] = (R)src[2 * i];
    dst[(tb * 2 + 1) * ts + k] = (R)src[2 * i + 1];
  } else {
    dst[i] = (R)src[i];
  }
}

}  // namespace

int launch_m2l(const M2LArgs& a, int dtype, int rows_per_wave, int waves, hipStream_t s) {
  if (a.n_items == 0) return FMM_OK;
  switch (dtype) {
    case FMM_F64: return launch_typed<double, false>(a, rows_per_wave, waves, s);
    case FMM_F32: return launch_typed<float, false>(a, rows_per_wave, waves, s);
    case FMM_C128: return launch_typed<double, true>(a, rows_per_wave, waves, s);
    case FMM_C64: return launch_typed<float, true>(a, rows_per_wave, waves, s);
  }
  return fail(FMM_EINVAL, "dtype");
}

int launch_m2l_table_layout(const double* src, void* dst, int64_t n, int ts, int dtype, hipStream_t s) {
  const int64_t tot = n * ts;
  if (tot == 0) return FMM_OK;
  dim3 g((unsigned)((tot + 255) / 256)), t(256);
  switch (dtype) {
    case FMM_F64: hipLaunchKernelGGL((m2l_table_layout_kernel<double, false>), g, t, 0, s, src, (double*)dst, n, ts); break;
    case FMM_F32: hipLaunchKernelGGL((m2l_table_layout_kernel<float, false>), g, t, 0, s, src, (float*)dst, n, ts); break;
    case FMM_C128: hipLaunchKernelGGL((m2l_table_layout_kernel<double, true>), g, t, 0, s, src, (double*)dst, n, ts); break;
    case FMM_C64: hipLaunchKernelGGL((m2l_table_layout_kernel<float, true>), g, t, 0, s, src, (float*)dst, n, ts); break;
    default: return fail(FMM_EINVAL, "dtype");
  }
  FMM_HIP_CHECK(hipGetLastError());
  return FMM_OK;
}

int launch_convert_f32(const double* src, float* dst, int64_t n, hipStream_t s) {
  if (n == 0) return FMM_OK;
  hipLaunchKernelGGL(convert_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
  FMM_HIP_CHECK(hipGetLastError());
  return FMM_OK;
}

}  // namespace fmm
