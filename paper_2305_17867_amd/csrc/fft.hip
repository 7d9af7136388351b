// M2L as a 3-D convolution evaluated with discrete Fourier transforms (eq. convolution_m2l).
//
// The compressed M2L  theta~_i = sum_{q in J} T~[i + q] beta~_q  is a correlation of the
// derivative grid g[m] = T~[m], m in [0, 2M] (M = (p, p, c - 1), grid (2c-1) x (2p+1) x (2p+1),
// index (m_z, m_x, m_y)), with the kept coefficients.  Embedding b[(-q) mod L] = beta~_q in the
// same grid turns it into a circular convolution: theta~ = IDFT(DFT(g) . DFT(b)) restricted to J.
// For real dtypes both inputs are real, so every spectrum is kept as its Hermitian half along y
// ((2p+1+1)/2 of the 2p+1 y frequencies); for complex dtypes (Helmholtz) the tables and the
// coefficients are complex and the full spectrum is kept.  To keep the transforms accurate the inputs are
// rescaled as in Sec. 4.1.1 with an extra parameter tau: g[m] tau^-|m|, beta~_q tau^|q|, and the
// outputs multiplied by tau^|i|.
//
// Kernels: forward transform of every table and of every source box's multipole (one
// workgroup each, dense per-axis DFTs in LDS), and per target box the accumulation of the
// spectral products over its interaction list followed by the inverse transform.
#include <cmath>

#include "../../include/fmm.h"
#include "common.hpp"
#include "device_util.hpp"
#include "kernels.hpp"

namespace fmm {

namespace {

constexpr int kFftThreads = 256;

template <typename R>
struct C2 {
  R re, im;
};

// y frequencies kept: the Hermitian half for real grids, all of them for complex grids
__host__ __device__ inline int half_y(int S, bool cplx) { return cplx ? S : (S + 1) / 2; }

// Forward 3-D DFT of the grid held in LDS ([Sz][S][S], real or complex) into the spectrum
// out[kz][kx][ky] (ky < Hy), using ping-pong complex LDS buffers.
template <typename R, bool CPLX>
__device__ void dft_forward(const void* gridv, C2<R>* b1, C2<R>* b2, const C2<R>* wS, const C2<R>* wZ,
                            int S, int Sz, int Hy, C2<R>* out_global) {
  const int nh = Sz * S * Hy;
  // y (real -> half complex, or complex -> complex)
  for (int f = threadIdx.x; f < nh; f += blockDim.x) {
    const int z = f / (S * Hy), r = f % (S * Hy), x = r / Hy, ky = r % Hy;
    R sr = 0, si = 0;
    int idx = 0;
    if constexpr (CPLX) {
      const C2<R>* line = reinterpret_cast<const C2<R>*>(gridv) + (z * S + x) * S;
      for (int y = 0; y < S; ++y) {
        const C2<R> v = line[y];
        const C2<R> w = wS[idx];
        sr += v.re * w.re - v.im * w.im;
        si += v.re * w.im + v.im * w.re;
        idx += ky;
        if (idx >= S) idx -= S;
      }
    } else {
      const R* line = reinterpret_cast<const R*>(gridv) + (z * S + x) * S;
      for (int y = 0; y < S; ++y) {
        const R v = line[y];
        sr += v * wS[idx].re;
        si += v * wS[idx].im;
        idx += ky;
        if (idx >= S) idx -= S;
      }
    }
    b1[f] = {sr, si};
  }
  __syncthreads();
  // x
  for (int f = threadIdx.x; f < nh; f += blockDim.x) {
    const int z = f / (S * Hy), r = f % (S * Hy), kx = r / Hy, ky = r % Hy;
    R sr = 0, si = 0;
    int idx = 0;
    for (int x = 0; x < S; ++x) {
      const C2<R> v = b1[(z * S + x) * Hy + ky];
      const C2<R> w = wS[idx];
      sr += v.re * w.re - v.im * w.im;
      si += v.re * w.im + v.im * w.re;
      idx += kx;
      if (idx >= S) idx -= S;
    }
    b2[f] = {sr, si};
  }
  __syncthreads();
  // z
  for (int f = threadIdx.x; f < nh; f += blockDim.x) {
    const int kz = f / (S * Hy), r = f % (S * Hy);
    R sr = 0, si = 0;
    int idx = 0;
    for (int z = 0; z < Sz; ++z) {
      const C2<R> v = b2[z * S * Hy + r];
      const C2<R> w = wZ[idx];
      sr += v.re * w.re - v.im * w.im;
      si += v.re * w.im + v.im * w.re;
      idx += kz;
      if (idx >= Sz) idx -= Sz;
    }
    out_global[f] = {sr, si};
  }
}

template <typename R>
__device__ void load_twiddles(C2<R>* wS, C2<R>* wZ, int S, int Sz) {
  for (int k = threadIdx.x; k < S; k += blockDim.x) {
    const double a = -2.0 * M_PI * k / S;
    wS[k] = {(R)cos(a), (R)sin(a)};
  }
  for (int k = threadIdx.x; k < Sz; k += blockDim.x) {
    const double a = -2.0 * M_PI * k / Sz;
    wZ[k] = {(R)cos(a), (R)sin(a)};
  }
}

// LDS layout of the transform kernels: [grid: ng values, real or complex][b1, b2: nh complex each]
// [twiddles S + Sz complex]
template <typename R, bool CPLX>
__device__ inline C2<R>* after_grid(char* smem, int ng) {
  return CPLX ? reinterpret_cast<C2<R>*>(smem) + ng : reinterpret_cast<C2<R>*>(reinterpret_cast<R*>(smem) + ((ng + 1) & ~1));
}

// tables: grid = T~[m] tau^-|m| (double input, layout of the derivative tables; complex tables
// interleaved)
template <typename R, bool CPLX>
__global__ __launch_bounds__(kFftThreads) void fft_tables_kernel(FftArgs a) {
  extern __shared__ __align__(16) char smem[];
  constexpr int W = CPLX ? 2 : 1;
  const int S = a.S, Sz = a.Sz, Hy = half_y(a.S, CPLX), ng = Sz * S * S, nh = Sz * S * Hy;
  R* grid = reinterpret_cast<R*>(smem);
  C2<R>* b1 = after_grid<R, CPLX>(smem, ng);
  C2<R>* b2 = b1 + nh;
  C2<R>* wS = b2 + nh;
  C2<R>* wZ = wS + S;
  load_twiddles(wS, wZ, S, Sz);
  const double* src = a.tab64 + (int64_t)blockIdx.x * ng * W;
  for (int k = threadIdx.x; k < ng; k += blockDim.x) {
    const int z = k / (S * S), r = k % (S * S), x = r / S, y = r % S;
    const double sc = pow(a.tau, -(double)(x + y + z));
#pragma unroll
    for (int u = 0; u < W; ++u) grid[k * W + u] = (R)(src[k * W + u] * sc);
  }
  __syncthreads();
  dft_forward<R, CPLX>(grid, b1, b2, wS, wZ, S, Sz, Hy,
                       reinterpret_cast<C2<R>*>(a.spec_tab) + (int64_t)blockIdx.x * nh);
}

// sources: grid = beta~ embedded at (-q) mod L, times tau^|q|
template <typename R, bool CPLX>
__global__ __launch_bounds__(kFftThreads) void fft_sources_kernel(FftArgs a) {
  extern __shared__ __align__(16) char smem[];
  constexpr int W = CPLX ? 2 : 1;
  const int S = a.S, Sz = a.Sz, Hy = half_y(a.S, CPLX), ng = Sz * S * S, nh = Sz * S * Hy;
  R* grid = reinterpret_cast<R*>(smem);
  C2<R>* b1 = after_grid<R, CPLX>(smem, ng);
  C2<R>* b2 = b1 + nh;
  C2<R>* wS = b2 + nh;
  C2<R>* wZ = wS + S;
  load_twiddles(wS, wZ, S, Sz);
  const int box = a.src_list[blockIdx.x];
  for (int k = threadIdx.x; k < ng * W; k += blockDim.x) grid[k] = R(0);
  __syncthreads();
  const R* beta = reinterpret_cast<const R*>(a.mpole) + (int64_t)box * a.nc * W;
  for (int k = threadIdx.x; k < a.nc; k += blockDim.x) {
    const int pk = a.jxyz[k];
    const int qx = pk & 255, qy = (pk >> 8) & 255, qz = pk >> 16;
    const int z = (Sz - qz) % Sz, x = (S - qx) % S, y = (S - qy) % S;
    const R t = (R)a.taupow[qx + qy + qz];
#pragma unroll
    for (int u = 0; u < W; ++u) grid[((z * S + x) * S + y) * W + u] = beta[k * W + u] * t;
  }
  __syncthreads();
  dft_forward<R, CPLX>(grid, b1, b2, wS, wZ, S, Sz, Hy,
                       reinterpret_cast<C2<R>*>(a.spec_src) + (int64_t)box * nh);
}

// per target: sum of spectral products over the interaction list, inverse transform, extract J
template <typename R, bool CPLX>
__global__ __launch_bounds__(kFftThreads) void fft_targets_kernel(FftArgs a) {
  extern __shared__ __align__(16) char smem[];
  const int S = a.S, Sz = a.Sz, Hy = half_y(a.S, CPLX), nh = Sz * S * Hy;
  C2<R>* b1 = reinterpret_cast<C2<R>*>(smem);
  C2<R>* b2 = b1 + nh;
  C2<R>* wS = b2 + nh;
  C2<R>* wZ = wS + S;
  load_twiddles(wS, wZ, S, Sz);
  const int tgt = a.tgt_list[blockIdx.x];
  const int e0 = a.tgt_ptr[blockIdx.x], e1 = a.tgt_ptr[blockIdx.x + 1];
  const C2<R>* st = reinterpret_cast<const C2<R>*>(a.spec_tab);
  const C2<R>* ss = reinterpret_cast<const C2<R>*>(a.spec_src);
  // accumulate in registers: thread owns frequencies tid + k blockDim
  C2<R> acc[kFftMaxPerThread];
#pragma unroll
  for (int k = 0; k < kFftMaxPerThread; ++k) acc[k] = {R(0), R(0)};
  for (int e = e0; e < e1; ++e) {
    const C2<R>* g = st + (int64_t)a.ent_tab[e] * nh;
    const C2<R>* b = ss + (int64_t)a.ent_src[e] * nh;
#pragma unroll
    for (int k = 0; k < kFftMaxPerThread; ++k) {
      const int f = threadIdx.x + k * blockDim.x;
      if (f < nh) {
        const C2<R> x = g[f], y = b[f];
        acc[k].re += x.re * y.re - x.im * y.im;
        acc[k].im += x.re * y.im + x.im * y.re;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kFftMaxPerThread; ++k) {
    const int f = threadIdx.x + k * blockDim.x;
    if (f < nh) b1[f] = acc[k];
  }
  __syncthreads();
  // inverse z (conjugate twiddles)
  for (int f = threadIdx.x; f < nh; f += blockDim.x) {
    const int z = f / (S * Hy), r = f % (S * Hy);
    R sr = 0, si = 0;
    int idx = 0;
    for (int kz = 0; kz < Sz; ++kz) {
      const C2<R> v = b1[kz * S * Hy + r];
      const C2<R> w = wZ[idx];
      sr += v.re * w.re + v.im * w.im;
      si += v.im * w.re - v.re * w.im;
      idx += z;
      if (idx >= Sz) idx -= Sz;
    }
    b2[f] = {sr, si};
  }
  __syncthreads();
  // inverse x
  for (int f = threadIdx.x; f < nh; f += blockDim.x) {
    const int z = f / (S * Hy), r = f % (S * Hy), x = r / Hy, ky = r % Hy;
    R sr = 0, si = 0;
    int idx = 0;
    for (int kx = 0; kx < S; ++kx) {
      const C2<R> v = b2[(z * S + kx) * Hy + ky];
      const C2<R> w = wS[idx];
      sr += v.re * w.re + v.im * w.im;
      si += v.im * w.re - v.re * w.im;
      idx += x;
      if (idx >= S) idx -= S;
    }
    b1[f] = {sr, si};
  }
  __syncthreads();
  // inverse y at the kept indices only (half complex -> real, or complex -> complex), scaled
  // and accumulated
  const double norm = 1.0 / ((double)Sz * S * S);
  constexpr int W = CPLX ? 2 : 1;
  R* out = reinterpret_cast<R*>(a.local) + (int64_t)tgt * a.nc * W;
  for (int k = threadIdx.x; k < a.nc; k += blockDim.x) {
    const int pk = a.jxyz[k];
    const int ix = pk & 255, iy = (pk >> 8) & 255, iz = pk >> 16;
    const C2<R>* line = b1 + (iz * S + ix) * Hy;
    const double sc = norm * a.taupow[ix + iy + iz];
    if constexpr (CPLX) {
      R sr = 0, si = 0;
      int idx = 0;
      for (int ky = 0; ky < S; ++ky) {
        const C2<R> v = line[ky], w = wS[idx];
        sr += v.re * w.re + v.im * w.im;
        si += v.im * w.re - v.re * w.im;
        idx += iy;
        if (idx >= S) idx -= S;
      }
      out[2 * k] = (R)((double)out[2 * k] + (double)sr * sc);
      out[2 * k + 1] = (R)((double)out[2 * k + 1] + (double)si * sc);
    } else {
      R s = line[0].re;
      int idx = iy;
      for (int ky = 1; ky < Hy; ++ky) {
        const C2<R> v = line[ky], w = wS[idx];
        s += R(2) * (v.re * w.re + v.im * w.im);
        idx += iy;
        if (idx >= S) idx -= S;
      }
      out[k] = (R)((double)out[k] + (double)s * sc);
    }
  }
}

size_t fft_lds(int S, int Sz, size_t rb, bool cplx, bool with_grid) {
  const int ng = Sz * S * S, nh = Sz * S * half_y(S, cplx);
  const size_t grid = cplx ? (size_t)ng * 2 * rb : (size_t)((ng + 1) & ~1) * rb;
  return (with_grid ? grid : 0) + (2 * (size_t)nh + S + Sz) * 2 * rb;
}

template <typename R, bool CPLX>
int launch_fft_t(const FftArgs& a, int which, hipStream_t s) {
  const bool grid = which != 2;
  const size_t lds = fft_lds(a.S, a.Sz, sizeof(R), CPLX, grid);
  auto set_lds = [&](const void* k) -> int {
    if (lds > 65536) {
      hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(FMM_EUNSUPPORTED, "FFT M2L needs too much LDS for this order");
      }
    }
    return FMM_OK;
  };
  if (which == 0) {
    if (a.n_tab == 0) return FMM_OK;
    if (int st = set_lds(reinterpret_cast<const void*>(fft_tables_kernel<R, CPLX>))) return st;
    hipLaunchKernelGGL((fft_tables_kernel<R, CPLX>), dim3((unsigned)a.n_tab), dim3(kFftThreads), lds, s, a);
  } else if (which == 1) {
    if (a.n_src == 0) return FMM_OK;
    if (int st = set_lds(reinterpret_cast<const void*>(fft_sources_kernel<R, CPLX>))) return st;
    hipLaunchKernelGGL((fft_sources_kernel<R, CPLX>), dim3((unsigned)a.n_src), dim3(kFftThreads), lds, s, a);
  } else {
    if (a.n_tgt == 0) return FMM_OK;
    if (int st = set_lds(reinterpret_cast<const void*>(fft_targets_kernel<R, CPLX>))) return st;
    hipLaunchKernelGGL((fft_targets_kernel<R, CPLX>), dim3((unsigned)a.n_tgt), dim3(kFftThreads), lds, s, a);
  }
  FMM_HIP_CHECK(hipGetLastError());
  return FMM_OK;
}

}  // namespace

size_t fft_lds_bytes(int S, int Sz, size_t real_bytes, bool cplx) { return fft_lds(S, Sz, real_bytes, cplx, true); }

int fft_half_y(int S, bool cplx) { return half_y(S, cplx); }

int launch_fft(const FftArgs& a, int dtype, int which, hipStream_t s) {
  switch (dtype) {
    case FMM_F64: return launch_fft_t<double, false>(a, which, s);
    case FMM_F32: return launch_fft_t<float, false>(a, which, s);
    case FMM_C128: return launch_fft_t<double, true>(a, which, s);
    case FMM_C64: return launch_fft_t<float, true>(a, which, s);
    default: return fail(FMM_EINVAL, "dtype");
  }
}

}  // namespace fmm
