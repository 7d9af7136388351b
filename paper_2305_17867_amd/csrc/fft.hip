// M2L as a 3-D convolution evaluated with discrete Fourier transforms (eq. convolution_m2l).
//
// The compressed M2L  theta~_i = sum_{q in J} T~[i + q] beta~_q  is a correlation of the
// derivative grid g[m] = T~[m], m in [0, 2M] (M = (p, p, c - 1), grid (2c-1) x (2p+1) x (2p+1),
// index (m_z, m_x, m_y)), with the kept coefficients.  Embedding b[(-q) mod L] = beta~_q in the
// same grid turns it into a circular convolution: theta~ = IDFT(DFT(g) . DFT(b)) restricted to J.
// Both inputs are real (real dtypes), so every spectrum is kept as its Hermitian half along y
// ((2p+1+1)/2 of the 2p+1 y frequencies).  To keep the transforms accurate the inputs are
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

// Forward real 3-D DFT of the grid held in LDS (real, [Sz][S][S]) into the half spectrum
// out[kz][kx][ky] (ky < Hy), using ping-pong complex LDS buffers.
template <typename R>
__device__ void dft_forward(const R* grid, C2<R>* b1, C2<R>* b2, const C2<R>* wS, const C2<R>* wZ,
                            int S, int Sz, int Hy, C2<R>* out_global) {
  const int nh = Sz * S * Hy;
  // y (real -> half complex)
  for (int f = threadIdx.x; f < nh; f += blockDim.x) {
    const int z = f / (S * Hy), r = f % (S * Hy), x = r / Hy, ky = r % Hy;
    const R* line = grid + (z * S + x) * S;
    R sr = 0, si = 0;
    int idx = 0;
    for (int y = 0; y < S; ++y) {
      const R v = line[y];
      sr += v * wS[idx].re;
      si += v * wS[idx].im;
      idx += ky;
      if (idx >= S) idx -= S;
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

// tables: grid = T~[m] tau^-|m| (double input, layout of the derivative tables)
template <typename R>
__global__ __launch_bounds__(kFftThreads) void fft_tables_kernel(FftArgs a) {
  extern __shared__ __align__(16) char smem[];
  const int S = a.S, Sz = a.Sz, Hy = (a.S + 1) / 2, ng = Sz * S * S, nh = Sz * S * Hy;
  R* grid = reinterpret_cast<R*>(smem);
  C2<R>* b1 = reinterpret_cast<C2<R>*>(grid + ((ng + 1) & ~1));
  C2<R>* b2 = b1 + nh;
  C2<R>* wS = b2 + nh;
  C2<R>* wZ = wS + S;
  load_twiddles(wS, wZ, S, Sz);
  const double* src = a.tab64 + (int64_t)blockIdx.x * ng;
  for (int k = threadIdx.x; k < ng; k += blockDim.x) {
    const int z = k / (S * S), r = k % (S * S), x = r / S, y = r % S;
    grid[k] = (R)(src[k] * pow(a.tau, -(double)(x + y + z)));
  }
  __syncthreads();
  dft_forward<R>(grid, b1, b2, wS, wZ, S, Sz, Hy,
                 reinterpret_cast<C2<R>*>(a.spec_tab) + (int64_t)blockIdx.x * nh);
}

// sources: grid = beta~ embedded at (-q) mod L, times tau^|q|
template <typename R>
__global__ __launch_bounds__(kFftThreads) void fft_sources_kernel(FftArgs a) {
  extern __shared__ __align__(16) char smem[];
  const int S = a.S, Sz = a.Sz, Hy = (a.S + 1) / 2, ng = Sz * S * S, nh = Sz * S * Hy;
  R* grid = reinterpret_cast<R*>(smem);
  C2<R>* b1 = reinterpret_cast<C2<R>*>(grid + ((ng + 1) & ~1));
  C2<R>* b2 = b1 + nh;
  C2<R>* wS = b2 + nh;
  C2<R>* wZ = wS + S;
  load_twiddles(wS, wZ, S, Sz);
  const int box = a.src_list[blockIdx.x];
  for (int k = threadIdx.x; k < ng; k += blockDim.x) grid[k] = R(0);
  __syncthreads();
  const R* beta = reinterpret_cast<const R*>(a.mpole) + (int64_t)box * a.nc;
  for (int k = threadIdx.x; k < a.nc; k += blockDim.x) {
    const int pk = a.jxyz[k];
    const int qx = pk & 255, qy = (pk >> 8) & 255, qz = pk >> 16;
    const int z = (Sz - qz) % Sz, x = (S - qx) % S, y = (S - qy) % S;
    grid[(z * S + x) * S + y] = beta[k] * (R)a.taupow[qx + qy + qz];
  }
  __syncthreads();
  dft_forward<R>(grid, b1, b2, wS, wZ, S, Sz, Hy,
                 reinterpret_cast<C2<R>*>(a.spec_src) + (int64_t)box * nh);
}

// per target: sum of spectral products over the interaction list, inverse transform, extract J
template <typename R>
__global__ __launch_bounds__(kFftThreads) void fft_targets_kernel(FftArgs a) {
  extern __shared__ __align__(16) char smem[];
  const int S = a.S, Sz = a.Sz, Hy = (a.S + 1) / 2, nh = Sz * S * Hy;
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
  // inverse y (half complex -> real) at the kept indices only, scaled and accumulated
  const double norm = 1.0 / ((double)Sz * S * S);
  R* out = reinterpret_cast<R*>(a.local) + (int64_t)tgt * a.nc;
  for (int k = threadIdx.x; k < a.nc; k += blockDim.x) {
    const int pk = a.jxyz[k];
    const int ix = pk & 255, iy = (pk >> 8) & 255, iz = pk >> 16;
    const C2<R>* line = b1 + (iz * S + ix) * Hy;
    R s = line[0].re;
    int idx = iy;
    for (int ky = 1; ky < Hy; ++ky) {
      const C2<R> v = line[ky], w = wS[idx];
      s += R(2) * (v.re * w.re + v.im * w.im);
      idx += iy;
      if (idx >= S) idx -= S;
    }
    out[k] = (R)((double)out[k] + (double)s * norm * a.taupow[ix + iy + iz]);
  }
}

size_t fft_lds(int S, int Sz, size_t rb, bool with_grid) {
  const int Hy = (S + 1) / 2, ng = Sz * S * S, nh = Sz * S * Hy;
  return (with_grid ? (size_t)((ng + 1) & ~1) * rb : 0) + (2 * (size_t)nh + S + Sz) * 2 * rb;
}

template <typename R>
int launch_fft_t(const FftArgs& a, int which, hipStream_t s) {
  const bool grid = which != 2;
  const size_t lds = fft_lds(a.S, a.Sz, sizeof(R), grid);
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
    if (int st = set_lds(reinterpret_cast<const void*>(fft_tables_kernel<R>))) return st;
    hipLaunchKernelGGL(fft_tables_kernel<R>, dim3((unsigned)a.n_tab), dim3(kFftThreads), lds, s, a);
  } else if (which == 1) {
    if (a.n_src == 0) return FMM_OK;
    if (int st = set_lds(reinterpret_cast<const void*>(fft_sources_kernel<R>))) return st;
    hipLaunchKernelGGL(fft_sources_kernel<R>, dim3((unsigned)a.n_src), dim3(kFftThreads), lds, s, a);
  } else {
    if (a.n_tgt == 0) return FMM_OK;
    if (int st = set_lds(reinterpret_cast<const void*>(fft_targets_kernel<R>))) return st;
    hipLaunchKernelGGL(fft_targets_kernel<R>, dim3((unsigned)a.n_tgt), dim3(kFftThreads), lds, s, a);
  }
  FMM_HIP_CHECK(hipGetLastError());
  return FMM_OK;
}

}  // namespace

size_t fft_lds_bytes(int S, int Sz, size_t real_bytes) { return fft_lds(S, Sz, real_bytes, true); }

int launch_fft(const FftArgs& a, int dtype, int which, hipStream_t s) {
  if (dtype == FMM_F64) return launch_fft_t<double>(a, which, s);
  if (dtype == FMM_F32) return launch_fft_t<float>(a, which, s);
  return fail(FMM_EUNSUPPORTED, "the FFT M2L path is implemented for real dtypes");
}

}  // namespace fmm
