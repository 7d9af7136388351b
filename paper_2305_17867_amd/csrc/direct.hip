// Direct sum eq. (1): phi(x) = sum_y G(x - y) w(y), terms with x == y skipped.
// One thread per target; sources are staged through LDS in tiles of the block size.
#include <cmath>

#include "../../include/fmm.h"
#include "common.hpp"
#include "device_util.hpp"
#include "kernels.hpp"

namespace fmm {

namespace {

constexpr int kThreads = 256;

template <typename R>
__device__ inline R r_sqrt(R v) { return sqrt(v); }
__device__ inline float r_sqrt(float v) { return sqrtf(v); }

template <typename R, bool CPLX>
__global__ __launch_bounds__(kThreads) void direct_kernel(DirectArgs a) {
  using T = typename Val<R, CPLX>::T;
  __shared__ R sx[kThreads], sy[kThreads], sz[kThreads];
  __shared__ T sw[kThreads];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const R* tg = reinterpret_cast<const R*>(a.tgt);
  const R* sr = reinterpret_cast<const R*>(a.src);
  const T* w = reinterpret_cast<const T*>(a.w);
  R x = 0, y = 0, z = 0;
  if (t < a.n_tgt) {
    x = tg[3 * t];
    y = tg[3 * t + 1];
    z = tg[3 * t + 2];
  }
  T acc{};
  const R inv4pi = R(1.0 / (4.0 * M_PI));
  const R prm = (R)a.param;
  for (int64_t base = 0; base < a.n_src; base += kThreads) {
    __syncthreads();
    const int64_t j = base + threadIdx.x;
    if (j < a.n_src) {
      sx[threadIdx.x] = sr[3 * j];
      sy[threadIdx.x] = sr[3 * j + 1];
      sz[threadIdx.x] = sr[3 * j + 2];
      sw[threadIdx.x] = w[j];
    }
    __syncthreads();
    const int cnt = (int)((a.n_src - base) < kThreads ? (a.n_src - base) : kThreads);
    for (int k = 0; k < cnt; ++k) {
      const R dx = x - sx[k], dy = y - sy[k], dz = z - sz[k];
      const R r2 = dx * dx + dy * dy + dz * dz;
      if (r2 == R(0)) continue;
      const R r = r_sqrt(r2);
      if constexpr (CPLX) {
        // Helmholtz exp(i k r) / (4 pi r)
        R sn, cs;
        if constexpr (sizeof(R) == 8) sincos(prm * r, &sn, &cs);
        else sincosf(prm * r, &sn, &cs);
        const R g = inv4pi / r;
        const T G(g * cs, g * sn);
        acc += G * sw[k];
      } else {
        R G;
        if (a.kernel == FMM_LAPLACE) G = inv4pi / r;
        else if (a.kernel == FMM_YUKAWA) G = exp(-prm * r) * inv4pi / r;
        else G = r;
        acc += G * sw[k];
      }
    }
  }
  if (t < a.n_tgt) reinterpret_cast<T*>(a.pot)[t] = acc;
}

}  // namespace

int launch_direct(const DirectArgs& a, int dtype, hipStream_t s) {
  if (a.n_tgt == 0) return FMM_OK;
  dim3 g((unsigned)((a.n_tgt + kThreads - 1) / kThreads)), t(kThreads);
  switch (dtype) {
    case FMM_F64: hipLaunchKernelGGL((direct_kernel<double, false>), g, t, 0, s, a); break;
    case FMM_F32: hipLaunchKernelGGL((direct_kernel<float, false>), g, t, 0, s, a); break;
    case FMM_C128: hipLaunchKernelGGL((direct_kernel<double, true>), g, t, 0, s, a); break;
    case FMM_C64: hipLaunchKernelGGL((direct_kernel<float, true>), g, t, 0, s, a); break;
    default: return fail(FMM_EINVAL, "dtype");
  }
  FMM_HIP_CHECK(hipGetLastError());
  return FMM_OK;
}

}  // namespace fmm
