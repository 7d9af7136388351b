// FP64 derivative tables for the compressed M2L (Sec. 4.1: the derivatives G^(i+q) at the
// translation vector, |i + q| <= 2p, (i + q)_z <= 2(c - 1), precomputed per offset): one
// workgroup per table runs the Taylor-coefficient recurrences of taylor_grid.hpp order by order.
#include "../../include/fmm.h"
#include "common.hpp"
#include "device_util.hpp"
#include "kernels.hpp"
#include "taylor_grid.hpp"

namespace fmm {

namespace {

constexpr int kTabThreads = 256;

template <bool CPLX>
__global__ __launch_bounds__(kTabThreads) void tables_kernel(TableArgs a) {
  using T = typename Val<double, CPLX>::T;
  const int64_t tb = blockIdx.x;
  if (tb >= a.n) return;
  const int S = a.S, Sz = a.Sz, P2 = a.p2;
  const double x0[3] = {a.offset[tb * 3 + 0], a.offset[tb * 3 + 1], a.offset[tb * 3 + 2]};
  __shared__ TaylorRing<CPLX> ring;
  T* out = reinterpret_cast<T*>(a.out) + tb * (int64_t)(Sz * S * S);
  // entries with |m| > 2p: zero
  for (int k = threadIdx.x; k < Sz * S * S; k += blockDim.x) {
    int mz = k / (S * S), rem = k % (S * S), mx = rem / S, my = rem % S;
    if (mx + my + mz > P2) out[k] = T(0.0);
  }
  taylor_grid<CPLX>(a.kernel, a.param, x0, a.h[tb], P2, S, Sz, out, ring);
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
