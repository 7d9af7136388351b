// Dispatch of P2M launches to the per-order instantiations (p2m_orders_*.hip).
#include "../../include/fmm.h"
#include "common.hpp"
#include "kernels.hpp"

namespace fmm {

int launch_p2m_order_0(const P2MArgs& a, int dtype, hipStream_t s);
int launch_p2m_order_1(const P2MArgs& a, int dtype, hipStream_t s);
int launch_p2m_order_2(const P2MArgs& a, int dtype, hipStream_t s);
int launch_p2m_order_3(const P2MArgs& a, int dtype, hipStream_t s);
int launch_p2m_order_4(const P2MArgs& a, int dtype, hipStream_t s);
int launch_p2m_order_5(const P2MArgs& a, int dtype, hipStream_t s);
int launch_p2m_order_6(const P2MArgs& a, int dtype, hipStream_t s);
int launch_p2m_order_7(const P2MArgs& a, int dtype, hipStream_t s);
int launch_p2m_order_8(const P2MArgs& a, int dtype, hipStream_t s);
int launch_p2m_order_9(const P2MArgs& a, int dtype, hipStream_t s);
int launch_p2m_order_10(const P2MArgs& a, int dtype, hipStream_t s);
int launch_p2m_order_11(const P2MArgs& a, int dtype, hipStream_t s);
int launch_p2m_order_12(const P2MArgs& a, int dtype, hipStream_t s);
int launch_p2m_order_13(const P2MArgs& a, int dtype, hipStream_t s);
int launch_p2m_order_14(const P2MArgs& a, int dtype, hipStream_t s);
int launch_p2m_order_15(const P2MArgs& a, int dtype, hipStream_t s);
int launch_p2m_order_16(const P2MArgs& a, int dtype, hipStream_t s);


namespace {

// out[b][k] = sum over the chunks y (in order) of part[b][y][k]: the multipoles of boxes whose
// points were spread over several workgroups
template <typename R>
__global__ void p2m_chunk_sum_kernel(const double* part, R* out, int64_t n_box, int ny, int width) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_box * width) return;
  const int64_t b = i / width, k = i - b * width;
  const double* p = part + b * ny * (int64_t)width + k;
  double acc = 0.0;
  for (int y = 0; y < ny; ++y) acc += p[(int64_t)y * width];
  out[i] = (R)acc;
}

int launch_orders(const P2MArgs& a, int p, int dtype, hipStream_t s);

}  // namespace

int launch_p2m(const P2MArgs& a, int p, int dtype, hipStream_t s) {
  if (a.n_box == 0) return FMM_OK;
  const int st = launch_orders(a, p, dtype, s);
  if (st || a.ny <= 1) return st;
  const int width = a.nc * (dtype_complex(dtype) ? 2 : 1);
  const int64_t n = a.n_box * width;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (real_size(dtype) == 8)
    hipLaunchKernelGGL(p2m_chunk_sum_kernel<double>, dim3(blocks), dim3(256), 0, s, a.part,
                       reinterpret_cast<double*>(a.out), a.n_box, a.ny, width);
  else
    hipLaunchKernelGGL(p2m_chunk_sum_kernel<float>, dim3(blocks), dim3(256), 0, s, a.part,
                       reinterpret_cast<float*>(a.out), a.n_box, a.ny, width);
  FMM_HIP_CHECK(hipGetLastError());
  return FMM_OK;
}

namespace {

int launch_orders(const P2MArgs& a, int p, int dtype, hipStream_t s) {
  switch (p) {
    case 0: return launch_p2m_order_0(a, dtype, s);
    case 1: return launch_p2m_order_1(a, dtype, s);
    case 2: return launch_p2m_order_2(a, dtype, s);
    case 3: return launch_p2m_order_3(a, dtype, s);
    case 4: return launch_p2m_order_4(a, dtype, s);
    case 5: return launch_p2m_order_5(a, dtype, s);
    case 6: return launch_p2m_order_6(a, dtype, s);
    case 7: return launch_p2m_order_7(a, dtype, s);
    case 8: return launch_p2m_order_8(a, dtype, s);
    case 9: return launch_p2m_order_9(a, dtype, s);
    case 10: return launch_p2m_order_10(a, dtype, s);
    case 11: return launch_p2m_order_11(a, dtype, s);
    case 12: return launch_p2m_order_12(a, dtype, s);
    case 13: return launch_p2m_order_13(a, dtype, s);
    case 14: return launch_p2m_order_14(a, dtype, s);
    case 15: return launch_p2m_order_15(a, dtype, s);
    case 16: return launch_p2m_order_16(a, dtype, s);
  }
  return fail(FMM_EUNSUPPORTED, "order");
}

}  // namespace

}  // namespace fmm
