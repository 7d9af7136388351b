// Two-dimensional expansions (kernels log r and r^2 log r, Sec. 4.4): index helpers shared by the
// 2-D sources and the launcher of the unrolled M2L.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fmm2d {

// |J| for J = {(a, b) : a + b <= p, b < c}
__host__ __device__ constexpr int n_kept(int p, int c) {
  int n = 0;
  for (int b = 0; b < c && b <= p; ++b) n += p - b + 1;
  return n;
}

__host__ __device__ constexpr int n_full(int p) { return (p + 1) * (p + 2) / 2; }

// storage position of (a, b) in J: layers b = 0, 1, ... with a fastest
__host__ __device__ constexpr int kept_pos(int p, int a, int b) { return b * (p + 1) - b * (b - 1) / 2 + a; }

struct M2LArgs2D {
  int64_t n_tbox;
  const int32_t* tbox;
  const int32_t* pair_ptr;
  int64_t n_pair;
  const int32_t* pair_src;
  const int32_t* pair_tab;
  int64_t n_tab;
  const double* tables;  // [n_tab][2c - 1][2p + 1]
  int64_t n_box;
  const double* mpole;  // [n_box][Nc]
  double* local;        // [n_box][Nc]
};

// Enqueue the M2L; false when (p, c) has no instantiation.
bool launch_m2l2d(const M2LArgs2D& a, int p, int c, hipStream_t s);

}  // namespace fmm2d
