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

// One degree of the kept moments: v holds the C kept coefficients (powers of d_y 0 .. C-1) of the
// reduced (X d_x + Y d_y)^(n-1) / (n-1)!; afterwards those of degree n.  The product by
// (X d_x + Y d_y) / n raises one power of d_y to C, which the PDE's symbol reduces: d_y^2 ->
// -d_x^2 (C = 2, the Laplace equation); d_y^4 -> -d_x^4 - 2 d_x^2 d_y^2 (C = 4, biharmonic).
template <int C>
__device__ __forceinline__ void moment_step(double* v, double X, double Y, double inv_n) {
  double u[C];
  u[0] = X * v[0];
#pragma unroll
  for (int b = 1; b < C; ++b) u[b] = fma(Y, v[b - 1], X * v[b]);
  const double o = Y * v[C - 1];
  u[0] -= o;
  if constexpr (C == 4) u[2] = fma(-2.0, o, u[2]);
#pragma unroll
  for (int b = 0; b < C; ++b) v[b] = u[b] * inv_n;
}

// Kept moments of one point (X, Y) in storage order: m[kept_pos(P, n - b, b)] = the coefficient
// of d_x^(n-b) d_y^b in (X d_x + Y d_y)^n / n! reduced modulo the PDE's symbol (d_x^2 + d_y^2)^(C/2)
// to powers of d_y below C.  The symbol is monic in d_y, so the remainder is unique and equals the
// compression M^T of the point's full moments X^a Y^b / (a! b!) (Thm. mult_decompression for
// d = 2); each degree costs O(C) (moment_step).  For C = 2 the pairs are Re and Im of
// (X + iY)^n / n!.
template <int P, int C>
__device__ __forceinline__ void kept_moments(double X, double Y, double* m) {
  double v[C];
  v[0] = 1.0;
#pragma unroll
  for (int b = 1; b < C; ++b) v[b] = 0.0;
  m[0] = 1.0;
#pragma unroll
  for (int n = 1; n <= P; ++n) {
    moment_step<C>(v, X, Y, 1.0 / n);  // a constant once the loop is unrolled
#pragma unroll
    for (int b = 0; b < C && b <= n; ++b) m[kept_pos(P, n - b, b)] = v[b];
  }
}

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

struct PointArgs2D {
  int64_t n_box;
  const double* center;   // [n_box][2]
  const double* box_h;    // [n_box]
  const int64_t* range;   // [n_box][2], clamped to [0, n_pt]
  int64_t n_pt;
  const double* xy;       // [n_pt][2]
  const double* w;        // [n_pt] source weights (P2M)
  double* pot;            // [n_pt] potentials (L2P), accumulated
  double* coef;           // [n_box][Nc]: multipoles accumulated (P2M) or locals read (L2P)
  int lg;                 // log2 of the lanes per box
  int per_lane;           // points per lane and chunk
};

// Launch shape for boxes of at most max_per_box points (a sizing hint: every point is taken).
void point_launch_shape(int64_t max_per_box, int& lg, int& per_lane, unsigned& columns);

// Enqueue the P2M (l2p false) or the L2P; false when (p, c) has no instantiation.
bool launch_points2d(const PointArgs2D& a, bool l2p, int p, int c, unsigned columns, hipStream_t s);

struct ShiftArgs2D {
  int64_t n_parent;
  const int32_t* parent;  // [n_parent]
  const int32_t* child;   // [n_parent][4], ids outside [0, n_box) mean no child
  int64_t n_box;
  const double* center;   // [n_box][2]
  const double* box_h;    // [n_box]
  double* coef;           // [n_box][Nc] multipoles (M2M) or locals (L2L)
};

// Enqueue the M2M (l2l false) or the L2L; false when (p, c) has no instantiation.
bool launch_shift2d(const ShiftArgs2D& a, bool l2l, int p, int c, hipStream_t s);

}  // namespace fmm2d
