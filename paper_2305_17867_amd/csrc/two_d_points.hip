// Compressed 2-D P2M and L2P (Secs. 3.1-3.4 for d = 2), one point per lane.
//
// Both take each point's kept moments M^T alpha~(X, Y) directly (kept_moments in two_d.hpp: the
// reduction of (X d_x + Y d_y)^n / n! modulo the PDE's symbol, O(p c) per point):
//
//   P2M: beta~ += sum_y w (M^T alpha~(X, Y)), (X, Y) = (c - y) / h (eq. define_beta_multipole,
//        linear in the points, so the compression is applied per point);
//   L2P: phi(x) += <M theta~, alpha~(X, Y)> = <theta~, M^T alpha~(X, Y)>, (X, Y) = (x - c) / h
//        (eq. compressed-local-form evaluated through the transpose, as eq. multipole_eval_beta
//        does for multipoles), so no decompressed local is formed.
//
// A group of G lanes (a power of two up to 64) owns one box, so a wavefront serves 64 / G boxes
// of a level of small boxes at once; the launcher sizes G from the largest box.  Each lane takes
// every G-th point of the group's chunk; P2M adds the group's sums by lane exchanges.
#include "two_d.hpp"

namespace fmm2d {
namespace {

__device__ __forceinline__ void clamp_range(const int64_t* range, int64_t box, int64_t n, int64_t& lo,
                                            int64_t& hi) {
  lo = range[2 * box];
  hi = range[2 * box + 1];
  lo = lo < 0 ? 0 : (lo > n ? n : lo);
  hi = hi < lo ? lo : (hi > n ? n : hi);
}

// Group (box, blockIdx.y) sums the chunks y, y + gridDim.y, ... of G * per_lane points of its box.
// With one chunk column (gridDim.y == 1) the group holds the whole box and adds its row plainly;
// otherwise the columns add atomically.
template <int P, int C>
__global__ __launch_bounds__(64) void p2m2d_points_kernel(PointArgs2D a) {
  constexpr int NC = n_kept(P, C);
  const int G = 1 << a.lg;
  const int gl = threadIdx.x & (G - 1);
  const int64_t box = (int64_t)blockIdx.x * (64 >> a.lg) + (threadIdx.x >> a.lg);
  int64_t lo = 0, hi = 0;
  double cx = 0.0, cy = 0.0, ih = 0.0;
  if (box < a.n_box) {
    clamp_range(a.range, box, a.n_pt, lo, hi);
    cx = a.center[2 * box];
    cy = a.center[2 * box + 1];
    ih = 1.0 / a.box_h[box];
  }
  const int64_t chunk = (int64_t)G * a.per_lane;
  const int64_t first = lo + (int64_t)blockIdx.y * chunk;
  double acc[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) acc[j] = 0.0;
  for (int64_t c0 = first; c0 < hi; c0 += (int64_t)gridDim.y * chunk) {
    const int64_t c1 = c0 + chunk < hi ? c0 + chunk : hi;
    for (int64_t i = c0 + gl; i < c1; i += G) {
      const double X = (cx - a.xy[2 * i]) * ih, Y = (cy - a.xy[2 * i + 1]) * ih, w = a.w[i];
      double m[NC];
      kept_moments<P, C>(X, Y, m);
#pragma unroll
      for (int j = 0; j < NC; ++j) acc[j] = fma(w, m[j], acc[j]);
    }
  }
  // every lane of the wavefront takes part in the exchanges
  for (int s = 1; s < G; s <<= 1)
#pragma unroll
    for (int j = 0; j < NC; ++j) acc[j] += __shfl_xor(acc[j], s, 64);
  if (box >= a.n_box || first >= hi) return;
  double* out = a.coef + box * NC;
#pragma unroll
  for (int j = 0; j < NC; ++j)
    if ((j & (G - 1)) == gl) {
      if (gridDim.y > 1)
        atomicAdd(out + j, acc[j]);
      else
        out[j] += acc[j];
    }
}

template <int P, int C>
__global__ __launch_bounds__(64) void l2p2d_points_kernel(PointArgs2D a) {
  constexpr int NC = n_kept(P, C);
  const int G = 1 << a.lg;
  const int gl = threadIdx.x & (G - 1);
  const int64_t box = (int64_t)blockIdx.x * (64 >> a.lg) + (threadIdx.x >> a.lg);
  if (box >= a.n_box) return;
  int64_t lo, hi;
  clamp_range(a.range, box, a.n_pt, lo, hi);
  const int64_t chunk = (int64_t)G * a.per_lane;
  const int64_t first = lo + (int64_t)blockIdx.y * chunk;
  if (first >= hi) return;
  const double cx = a.center[2 * box], cy = a.center[2 * box + 1], ih = 1.0 / a.box_h[box];
  double th[NC];
  const double* T = a.coef + box * NC;
#pragma unroll
  for (int j = 0; j < NC; ++j) th[j] = T[j];
  for (int64_t c0 = first; c0 < hi; c0 += (int64_t)gridDim.y * chunk) {
    const int64_t c1 = c0 + chunk < hi ? c0 + chunk : hi;
    for (int64_t i = c0 + gl; i < c1; i += G) {
      const double X = (a.xy[2 * i] - cx) * ih, Y = (a.xy[2 * i + 1] - cy) * ih;
      double m[NC];
      kept_moments<P, C>(X, Y, m);
      double phi = 0.0;
#pragma unroll
      for (int j = 0; j < NC; ++j) phi = fma(th[j], m[j], phi);
      a.pot[i] += phi;
    }
  }
}

template <int C, int P>
bool launch_p(const PointArgs2D& a, bool l2p, int p, dim3 grid, hipStream_t s) {
  if constexpr (P > 16) {
    return false;
  } else {
    if (p != P) return launch_p<C, P + 1>(a, l2p, p, grid, s);
    if (l2p)
      l2p2d_points_kernel<P, C><<<grid, 64, 0, s>>>(a);
    else
      p2m2d_points_kernel<P, C><<<grid, 64, 0, s>>>(a);
    return true;
  }
}

}  // namespace

// Launch shape from the largest box of the call: boxes of up to 8 * 64 points take a group of
// pow2(ceil(max / 8)) lanes, eight points per lane, one chunk column; larger boxes a full
// wavefront per chunk of 1024 points, ceil(max / 1024) chunk columns (at most 65535).
void point_launch_shape(int64_t max_per_box, int& lg, int& per_lane, unsigned& columns) {
  const int64_t m = max_per_box < 1 ? 1 : max_per_box;
  if (m <= 8 * 64) {
    per_lane = 8;
    const int64_t lanes = (m + 7) / 8;
    lg = 0;
    while ((int64_t(1) << lg) < lanes) ++lg;
    columns = 1;
  } else {
    per_lane = 16;
    lg = 6;
    const int64_t c = (m + 1023) / 1024;
    columns = (unsigned)(c > 65535 ? 65535 : c);
  }
}

bool launch_points2d(const PointArgs2D& a, bool l2p, int p, int c, unsigned columns, hipStream_t s) {
  if (a.n_box == 0) return true;
  const int64_t per_wave = 64 >> a.lg;
  const dim3 grid((unsigned)((a.n_box + per_wave - 1) / per_wave), columns);
  if (c == 2) return launch_p<2, 0>(a, l2p, p, grid, s);
  if (c == 4) return launch_p<4, 0>(a, l2p, p, grid, s);
  return false;
}

}  // namespace fmm2d
