// Two-dimensional kernels G = log r and G = r^2 log r (Sec. 4.4) with the compressed Cartesian
// Taylor expansions of Secs. 2-3 for d = 2: derivative tables by the paper's recurrences
// (eqs. deriv_laplace_2d and deriv_biharmonic_2d), the direct sum, the near field and the
// launchers of P2M, L2P (two_d_points.hip), M2L (two_d_m2l.hip), M2M and L2L (two_d_shift.hip).
// FP64.
//
// Index sets: M(p) = {(a, b) : a + b <= p}, J = {(a, b) in M(p) : b < c} (c = 2 for the Laplace
// equation, 4 for the biharmonic one; y is the compressed axis).  Compressing and decompressing
// use the PDE as a rewriting rule for d_y^c (Laplace: d_y^2 -> -d_x^2; biharmonic:
// d_y^4 -> -d_x^4 - 2 d_x^2 d_y^2); both PDEs are homogeneous, so the rule is the same for the
// scaled coefficients of every box size.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "common.hpp"
#include "two_d.hpp"

using namespace fmm;
using namespace fmm2d;

namespace {

constexpr int kTpb = 256;

inline unsigned blocks_for(int64_t n, int tpb) { return (unsigned)((n + tpb - 1) / tpb); }

// ----------------------------------------------------------------------------- tables

// Scaled tables T~_(a, b) = G^(a, b)(h o) h^(a + b) at offsets o given in units of h, for
// a + b <= 2p, b <= 2(c - 1), stored [m_y][m_x] with row length 2p + 1 (entries a + b > 2p
// zero).  The derivatives are taken at the unit-free vector o, where they are of moderate size,
// and the box size enters exactly: log(h r) = log h + log r, and
// (h r)^2 log(h r) = h^2 (r^2 log r + log h r^2).
__global__ void tables2d_kernel(int64_t n, const double* __restrict__ offset, const double* __restrict__ h,
                                double* __restrict__ out, int kernel, int p) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int c = kernel == FMM_BIHARMONIC2D ? 4 : 2;
  const int SX = 2 * p + 1, SY = 2 * c - 1, P2 = 2 * p;
  double* G = out + t * (int64_t)SX * SY;
  auto at = [&](int a, int b) -> double& { return G[b * SX + a]; };
  for (int k = 0; k < SX * SY; ++k) G[k] = 0.0;
  const double x = offset[2 * t], y = offset[2 * t + 1];
  const double r2 = x * x + y * y, ir2 = 1.0 / r2, L = 0.5 * log(r2);
  const double hh = h[t], lh = log(hh);
  // The recurrence for column m (m = number of y derivatives), valid from n = n0(m) on:
  //   r^2 G(n, m) = -A(n) x G(n-1, m) - B(n) G(n-2, m) - 2 m y G(n, m-1) - m (m-1) G(n, m-2)
  // with A = 2(n-1), B = (n-1)(n-2) for log r and A = 2(n-2), B = (n-1)(n-4) for r^2 log r.
  auto step = [&](int nn, int m) {
    double v = 0.0;
    const double A = kernel == FMM_BIHARMONIC2D ? 2.0 * (nn - 2) : 2.0 * (nn - 1);
    const double B = kernel == FMM_BIHARMONIC2D ? (double)(nn - 1) * (nn - 4) : (double)(nn - 1) * (nn - 2);
    if (nn >= 1) v -= A * x * at(nn - 1, m);
    if (nn >= 2) v -= B * at(nn - 2, m);
    if (m >= 1) v -= 2.0 * m * y * at(nn, m - 1);
    if (m >= 2) v -= (double)m * (m - 1) * at(nn, m - 2);
    at(nn, m) = v * ir2;
  };
  if (kernel == FMM_LAPLACE2D) {
    // base values: G, G_x, G_xx, G_y, G_yy
    at(0, 0) = L;
    if (P2 >= 1) {
      at(1, 0) = x * ir2;
      at(0, 1) = y * ir2;
    }
    if (P2 >= 2) {
      at(2, 0) = (y * y - x * x) * ir2 * ir2;
      at(0, 2) = (x * x - y * y) * ir2 * ir2;
    }
    for (int nn = 3; nn <= P2; ++nn) step(nn, 0);
    for (int m = 1; m <= 2 && m <= P2; ++m)
      for (int nn = 1; nn <= P2 - m; ++nn) step(nn, m);
    at(0, 0) += lh;  // every other entry of the scaled table is free of h
  } else {
    const double x2 = x * x, y2 = y * y;
    const double base[5][5] = {
        // [n][m]: closed forms of the derivatives of r^2 log r with n + m <= 4 that the
        // recurrences do not reach (m = 0: n <= 4; m = 1, 2: n <= 2; m = 3, 4: n = 0)
        {r2 * L, 2 * y * L + y, 2 * L + 1 + 2 * y2 * ir2, 6 * y * ir2 - 4 * y2 * y * ir2 * ir2,
         6 * ir2 - 24 * y2 * ir2 * ir2 + 16 * y2 * y2 * ir2 * ir2 * ir2},
        {2 * x * L + x, 2 * x * y * ir2, 2 * x * ir2 - 4 * x * y2 * ir2 * ir2, 0, 0},
        {2 * L + 1 + 2 * x2 * ir2, 2 * y * ir2 - 4 * x2 * y * ir2 * ir2, -2 * ir2 + 16 * x2 * y2 * ir2 * ir2 * ir2, 0, 0},
        {6 * x * ir2 - 4 * x2 * x * ir2 * ir2, 0, 0, 0, 0},
        {6 * ir2 - 24 * x2 * ir2 * ir2 + 16 * x2 * x2 * ir2 * ir2 * ir2, 0, 0, 0, 0}};
    for (int m = 0; m < SY; ++m) {
      const int nb = m == 0 ? 4 : (m <= 2 ? 2 : 0);  // last base value of the column
      for (int nn = 0; nn <= nb && nn + m <= P2; ++nn) {
        if (m <= 4) {
          at(nn, m) = base[nn][m];
        } else {
          // pure y derivatives: the recurrence along y (x and y exchanged)
          double v = -2.0 * (m - 2) * y * at(0, m - 1) - (double)(m - 1) * (m - 4) * at(0, m - 2);
          at(0, m) = v * ir2;
        }
      }
      for (int nn = nb + 1; nn + m <= P2; ++nn) step(nn, m);
    }
    // h^2 (G(o) + log h * d^m |o|^2)
    const double h2 = hh * hh;
    for (int m = 0; m < SY; ++m)
      for (int nn = 0; nn + m <= P2; ++nn) at(nn, m) *= h2;
    at(0, 0) += h2 * lh * r2;
    if (P2 >= 1) {
      at(1, 0) += h2 * lh * 2 * x;
      at(0, 1) += h2 * lh * 2 * y;
    }
    if (P2 >= 2) {
      at(2, 0) += h2 * lh * 2;
      at(0, 2) += h2 * lh * 2;
    }
  }
}

// ----------------------------------------------------------------------------- direct, P2P

// Natural logarithm of a positive finite x, by the series log m = 2 atanh(s) = 2 (s + s^3/3 +
// s^5/5 + ...), s = (m - 1) / (m + 1), after x = m 2^e with m in [sqrt(1/2), sqrt(2)) (frexp):
// |s| <= 0.1716, so ten terms leave a truncation below 2^-55.  ln 2 is split into a high part
// with eleven trailing zero bits (e ln2_hi is exact) and the rest.  Within 2 ulp of log x
// (checked against 50-digit logarithms); about a third of the instructions of the library's
// log, which the near field's interactions are bound by.
__device__ __forceinline__ double log_series(double x) {
  constexpr double kLn2Hi = 0x1.62e42fefa3800p-1, kLn2Lo = 0x1.ef35793c76730p-45;
  int e;
  double m = frexp(x, &e);
  if (m < 0.70710678118654752440) {
    m += m;
    --e;
  }
  const double s = (m - 1.0) / (m + 1.0), s2 = s * s;
  double poly = 1.0 / 19.0;
  poly = fma(poly, s2, 1.0 / 17.0);
  poly = fma(poly, s2, 1.0 / 15.0);
  poly = fma(poly, s2, 1.0 / 13.0);
  poly = fma(poly, s2, 1.0 / 11.0);
  poly = fma(poly, s2, 1.0 / 9.0);
  poly = fma(poly, s2, 1.0 / 7.0);
  poly = fma(poly, s2, 1.0 / 5.0);
  poly = fma(poly, s2, 1.0 / 3.0);
  poly = fma(poly, s2, 1.0);
  const double de = (double)e;
  return fma(de, kLn2Hi, fma(de, kLn2Lo, 2.0 * s * poly));
}

template <int KERNEL>
__device__ __forceinline__ double green2d_t(double r2) {
  const double l = 0.5 * log_series(r2 == 0.0 ? 1.0 : r2);
  const double g = KERNEL == FMM_BIHARMONIC2D ? r2 * l : l;
  return r2 == 0.0 ? 0.0 : g;  // the x == y term is skipped
}

constexpr int kTile = 256;

// Direct sum: sources staged through LDS in tiles of kTile; each target is taken by `split`
// adjacent lanes (doubled until the launch has about 1,024 workgroups, at most a wavefront), each
// on every split-th source of a tile; a butterfly of lane exchanges adds their sums.
template <int KERNEL>
__global__ __launch_bounds__(kTpb) void direct2d_kernel(int64_t n_src, const double* __restrict__ src,
                                                       const double* __restrict__ w, int64_t n_tgt,
                                                       const double* __restrict__ tgt, double* __restrict__ pot,
                                                       int split) {
  __shared__ double sx[kTile], sy[kTile], sw[kTile];
  const int tl = threadIdx.x / split, sp = threadIdx.x % split;
  const int64_t i = (int64_t)blockIdx.x * (kTpb / split) + tl;
  const bool active = i < n_tgt;
  const double x = active ? tgt[2 * i] : 0.0, y = active ? tgt[2 * i + 1] : 0.0;
  double acc = 0.0;
  for (int64_t t0 = 0; t0 < n_src; t0 += kTile) {
    const int64_t j = t0 + threadIdx.x;
    sx[threadIdx.x] = j < n_src ? src[2 * j] : 0.0;
    sy[threadIdx.x] = j < n_src ? src[2 * j + 1] : 0.0;
    sw[threadIdx.x] = j < n_src ? w[j] : 0.0;
    __syncthreads();
    const int nt = (int)(n_src - t0 < kTile ? n_src - t0 : kTile);
    for (int k = sp; k < nt; k += split) {
      const double dx = x - sx[k], dy = y - sy[k];
      acc = fma(green2d_t<KERNEL>(fma(dx, dx, dy * dy)), sw[k], acc);
    }
    __syncthreads();
  }
  for (int m = 1; m < split; m <<= 1) acc += __shfl_xor(acc, m, 64);
  if (active && sp == 0) pot[i] = acc;
}

struct NearArgs2D {
  int64_t n_tbox;
  const int32_t* tbox;
  const int32_t* nbr_ptr;
  int64_t n_nbr;
  const int32_t* nbr;
  int64_t n_box;
  const int64_t* trange;
  const int64_t* srange;
  int64_t n_src;
  const double* src;
  const double* w;
  int64_t n_tgt;
  const double* tgt;
  double* pot;
};

// Near field: one wavefront per (target box of the list, chunk of 64 of its targets).  A chunk of
// n targets gives each target `split` adjacent lanes (the largest power of two up to 16 with
// n * split <= 64), each summing every split-th source of the listed boxes (unrolled by four); a
// butterfly of lane exchanges adds them up.  The list is read 64 entries at a time, one entry per
// lane (its id, then its source range), and each range is broadcast by a lane exchange, so no
// chain of dependent loads stands before every listed box.
template <int KERNEL>
__global__ __launch_bounds__(64) void p2p2d_kernel(NearArgs2D a) {
  const int64_t k = blockIdx.x;
  const int32_t t = a.tbox[k];
  if (t < 0 || t >= a.n_box) return;  // uniform
  int64_t lo = a.trange[2 * (int64_t)t], hi = a.trange[2 * (int64_t)t + 1];
  lo = lo < 0 ? 0 : (lo > a.n_tgt ? a.n_tgt : lo);
  hi = hi < lo ? lo : (hi > a.n_tgt ? a.n_tgt : hi);
  int64_t e0 = a.nbr_ptr[k], e1 = a.nbr_ptr[k + 1];
  e0 = e0 < 0 ? 0 : (e0 > a.n_nbr ? a.n_nbr : e0);
  e1 = e1 < e0 ? e0 : (e1 > a.n_nbr ? a.n_nbr : e1);
  const int lane = threadIdx.x;
  for (int64_t c0 = lo + (int64_t)blockIdx.y * 64; c0 < hi; c0 += (int64_t)gridDim.y * 64) {
    const int n = (int)(hi - c0 < 64 ? hi - c0 : 64);
    int split = 1;
    while (split < 16 && n * split * 2 <= 64) split *= 2;
    const int tl = lane / split, sp = lane % split;
    const bool active = tl < n;
    const int64_t i = c0 + tl;
    double x = 0.0, y = 0.0;
    if (active) {
      x = a.tgt[2 * i];
      y = a.tgt[2 * i + 1];
    }
    double acc = 0.0;
    for (int64_t base = e0; base < e1; base += 64) {
      int64_t s0 = 0, cnt = 0;
      if (base + lane < e1) {
        const int32_t s = a.nbr[base + lane];
        if (s >= 0 && s < a.n_box) {
          int64_t b0 = a.srange[2 * (int64_t)s], b1 = a.srange[2 * (int64_t)s + 1];
          b0 = b0 < 0 ? 0 : (b0 > a.n_src ? a.n_src : b0);
          b1 = b1 < b0 ? b0 : (b1 > a.n_src ? a.n_src : b1);
          s0 = b0;
          cnt = b1 - b0;
        }
      }
      const int jn = (int)(e1 - base < 64 ? e1 - base : 64);
      for (int j = 0; j < jn; ++j) {
        const int64_t j0 = __shfl(s0, j, 64);
        const int64_t j1 = j0 + __shfl(cnt, j, 64);
        if (!active) continue;
        int64_t m = j0 + sp;
        for (; m + 3 * split < j1; m += 4 * split) {
          double g[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int64_t q = m + u * split;
            const double dx = x - a.src[2 * q], dy = y - a.src[2 * q + 1];
            g[u] = green2d_t<KERNEL>(fma(dx, dx, dy * dy));
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) acc = fma(g[u], a.w[m + u * split], acc);
        }
        for (; m < j1; m += split) {
          const double dx = x - a.src[2 * m], dy = y - a.src[2 * m + 1];
          acc = fma(green2d_t<KERNEL>(fma(dx, dx, dy * dy)), a.w[m], acc);
        }
      }
    }
    for (int s = 1; s < split; s <<= 1) acc += __shfl_xor(acc, s, 64);  // every lane takes part
    if (active && sp == 0) a.pot[i] += acc;
  }
}

int check_desc2d(const fmm_desc* d) {
  if (!d) return fail(FMM_EINVAL, "desc is NULL");
  if (d->kernel != FMM_LAPLACE2D && d->kernel != FMM_BIHARMONIC2D)
    return fail(FMM_EINVAL, "2-D calls take FMM_LAPLACE2D or FMM_BIHARMONIC2D");
  if (d->dtype != FMM_F64) return fail(FMM_EUNSUPPORTED, "2-D kernels run in FMM_F64 only");
  if (d->order < 0 || d->order > FMM_MAX_ORDER)
    return fail(FMM_EUNSUPPORTED, "order " + std::to_string(d->order) + " outside [0, 16]");
  if (d->flags != 0) return fail(FMM_EINVAL, "flags must be 0");
  return FMM_OK;
}

inline int pde_c(const fmm_desc* d) { return d->kernel == FMM_BIHARMONIC2D ? 4 : 2; }

int launched(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(FMM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  return FMM_OK;
}

}  // namespace

extern "C" {

int fmm2d_sizes(const fmm_desc* desc, int32_t* n_full_out, int32_t* n_compressed) {
  int st = check_desc2d(desc);
  if (st) return st;
  if (n_full_out) *n_full_out = fmm2d::n_full(desc->order);
  if (n_compressed) *n_compressed = fmm2d::n_kept(desc->order, pde_c(desc));
  return FMM_OK;
}

int fmm2d_index_table(const fmm_desc* desc, int32_t* mxy) {
  int st = check_desc2d(desc);
  if (st) return st;
  FMM_REQUIRE(mxy, FMM_EINVAL, "mxy is NULL");
  const int p = desc->order, c = pde_c(desc);
  int k = 0;
  for (int b = 0; b < c && b <= p; ++b)
    for (int a = 0; a <= p - b; ++a) {
      mxy[2 * k] = a;
      mxy[2 * k + 1] = b;
      ++k;
    }
  return FMM_OK;
}

int fmm2d_deriv_tables(const fmm_desc* desc, int64_t n, const double* offset, const double* h, double* out,
                       void* stream) {
  int st = check_desc2d(desc);
  if (st) return st;
  FMM_REQUIRE(n >= 0, FMM_EINVAL, "n < 0");
  if (n == 0) return FMM_OK;
  FMM_REQUIRE(offset && h && out, FMM_EINVAL, "NULL pointer");
  tables2d_kernel<<<blocks_for(n, kTpb), kTpb, 0, (hipStream_t)stream>>>(n, offset, h, out, desc->kernel, desc->order);
  return launched("tables2d_kernel");
}

int fmm2d_p2m(const fmm_desc* desc, int64_t n_box, const double* box_center, const double* box_h,
              const int64_t* pt_range, int64_t n_src, const double* src_xy, const double* weight, double* mpole,
              int32_t max_src_per_box, void* stream) {
  int st = check_desc2d(desc);
  if (st) return st;
  FMM_REQUIRE(n_box >= 0 && n_src >= 0, FMM_EINVAL, "negative size");
  if (n_box == 0) return FMM_OK;
  FMM_REQUIRE(n_box <= 0x7fffffff, FMM_EINVAL, "too many boxes");
  FMM_REQUIRE(box_center && box_h && pt_range && mpole, FMM_EINVAL, "NULL pointer");
  FMM_REQUIRE(n_src == 0 || (src_xy && weight), FMM_EINVAL, "NULL source pointer");
  PointArgs2D a{n_box, box_center, box_h, pt_range, n_src, src_xy, weight, nullptr, mpole, 0, 0};
  unsigned columns = 1;
  point_launch_shape(max_src_per_box, a.lg, a.per_lane, columns);
  if (!launch_points2d(a, false, desc->order, pde_c(desc), columns, (hipStream_t)stream))
    return fail(FMM_EUNSUPPORTED, "no 2-D P2M for this order");
  return launched("p2m2d_points_kernel");
}

int fmm2d_m2l(const fmm_desc* desc, int64_t n_tbox, const int32_t* tbox, const int32_t* pair_ptr, int64_t n_pair,
              const int32_t* pair_src, const int32_t* pair_tab, int64_t n_tab, const double* tables, int64_t n_box,
              const double* mpole, double* local, void* stream) {
  int st = check_desc2d(desc);
  if (st) return st;
  FMM_REQUIRE(n_tbox >= 0 && n_pair >= 0 && n_tab >= 0 && n_box >= 0, FMM_EINVAL, "negative size");
  if (n_tbox == 0) return FMM_OK;
  FMM_REQUIRE(tbox && pair_ptr && mpole && local, FMM_EINVAL, "NULL pointer");
  FMM_REQUIRE(n_pair == 0 || (pair_src && pair_tab && tables), FMM_EINVAL, "NULL pair pointer");
  M2LArgs2D a{n_tbox, tbox, pair_ptr, n_pair, pair_src, pair_tab, n_tab, tables, n_box, mpole, local};
  if (!launch_m2l2d(a, desc->order, pde_c(desc), (hipStream_t)stream))
    return fail(FMM_EUNSUPPORTED, "no 2-D M2L for this order");
  return launched("m2l2d_kernel");
}

int fmm2d_l2p(const fmm_desc* desc, int64_t n_box, const double* box_center, const double* box_h,
              const int64_t* pt_range, int64_t n_tgt, const double* tgt_xy, const double* local, double* potential,
              int32_t max_tgt_per_box, void* stream) {
  int st = check_desc2d(desc);
  if (st) return st;
  FMM_REQUIRE(n_box >= 0 && n_tgt >= 0, FMM_EINVAL, "negative size");
  if (n_box == 0) return FMM_OK;
  FMM_REQUIRE(n_box <= 0x7fffffff, FMM_EINVAL, "too many boxes");
  FMM_REQUIRE(box_center && box_h && pt_range && local, FMM_EINVAL, "NULL pointer");
  FMM_REQUIRE(n_tgt == 0 || (tgt_xy && potential), FMM_EINVAL, "NULL target pointer");
  PointArgs2D a{n_box, box_center, box_h, pt_range, n_tgt, tgt_xy, nullptr, potential,
                const_cast<double*>(local), 0, 0};
  unsigned columns = 1;
  point_launch_shape(max_tgt_per_box, a.lg, a.per_lane, columns);
  if (!launch_points2d(a, true, desc->order, pde_c(desc), columns, (hipStream_t)stream))
    return fail(FMM_EUNSUPPORTED, "no 2-D L2P for this order");
  return launched("l2p2d_points_kernel");
}

int fmm2d_m2m(const fmm_desc* desc, int64_t n_parent, const int32_t* parent, const int32_t* child, int64_t n_box,
              const double* box_center, const double* box_h, double* mpole, void* stream) {
  int st = check_desc2d(desc);
  if (st) return st;
  FMM_REQUIRE(n_parent >= 0 && n_box >= 0, FMM_EINVAL, "negative size");
  if (n_parent == 0) return FMM_OK;
  FMM_REQUIRE(n_parent <= 0x7fffffff, FMM_EINVAL, "too many parents");
  FMM_REQUIRE(parent && child && box_center && box_h && mpole, FMM_EINVAL, "NULL pointer");
  const ShiftArgs2D a{n_parent, parent, child, n_box, box_center, box_h, mpole};
  if (!launch_shift2d(a, false, desc->order, pde_c(desc), (hipStream_t)stream))
    return fail(FMM_EUNSUPPORTED, "no 2-D M2M for this order");
  return launched("m2m2d_ring_kernel");
}

int fmm2d_l2l(const fmm_desc* desc, int64_t n_parent, const int32_t* parent, const int32_t* child, int64_t n_box,
              const double* box_center, const double* box_h, double* local, void* stream) {
  int st = check_desc2d(desc);
  if (st) return st;
  FMM_REQUIRE(n_parent >= 0 && n_box >= 0, FMM_EINVAL, "negative size");
  if (n_parent == 0) return FMM_OK;
  FMM_REQUIRE(n_parent <= 0x7fffffff, FMM_EINVAL, "too many parents");
  FMM_REQUIRE(parent && child && box_center && box_h && local, FMM_EINVAL, "NULL pointer");
  const ShiftArgs2D a{n_parent, parent, child, n_box, box_center, box_h, local};
  if (!launch_shift2d(a, true, desc->order, pde_c(desc), (hipStream_t)stream))
    return fail(FMM_EUNSUPPORTED, "no 2-D L2L for this order");
  return launched("l2l2d_ring_kernel");
}

int fmm2d_direct(const fmm_desc* desc, int64_t n_src, const double* src_xy, const double* weight, int64_t n_tgt,
                 const double* tgt_xy, double* potential, void* stream) {
  int st = check_desc2d(desc);
  if (st) return st;
  FMM_REQUIRE(n_src >= 0 && n_tgt >= 0, FMM_EINVAL, "negative size");
  if (n_tgt == 0) return FMM_OK;
  FMM_REQUIRE(tgt_xy && potential, FMM_EINVAL, "NULL target pointer");
  FMM_REQUIRE(n_src == 0 || (src_xy && weight), FMM_EINVAL, "NULL source pointer");
  int split = 1;
  while (split < 64 && (n_tgt * split + kTpb - 1) / kTpb < 1024) split *= 2;
  const unsigned grid = blocks_for(n_tgt, kTpb / split);
  if (desc->kernel == FMM_BIHARMONIC2D)
    direct2d_kernel<FMM_BIHARMONIC2D><<<grid, kTpb, 0, (hipStream_t)stream>>>(n_src, src_xy, weight, n_tgt, tgt_xy,
                                                                              potential, split);
  else
    direct2d_kernel<FMM_LAPLACE2D><<<grid, kTpb, 0, (hipStream_t)stream>>>(n_src, src_xy, weight, n_tgt, tgt_xy,
                                                                           potential, split);
  return launched("direct2d_kernel");
}

int fmm2d_p2p(const fmm_desc* desc, int64_t n_tbox, const int32_t* tbox, const int32_t* nbr_ptr, int64_t n_nbr,
              const int32_t* nbr, int64_t n_box, const int64_t* tgt_range, const int64_t* src_range, int64_t n_src,
              const double* src_xy, const double* weight, int64_t n_tgt, const double* tgt_xy, double* potential,
              int32_t max_tgt_per_box, void* stream) {
  int st = check_desc2d(desc);
  if (st) return st;
  FMM_REQUIRE(n_tbox >= 0 && n_nbr >= 0 && n_box >= 0 && n_src >= 0 && n_tgt >= 0, FMM_EINVAL, "negative size");
  if (n_tbox == 0) return FMM_OK;
  FMM_REQUIRE(n_tbox <= 0x7fffffff, FMM_EINVAL, "too many target boxes");
  FMM_REQUIRE(max_tgt_per_box >= 1, FMM_EINVAL, "max_tgt_per_box < 1");
  FMM_REQUIRE(tbox && nbr_ptr && tgt_range && src_range && tgt_xy && potential, FMM_EINVAL, "NULL pointer");
  FMM_REQUIRE(n_nbr == 0 || nbr, FMM_EINVAL, "NULL list");
  FMM_REQUIRE(n_src == 0 || (src_xy && weight), FMM_EINVAL, "NULL source pointer");
  // workgroups per box along y: one per 64 targets of the largest box
  const NearArgs2D a{n_tbox, tbox, nbr_ptr, n_nbr, nbr, n_box, tgt_range, src_range, n_src, src_xy, weight, n_tgt,
                     tgt_xy, potential};
  const int64_t chunks = ((int64_t)max_tgt_per_box + 63) / 64;
  const dim3 grid((unsigned)n_tbox, (unsigned)(chunks > 65535 ? 65535 : chunks));
  if (desc->kernel == FMM_BIHARMONIC2D)
    p2p2d_kernel<FMM_BIHARMONIC2D><<<grid, 64, 0, (hipStream_t)stream>>>(a);
  else
    p2p2d_kernel<FMM_LAPLACE2D><<<grid, 64, 0, (hipStream_t)stream>>>(a);
  return launched("p2p2d_kernel");
}

}  // extern "C"
