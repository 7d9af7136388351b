// Two-dimensional kernels G = log r and G = r^2 log r (Sec. 4.4) with the compressed Cartesian
// Taylor expansions of Secs. 2-3 for d = 2: derivative tables by the paper's recurrences
// (eqs. deriv_laplace_2d and deriv_biharmonic_2d), P2M with the compression, L2P with the
// decompression, the direct sum and the near field.  FP64.
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

// ----------------------------------------------------------------------------- P2M, L2P

// Compression in place: alpha over the square grid (a, b), a + b <= p (row length p + 1); the
// layers b >= c are pushed down by the PDE rule, highest first, so that afterwards the entries
// with b < c hold beta = M^T alpha.
__device__ void compress_grid(double* g, int p, int c, int lane, int nl) {
  const int R = p + 1;
  for (int b = p; b >= c; --b) {
    for (int a = lane; a <= p - b; a += nl) {
      const double v = g[a + b * R];
      if (c == 2) {
        g[(a + 2) + (b - 2) * R] -= v;
      } else {
        g[(a + 4) + (b - 4) * R] -= v;
        g[(a + 2) + (b - 2) * R] -= 2.0 * v;
      }
    }
    __syncthreads();
  }
}

// Decompression in place: entries with b < c hold theta; layers b >= c are filled lowest first.
__device__ void decompress_grid(double* g, int p, int c, int lane, int nl) {
  const int R = p + 1;
  for (int b = c; b <= p; ++b) {
    for (int a = lane; a <= p - b; a += nl) {
      if (c == 2)
        g[a + b * R] = -g[(a + 2) + (b - 2) * R];
      else
        g[a + b * R] = -g[(a + 4) + (b - 4) * R] - 2.0 * g[(a + 2) + (b - 2) * R];
    }
    __syncthreads();
  }
}

constexpr int kRow = FMM_MAX_ORDER + 1;  // grid row length bound
constexpr int kWg = 64;                  // one wavefront per (box, chunk)
constexpr int kChunk = 256;              // points of a box per workgroup (P2M, L2P)

// alpha~_(a, b) = sum_y w X^a Y^b / (a! b!), (X, Y) = (c - y) / h; beta~ = M^T alpha~.  Workgroup
// (box, y) takes the chunks y, y + gridDim.y, ... of kChunk points of the box and adds the
// compressed sum of its points to the box's row atomically (compression is linear).
__global__ __launch_bounds__(kWg) void p2m2d_kernel(int64_t n_box, const double* __restrict__ center,
                                                   const double* __restrict__ bh, const int64_t* __restrict__ range,
                                                   int64_t n_src, const double* __restrict__ xy,
                                                   const double* __restrict__ w, double* __restrict__ mpole, int p,
                                                   int c, int nc) {
  __shared__ double px[kWg][kRow];
  __shared__ double py[kWg][kRow];
  __shared__ double ws[kWg];
  __shared__ double grid[kRow * kRow];
  const int64_t box = blockIdx.x;
  const int lane = threadIdx.x;
  const int R = p + 1;
  const double cx = center[2 * box], cy = center[2 * box + 1], ih = 1.0 / bh[box];
  int64_t lo = range[2 * box], hi = range[2 * box + 1];
  lo = lo < 0 ? 0 : (lo > n_src ? n_src : lo);
  hi = hi < lo ? lo : (hi > n_src ? n_src : hi);
  if (lo + (int64_t)blockIdx.y * kChunk >= hi) return;  // no points for this workgroup (uniform)
  constexpr int kSlots = (kRow * kRow + kWg - 1) / kWg;
  double acc[kSlots];
#pragma unroll
  for (int k = 0; k < kSlots; ++k) acc[k] = 0.0;
  for (int64_t c0 = lo + (int64_t)blockIdx.y * kChunk; c0 < hi; c0 += (int64_t)gridDim.y * kChunk) {
  const int64_t c1 = c0 + kChunk < hi ? c0 + kChunk : hi;
  for (int64_t t0 = c0; t0 < c1; t0 += kWg) {
    const int64_t i = t0 + lane;
    double X = 0.0, Y = 0.0, wi = 0.0;
    if (i < c1) {
      X = (cx - xy[2 * i]) * ih;
      Y = (cy - xy[2 * i + 1]) * ih;
      wi = w[i];
    }
    px[lane][0] = 1.0;
    py[lane][0] = 1.0;
    for (int a = 1; a <= p; ++a) {
      px[lane][a] = px[lane][a - 1] * X / a;
      py[lane][a] = py[lane][a - 1] * Y / a;
    }
    ws[lane] = wi;
    __syncthreads();
    const int np = (int)(c1 - t0 < kWg ? c1 - t0 : kWg);
#pragma unroll
    for (int k = 0; k < kSlots; ++k) {
      const int e = lane + k * kWg;
      const int a = e % R, b = e / R;
      if (b <= p && a + b <= p) {
        double s = acc[k];
        for (int j = 0; j < np; ++j) s = fma(ws[j] * px[j][a], py[j][b], s);
        acc[k] = s;
      }
    }
    __syncthreads();
  }
  }
#pragma unroll
  for (int k = 0; k < kSlots; ++k) {
    const int e = lane + k * kWg;
    if (e < R * R) grid[e] = acc[k];
  }
  __syncthreads();
  compress_grid(grid, p, c, lane, kWg);
  for (int j = lane; j < nc; j += kWg) {
    // position j of J -> (a, b)
    int b = 0, off = 0;
    while (j >= off + (p - b + 1)) {
      off += p - b + 1;
      ++b;
    }
    atomicAdd(&mpole[box * nc + j], grid[(j - off) + b * R]);
  }
}

// phi(x) += sum_(a, b) L~_(a, b) X^a Y^b / (a! b!), (X, Y) = (x - c) / h, L~ = M theta~.  Workgroup
// (box, y) decompresses the box's local and evaluates it at the chunks y, y + gridDim.y, ... of
// kChunk targets.
__global__ __launch_bounds__(kWg) void l2p2d_kernel(int64_t n_box, const double* __restrict__ center,
                                                   const double* __restrict__ bh, const int64_t* __restrict__ range,
                                                   int64_t n_tgt, const double* __restrict__ xy,
                                                   const double* __restrict__ local, double* __restrict__ pot, int p,
                                                   int c, int nc) {
  __shared__ double grid[kRow * kRow];
  const int64_t box = blockIdx.x;
  const int lane = threadIdx.x;
  const int R = p + 1;
  int64_t lo = range[2 * box], hi = range[2 * box + 1];
  lo = lo < 0 ? 0 : (lo > n_tgt ? n_tgt : lo);
  hi = hi < lo ? lo : (hi > n_tgt ? n_tgt : hi);
  if (lo + (int64_t)blockIdx.y * kChunk >= hi) return;  // no targets for this workgroup (uniform)
  for (int e = lane; e < R * R; e += kWg) grid[e] = 0.0;
  __syncthreads();
  for (int j = lane; j < nc; j += kWg) {
    int b = 0, off = 0;
    while (j >= off + (p - b + 1)) {
      off += p - b + 1;
      ++b;
    }
    grid[(j - off) + b * R] = local[box * nc + j];
  }
  __syncthreads();
  decompress_grid(grid, p, c, lane, kWg);
  const double cx = center[2 * box], cy = center[2 * box + 1], ih = 1.0 / bh[box];
  for (int64_t c0 = lo + (int64_t)blockIdx.y * kChunk; c0 < hi; c0 += (int64_t)gridDim.y * kChunk)
  for (int64_t i = c0 + lane; i < (c0 + kChunk < hi ? c0 + kChunk : hi); i += kWg) {
    const double X = (xy[2 * i] - cx) * ih, Y = (xy[2 * i + 1] - cy) * ih;
    double outer = 0.0;
    for (int b = p; b >= 0; --b) {
      // inner Horner over a with the 1/a! folded in: c_0 + X (c_1 + X/2 (c_2 + ...))
      double s = grid[(p - b) + b * R];
      for (int a = p - b - 1; a >= 0; --a) s = fma(s, X / (a + 1), grid[a + b * R]);
      outer = b == p ? s : fma(outer, Y / (b + 1), s);
    }
    pot[i] += outer;
  }
}

// ----------------------------------------------------------------------------- M2M, L2L

// Powers d^k / k! (k <= p) of the two components of a translation vector, in LDS.
__device__ void stage_powers(double* px, double* py, double dx, double dy, int p, int lane) {
  if (lane == 0) {
    double a = 1.0, b = 1.0;
    px[0] = py[0] = 1.0;
    for (int k = 1; k <= p; ++k) {
      a *= dx / k;
      b *= dy / k;
      px[k] = a;
      py[k] = b;
    }
  }
}

// Compressed M2M (Sec. 4.3, eq. define_psi for d = 2), in the parent's scaled variables: each
// child's kept coefficients, rescaled to the parent's size ((h_c / h_p)^|q|), are embedded in
// M(p), translated by the binomial sums alpha'_r = sum_{q <= r} b_q D^(r-q) / (r-q)! with
// D = (c_p - c_c) / h_p (eq. mpole_translated_full_coeffs), summed over the children and
// compressed in place.  One wavefront per parent; the parent's row is overwritten.
__global__ __launch_bounds__(kWg) void m2m2d_kernel(int64_t n_parent, const int32_t* __restrict__ parent,
                                                   const int32_t* __restrict__ child, int64_t n_box,
                                                   const double* __restrict__ center, const double* __restrict__ bh,
                                                   double* __restrict__ mpole, int p, int c, int nc) {
  __shared__ double grid[kRow * kRow];   // alpha' of the parent (full)
  __shared__ double emb[kRow * kRow];    // the current child's embedded coefficients
  __shared__ double px[kRow], py[kRow];
  const int64_t k = blockIdx.x;
  const int par = parent[k];
  if (par < 0 || par >= n_box) return;  // uniform
  const int lane = threadIdx.x, R = p + 1;
  for (int e = lane; e < R * R; e += kWg) grid[e] = 0.0;
  const double hp = bh[par];
  for (int o = 0; o < 4; ++o) {
    const int ch = child[4 * k + o];
    if (ch < 0 || ch >= n_box) continue;  // uniform
    const double ratio = bh[ch] / hp;
    for (int e = lane; e < R * R; e += kWg) emb[e] = 0.0;
    __syncthreads();
    for (int j = lane; j < nc; j += kWg) {
      int b = 0, off = 0;
      while (j >= off + (p - b + 1)) {
        off += p - b + 1;
        ++b;
      }
      const int a = j - off;
      emb[a + b * R] = mpole[(int64_t)ch * nc + j] * pow(ratio, (double)(a + b));
    }
    stage_powers(px, py, (center[2 * par] - center[2 * ch]) / hp, (center[2 * par + 1] - center[2 * ch + 1]) / hp, p,
                 lane);
    __syncthreads();
    for (int e = lane; e < R * R; e += kWg) {
      const int ra = e % R, rb = e / R;
      if (ra + rb > p) continue;
      double acc = 0.0;
      for (int qb = 0; qb <= rb && qb < c; ++qb)
        for (int qa = 0; qa <= ra; ++qa) acc = fma(emb[qa + qb * R], px[ra - qa] * py[rb - qb], acc);
      grid[e] += acc;
    }
    __syncthreads();
  }
  __syncthreads();
  compress_grid(grid, p, c, lane, kWg);
  for (int j = lane; j < nc; j += kWg) {
    int b = 0, off = 0;
    while (j >= off + (p - b + 1)) {
      off += p - b + 1;
      ++b;
    }
    mpole[(int64_t)par * nc + j] = grid[(j - off) + b * R];
  }
}

// Compressed L2L (Sec. 4.2, eq. l2l-expr for d = 2): the parent's kept local is decompressed in
// place, its Taylor polynomial re-expanded about each child's centre (L'_i = sum_k L_(i+k)
// D^k / k!, D = (c_c - c_p) / h_p, scaled variables) and the kept entries, rescaled to the
// child's size, are added to the child's row.  One wavefront per parent.
__global__ __launch_bounds__(kWg) void l2l2d_kernel(int64_t n_parent, const int32_t* __restrict__ parent,
                                                   const int32_t* __restrict__ child, int64_t n_box,
                                                   const double* __restrict__ center, const double* __restrict__ bh,
                                                   double* __restrict__ local, int p, int c, int nc) {
  __shared__ double grid[kRow * kRow];
  __shared__ double px[kRow], py[kRow];
  const int64_t k = blockIdx.x;
  const int par = parent[k];
  if (par < 0 || par >= n_box) return;  // uniform
  const int lane = threadIdx.x, R = p + 1;
  for (int e = lane; e < R * R; e += kWg) grid[e] = 0.0;
  __syncthreads();
  for (int j = lane; j < nc; j += kWg) {
    int b = 0, off = 0;
    while (j >= off + (p - b + 1)) {
      off += p - b + 1;
      ++b;
    }
    grid[(j - off) + b * R] = local[(int64_t)par * nc + j];
  }
  __syncthreads();
  decompress_grid(grid, p, c, lane, kWg);
  const double hp = bh[par];
  for (int o = 0; o < 4; ++o) {
    const int ch = child[4 * k + o];
    if (ch < 0 || ch >= n_box) continue;  // uniform
    stage_powers(px, py, (center[2 * ch] - center[2 * par]) / hp, (center[2 * ch + 1] - center[2 * par + 1]) / hp, p,
                 lane);
    __syncthreads();
    const double ratio = bh[ch] / hp;
    for (int j = lane; j < nc; j += kWg) {
      int b = 0, off = 0;
      while (j >= off + (p - b + 1)) {
        off += p - b + 1;
        ++b;
      }
      const int a = j - off;
      double acc = 0.0;
      for (int ky = 0; ky <= p - a - b; ++ky)
        for (int kx = 0; kx <= p - a - b - ky; ++kx) acc = fma(grid[(a + kx) + (b + ky) * R], px[kx] * py[ky], acc);
      local[(int64_t)ch * nc + j] += acc * pow(ratio, (double)(a + b));
    }
    __syncthreads();  // px, py are rewritten for the next child
  }
}

// ----------------------------------------------------------------------------- direct, P2P

__device__ __forceinline__ double green2d(int kernel, double r2) {
  if (r2 == 0.0) return 0.0;
  const double l = 0.5 * log(r2);
  return kernel == FMM_BIHARMONIC2D ? r2 * l : l;
}

constexpr int kTile = 256;

__global__ __launch_bounds__(kTpb) void direct2d_kernel(int kernel, int64_t n_src, const double* __restrict__ src,
                                                       const double* __restrict__ w, int64_t n_tgt,
                                                       const double* __restrict__ tgt, double* __restrict__ pot) {
  __shared__ double sx[kTile], sy[kTile], sw[kTile];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
    for (int k = 0; k < nt; ++k) {
      const double dx = x - sx[k], dy = y - sy[k];
      acc = fma(green2d(kernel, dx * dx + dy * dy), sw[k], acc);
    }
    __syncthreads();
  }
  if (active) pot[i] = acc;
}

// Near field: one wavefront per (target box of the list, chunk of 64 of its targets).  A chunk of
// n targets gives each target `split` adjacent lanes (the largest power of two up to 16 with
// n * split <= 64), each summing every split-th source of the listed boxes; a butterfly of lane
// exchanges adds them up.  Sources are read straight from memory (lanes of one target read
// consecutive sources, the targets of a chunk read the same ones).
constexpr int kNearWg = 64;

__global__ __launch_bounds__(kNearWg) void p2p2d_kernel(int kernel, int64_t n_tbox, const int32_t* __restrict__ tbox,
                                                       const int32_t* __restrict__ nbr_ptr, int64_t n_nbr,
                                                       const int32_t* __restrict__ nbr, int64_t n_box,
                                                       const int64_t* __restrict__ trange,
                                                       const int64_t* __restrict__ srange, int64_t n_src,
                                                       const double* __restrict__ src, const double* __restrict__ w,
                                                       int64_t n_tgt, const double* __restrict__ tgt,
                                                       double* __restrict__ pot) {
  const int64_t k = blockIdx.x;
  const int32_t t = tbox[k];
  if (t < 0 || t >= n_box) return;
  int64_t lo = trange[2 * (int64_t)t], hi = trange[2 * (int64_t)t + 1];
  lo = lo < 0 ? 0 : (lo > n_tgt ? n_tgt : lo);
  hi = hi < lo ? lo : (hi > n_tgt ? n_tgt : hi);
  int64_t e0 = nbr_ptr[k], e1 = nbr_ptr[k + 1];
  e0 = e0 < 0 ? 0 : (e0 > n_nbr ? n_nbr : e0);
  e1 = e1 < e0 ? e0 : (e1 > n_nbr ? n_nbr : e1);
  const int lane = threadIdx.x;
  for (int64_t c0 = lo + (int64_t)blockIdx.y * kNearWg; c0 < hi; c0 += (int64_t)gridDim.y * kNearWg) {
    const int n = (int)(hi - c0 < kNearWg ? hi - c0 : kNearWg);
    int split = 1;
    while (split < 16 && n * split * 2 <= kNearWg) split *= 2;
    const int tl = lane / split, sp = lane % split;
    const bool active = tl < n;
    const int64_t i = c0 + tl;
    const double x = active ? tgt[2 * i] : 0.0, y = active ? tgt[2 * i + 1] : 0.0;
    double acc = 0.0;
    for (int64_t e = e0; e < e1; ++e) {
      const int32_t s = nbr[e];
      if (s < 0 || s >= n_box) continue;
      int64_t s0 = srange[2 * (int64_t)s], s1 = srange[2 * (int64_t)s + 1];
      s0 = s0 < 0 ? 0 : (s0 > n_src ? n_src : s0);
      s1 = s1 < s0 ? s0 : (s1 > n_src ? n_src : s1);
      if (!active) continue;
      for (int64_t j = s0 + sp; j < s1; j += split) {
        const double dx = x - src[2 * j], dy = y - src[2 * j + 1];
        acc = fma(green2d(kernel, dx * dx + dy * dy), w[j], acc);
      }
    }
    for (int m = 1; m < split; m <<= 1) acc += __shfl_xor(acc, m, 64);  // every lane takes part
    if (active && sp == 0) pot[i] += acc;
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

// workgroups per box along y for boxes of up to max_per_box points, `per` points each
inline unsigned chunks(int32_t max_per_box, int per) {
  const int64_t c = ((int64_t)(max_per_box < 1 ? 1 : max_per_box) + per - 1) / per;
  return (unsigned)(c > 65535 ? 65535 : c);
}

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
  const int p = desc->order, c = pde_c(desc);
  p2m2d_kernel<<<dim3((unsigned)n_box, chunks(max_src_per_box, kChunk)), kWg, 0, (hipStream_t)stream>>>(n_box, box_center, box_h, pt_range, n_src, src_xy,
                                                                  weight, mpole, p, c, fmm2d::n_kept(p, c));
  return launched("p2m2d_kernel");
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
  const int p = desc->order, c = pde_c(desc);
  l2p2d_kernel<<<dim3((unsigned)n_box, chunks(max_tgt_per_box, kChunk)), kWg, 0, (hipStream_t)stream>>>(n_box, box_center, box_h, pt_range, n_tgt, tgt_xy,
                                                                  local, potential, p, c, fmm2d::n_kept(p, c));
  return launched("l2p2d_kernel");
}

int fmm2d_m2m(const fmm_desc* desc, int64_t n_parent, const int32_t* parent, const int32_t* child, int64_t n_box,
              const double* box_center, const double* box_h, double* mpole, void* stream) {
  int st = check_desc2d(desc);
  if (st) return st;
  FMM_REQUIRE(n_parent >= 0 && n_box >= 0, FMM_EINVAL, "negative size");
  if (n_parent == 0) return FMM_OK;
  FMM_REQUIRE(n_parent <= 0x7fffffff, FMM_EINVAL, "too many parents");
  FMM_REQUIRE(parent && child && box_center && box_h && mpole, FMM_EINVAL, "NULL pointer");
  const int p = desc->order, c = pde_c(desc);
  m2m2d_kernel<<<(unsigned)n_parent, kWg, 0, (hipStream_t)stream>>>(n_parent, parent, child, n_box, box_center, box_h,
                                                                     mpole, p, c, fmm2d::n_kept(p, c));
  return launched("m2m2d_kernel");
}

int fmm2d_l2l(const fmm_desc* desc, int64_t n_parent, const int32_t* parent, const int32_t* child, int64_t n_box,
              const double* box_center, const double* box_h, double* local, void* stream) {
  int st = check_desc2d(desc);
  if (st) return st;
  FMM_REQUIRE(n_parent >= 0 && n_box >= 0, FMM_EINVAL, "negative size");
  if (n_parent == 0) return FMM_OK;
  FMM_REQUIRE(n_parent <= 0x7fffffff, FMM_EINVAL, "too many parents");
  FMM_REQUIRE(parent && child && box_center && box_h && local, FMM_EINVAL, "NULL pointer");
  const int p = desc->order, c = pde_c(desc);
  l2l2d_kernel<<<(unsigned)n_parent, kWg, 0, (hipStream_t)stream>>>(n_parent, parent, child, n_box, box_center, box_h,
                                                                     local, p, c, fmm2d::n_kept(p, c));
  return launched("l2l2d_kernel");
}

int fmm2d_direct(const fmm_desc* desc, int64_t n_src, const double* src_xy, const double* weight, int64_t n_tgt,
                 const double* tgt_xy, double* potential, void* stream) {
  int st = check_desc2d(desc);
  if (st) return st;
  FMM_REQUIRE(n_src >= 0 && n_tgt >= 0, FMM_EINVAL, "negative size");
  if (n_tgt == 0) return FMM_OK;
  FMM_REQUIRE(tgt_xy && potential, FMM_EINVAL, "NULL target pointer");
  FMM_REQUIRE(n_src == 0 || (src_xy && weight), FMM_EINVAL, "NULL source pointer");
  direct2d_kernel<<<blocks_for(n_tgt, kTpb), kTpb, 0, (hipStream_t)stream>>>(desc->kernel, n_src, src_xy, weight,
                                                                            n_tgt, tgt_xy, potential);
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
  const dim3 grid((unsigned)n_tbox, chunks(max_tgt_per_box, kNearWg));
  p2p2d_kernel<<<grid, kNearWg, 0, (hipStream_t)stream>>>(desc->kernel, n_tbox, tbox, nbr_ptr, n_nbr, nbr, n_box,
                                                       tgt_range, src_range, n_src, src_xy, weight, n_tgt, tgt_xy,
                                                       potential);
  return launched("p2p2d_kernel");
}

}  // extern "C"
