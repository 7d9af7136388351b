// Compressed P2M (Sec. 3.4): per box, the Cartesian moments
//   alpha~_q = sum_s w_s X_s^q / q!,   X_s = (c - y_s) / h        (eq. mpole, scaled t = 1/h)
// followed by the compression beta~ = M~^T alpha~ (eq. define_beta_multipole; Thm.
// mult_decompression: back substitution over the PDE recursion, O(p^3)).
//
// Layout of the work: one workgroup (4 wavefronts) per box.  The box's points are staged in
// LDS once as (X, Y, Z, w) (tiles of 256 points).  Each wavefront owns a contiguous quarter of
// M(p) in the full order (rows (m_z, m_x) of consecutive m_y), cut into pieces of at most 48
// coefficients (24 complex) that stay in registers: per point, the powers of Y once, the
// factor w Z^z X^x of each row as a running product, then one fused multiply-add per
// coefficient.  The monomials carry no factorials; 1/q! is applied to the sums.  A piece's
// sums over the 64 lanes go through a padded LDS transpose (8 values per pass in FP64, 16 in
// FP32: each lane adds one value over a group of lanes, then lane exchanges combine the groups),
// and land in the box's alpha~ in LDS.  The
// compression beta~ = M~^T alpha~ is one sparse row of the level's M~^T per coefficient (the
// matrix formed once per level on the host from the recursion of Thm. mult_decompression).
#pragma once

#include "../../include/fmm.h"
#include "common.hpp"
#include "device_util.hpp"
#include "kernels.hpp"

namespace fmm {

namespace detail_p2m {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

template <int P>
struct FullIdx {
  int x[nfull(P)], y[nfull(P)], z[nfull(P)];
  constexpr FullIdx() : x(), y(), z() {
    int k = 0;
    for (int mz = 0; mz <= P; ++mz)
      for (int mx = 0; mx <= P - mz; ++mx)
        for (int my = 0; my <= P - mz - mx; ++my) {
          x[k] = mx;
          y[k] = my;
          z[k] = mz;
          ++k;
        }
  }
};

// 1 / (x! y! z!) of every full index of M(P)
template <int P>
struct InvFactFull {
  double v[nfull(P)];
  constexpr InvFactFull() : v() {
    double f[P + 1] = {};
    f[0] = 1.0;
    for (int i = 1; i <= P; ++i) f[i] = f[i - 1] * i;
    constexpr FullIdx<P> I{};
    for (int q = 0; q < nfull(P); ++q) v[q] = 1.0 / (f[I.x[q]] * f[I.y[q]] * f[I.z[q]]);
  }
};
template <int P>
__device__ constexpr InvFactFull<P> kInvFact{};

constexpr int kTile = kThreads;  // points staged per pass
// values per pass of the reduction transpose: 8 for FP64, whose buffers would otherwise limit
// the resident workgroups (44 KB per workgroup instead of 28 KB at p = 8), 16 for FP32
template <typename R>
constexpr int kRedW = sizeof(R) == 8 ? 8 : 16;
template <typename R>
constexpr int kRedStride = kRedW<R> + 1;  // LDS row stride (one element of padding against bank conflicts)

template <typename R, bool CPLX>
struct Stage {
  R x[kTile], y[kTile], z[kTile], wr[kTile], wi[CPLX ? kTile : 1];
};

// Coefficients of wavefront W_ of a box: the full order cut into kWaves contiguous ranges, each
// cut into NS pieces (NS the same for every wavefront, so that their barriers match).
template <int P, bool CPLX>
struct Pieces {
  static constexpr int NP = nfull(P);
  static constexpr int QMAX = CPLX ? 24 : 48;
  static constexpr int QW = (NP + kWaves - 1) / kWaves;  // largest range
  static constexpr int NS = (QW + QMAX - 1) / QMAX;
  template <int W_, int S_>
  static constexpr int q0() {
    constexpr int a = NP * W_ / kWaves, b = NP * (W_ + 1) / kWaves;
    return a + (b - a) * S_ / NS;
  }
  template <int W_, int S_>
  static constexpr int q1() {
    constexpr int a = NP * W_ / kWaves, b = NP * (W_ + 1) / kWaves;
    return a + (b - a) * (S_ + 1) / NS;
  }
};

// acc[q - A] += w X^x Y^y Z^z for the coefficients q in [A, B) of the full order, one point.
template <int P, int A, int B, typename R, bool CPLX>
__device__ __forceinline__ void accumulate_point(R (&ar)[B - A > 0 ? B - A : 1], R (&ai)[B - A > 0 ? B - A : 1],
                                                 R X, R Y, R Z, R wr, R wi) {
  constexpr FullIdx<P> I{};
  if constexpr (B > A) {
    R py[P + 1];
    py[0] = R(1);
#pragma unroll
    for (int k = 1; k <= P; ++k) py[k] = py[k - 1] * Y;
    R zr = wr, zi = wi;  // w Z^z
#pragma unroll
    for (int e = 0; e < I.z[A]; ++e) {
      zr *= Z;
      if constexpr (CPLX) zi *= Z;
    }
    R rr = zr, ri = zi;  // w Z^z X^x
#pragma unroll
    for (int e = 0; e < I.x[A]; ++e) {
      rr *= X;
      if constexpr (CPLX) ri *= X;
    }
#pragma unroll
    for (int q = A; q < B; ++q) {
      if (q > A && I.y[q] == 0) {  // next row: x + 1, or the next slab (z + 1, x = 0)
        if (I.x[q] == 0) {
          zr *= Z;
          rr = zr;
          if constexpr (CPLX) {
            zi *= Z;
            ri = zi;
          }
        } else {
          rr *= X;
          if constexpr (CPLX) ri *= X;
        }
      }
      ar[q - A] += rr * py[I.y[q]];
      if constexpr (CPLX) ai[q - A] += ri * py[I.y[q]];
    }
  }
}

// Sum over the 64 lanes of v[0 .. N-1] (one value per lane each) into dst[k * DS] * scale[k],
// through the wavefront's LDS transpose buffer buf [64][kRedStride<R>], kRedW<R> values per pass:
// lane (g, k) adds value k of the kRedW lanes of group g, then the groups are combined by
// lane exchanges.
template <int N, int DS, typename R>
__device__ __forceinline__ void wave_sum(const R (&v)[N > 0 ? N : 1], R* buf, int lane, double* dst,
                                         const double* scale) {
  constexpr int RW = kRedW<R>, RS = kRedStride<R>;
  const int k = lane & (RW - 1), g = lane / RW;
#pragma unroll
  for (int j = 0; j < (N + RW - 1) / RW; ++j) {
#pragma unroll
    for (int i = 0; i < RW; ++i) buf[lane * RS + i] = (RW * j + i < N) ? v[RW * j + i] : R(0);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // this wavefront's writes are in LDS
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < RW; ++r) s += (double)buf[(RW * g + r) * RS + k];
    if constexpr (RW <= 8) s += xchg<8>(s);
    s += xchg<16>(s);
    s += xchg<32>(s);
    if (g == 0 && RW * j + k < N) dst[(RW * j + k) * DS] = s * scale[RW * j + k];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // reads done before the next writes
  }
}

// Stage points [lo + t0, lo + t0 + cnt) of the box: X = s (c - y) h^-1 and the weights.
template <typename R, bool CPLX>
__device__ __forceinline__ void stage_tile(const P2MArgs& a, Stage<R, CPLX>& st, int64_t first, int cnt,
                                           const double (&cen)[3], double inv_h) {
  const int t = threadIdx.x;
  if (t < cnt) {
    const R* xyz = reinterpret_cast<const R*>(a.xyz);
    const int64_t s = first + t;
    const R ih = (R)inv_h;
    st.x[t] = ((R)cen[0] - xyz[s * 3 + 0]) * ih;
    st.y[t] = ((R)cen[1] - xyz[s * 3 + 1]) * ih;
    st.z[t] = ((R)cen[2] - xyz[s * 3 + 2]) * ih;
    if constexpr (CPLX) {
      st.wr[t] = reinterpret_cast<const R*>(a.w)[2 * s];
      st.wi[t] = reinterpret_cast<const R*>(a.w)[2 * s + 1];
    } else {
      st.wr[t] = reinterpret_cast<const R*>(a.w)[s];
    }
  }
}

// Piece S_ of wavefront W_: accumulate over every point of the box, then sum into alpha (LDS).
template <int P, typename R, bool CPLX, int W_, int S_>
__device__ __forceinline__ void run_piece(const P2MArgs& a, Stage<R, CPLX>& st, R* buf, int64_t lo, int n,
                                          const double (&cen)[3], double inv_h, int lane, double* alpha) {
  using PC = Pieces<P, CPLX>;
  constexpr int A = PC::template q0<W_, S_>(), B = PC::template q1<W_, S_>(), N = B - A;
  R ar[N > 0 ? N : 1], ai[N > 0 ? N : 1];
#pragma unroll
  for (int k = 0; k < (N > 0 ? N : 1); ++k) ar[k] = ai[k] = R(0);
  const bool one_tile = n <= kTile;
  for (int t0 = 0; t0 < n; t0 += kTile) {
    const int cnt = n - t0 < kTile ? n - t0 : kTile;
    if (!one_tile) {  // the single tile of a small box was staged once before the pieces
      __syncthreads();
      stage_tile<R, CPLX>(a, st, lo + t0, cnt, cen, inv_h);
      __syncthreads();
    }
    for (int j = lane; j < cnt; j += 64)
      accumulate_point<P, A, B, R, CPLX>(ar, ai, st.x[j], st.y[j], st.z[j], st.wr[j], CPLX ? st.wi[j] : R(0));
  }
  const double* scale = kInvFact<P>.v + A;
  if constexpr (CPLX) {
    wave_sum<N, 2, R>(ar, buf, lane, alpha + 2 * A, scale);
    wave_sum<N, 2, R>(ai, buf, lane, alpha + 2 * A + 1, scale);
  } else {
    wave_sum<N, 1, R>(ar, buf, lane, alpha + A, scale);
  }
}

template <int P, typename R, bool CPLX, int W_, int S_>
__device__ __forceinline__ void run_pieces(const P2MArgs& a, Stage<R, CPLX>& st, R* buf, int64_t lo, int n,
                                           const double (&cen)[3], double inv_h, int lane, double* alpha) {
  if constexpr (S_ < Pieces<P, CPLX>::NS) {
    run_piece<P, R, CPLX, W_, S_>(a, st, buf, lo, n, cen, inv_h, lane, alpha);
    run_pieces<P, R, CPLX, W_, S_ + 1>(a, st, buf, lo, n, cen, inv_h, lane, alpha);
  }
}

// In-LDS back substitution beta = M^T alpha over the recursion terms (gather form, levels
// of m_z from P down to 0).  Values in double (complex interleaved).  Entry k of level z is
// full index slab(z) + k, decoded arithmetically; the recursion terms are unrolled, so nothing
// is indexed dynamically in registers.
template <int P, bool CPLX>
__device__ inline void compress_lds(double* al, const RecArgs& rec, int c, double h) {
  double cf[kMaxRecTerms];
#pragma unroll
  for (int t = 0; t < kMaxRecTerms; ++t) {
    double f = rec.coef[t];
    for (int e = 0; e < rec.hpow[t]; ++e) f *= h;
    cf[t] = f;
  }
  // a level gathers only from levels at least dmin above it, so dmin consecutive levels are
  // independent and share one barrier
  int dmin = P + 1;
#pragma unroll
  for (int t = 0; t < kMaxRecTerms; ++t)
    if (t < rec.n) dmin = min(dmin, -rec.dz[t]);
  dmin = max(dmin, 1);
  for (int z1 = P; z1 >= 0; z1 -= dmin) {
    const int z0 = max(0, z1 - dmin + 1);  // levels z0 .. z1
    const int s0 = nfull(P) - nfull(P - z0), cnt = nfull(P - z0) - nfull(P - z1 - 1);
    for (int k = threadIdx.x; k < cnt; k += blockDim.x) {
      const int n = s0 + k;
      int z = z0, kk = k;
      while (kk >= tri(P - z)) {
        kk -= tri(P - z);
        ++z;
      }
      int x, y;
      slab_decode(P - z, kk, x, y);
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int t = 0; t < kMaxRecTerms; ++t) {
        if (t >= rec.n) break;
        // m = n - d with m_z >= c feeds n
        const int mx = x - rec.dx[t], my = y - rec.dy[t], mz = z - rec.dz[t];
        if (mx < 0 || my < 0 || mz < c || mx + my + mz > P) continue;
        const int m = full_index(P, mx, my, mz);
        if constexpr (CPLX) {
          sr += cf[t] * al[2 * m];
          si += cf[t] * al[2 * m + 1];
        } else {
          sr += cf[t] * al[m];
        }
      }
      if constexpr (CPLX) {
        al[2 * n] += sr;
        al[2 * n + 1] += si;
      } else {
        al[n] += sr;
      }
    }
    __syncthreads();
  }
}

template <int P, typename R, bool CPLX>
__global__ __launch_bounds__(kThreads) void p2m_kernel(P2MArgs a) {
  constexpr int NP = nfull(P);
  __shared__ double alpha[NP * (CPLX ? 2 : 1)];
  __shared__ Stage<R, CPLX> st;
  __shared__ R red[kWaves][64 * kRedStride<R>];
  const int64_t b = blockIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  int lev = a.level[b];
  lev = lev < 0 ? 0 : (lev >= a.n_levels ? a.n_levels - 1 : lev);
  const double h = a.level_h[lev];
  const double cen[3] = {a.center[3 * b], a.center[3 * b + 1], a.center[3 * b + 2]};
  int64_t lo = a.range[2 * b], hi = a.range[2 * b + 1];
  lo = lo < 0 ? 0 : (lo > a.n_pts ? a.n_pts : lo);
  hi = hi < lo ? lo : (hi > a.n_pts ? a.n_pts : hi);
  if (gridDim.y > 1) {  // chunk blockIdx.y of the box's points (compression is linear)
    const int64_t len = (hi - lo + gridDim.y - 1) / gridDim.y;
    const int64_t c0 = lo + (int64_t)blockIdx.y * len;
    hi = c0 + len < hi ? c0 + len : hi;
    lo = c0 < hi ? c0 : hi;
  }
  const int n = (int)(hi - lo);
  const double inv_h = a.xsign / h;
  if (n <= kTile) {
    stage_tile<R, CPLX>(a, st, lo, n, cen, inv_h);
    __syncthreads();
  }
  R* buf = red[wave];
  switch (wave) {
    case 0: run_pieces<P, R, CPLX, 0, 0>(a, st, buf, lo, n, cen, inv_h, lane, alpha); break;
    case 1: run_pieces<P, R, CPLX, 1, 0>(a, st, buf, lo, n, cen, inv_h, lane, alpha); break;
    case 2: run_pieces<P, R, CPLX, 2, 0>(a, st, buf, lo, n, cen, inv_h, lane, alpha); break;
    default: run_pieces<P, R, CPLX, 3, 0>(a, st, buf, lo, n, cen, inv_h, lane, alpha); break;
  }
  __syncthreads();
  // compression beta~_j = sum_m M~[m][j] alpha~_m: one sparse row of M~^T per coefficient, the
  // level's matrix formed once on the host from the recursion
  const int nc = a.nc;
  const int32_t* rp = a.cmp_ptr + (int64_t)lev * (nc + 1);
  constexpr int W = CPLX ? 2 : 1;
  double* part = gridDim.y > 1 ? a.part + (b * gridDim.y + blockIdx.y) * (int64_t)nc * W : nullptr;
  R* out = reinterpret_cast<R*>(a.out) + b * (int64_t)nc * W;
  for (int j = threadIdx.x; j < nc; j += blockDim.x) {
    double sr = 0.0, si = 0.0;
    for (int e = rp[j]; e < rp[j + 1]; ++e) {
      const int m = a.cmp_col[e];
      const double v = a.cmp_val[e];
      sr += v * alpha[W * m];
      if constexpr (CPLX) si += v * alpha[W * m + 1];
    }
    if (part) {
      part[W * j] = sr;
      if constexpr (CPLX) part[W * j + 1] = si;
    } else {
      out[W * j] = (R)sr;
      if constexpr (CPLX) out[W * j + 1] = (R)si;
    }
  }
}

// ---- Several boxes per workgroup -------------------------------------------------------------
// With one box per workgroup, a box of a few hundred points gives each lane only a handful of
// points, the sums over 64 lanes cost as much as the accumulation, and the launch runs as
// several rounds of resident workgroups, each paying a whole load -> reduce -> store chain.
// Here a workgroup takes kQBoxes consecutive boxes: in every wavefront (which still owns a
// quarter of M(p)), the kQLanes lanes of row r take the points of box r, so each lane
// accumulates kQBoxes times more points and the sums run over kQLanes lanes only.

constexpr int kQBoxes = 4;
constexpr int kQLanes = 64 / kQBoxes;  // lanes per box in each wavefront (one DPP row)

// points per box staged per pass (16 KB of real points per workgroup)
template <typename R>
constexpr int kQTile = sizeof(R) == 8 ? 128 : 256;

template <typename R, bool CPLX>
struct QStage {
  R x[kQBoxes * kQTile<R>], y[kQBoxes * kQTile<R>], z[kQBoxes * kQTile<R>], wr[kQBoxes * kQTile<R>],
      wi[CPLX ? kQBoxes * kQTile<R> : 1];
};

struct QBox {
  double cx, cy, cz, inv_h;
  int64_t lo;
  int n, lev;
};

template <int P, typename R, bool CPLX>
constexpr size_t quad_lds_bytes() {
  return sizeof(double) * kQBoxes * nfull(P) * (CPLX ? 2 : 1) + sizeof(QStage<R, CPLX>) +
         sizeof(R) * kWaves * 64 * kRedStride<R> + sizeof(QBox) * kQBoxes;
}

// the form is used where its LDS leaves room for three workgroups per CU
template <int P, typename R, bool CPLX>
constexpr bool quad_ok() {
  return quad_lds_bytes<P, R, CPLX>() <= 52u * 1024u;
}

// Sum over the kQLanes lanes of each row of v[0 .. N-1] into dst_r[k * DS] * scale[k] (dst_r
// the row's box), through the wavefront's LDS transpose buffer buf [64][kRedStride<R>],
// kRedW<R> values per pass: each lane adds one value over a group of kRedW lanes of its row,
// and for kRedW = 8 the two groups of a row are combined by a lane exchange within the row.
template <int N, int DS, typename R>
__device__ __forceinline__ void row_sum(const R (&v)[N > 0 ? N : 1], R* buf, int lane, double* dst_r,
                                        const double* scale) {
  constexpr int RW = kRedW<R>, RS = kRedStride<R>;
  constexpr int G = kQLanes / RW;  // groups of lanes per row: 2 (FP64) or 1 (FP32)
  static_assert(G == 1 || G == 2, "row groups");
  const int r = lane / kQLanes, k = lane & (kQLanes - 1);
  const int val = k & (RW - 1), grp = k / RW;
  const int base = (r * kQLanes + grp * RW) * RS + val;
#pragma unroll
  for (int j = 0; j < (N + RW - 1) / RW; ++j) {
#pragma unroll
    for (int i = 0; i < RW; ++i) buf[lane * RS + i] = (RW * j + i < N) ? v[RW * j + i] : R(0);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // this wavefront's writes are in LDS
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < RW; ++i) s += (double)buf[base + i * RS];
    if constexpr (G == 2) s += xchg<8>(s);
    if (grp == 0 && RW * j + val < N) dst_r[(RW * j + val) * DS] = s * scale[RW * j + val];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // reads done before the next writes
  }
}

// Stage points [t0, t0 + kQTile) of every box of the workgroup (X = s (c - y) h^-1 and w).
// Every read is issued before any is used: slots past a box's end read point 0 (the workgroup
// holds at least one point, so the array is not empty) and store nothing.
template <typename R, bool CPLX>
__device__ __forceinline__ void quad_stage(const P2MArgs& a, QStage<R, CPLX>& st, const QBox* bx, int t0) {
  constexpr int T = kQTile<R>;
  constexpr int NS = kQBoxes * T / kThreads;  // slots per thread
  const R* xyz = reinterpret_cast<const R*>(a.xyz);
  const R* w = reinterpret_cast<const R*>(a.w);
  int64_t src[NS];
  bool ok[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const int slot = threadIdx.x + i * kThreads, r = slot / T, j = slot - r * T;
    ok[i] = t0 + j < bx[r].n;
    src[i] = ok[i] ? bx[r].lo + t0 + j : 0;
  }
  R px[NS], py[NS], pz[NS], wr[NS], wi[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    px[i] = xyz[src[i] * 3 + 0];
    py[i] = xyz[src[i] * 3 + 1];
    pz[i] = xyz[src[i] * 3 + 2];
    if constexpr (CPLX) {
      wr[i] = w[2 * src[i]];
      wi[i] = w[2 * src[i] + 1];
    } else {
      wr[i] = w[src[i]];
      wi[i] = R(0);
    }
  }
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const int slot = threadIdx.x + i * kThreads, r = slot / T;
    if (ok[i]) {
      const R ih = (R)bx[r].inv_h;
      st.x[slot] = ((R)bx[r].cx - px[i]) * ih;
      st.y[slot] = ((R)bx[r].cy - py[i]) * ih;
      st.z[slot] = ((R)bx[r].cz - pz[i]) * ih;
      st.wr[slot] = wr[i];
      if constexpr (CPLX) st.wi[slot] = wi[i];
    }
  }
}

template <int P, typename R, bool CPLX, int W_, int S_>
__device__ __forceinline__ void quad_piece(const P2MArgs& a, QStage<R, CPLX>& st, R* buf, const QBox* bx, int nmax,
                                           int lane, double* alpha) {
  using PC = Pieces<P, CPLX>;
  constexpr int A = PC::template q0<W_, S_>(), B = PC::template q1<W_, S_>(), N = B - A;
  constexpr int T = kQTile<R>;
  constexpr int WD = CPLX ? 2 : 1;
  R ar[N > 0 ? N : 1], ai[N > 0 ? N : 1];
#pragma unroll
  for (int k = 0; k < (N > 0 ? N : 1); ++k) ar[k] = ai[k] = R(0);
  const int r = lane / kQLanes, pl = lane & (kQLanes - 1);
  const int n = bx[r].n;
  const bool one_tile = nmax <= T;
  for (int t0 = 0; t0 < nmax; t0 += T) {  // uniform over the workgroup
    if (!one_tile) {  // the single tile of small boxes was staged once before the pieces
      __syncthreads();
      quad_stage<R, CPLX>(a, st, bx, t0);
      __syncthreads();
    }
    const int cnt = n - t0 < T ? n - t0 : T;
    for (int j = pl; j < cnt; j += kQLanes) {
      const int sl = r * T + j;
      accumulate_point<P, A, B, R, CPLX>(ar, ai, st.x[sl], st.y[sl], st.z[sl], st.wr[sl], CPLX ? st.wi[sl] : R(0));
    }
  }
  const double* scale = kInvFact<P>.v + A;
  double* dst = alpha + (size_t)r * nfull(P) * WD + (size_t)A * WD;
  if constexpr (CPLX) {
    row_sum<N, 2, R>(ar, buf, lane, dst, scale);
    row_sum<N, 2, R>(ai, buf, lane, dst + 1, scale);
  } else {
    row_sum<N, 1, R>(ar, buf, lane, dst, scale);
  }
}

template <int P, typename R, bool CPLX, int W_, int S_>
__device__ __forceinline__ void quad_pieces(const P2MArgs& a, QStage<R, CPLX>& st, R* buf, const QBox* bx, int nmax,
                                            int lane, double* alpha) {
  if constexpr (S_ < Pieces<P, CPLX>::NS) {
    quad_piece<P, R, CPLX, W_, S_>(a, st, buf, bx, nmax, lane, alpha);
    quad_pieces<P, R, CPLX, W_, S_ + 1>(a, st, buf, bx, nmax, lane, alpha);
  }
}

template <int P, typename R, bool CPLX>
__global__ __launch_bounds__(kThreads) void p2m_quad_kernel(P2MArgs a) {
  constexpr int NP = nfull(P);
  constexpr int WD = CPLX ? 2 : 1;
  __shared__ double alpha[kQBoxes * NP * WD];
  __shared__ QStage<R, CPLX> st;
  __shared__ R red[kWaves][64 * kRedStride<R>];
  __shared__ QBox bx[kQBoxes];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int64_t b0 = (int64_t)blockIdx.x * kQBoxes;
  if (threadIdx.x < kQBoxes) {
    const int64_t b = b0 + threadIdx.x;
    QBox q{};
    if (b < a.n_box) {
      int lev = a.level[b];
      lev = lev < 0 ? 0 : (lev >= a.n_levels ? a.n_levels - 1 : lev);
      int64_t lo = a.range[2 * b], hi = a.range[2 * b + 1];
      lo = lo < 0 ? 0 : (lo > a.n_pts ? a.n_pts : lo);
      hi = hi < lo ? lo : (hi > a.n_pts ? a.n_pts : hi);
      q.cx = a.center[3 * b];
      q.cy = a.center[3 * b + 1];
      q.cz = a.center[3 * b + 2];
      q.inv_h = a.xsign / a.level_h[lev];
      q.lo = lo;
      q.n = (int)(hi - lo);
      q.lev = lev;
    }
    bx[threadIdx.x] = q;
  }
  __syncthreads();
  int nmax = 0;
#pragma unroll
  for (int r = 0; r < kQBoxes; ++r) nmax = bx[r].n > nmax ? bx[r].n : nmax;
  if (nmax > 0 && nmax <= kQTile<R>) {
    quad_stage<R, CPLX>(a, st, bx, 0);
    __syncthreads();
  }
  R* buf = red[wave];
  switch (wave) {
    case 0: quad_pieces<P, R, CPLX, 0, 0>(a, st, buf, bx, nmax, lane, alpha); break;
    case 1: quad_pieces<P, R, CPLX, 1, 0>(a, st, buf, bx, nmax, lane, alpha); break;
    case 2: quad_pieces<P, R, CPLX, 2, 0>(a, st, buf, bx, nmax, lane, alpha); break;
    default: quad_pieces<P, R, CPLX, 3, 0>(a, st, buf, bx, nmax, lane, alpha); break;
  }
  __syncthreads();
  // compression beta~_j = sum_m M~[m][j] alpha~_m of every box of the workgroup (one sparse
  // row of the box level's M~^T per coefficient)
  const int nc = a.nc;
  for (int idx = threadIdx.x; idx < kQBoxes * nc; idx += kThreads) {
    const int r = idx / nc, j = idx - r * nc;
    const int64_t b = b0 + r;
    if (b >= a.n_box) break;  // boxes past the end come last
    const int32_t* rp = a.cmp_ptr + (int64_t)bx[r].lev * (nc + 1);
    const double* al = alpha + (size_t)r * NP * WD;
    double sr = 0.0, si = 0.0;
    for (int e = rp[j]; e < rp[j + 1]; ++e) {
      const int m = a.cmp_col[e];
      const double v = a.cmp_val[e];
      sr += v * al[WD * m];
      if constexpr (CPLX) si += v * al[WD * m + 1];
    }
    R* out = reinterpret_cast<R*>(a.out) + b * (int64_t)nc * WD;
    out[WD * j] = (R)sr;
    if constexpr (CPLX) out[WD * j + 1] = (R)si;
  }
}

template <int P>
int launch_p2m_p(const P2MArgs& a, int dtype, hipStream_t s) {
  if (a.ny <= 1) {  // boxes not split into chunks: several boxes per workgroup where it fits
    const dim3 gq((unsigned)((a.n_box + kQBoxes - 1) / kQBoxes)), tq(kThreads);
    switch (dtype) {
      case FMM_F64:
        if constexpr (quad_ok<P, double, false>()) {
          hipLaunchKernelGGL((p2m_quad_kernel<P, double, false>), gq, tq, 0, s, a);
          FMM_HIP_CHECK(hipGetLastError());
          return FMM_OK;
        }
        break;
      case FMM_F32:
        if constexpr (quad_ok<P, float, false>()) {
          hipLaunchKernelGGL((p2m_quad_kernel<P, float, false>), gq, tq, 0, s, a);
          FMM_HIP_CHECK(hipGetLastError());
          return FMM_OK;
        }
        break;
      default: break;
    }
  }
  dim3 g((unsigned)a.n_box, (unsigned)(a.ny > 1 ? a.ny : 1)), t(kThreads);
  switch (dtype) {
    case FMM_F64: hipLaunchKernelGGL((p2m_kernel<P, double, false>), g, t, 0, s, a); break;
    case FMM_F32: hipLaunchKernelGGL((p2m_kernel<P, float, false>), g, t, 0, s, a); break;
    case FMM_C128: hipLaunchKernelGGL((p2m_kernel<P, double, true>), g, t, 0, s, a); break;
    case FMM_C64: hipLaunchKernelGGL((p2m_kernel<P, float, true>), g, t, 0, s, a); break;
    default: return fail(FMM_EINVAL, "dtype");
  }
  FMM_HIP_CHECK(hipGetLastError());
  return FMM_OK;
}

}  // namespace detail_p2m

#define FMM_INSTANTIATE_P2M(P) \
  int launch_p2m_order_##P(const P2MArgs& a, int dtype, hipStream_t s) { \
    return detail_p2m::launch_p2m_p<P>(a, dtype, s); \
  }

}  // namespace fmm
