// Compressed L2P (Sec. 3.3, eq. compressed-local-form): per box, decompress the scaled
// local theta~ (L~ = M~ theta~, Thm. mult_decompression, one sparse row of the level's M~ per
// full index; the matrix is formed once per level on the host from the PDE recursion),
// multiply by 1/i!, and add
//   phi(x) = sum_{i in M(p)} L~_i / i! X^i,    X = (x - c) / h,
// to every target of the box.
//
// One wavefront per box (a workgroup of 64 lanes, so its barriers cost next to nothing).  The
// decompressed coefficients live in LDS and are read as wave-wide broadcasts; every lane
// evaluates KU targets at once with a nested Horner scheme, so that each coefficient read
// feeds KU fused multiply-adds.  KU is chosen per pass from the points left (1, 2 or 4), so
// that a pass is not mostly empty: small leaves of adaptive trees take KU = 1.  Memory reads
// are issued in groups before their first use (the targets of a pass, the rows of the
// decompression, the box's locals), never one per branch: a read inside a bounds check waits
// for its own round trip.  The index decode (full index -> (x, y, z)) comes from compile-time
// tables, so that no per-lane array is indexed dynamically.
#pragma once

#include "../../include/fmm.h"
#include "common.hpp"
#include "device_util.hpp"
#include "kernels.hpp"

#include <algorithm>

namespace fmm {

namespace detail_l2p {

constexpr int kThreads = 64;  // one wavefront per box
// most targets per lane and pass: 8 for real potentials, 4 where complex values or gradients
// leave fewer registers.  The unrolled evaluation (whose reads are all issued before it) takes
// at most 5: a box of a few more than 256 points (boxes of a uniform level of 2^20 points
// hold 256 +- 16) runs one pass of 5 instead of a pass of 4 and a short second one (which
// repeats the whole sweep over the coefficients); a pass of 6 measured slower than both.
template <bool CPLX, bool GRAD>
constexpr int kMaxU = (CPLX || GRAD) ? 4 : 8;
constexpr int kMaxUnrolledU = 5;
constexpr int kChunk = kThreads * 8;  // points of a box per workgroup of the 2-D grid
constexpr int kWavesPerEU = 4;  // register budget: at most 128 per lane

struct InvFact {
  double v[FMM_MAX_ORDER + 1];
  constexpr InvFact() : v() {
    double f = 1.0;
    for (int i = 0; i <= FMM_MAX_ORDER; ++i) {
      if (i > 0) f *= i;
      v[i] = 1.0 / f;
    }
  }
};

// (x, y, z) of every full index of M(P), and 1 / (x! y! z!)
template <int P>
struct FullDecode {
  unsigned char x[nfull(P)], y[nfull(P)], z[nfull(P)];
  double inv_fact[nfull(P)];
  constexpr FullDecode() : x(), y(), z(), inv_fact() {
    constexpr InvFact IF{};
    int k = 0;
    for (int mz = 0; mz <= P; ++mz)
      for (int mx = 0; mx <= P - mz; ++mx)
        for (int my = 0; my <= P - mz - mx; ++my) {
          x[k] = (unsigned char)mx;
          y[k] = (unsigned char)my;
          z[k] = (unsigned char)mz;
          inv_fact[k] = IF.v[mx] * IF.v[my] * IF.v[mz];
          ++k;
        }
  }
};

template <int P>
__device__ constexpr FullDecode<P> kDecode{};

// Forward substitution L = M theta in LDS, levels m_z = c .. P (values in double, complex
// interleaved).  Entry k of level z is full index slab(z) + k.
template <int P, bool CPLX>
__device__ inline void decompress_lds(double* L, const RecArgs& rec, int c, double h) {
  double cf[kMaxRecTerms];
#pragma unroll
  for (int t = 0; t < kMaxRecTerms; ++t) {
    double f = rec.coef[t];
    for (int e = 0; e < rec.hpow[t]; ++e) f *= h;
    cf[t] = f;
  }
  // a level reads only levels at least dmin below it, so dmin consecutive levels are
  // independent and share one barrier
  int dmin = P + 1;
#pragma unroll
  for (int t = 0; t < kMaxRecTerms; ++t)
    if (t < rec.n) dmin = min(dmin, -rec.dz[t]);
  dmin = max(dmin, 1);
  for (int z0 = c; z0 <= P; z0 += dmin) {
    const int z1 = min(P, z0 + dmin - 1);
    const int s0 = nfull(P) - nfull(P - z0), cnt = nfull(P - z0) - nfull(P - z1 - 1);
    for (int k = threadIdx.x; k < cnt; k += blockDim.x) {
      const int m = s0 + k;
      int z = z0, kk = k;
      while (kk >= tri(P - z)) {
        kk -= tri(P - z);
        ++z;
      }
      int x, y;
      slab_decode(P - z, kk, x, y);  // arithmetic: no memory wait on the level's critical path
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int t = 0; t < kMaxRecTerms; ++t) {
        if (t >= rec.n) break;
        const int n = full_index(P, x + rec.dx[t], y + rec.dy[t], z + rec.dz[t]);
        if constexpr (CPLX) {
          sr += cf[t] * L[2 * n];
          si += cf[t] * L[2 * n + 1];
        } else {
          sr += cf[t] * L[n];
        }
      }
      if constexpr (CPLX) {
        L[2 * m] = sr;
        L[2 * m + 1] = si;
      } else {
        L[m] = sr;
      }
    }
    __syncthreads();
  }
}

// Position of every full index of M(Q) in the order in which the nested Horner scheme below
// consumes the coefficients (z from Q down, then x down, then y down).
template <int Q>
struct HornerOrder {
  int pos[nfull(Q) > 0 ? nfull(Q) : 1];
  constexpr HornerOrder() : pos() {
    int k = 0;
    for (int z = Q; z >= 0; --z)
      for (int x = Q - z; x >= 0; --x)
        for (int y = Q - z - x; y >= 0; --y) pos[full_index(Q, x, y, z)] = k++;
  }
};

template <int Q>
__device__ constexpr HornerOrder<Q> kHorner{};

// out[j][u] = sum_{|m| <= Q} c_m,u X_j^m for KU points j at once (nested Horner: y innermost,
// then x, then z), the coefficients C[W * k + u] stored in Horner order.  The row loops are
// kept as loops so that the coefficients are read from LDS as they are consumed.
template <int KU, int Q, int W, typename R>
__device__ inline void horner_u(const R* C, const R (&X)[KU], const R (&Y)[KU], const R (&Z)[KU],
                                R (&out)[KU][W]) {
  R pz[KU][W];
#pragma unroll
  for (int j = 0; j < KU; ++j)
#pragma unroll
    for (int u = 0; u < W; ++u) pz[j][u] = R(0);
  // the coefficients are consumed strictly in storage order, so the reads run two steps ahead
  // of the products across row and slab boundaries (C holds two zero entries of padding)
  R c0[W], c1[W];
#pragma unroll
  for (int u = 0; u < W; ++u) {
    c0[u] = C[u];
    c1[u] = C[W + u];
  }
  int idx = 0;
#pragma unroll 1
  for (int z = Q; z >= 0; --z) {
    R qx[KU][W];
#pragma unroll
    for (int j = 0; j < KU; ++j)
#pragma unroll
      for (int u = 0; u < W; ++u) qx[j][u] = R(0);
#pragma unroll 1
    for (int x = Q - z; x >= 0; --x) {
      R ry[KU][W];
#pragma unroll
      for (int j = 0; j < KU; ++j)
#pragma unroll
        for (int u = 0; u < W; ++u) ry[j][u] = R(0);
      const int n = Q - z - x + 1;
#pragma unroll 2
      for (int y = 0; y < n; ++y, ++idx) {
#pragma unroll
        for (int u = 0; u < W; ++u) {
          const R cv = c0[u];
          c0[u] = c1[u];
          c1[u] = C[(idx + 2) * W + u];
#pragma unroll
          for (int j = 0; j < KU; ++j) ry[j][u] = ry[j][u] * Y[j] + cv;
        }
      }
#pragma unroll
      for (int j = 0; j < KU; ++j)
#pragma unroll
        for (int u = 0; u < W; ++u) qx[j][u] = qx[j][u] * X[j] + ry[j][u];
    }
#pragma unroll
    for (int j = 0; j < KU; ++j)
#pragma unroll
      for (int u = 0; u < W; ++u) pz[j][u] = pz[j][u] * Z[j] + qx[j][u];
  }
#pragma unroll
  for (int j = 0; j < KU; ++j)
#pragma unroll
    for (int u = 0; u < W; ++u) out[j][u] = pz[j][u];
}

// The same sum for real values, with the whole nested scheme unrolled at compile time: every
// row, slab and total starts from its first term (no products with zero), and no registers
// are moved between loop iterations.  The coefficients are read from LDS in groups of kHG,
// each group while the previous one is consumed; scheduling barriers between the groups keep
// the compiler from moving every read to the top (which would hold them all in registers).
constexpr int kHG = 8;

template <int Q>
struct HornerSteps {
  // for position k of the Horner order: the row ends (fold into the slab sum) and the slab ends
  // (fold into the total); the first row of a slab and the first slab start their sums
  bool row_start[nfull(Q) > 0 ? nfull(Q) : 1], row_end[nfull(Q) > 0 ? nfull(Q) : 1];
  bool first_row[nfull(Q) > 0 ? nfull(Q) : 1], slab_end[nfull(Q) > 0 ? nfull(Q) : 1];
  bool first_slab[nfull(Q) > 0 ? nfull(Q) : 1];
  constexpr HornerSteps() : row_start(), row_end(), first_row(), slab_end(), first_slab() {
    int k = 0;
    for (int z = Q; z >= 0; --z)
      for (int x = Q - z; x >= 0; --x)
        for (int y = Q - z - x; y >= 0; --y) {
          row_start[k] = y == Q - z - x;
          row_end[k] = y == 0;
          first_row[k] = x == Q - z;
          slab_end[k] = y == 0 && x == 0;
          first_slab[k] = z == Q;
          ++k;
        }
  }
};

template <int Q>
__device__ constexpr HornerSteps<Q> kSteps{};

template <int KU, int Q, typename R>
__device__ inline void horner_unrolled(const R* C, const R (&X)[KU], const R (&Y)[KU], const R (&Z)[KU],
                                       R (&out)[KU][1]) {
  constexpr int NP = nfull(Q);
  constexpr int G = kHG;
  constexpr int NG = (NP + G - 1) / G;
  constexpr HornerSteps<Q> S{};
  R pz[KU], qx[KU], ry[KU];
  R cb[2][G];
#pragma unroll
  for (int i = 0; i < G; ++i) cb[0][i] = i < NP ? C[i] : R(0);
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    if (g + 1 < NG) {
#pragma unroll
      for (int i = 0; i < G; ++i)
        if ((g + 1) * G + i < NP) cb[(g + 1) & 1][i] = C[(g + 1) * G + i];
    }
#pragma unroll
    for (int i = 0; i < G; ++i) {
      const int k = g * G + i;
      if (k < NP) {
        const R c = cb[g & 1][i];
#pragma unroll
        for (int j = 0; j < KU; ++j) ry[j] = S.row_start[k] ? c : ry[j] * Y[j] + c;
        if (S.row_end[k]) {
#pragma unroll
          for (int j = 0; j < KU; ++j) qx[j] = S.first_row[k] ? ry[j] : qx[j] * X[j] + ry[j];
        }
        if (S.slab_end[k]) {
#pragma unroll
          for (int j = 0; j < KU; ++j) pz[j] = S.first_slab[k] ? qx[j] : pz[j] * Z[j] + qx[j];
        }
      }
    }
    // the group's products happen here, before the next group's reads are issued (the
    // compiler would otherwise place every product after the last read)
#pragma unroll
    for (int j = 0; j < KU; ++j) asm volatile("" : "+v"(ry[j]), "+v"(qx[j]), "+v"(pz[j]));
  }
  __builtin_amdgcn_sched_barrier(0);
  // the sums are used only under the callers' bounds checks; without this use here the
  // compiler sinks every product chain into those branches, past the grouped reads
#pragma unroll
  for (int j = 0; j < KU; ++j) {
    asm volatile("" : "+v"(pz[j]));
    out[j][0] = pz[j];
  }
}

// orders whose real potentials take the unrolled scheme: its code grows with N(p) times the
// targets per lane, and at p = 12 (455 coefficients) it ran 2.5x slower than the loop form
constexpr int kMaxUnrolledOrder = 9;

// One pass over the next KU * 64 targets of the box from s0 (each lane takes KU of them, 64
// apart): potentials and, for GRAD, gradients.  Returns the number of targets covered.
// The pass for the loop form of the evaluation (orders above the unrolled ones, complex values,
// gradients): each target's reads sit in its bounds check.  Grouping them ahead, as in pass()
// below, gained nothing with the loop form at p = 8 and made p = 12 slower.
template <int P, typename R, bool CPLX, bool GRAD, int KU, typename LG>
__device__ inline int pass_loop(const L2PArgs& a, const R* Lc, const LG& Lg, const R* xyz, int64_t s0, int64_t hi,
                                R cx, R cy, R cz, R ih) {
  constexpr int W = CPLX ? 2 : 1;
  const int64_t t0 = s0 + threadIdx.x;
  R X[KU], Y[KU], Z[KU];
#pragma unroll
  for (int j = 0; j < KU; ++j) {
    const int64_t s = t0 + (int64_t)j * kThreads;
    const bool ok = s < hi;
    X[j] = ok ? (xyz[3 * s + 0] - cx) * ih : R(0);
    Y[j] = ok ? (xyz[3 * s + 1] - cy) * ih : R(0);
    Z[j] = ok ? (xyz[3 * s + 2] - cz) * ih : R(0);
  }
  if (a.pot) {
    R v[KU][W];
    horner_u<KU, P, W, R>(Lc, X, Y, Z, v);
    R* pot = reinterpret_cast<R*>(a.pot);
#pragma unroll
    for (int j = 0; j < KU; ++j) {
      const int64_t s = t0 + (int64_t)j * kThreads;
      if (s < hi) {
#pragma unroll
        for (int u = 0; u < W; ++u) pot[s * W + u] = a.overwrite ? v[j][u] : pot[s * W + u] + v[j][u];
      }
    }
  }
  if constexpr (GRAD && P > 0 && !CPLX) {
    R g[3][KU][1];
    horner_u<KU, P - 1, 1, R>(Lg[0], X, Y, Z, g[0]);
    horner_u<KU, P - 1, 1, R>(Lg[1], X, Y, Z, g[1]);
    horner_u<KU, P - 1, 1, R>(Lg[2], X, Y, Z, g[2]);
    R* gout = reinterpret_cast<R*>(a.grad);
#pragma unroll
    for (int j = 0; j < KU; ++j) {
      const int64_t s = t0 + (int64_t)j * kThreads;
      if (s < hi) {
        const R sc = a.gscale ? reinterpret_cast<const R*>(a.gscale)[s] : R(1);
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) gout[3 * s + ax] += sc * ih * g[ax][j][0];
      }
    }
  }
  return KU * kThreads;
}

// The pass for real potentials with the unrolled evaluation (orders up to kMaxUnrolledOrder).
// Every read of a group is issued before any of it is used: lanes past the end read point s0
// (in range: s0 < hi) and drop the value, so no read sits in a branch of its own that waits for
// it.  The old potentials (when adding) are read after the evaluation, so they hold no
// registers during it.
template <int P, typename R, int KU, bool PRE = false>
__device__ inline int pass(const L2PArgs& a, const R* Lc, const R* xyz, int64_t s0, int64_t hi, R cx, R cy, R cz,
                           R ih, const R (*pre)[kMaxUnrolledU] = nullptr) {
  const int64_t t0 = s0 + threadIdx.x;
  const auto at = [&](int j) {
    const int64_t s = t0 + (int64_t)j * kThreads;
    return s < hi ? s : s0;
  };
  R X[KU], Y[KU], Z[KU];
#pragma unroll
  for (int j = 0; j < KU; ++j) {
    R x, y, z;
    if constexpr (PRE) {  // read at the start of the kernel
      x = pre[0][j];
      y = pre[1][j];
      z = pre[2][j];
    } else {
      const int64_t s = at(j);
      x = xyz[3 * s + 0];
      y = xyz[3 * s + 1];
      z = xyz[3 * s + 2];
    }
    const bool ok = t0 + (int64_t)j * kThreads < hi;
    X[j] = ok ? (x - cx) * ih : R(0);
    Y[j] = ok ? (y - cy) * ih : R(0);
    Z[j] = ok ? (z - cz) * ih : R(0);
  }
  R* pot = reinterpret_cast<R*>(a.pot);
  if (pot) {
    R v[KU][1];
    horner_unrolled<KU, P, R>(Lc, X, Y, Z, v);
    if (!a.overwrite) {
#pragma unroll
      for (int j = 0; j < KU; ++j) v[j][0] += pot[at(j)];
    }
#pragma unroll
    for (int j = 0; j < KU; ++j)
      if (t0 + (int64_t)j * kThreads < hi) pot[at(j)] = v[j][0];
  }
  return KU * kThreads;
}

// The unrolled evaluation with grouped reads where it applies (a pass of 8 targets per lane
// becomes one of 5), else the loop form.
template <int P, typename R, bool CPLX, bool GRAD, int KU, typename LG>
__device__ inline int any_pass(const L2PArgs& a, const R* Lc, const LG& Lg, const R* xyz, int64_t s0, int64_t hi, R cx,
                               R cy, R cz, R ih) {
  if constexpr (!CPLX && !GRAD && P <= kMaxUnrolledOrder)
    return pass<P, R, (KU < kMaxUnrolledU ? KU : kMaxUnrolledU)>(a, Lc, xyz, s0, hi, cx, cy, cz, ih);
  else return pass_loop<P, R, CPLX, GRAD, KU>(a, Lc, Lg, xyz, s0, hi, cx, cy, cz, ih);
}

// Rows k = lane + i * 64 (i < NK) of a level's sparse decompression: out[i] = theta~_k for kept
// rows (k < nc), and sum_e val[e] src[col[e]] over the row's entries otherwise.  The row bounds
// of all NK rows, then the first PRE entries of every row, are read before any of them is
// used, so a lane waits for two memory round trips instead of one per entry (rows longer than
// PRE finish in a loop).  About 24 entries per lane are read ahead.
template <int NK>
constexpr int kPre = 24 / NK > 8 ? 8 : (24 / NK < 2 ? 2 : 24 / NK);

template <int NK, int W, int PRE = kPre<NK * W>>
__device__ inline void sparse_rows(const int32_t* rp, const int32_t* col, const double* val, const double* src,
                                   int nc, int np, double (&out)[NK][W]) {
  int e0[NK], e1[NK];
#pragma unroll
  for (int i = 0; i < NK; ++i) {
    const int k = threadIdx.x + i * kThreads;
    const bool dec = k >= nc && k < np;
    const int kk = k < np ? k : 0;
    const int lo = rp[kk], hi = rp[kk + 1];
    e0[i] = dec ? lo : 0;
    e1[i] = dec ? hi : 0;
  }
  int cj[NK][PRE];
  double cv[NK][PRE];
#pragma unroll
  for (int i = 0; i < NK; ++i)
#pragma unroll
    for (int t = 0; t < PRE; ++t) {
      const int e = e0[i] + t < e1[i] ? e0[i] + t : 0;  // the arrays hold at least one entry
      cj[i][t] = col[e];
      cv[i][t] = val[e];
    }
#pragma unroll
  for (int i = 0; i < NK; ++i) {
    const int k = threadIdx.x + i * kThreads;
#pragma unroll
    for (int u = 0; u < W; ++u) out[i][u] = k < nc ? src[k * W + u] : 0.0;
#pragma unroll
    for (int t = 0; t < PRE; ++t)
      if (e0[i] + t < e1[i]) {
#pragma unroll
        for (int u = 0; u < W; ++u) out[i][u] += cv[i][t] * src[cj[i][t] * W + u];
      }
    for (int e = e0[i] + PRE; e < e1[i]; ++e) {
      const int j = col[e];
      const double v = val[e];
#pragma unroll
      for (int u = 0; u < W; ++u) out[i][u] += v * src[j * W + u];
    }
  }
}

template <int P, typename R, bool CPLX, bool GRAD>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kWavesPerEU))) void l2p_kernel(L2PArgs a) {
  constexpr int NP = nfull(P);
  constexpr int NG = GRAD ? nfull(P - 1) : 0;
  constexpr int W = CPLX ? 2 : 1;
  __shared__ double Ld[NP * W];
  __shared__ R Lc[(NP + 2) * W];  // + 2 zero entries read ahead by horner_u
  __shared__ R Lg[3][((NG > 0 ? NG : 1) + 2) * W];
  const int64_t b = blockIdx.x;
  // points of the box: workgroup y of the box takes the chunks y, y + gridDim.y, ... of ch
  // points (large boxes of coarse levels are spread over several workgroups)
  const int64_t ch = a.chunk > 0 ? a.chunk : kChunk;
  int64_t lo = a.range[2 * b], hi = a.range[2 * b + 1];
  lo = lo < 0 ? 0 : (lo > a.n_pts ? a.n_pts : lo);
  hi = hi < lo ? lo : (hi > a.n_pts ? a.n_pts : hi);
  if (lo + (int64_t)blockIdx.y * ch >= hi) return;  // uniform: no points for this workgroup
  constexpr bool UNR = !CPLX && !GRAD && P <= kMaxUnrolledOrder;
  const R* xyz = reinterpret_cast<const R*>(a.xyz);
  // the unrolled form reads the coordinates of its first pass here, so that they arrive while
  // the locals are read and decompressed (lanes past the chunk read its first point)
  const int64_t f0 = lo + (int64_t)blockIdx.y * ch, f1 = f0 + ch < hi ? f0 + ch : hi;
  R pre[3][kMaxUnrolledU];
  const bool use_pre = UNR && f1 - f0 > 2 * kThreads;  // small leaves keep their narrow passes
  if (use_pre) {
#pragma unroll
    for (int j = 0; j < kMaxUnrolledU; ++j) {
      const int64_t s = f0 + threadIdx.x + (int64_t)j * kThreads;
      const int64_t sc = s < f1 ? s : f0;
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) pre[ax][j] = xyz[3 * sc + ax];
    }
  }
  int lev = a.level[b];
  lev = lev < 0 ? 0 : (lev >= a.n_levels ? a.n_levels - 1 : lev);
  const double h = a.level_h[lev];
  const int nc = a.nc;
  const R* loc = reinterpret_cast<const R*>(a.local) + b * (int64_t)nc * W;
  constexpr int NK = (NP + kThreads - 1) / kThreads;  // full indices per lane
  if constexpr (NK > 4) {  // high orders: the plain loop (grouping the reads was slower at p = 12)
    for (int k = threadIdx.x; k < nc * W; k += kThreads) Ld[k] = (double)loc[k];
  } else {  // all reads of the box's locals first (the last lanes re-read entry 0), then the LDS stores
    constexpr int NL = (NP * W + kThreads - 1) / kThreads;
    R lv[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const int k = threadIdx.x + i * kThreads;
      lv[i] = loc[k < nc * W ? k : 0];
    }
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const int k = threadIdx.x + i * kThreads;
      if (k < nc * W) Ld[k] = (double)lv[i];
    }
  }
  if (threadIdx.x < 2 * W) {
    Lc[NP * W + threadIdx.x] = R(0);
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) Lg[ax][(NG > 0 ? NG : 1) * W + threadIdx.x] = R(0);
  }
  __syncthreads();
  // decompression L~_m = sum_j M~[m][j] theta~_j (kept rows are theta~ itself): one sparse row
  // of the level's M~ per full index, read from the kept prefix only, so no level waits for
  // another
  const int32_t* rp = a.dec_ptr + (int64_t)lev * (NP + 1);
  // the coefficient of full index k (decompressed value lv) in Horner order, scaled by 1 / k!,
  // and for GRAD the coefficients of its derivatives
  const auto put = [&](int k, const double (&lv)[W]) {
    const double f = kDecode<P>.inv_fact[k];
    const int hk = kHorner<P>.pos[k];
#pragma unroll
    for (int u = 0; u < W; ++u) Lc[hk * W + u] = (R)(lv[u] * f);
    if constexpr (GRAD) {
      // d/dX_ax of L_m X^m / m!: the coefficient of X^(m - e_ax) is L_m / (m - e_ax)!
      const int mm[3] = {kDecode<P>.x[k], kDecode<P>.y[k], kDecode<P>.z[k]};
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        if (mm[ax] == 0) continue;
        const int d0 = mm[0] - (ax == 0), d1 = mm[1] - (ax == 1), d2 = mm[2] - (ax == 2);
        const int g = kHorner<P - 1>.pos[full_index(P - 1, d0, d1, d2)];
        const double fg = f * mm[ax];
#pragma unroll
        for (int u = 0; u < W; ++u) Lg[ax][g * W + u] = (R)(lv[u] * fg);
      }
    }
  };
  if constexpr (NK <= 4) {
    double lvs[NK][W];
    // (about 12 entries per lane read ahead where the first pass's coordinates are in flight)
    constexpr int PRE = UNR ? (12 / NK > 8 ? 8 : (12 / NK < 2 ? 2 : 12 / NK)) : kPre<NK * W>;
    sparse_rows<NK, W, PRE>(rp, a.dec_col, a.dec_val, Ld, nc, NP, lvs);
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      const int k = threadIdx.x + i * kThreads;
      if (k >= NP) break;
      put(k, lvs[i]);
    }
  } else {  // high orders: too many rows per lane to read ahead
    for (int k = threadIdx.x; k < NP; k += kThreads) {
      double lv[W];
#pragma unroll
      for (int u = 0; u < W; ++u) lv[u] = k < nc ? Ld[k * W + u] : 0.0;
      if (k >= nc) {
        for (int e = rp[k]; e < rp[k + 1]; ++e) {
          const int j = a.dec_col[e];
          const double v = a.dec_val[e];
#pragma unroll
          for (int u = 0; u < W; ++u) lv[u] += v * Ld[j * W + u];
        }
      }
      put(k, lv);
    }
  }
  __syncthreads();
  const double cen[3] = {a.center[3 * b], a.center[3 * b + 1], a.center[3 * b + 2]};
  const R cx = (R)cen[0], cy = (R)cen[1], cz = (R)cen[2], ih = (R)(a.xsign / h);
  constexpr int KM = kMaxU<CPLX, GRAD>;
  int64_t first_end = f0;  // the first pass, with the coordinates read at the start
  if constexpr (UNR) {
    if (use_pre) {
      if (f1 - f0 <= 4 * kThreads) first_end += pass<P, R, 4, true>(a, Lc, xyz, f0, f1, cx, cy, cz, ih, pre);
      else first_end += pass<P, R, kMaxUnrolledU, true>(a, Lc, xyz, f0, f1, cx, cy, cz, ih, pre);
    }
  }
  for (int64_t c0 = f0; c0 < hi; c0 += (int64_t)gridDim.y * ch) {  // uniform
    const int64_t c1 = c0 + ch < hi ? c0 + ch : hi;
    for (int64_t s0 = c0 == f0 ? first_end : c0; s0 < c1;) {  // passes sized to the points left in the chunk
      const int64_t left = c1 - s0;
      int step;
      if (left <= kThreads) step = any_pass<P, R, CPLX, GRAD, 1>(a, Lc, Lg, xyz, s0, c1, cx, cy, cz, ih);
      else if (left <= 2 * kThreads) step = any_pass<P, R, CPLX, GRAD, 2>(a, Lc, Lg, xyz, s0, c1, cx, cy, cz, ih);
      else if (KM == 4 || left <= 4 * kThreads) step = any_pass<P, R, CPLX, GRAD, 4>(a, Lc, Lg, xyz, s0, c1, cx, cy, cz, ih);
      else step = any_pass<P, R, CPLX, GRAD, KM>(a, Lc, Lg, xyz, s0, c1, cx, cy, cz, ih);
      s0 += step;
    }
  }
}

template <int P>
int launch_l2p_p(const L2PArgs& a_in, int dtype, hipStream_t s) {
  // workgroups per box: enough that the average box gets one per kChunk targets; with few
  // boxes (coarse levels), more and smaller chunks (at least 2 kThreads points, a multiple of
  // kThreads) so that the launch has about kFillGroups workgroups
  constexpr int64_t kFillGroups = 4096;
  const int64_t per_box = a_in.n_box > 0 ? (a_in.n_pts + a_in.n_box - 1) / a_in.n_box : 1;
  int64_t ny = (per_box + kChunk - 1) / kChunk, ch = kChunk;
  const int64_t fill = a_in.n_box > 0 ? std::min<int64_t>((kFillGroups + a_in.n_box - 1) / a_in.n_box, per_box / (2 * kThreads)) : 0;
  if (fill > ny) {
    ch = ((per_box + fill - 1) / fill + kThreads - 1) / kThreads * kThreads;
    ny = (per_box + ch - 1) / ch;
  }
  ny = std::max<int64_t>(1, std::min<int64_t>(1024, ny));
  L2PArgs a = a_in;
  a.chunk = ch;
  dim3 g((unsigned)a.n_box, (unsigned)ny), t(kThreads);
  const bool grad = a.grad != nullptr;
  switch (dtype) {
    case FMM_F64:
      if (grad) hipLaunchKernelGGL((l2p_kernel<P, double, false, true>), g, t, 0, s, a);
      else hipLaunchKernelGGL((l2p_kernel<P, double, false, false>), g, t, 0, s, a);
      break;
    case FMM_F32:
      if (grad) hipLaunchKernelGGL((l2p_kernel<P, float, false, true>), g, t, 0, s, a);
      else hipLaunchKernelGGL((l2p_kernel<P, float, false, false>), g, t, 0, s, a);
      break;
    case FMM_C128: hipLaunchKernelGGL((l2p_kernel<P, double, true, false>), g, t, 0, s, a); break;
    case FMM_C64: hipLaunchKernelGGL((l2p_kernel<P, float, true, false>), g, t, 0, s, a); break;
    default: return fail(FMM_EINVAL, "dtype");
  }
  FMM_HIP_CHECK(hipGetLastError());
  return FMM_OK;
}

}  // namespace detail_l2p

#define FMM_INSTANTIATE_L2P(P) \
  int launch_l2p_order_##P(const L2PArgs& a, int dtype, hipStream_t s) { \
    return detail_l2p::launch_l2p_p<P>(a, dtype, s); \
  }

}  // namespace fmm
