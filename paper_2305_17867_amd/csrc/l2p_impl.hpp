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
// feeds KU fused multiply-adds.  KU is chosen per pass from the points left (1, 2, 4 or 8),
// so that a pass is not mostly empty: small leaves of adaptive trees take KU = 1, and boxes
// of a few more than 256 points one pass of KU = 8 instead of two.  The index decode (full index -> (x, y, z)) comes from
// compile-time tables, and the recursion terms are unrolled so that no per-lane array is
// indexed dynamically.
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
// leave fewer registers
template <bool CPLX, bool GRAD>
constexpr int kMaxU = (CPLX || GRAD) ? 4 : 8;
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

// One pass over the next KU * 64 targets of the box from s0 (each lane takes KU of them, 64
// apart): potentials and, for GRAD, gradients.  Returns the number of targets covered.
template <int P, typename R, bool CPLX, bool GRAD, int KU, typename LG>
__device__ inline int pass(const L2PArgs& a, const R* Lc, const LG& Lg, const R* xyz, int64_t s0, int64_t hi, R cx,
                           R cy, R cz, R ih) {
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
  int lev = a.level[b];
  lev = lev < 0 ? 0 : (lev >= a.n_levels ? a.n_levels - 1 : lev);
  const double h = a.level_h[lev];
  const int nc = a.nc;
  const R* loc = reinterpret_cast<const R*>(a.local) + b * (int64_t)nc * W;
  for (int k = threadIdx.x; k < nc * W; k += kThreads) Ld[k] = (double)loc[k];
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
  }
  __syncthreads();
  const double cen[3] = {a.center[3 * b], a.center[3 * b + 1], a.center[3 * b + 2]};
  const R* xyz = reinterpret_cast<const R*>(a.xyz);
  const R cx = (R)cen[0], cy = (R)cen[1], cz = (R)cen[2], ih = (R)(a.xsign / h);
  constexpr int KM = kMaxU<CPLX, GRAD>;
  for (int64_t c0 = lo + (int64_t)blockIdx.y * ch; c0 < hi; c0 += (int64_t)gridDim.y * ch) {  // uniform
    const int64_t c1 = c0 + ch < hi ? c0 + ch : hi;
    for (int64_t s0 = c0; s0 < c1;) {  // passes sized to the points left in the chunk
      const int64_t left = c1 - s0;
      int step;
      if (left <= kThreads) step = pass<P, R, CPLX, GRAD, 1>(a, Lc, Lg, xyz, s0, c1, cx, cy, cz, ih);
      else if (left <= 2 * kThreads) step = pass<P, R, CPLX, GRAD, 2>(a, Lc, Lg, xyz, s0, c1, cx, cy, cz, ih);
      else if (KM == 4 || left <= 4 * kThreads) step = pass<P, R, CPLX, GRAD, 4>(a, Lc, Lg, xyz, s0, c1, cx, cy, cz, ih);
      else step = pass<P, R, CPLX, GRAD, KM>(a, Lc, Lg, xyz, s0, c1, cx, cy, cz, ih);
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
