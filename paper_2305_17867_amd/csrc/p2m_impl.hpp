// Compressed P2M (Sec. 3.4): per box, the Cartesian moments
//   alpha~_q = sum_s w_s X_s^q / q!,   X_s = (c - y_s) / h        (eq. mpole, scaled t = 1/h)
// followed by the compression beta~ = M~^T alpha~ (eq. define_beta_multipole; Thm.
// mult_decompression: back substitution over the PDE recursion, O(p^3)).
//
// Layout of the work: one workgroup (4 wavefronts) per box.  The q set M(p) is cut into
// chunks of at most 32 (real) / 16 (complex) coefficients; each wavefront owns every
// fourth chunk.  Lanes stride over the box's points (coalesced loads), keep the chunk's
// partial sums in registers, and a reduce-scatter over the wavefront leaves one sum per
// lane, which is stored to LDS.  The compression then runs in LDS level by level in m_z
// (descending) and the kept prefix is written out.
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

template <typename R>
__device__ inline R load_real(const void* p, int64_t i) {
  return reinterpret_cast<const R*>(p)[i];
}

// Accumulate chunk [Q0, Q0 + QN) of the full order for one point.
template <int P, int Q0, int QN, int QP, typename R, bool CPLX>
__device__ inline void accumulate_chunk(R (&acc)[2][QP], const R (&px)[P + 1], const R (&py)[P + 1],
                                        const R (&pz)[P + 1], R wr, R wi) {
  constexpr FullIdx<P> I{};
  // the weight times the (z, x) factor is shared by a row of the chunk (the compiler computes
  // it once per row), so each coefficient costs one fused multiply-add per component
#pragma unroll
  for (int k = 0; k < QN; ++k) {
    const int q = Q0 + k;
    const R zx = pz[I.z[q]] * px[I.x[q]];
    acc[0][k] += (wr * zx) * py[I.y[q]];
    if constexpr (CPLX) acc[1][k] += (wi * zx) * py[I.y[q]];
  }
}

template <int P, typename R, bool CPLX, int QMAX>
struct Chunks {
  static constexpr int NP = nfull(P);
  // number of chunks: a multiple of the wavefront count when there is enough work, so that
  // the wavefronts of a box get the same number of chunks
  static constexpr int N0 = (NP + QMAX - 1) / QMAX;
  static constexpr int N = N0 >= kWaves ? (N0 + kWaves - 1) / kWaves * kWaves : N0;
  static constexpr int Q = (NP + N - 1) / N;  // balanced chunk size <= QMAX
  static constexpr int M = Q <= 1 ? 0 : Q <= 2 ? 1 : Q <= 4 ? 2 : Q <= 8 ? 3 : Q <= 16 ? 4 : Q <= 32 ? 5 : 6;
  static constexpr int QP = 1 << M;
};

template <int P, typename R, bool CPLX, int CH>
__device__ inline void run_chunk(const P2MArgs& a, int64_t lo, int64_t hi, const double (&cen)[3],
                                 double inv_h, int lane, double* alpha) {
  constexpr int QMAX = CPLX ? 16 : 32;
  using C = Chunks<P, R, CPLX, QMAX>;
  constexpr int Q0 = CH * C::Q;
  constexpr int QN = (Q0 + C::Q <= C::NP) ? C::Q : C::NP - Q0;
  R acc[2][C::QP];
#pragma unroll
  for (int k = 0; k < C::QP; ++k) acc[0][k] = acc[1][k] = R(0);
  const R* xyz = reinterpret_cast<const R*>(a.xyz);
  const R cx = (R)cen[0], cy = (R)cen[1], cz = (R)cen[2], ih = (R)inv_h;
  for (int64_t s = lo + lane; s < hi; s += 64) {
    const R X = (cx - xyz[s * 3 + 0]) * ih;
    const R Y = (cy - xyz[s * 3 + 1]) * ih;
    const R Z = (cz - xyz[s * 3 + 2]) * ih;
    R wr, wi = R(0);
    if constexpr (CPLX) {
      wr = reinterpret_cast<const R*>(a.w)[2 * s];
      wi = reinterpret_cast<const R*>(a.w)[2 * s + 1];
    } else {
      wr = reinterpret_cast<const R*>(a.w)[s];
    }
    R px[P + 1], py[P + 1], pz[P + 1];
    px[0] = py[0] = pz[0] = R(1);
#pragma unroll
    for (int k = 1; k <= P; ++k) {
      const R inv = R(1) / R(k);
      px[k] = px[k - 1] * (X * inv);
      py[k] = py[k - 1] * (Y * inv);
      pz[k] = pz[k - 1] * (Z * inv);
    }
    accumulate_chunk<P, Q0, QN, C::QP, R, CPLX>(acc, px, py, pz, wr, wi);
  }
  R re = wave_reduce_scatter<C::M, R>(acc[0], lane);
  R im = R(0);
  if constexpr (CPLX) im = wave_reduce_scatter<C::M, R>(acc[1], lane);
  const int k = rs_index<C::M>(lane);
  if (rs_owner<C::M>(lane) && k < QN) {
    if constexpr (CPLX) {
      alpha[2 * (Q0 + k)] = (double)re;
      alpha[2 * (Q0 + k) + 1] = (double)im;
    } else {
      alpha[Q0 + k] = (double)re;
    }
  }
}

template <int P, typename R, bool CPLX, int CH, int NCH>
__device__ inline void run_chunks(const P2MArgs& a, int64_t lo, int64_t hi, const double (&cen)[3],
                                  double inv_h, int wave, int lane, double* alpha) {
  if constexpr (CH < NCH) {
    if (CH % kWaves == wave) run_chunk<P, R, CPLX, CH>(a, lo, hi, cen, inv_h, lane, alpha);
    run_chunks<P, R, CPLX, CH + 1, NCH>(a, lo, hi, cen, inv_h, wave, lane, alpha);
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

// occupancy hint: real FP64 at p = 8 fits 80 VGPRs (6 wavefronts per SIMD) without spills
// (the chunk layouts of the other orders spill under it); the other forms keep the compiler's
// own budget
template <int P, typename R, bool CPLX>
constexpr int p2m_waves_hint() {
  return (P == 8 && sizeof(R) == 8 && !CPLX) ? 6 : 1;
}

template <int P, typename R, bool CPLX>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(p2m_waves_hint<P, R, CPLX>()))) void p2m_kernel(P2MArgs a) {
  constexpr int NP = nfull(P);
  __shared__ double alpha[NP * (CPLX ? 2 : 1)];
  const int64_t b = blockIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
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
  constexpr int QMAX = CPLX ? 16 : 32;
  constexpr int NCH = Chunks<P, R, CPLX, QMAX>::N;
  run_chunks<P, R, CPLX, 0, NCH>(a, lo, hi, cen, a.xsign / h, wave, lane, alpha);
  __syncthreads();
  compress_lds<P, CPLX>(alpha, a.rec, a.c, h);
  // the kept set is the prefix [0, nc) of the full order
  const int nc = a.nc;
  if (gridDim.y > 1) {
    constexpr int W = CPLX ? 2 : 1;
    double* part = a.part + (b * gridDim.y + blockIdx.y) * (int64_t)nc * W;
    for (int k = threadIdx.x; k < W * nc; k += blockDim.x) part[k] = alpha[k];
    return;
  }
  if constexpr (CPLX) {
    R* out = reinterpret_cast<R*>(a.out) + b * (int64_t)nc * 2;
    for (int k = threadIdx.x; k < 2 * nc; k += blockDim.x) out[k] = (R)alpha[k];
  } else {
    R* out = reinterpret_cast<R*>(a.out) + b * (int64_t)nc;
    for (int k = threadIdx.x; k < nc; k += blockDim.x) out[k] = (R)alpha[k];
  }
}

template <int P>
int launch_p2m_p(const P2MArgs& a, int dtype, hipStream_t s) {
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
