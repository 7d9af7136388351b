// Direct sum eq. (1): phi(x) = sum_y G(x - y) w(y), terms with x == y skipped.
// Sources are staged through LDS in tiles of the block size.  Each target is taken by `split`
// adjacent lanes (one when there are many targets; up to a wavefront when there are few, so
// that the launch still fills the chip), each summing every split-th source of a tile; the
// lanes' sums are added by a butterfly of lane exchanges in a fixed order.
// The near field (P2P) is the same sum restricted, per target box, to the sources of its
// neighbour boxes: one workgroup per (target box, chunk of up to 512 targets).
#include <cmath>

#include "../../include/fmm.h"
#include "common.hpp"
#include "device_util.hpp"
#include "kernels.hpp"

namespace fmm {

namespace {

constexpr int kThreads = 256;

// 1 / sqrt(v), v > 0: in double precision the hardware estimate refined by two Newton steps
// y <- y (3 - v y^2) / 2 (each roughly squares the relative error); in single precision the
// hardware result as it is
__device__ inline double inv_sqrt(double v) {
  double y = __builtin_amdgcn_rsq(v);
#pragma unroll
  for (int it = 0; it < 2; ++it) y = fma(0.5 * y, fma(-v * y, y, 1.0), y);
  return y;
}
__device__ inline float inv_sqrt(float v) {
  return __builtin_amdgcn_rsqf(v);  // the hardware result is within about an ulp in FP32
}

// acc += G(d) w for one source at offset d = x - y; d = 0 adds nothing (1/r is taken as 0
// there, which zeroes every kernel's term without a branch).  K is the kernel (compile time).
template <typename R, bool CPLX, int K, typename T>
__device__ inline void add_green(T& acc, R prm, R dx, R dy, R dz, const T& w) {
  const R inv4pi = R(1.0 / (4.0 * M_PI));
  const R r2 = dx * dx + dy * dy + dz * dz;
  const R ir0 = inv_sqrt(r2);
  const R ir = r2 > R(0) ? ir0 : R(0);
  if constexpr (CPLX) {
    // Helmholtz exp(i k r) / (4 pi r)
    const R r = r2 * ir;
    R sn, cs;
    if constexpr (sizeof(R) == 8) sincos(prm * r, &sn, &cs);
    else sincosf(prm * r, &sn, &cs);
    const R g = inv4pi * ir;
    const T G(g * cs, g * sn);
    acc += G * w;
  } else if constexpr (K == FMM_LAPLACE) {
    acc += (inv4pi * ir) * w;
  } else if constexpr (K == FMM_YUKAWA) {
    const R r = r2 * ir;
    acc += (exp(-prm * r) * inv4pi * ir) * w;
  } else {  // biharmonic: G = r
    acc += (r2 * ir) * w;
  }
}

template <typename R>
__device__ inline R lane_xor(R v, int m) { return shfl_xor_d(v, m); }
template <typename R>
__device__ inline Cx<R> lane_xor(Cx<R> v, int m) { return {shfl_xor_d(v.re, m), shfl_xor_d(v.im, m)}; }

// One staged source: position and weight side by side, so that the inner loop reads it with
// 128-bit LDS loads (two for FP64, one for FP32) instead of one load per component.
template <typename R, bool CPLX>
struct alignas(16) Staged;
template <typename R>
struct alignas(16) Staged<R, false> {
  R x, y, z, w;
};
template <typename R>
struct alignas(16) Staged<R, true> {
  R x, y, z, pad;
  Cx<R> w;
};

template <typename R, bool CPLX, int K>
__global__ __launch_bounds__(kThreads) void direct_kernel(DirectArgs a) {
  using T = typename Val<R, CPLX>::T;
  __shared__ Staged<R, CPLX> st[kThreads];
  const int split = a.split;
  const int ls = threadIdx.x & (split - 1);  // lane within the target's group
  const int64_t t = (int64_t)blockIdx.x * (kThreads / split) + threadIdx.x / split;
  const R* tg = reinterpret_cast<const R*>(a.tgt);
  const R* sr = reinterpret_cast<const R*>(a.src);
  const T* w = reinterpret_cast<const T*>(a.w);
  R x = 0, y = 0, z = 0;
  if (t < a.n_tgt) {
    x = tg[3 * t];
    y = tg[3 * t + 1];
    z = tg[3 * t + 2];
  }
  T acc{};
  const R prm = (R)a.param;
  for (int64_t base = 0; base < a.n_src; base += kThreads) {
    __syncthreads();
    const int64_t j = base + threadIdx.x;
    if (j < a.n_src) {
      Staged<R, CPLX> v;
      v.x = sr[3 * j];
      v.y = sr[3 * j + 1];
      v.z = sr[3 * j + 2];
      if constexpr (CPLX) v.pad = R(0);
      v.w = w[j];
      st[threadIdx.x] = v;
    }
    __syncthreads();
    const int cnt = (int)((a.n_src - base) < kThreads ? (a.n_src - base) : kThreads);
    for (int k = ls; k < cnt; k += split) {
      const Staged<R, CPLX> v = st[k];
      add_green<R, CPLX, K>(acc, prm, x - v.x, y - v.y, z - v.z, v.w);
    }
  }
  for (int m = 1; m < split; m <<= 1) acc += lane_xor(acc, m);  // all lanes active here
  if (ls == 0 && t < a.n_tgt) reinterpret_cast<T*>(a.pot)[t] = acc;
}

__device__ inline void clamp_range(const int64_t* rng, int64_t b, int64_t n, int64_t& lo, int64_t& hi) {
  lo = rng[2 * b];
  hi = rng[2 * b + 1];
  lo = lo < 0 ? 0 : (lo > n ? n : lo);
  hi = hi < lo ? lo : (hi > n ? n : hi);
}

// Targets [t0, t1) of one box against the sources of its neighbour boxes.  The sources of the
// list are one stream: a scan of the boxes' point counts (a segment of up to kThreads list
// entries at a time) maps a stream position to its box, so every staged tile holds kThreads
// sources however small the boxes are.  Thread layout: `split` consecutive lanes share a target
// and take every split-th source of a tile (their sums are combined by butterfly shuffles at
// the end); KT targets per thread, kThreads / split apart.
template <typename R, bool CPLX, int K, int KT>
__device__ inline void p2p_chunk(const P2PArgs& a, int64_t t0, int64_t t1, int64_t e0, int64_t e1, int split,
                                 Staged<R, CPLX>* st, int64_t* s_lo, int64_t* s_cum) {
  using T = typename Val<R, CPLX>::T;
  const R* tg = reinterpret_cast<const R*>(a.tgt);
  const R* sr = reinterpret_cast<const R*>(a.src);
  const T* w = reinterpret_cast<const T*>(a.w);
  const R prm = (R)a.param;
  const int tid = threadIdx.x;
  const int tl = tid / split, sp = tid % split, per = kThreads / split;
  R x[KT], y[KT], z[KT];
  T acc[KT];
#pragma unroll
  for (int j = 0; j < KT; ++j) {
    const int64_t t = t0 + tl + (int64_t)j * per;
    x[j] = y[j] = z[j] = R(0);
    if (t < t1) {
      x[j] = tg[3 * t];
      y[j] = tg[3 * t + 1];
      z[j] = tg[3 * t + 2];
    }
    acc[j] = T{};
  }
  for (int64_t seg = e0; seg < e1; seg += kThreads) {
    const int ns = (int)((e1 - seg) < kThreads ? (e1 - seg) : kThreads);
    int64_t lo = 0, cnt = 0;
    if (tid < ns) {
      const int sb = a.nbr[seg + tid];
      if (sb >= 0 && sb < a.n_box) {
        int64_t hi;
        clamp_range(a.src_range, sb, a.n_src, lo, hi);
        cnt = hi - lo;
      }
    }
    __syncthreads();  // the previous segment's tables are no longer read
    s_lo[tid] = lo;
    s_cum[tid] = cnt;
    __syncthreads();
    for (int off = 1; off < kThreads; off <<= 1) {  // inclusive scan of the counts
      const int64_t v = tid >= off ? s_cum[tid - off] : 0;
      __syncthreads();
      s_cum[tid] += v;
      __syncthreads();
    }
    const int64_t total = s_cum[kThreads - 1];
    for (int64_t base = 0; base < total; base += kThreads) {
      __syncthreads();  // the previous tile has been used
      const int64_t f = base + tid;
      if (f < total) {
        int l = 0, h = ns - 1;  // first entry whose inclusive count exceeds f
        while (l < h) {
          const int m = (l + h) >> 1;
          if (s_cum[m] > f) h = m;
          else l = m + 1;
        }
        const int64_t j = s_lo[l] + (f - (l > 0 ? s_cum[l - 1] : 0));
        Staged<R, CPLX> v;
        v.x = sr[3 * j];
        v.y = sr[3 * j + 1];
        v.z = sr[3 * j + 2];
        if constexpr (CPLX) v.pad = R(0);
        v.w = w[j];
        st[tid] = v;
      }
      __syncthreads();
      const int n = (int)((total - base) < kThreads ? (total - base) : kThreads);
#pragma unroll 4
      for (int k = sp; k < n; k += split) {
        const Staged<R, CPLX> v = st[k];
#pragma unroll
        for (int j = 0; j < KT; ++j) add_green<R, CPLX, K>(acc[j], prm, x[j] - v.x, y[j] - v.y, z[j] - v.z, v.w);
      }
    }
  }
  // combine the split lanes of each target; a target box may be listed several times with
  // different source lists, and those entries run in parallel: the sums are added atomically
  for (int m = 1; m < split; m <<= 1) {
#pragma unroll
    for (int j = 0; j < KT; ++j) {
      if constexpr (CPLX) {
        acc[j].re += shfl_xor_d(acc[j].re, m);
        acc[j].im += shfl_xor_d(acc[j].im, m);
      } else {
        acc[j] += shfl_xor_d(acc[j], m);
      }
    }
  }
  R* pot = reinterpret_cast<R*>(a.pot);
#pragma unroll
  for (int j = 0; j < KT; ++j) {
    const int64_t t = t0 + tl + (int64_t)j * per;
    if (sp == 0 && t < t1) {
      if constexpr (CPLX) {
        atomicAdd(pot + 2 * t, acc[j].re);
        atomicAdd(pot + 2 * t + 1, acc[j].im);
      } else {
        atomicAdd(pot + t, acc[j]);
      }
    }
  }
}

template <typename R, bool CPLX, int K>
__global__ __launch_bounds__(kThreads) void p2p_kernel(P2PArgs a) {
  using T = typename Val<R, CPLX>::T;
  __shared__ Staged<R, CPLX> st[kThreads];
  __shared__ int64_t s_lo[kThreads], s_cum[kThreads];
  const int tb = a.tbox[blockIdx.x];
  if (tb < 0 || tb >= a.n_box) return;  // uniform
  int64_t tlo, thi;
  clamp_range(a.tgt_range, tb, a.n_tgt, tlo, thi);
  // the list range, clamped to the list (the CSR pointers are device data)
  int64_t e0 = a.nbr_ptr[blockIdx.x], e1 = a.nbr_ptr[blockIdx.x + 1];
  e0 = e0 < 0 ? 0 : (e0 > a.n_nbr ? a.n_nbr : e0);
  e1 = e1 < e0 ? e0 : (e1 > a.n_nbr ? a.n_nbr : e1);
  // workgroup y takes the chunks y, y + gridDim.y, ... of 2 kThreads targets; a chunk of more
  // than kThreads targets is taken two per thread, a smaller one by as many lanes per target
  // (a power of two up to 16) as fill the workgroup
  for (int64_t t0 = tlo + (int64_t)blockIdx.y * 2 * kThreads; t0 < thi; t0 += (int64_t)gridDim.y * 2 * kThreads) {
    const int64_t t1 = t0 + 2 * kThreads < thi ? t0 + 2 * kThreads : thi;
    const int64_t n = t1 - t0;
    if (n > kThreads) {
      p2p_chunk<R, CPLX, K, 2>(a, t0, t1, e0, e1, 1, st, s_lo, s_cum);
    } else {
      int split = 1;
      while (split < 16 && n * split * 2 <= kThreads) split *= 2;
      p2p_chunk<R, CPLX, K, 1>(a, t0, t1, e0, e1, split, st, s_lo, s_cum);
    }
  }
}

}  // namespace

// Launch KERNEL<R, CPLX, K> for the dtype and the kernel of the arguments (complex dtypes are
// Helmholtz); returns from the enclosing function on a bad dtype or kernel.
#define FMM_GREEN_DISPATCH(KERNEL, G, T, S, A, DTYPE)                                                     \
  switch ((DTYPE) * 8 + ((DTYPE) == FMM_C128 || (DTYPE) == FMM_C64 ? 0 : (A).kernel)) {                     \
    case FMM_F64 * 8 + FMM_LAPLACE: hipLaunchKernelGGL((KERNEL<double, false, FMM_LAPLACE>), G, T, 0, S, A); break;       \
    case FMM_F64 * 8 + FMM_YUKAWA: hipLaunchKernelGGL((KERNEL<double, false, FMM_YUKAWA>), G, T, 0, S, A); break;         \
    case FMM_F64 * 8 + FMM_BIHARMONIC: hipLaunchKernelGGL((KERNEL<double, false, FMM_BIHARMONIC>), G, T, 0, S, A); break; \
    case FMM_F32 * 8 + FMM_LAPLACE: hipLaunchKernelGGL((KERNEL<float, false, FMM_LAPLACE>), G, T, 0, S, A); break;        \
    case FMM_F32 * 8 + FMM_YUKAWA: hipLaunchKernelGGL((KERNEL<float, false, FMM_YUKAWA>), G, T, 0, S, A); break;          \
    case FMM_F32 * 8 + FMM_BIHARMONIC: hipLaunchKernelGGL((KERNEL<float, false, FMM_BIHARMONIC>), G, T, 0, S, A); break;  \
    case FMM_C128 * 8: hipLaunchKernelGGL((KERNEL<double, true, FMM_HELMHOLTZ>), G, T, 0, S, A); break;                 \
    case FMM_C64 * 8: hipLaunchKernelGGL((KERNEL<float, true, FMM_HELMHOLTZ>), G, T, 0, S, A); break;                   \
    default: return fail(FMM_EINVAL, "dtype and kernel");                                                 \
  }

int launch_p2p(const P2PArgs& a, int dtype, hipStream_t s) {
  if (a.n_tbox == 0) return FMM_OK;
  // workgroups per target box: enough that the average box gets one per 2 kThreads targets
  const int64_t per_box = (a.n_tgt + a.n_tbox - 1) / a.n_tbox;
  const int64_t chunks = (per_box + 2 * kThreads - 1) / (2 * kThreads);
  const int64_t ny = chunks < 1 ? 1 : (chunks < 1024 ? chunks : 1024);
  dim3 g((unsigned)a.n_tbox, (unsigned)ny), t(kThreads);
  FMM_GREEN_DISPATCH(p2p_kernel, g, t, s, a, dtype);
  FMM_HIP_CHECK(hipGetLastError());
  return FMM_OK;
}

int launch_direct(const DirectArgs& a_in, int dtype, hipStream_t s) {
  if (a_in.n_tgt == 0) return FMM_OK;
  // lanes per target: double until the launch has about 1,024 workgroups (or one wavefront
  // per target)
  DirectArgs a = a_in;
  a.split = 1;
  while (a.split < 64 && (a.n_tgt * a.split + kThreads - 1) / kThreads < 1024) a.split *= 2;
  const int64_t per_block = kThreads / a.split;
  dim3 g((unsigned)((a.n_tgt + per_block - 1) / per_block)), t(kThreads);
  FMM_GREEN_DISPATCH(direct_kernel, g, t, s, a, dtype);
  FMM_HIP_CHECK(hipGetLastError());
  return FMM_OK;
}

}  // namespace fmm
