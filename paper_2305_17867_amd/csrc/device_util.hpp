// Small device helpers: complex arithmetic, dtype traits, wavefront reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fmm {

// Trivially default-constructible (usable in __shared__ arrays); T{} / T(0) give zero.
template <typename R>
struct Cx {
  R re, im;
  Cx() = default;
  __host__ __device__ constexpr Cx(R r, R i = 0) : re(r), im(i) {}
};
template <typename R>
__device__ inline Cx<R> operator+(Cx<R> a, Cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ inline Cx<R> operator-(Cx<R> a, Cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ inline Cx<R> operator*(Cx<R> a, Cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ inline Cx<R> operator*(R s, Cx<R> a) { return {s * a.re, s * a.im}; }
template <typename R>
__device__ inline Cx<R> operator*(Cx<R> a, R s) { return {s * a.re, s * a.im}; }
template <typename R>
__device__ inline Cx<R>& operator+=(Cx<R>& a, Cx<R> b) {
  a.re += b.re;
  a.im += b.im;
  return a;
}

// Value type for a (real type, complex?) pair.
template <typename R, bool CPLX>
struct Val;
template <typename R>
struct Val<R, false> {
  using T = R;
};
template <typename R>
struct Val<R, true> {
  using T = Cx<R>;
};

__device__ inline double shfl_xor_d(double v, int m) { return __shfl_xor(v, m, 64); }
__device__ inline float shfl_xor_d(float v, int m) { return __shfl_xor(v, m, 64); }

// c ? a : b by bit masks.  A plain select of two elements of a register array can be turned
// by the compiler into one load with a lane-dependent index, which moves the whole array to
// scratch memory; the masks keep it in registers.
template <typename R>
__device__ inline R pick_bits(bool c, R a, R b) {
  if constexpr (sizeof(R) == 8) {
    const uint64_t m = 0ull - (uint64_t)c;
    return __builtin_bit_cast(R, (__builtin_bit_cast(uint64_t, a) & m) | (__builtin_bit_cast(uint64_t, b) & ~m));
  } else {
    const uint32_t m = 0u - (uint32_t)c;
    return __builtin_bit_cast(R, (__builtin_bit_cast(uint32_t, a) & m) | (__builtin_bit_cast(uint32_t, b) & ~m));
  }
}

// Wavefront exchanges used by the reduce-scatter below: the value of the lane l ^ mask for
// mask = 15, 7, 2, 1 (lane moves within rows of 16 lanes: row mirror, half-row mirror, quad
// permutations), 16 (swizzle within 32 lanes) and 32 (LDS permute).
constexpr int kRsMasks[6] = {15, 7, 2, 1, 16, 32};
constexpr int kRsUpBit[6] = {3, 2, 1, 0, 4, 5};  // the lane bit that tells the two partners apart

template <int MASK>
__device__ inline int xchg32(int v) {
  if constexpr (MASK == 15) return __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, false);      // row_mirror
  else if constexpr (MASK == 7) return __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false);  // row_half_mirror
  else if constexpr (MASK == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
  else if constexpr (MASK == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
  else if constexpr (MASK == 8) return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, false);   // row_ror:8 (xor 8)
  else if constexpr (MASK == 16) return __builtin_amdgcn_ds_swizzle(v, 0x401F);             // xor 16 in 32 lanes
  else return __shfl_xor(v, 32, 64);
}

template <int MASK, typename R>
__device__ inline R xchg(R v) {
  if constexpr (sizeof(R) == 8) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)xchg32<MASK>((int)(uint32_t)b);
    const uint32_t hi = (uint32_t)xchg32<MASK>((int)(uint32_t)(b >> 32));
    return __builtin_bit_cast(R, ((uint64_t)hi << 32) | lo);
  } else {
    return __builtin_bit_cast(R, xchg32<MASK>(__builtin_bit_cast(int, v)));
  }
}

// Reduce-scatter of the 2^M values v[] over the 64 lanes of a wavefront by halving exchanges,
// the stages with the most values first on the cheapest exchanges (lane moves within rows).
// Stage i pairs lane l with l ^ kRsMasks[i]; the masks are independent over GF(2), so after
// all six stages every lane holds a sum over all 64 lanes.  The lane keeps the upper half when
// its bit kRsUpBit[i] is set.  Afterwards lane l holds the wave-wide sum of v[rs_index<M>(l)],
// and rs_owner<M>(l) marks one lane per index.
template <int M>
__device__ inline int rs_index(int lane) {
  int k = 0;
#pragma unroll
  for (int i = 0; i < M; ++i) k |= ((lane >> kRsUpBit[i]) & 1) << (M - 1 - i);
  return k;
}
template <int M>
__device__ inline bool rs_owner(int lane) {
  int used = 0;
#pragma unroll
  for (int i = 0; i < M; ++i) used |= 1 << kRsUpBit[i];
  return (lane & (63 & ~used)) == 0;
}

template <int M, int I, typename R>
__device__ inline void rs_stage(R (&v)[1 << M], int lane) {
  if constexpr (I < M) {
    constexpr int L = (1 << M) >> I;
    const bool up = ((lane >> kRsUpBit[I]) & 1) != 0;
#pragma unroll
    for (int k = 0; k < L / 2; ++k) {
      const R lo = v[k], hi = v[L / 2 + k];
      v[k] = pick_bits(up, hi, lo) + xchg<kRsMasks[I]>(pick_bits(up, lo, hi));
    }
    rs_stage<M, I + 1, R>(v, lane);
  }
}

template <int I, typename R>
__device__ inline R rs_allreduce(R r) {
  if constexpr (I < 6) return rs_allreduce<I + 1, R>(r + xchg<kRsMasks[I]>(r));
  else return r;
}

template <int M, typename R>
__device__ inline R wave_reduce_scatter(R (&v)[1 << M], int lane) {
  static_assert(M >= 0 && M <= 5, "at most 32 values per lane");
  rs_stage<M, 0, R>(v, lane);
  return rs_allreduce<M, R>(v[0]);
}

__host__ __device__ constexpr int tri(int n) { return n < 0 ? 0 : (n + 1) * (n + 2) / 2; }
__host__ __device__ constexpr int nfull(int p) { return p < 0 ? 0 : (p + 1) * (p + 2) * (p + 3) / 6; }

// Position of (x, y, z) in the internal full order of M(p): (m_z, m_x, m_y) lexicographic.
// The kept set J = {m_z < c} is a prefix of this order.
__host__ __device__ constexpr int full_index(int p, int x, int y, int z) {
  // slab start: sum_{z' < z} tri(p - z')
  int s = nfull(p) - nfull(p - z);
  // row start within slab: sum_{x' < x} (p - z - x' + 1)
  int r = x * (p - z + 1) - x * (x - 1) / 2;
  return s + r + y;
}

// (x, y) of entry k of a slab of M(p) with x + y <= n, rows x ascending, y fastest (the
// order of full_index within one m_z).  Arithmetic only: no table lookups.
__device__ inline void slab_decode(int n, int k, int& x, int& y) {
  x = 0;
  while (k > n - x) {
    k -= n - x + 1;
    ++x;
  }
  y = k;
}

// (x, y, z) of full index k of M(p): the inverse of full_index.
__device__ inline void full_decode(int p, int k, int& x, int& y, int& z) {
  z = 0;
  while (z < p && k >= tri(p - z)) {
    k -= tri(p - z);
    ++z;
  }
  slab_decode(p - z, k, x, y);
}

// 1 / n!
__device__ inline double inv_factorial(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return 1.0 / f;
}

// Position of (x, y, z), |m| <= p, in the order of a nested Horner scheme that runs z from p
// down, then x down, then y down: the slabs above z, the rows above x in slab z, then y.
__host__ __device__ constexpr int horner_pos(int p, int x, int y, int z) {
  return nfull(p - z - 1) + tri(p - z - x - 1) + (p - z - x - y);
}

}  // namespace fmm
