// Batched compressed M2L in two dimensions (eq. m2l_toeplitz for d = 2):
//   theta~_i[t] += sum over the pairs (t, s) of sum_{q in J} T~_(i + q) beta~_q[s],  i in J,
// with T~ the scaled derivative table of the pair's translation vector.
//
// J holds at most 4p - 2 coefficients, so one pair is a small dense product that does not
// fill a matrix-core tile; it runs on the vector units (FP64 vector and matrix peaks are the
// same on this chip).  kSplit adjacent lanes own one target box and one layer m_y = IY of its
// outputs (the launch's y dimension picks the layer, so a wavefront never diverges on it); each
// takes every kSplit-th pair of the target, holds the layer's accumulators and the source's
// coefficients in registers and reads each table entry it needs once per pair; a butterfly of
// lane exchanges adds the kSplit partial sums.  Splitting a target's pairs over lanes gives the
// launch kSplit times the wavefronts, which the memory latency of the pair loop needs.  Every
// index is a compile-time constant (p, c and the layer are template parameters and the loops
// are unrolled).  A workgroup reads its tables from LDS where they fit (one copy per workgroup).
#include "two_d.hpp"

namespace fmm2d {
namespace {

constexpr int kSplit = 4;
constexpr int kStageTables = 40;             // tables a workgroup stages in LDS (one level's offsets)
constexpr int kStageBytes = 64 * 1024;       // the largest static LDS array of a workgroup

template <int P, int C>
constexpr int table_size() { return (2 * C - 1) * (2 * P + 1); }

template <int P, int C>
constexpr bool stages() { return kStageTables * table_size<P, C>() * 8 <= kStageBytes; }

// TB: the tables, in LDS (staged: ids from t0 on) or in global memory (t0 = 0)
template <int P, int C, int IY, typename TB>
__device__ __forceinline__ void m2l_layer(const M2LArgs2D& a, int64_t k, int part, TB tables, int t0) {
  constexpr int NC = n_kept(P, C);
  constexpr int SX = 2 * P + 1;
  constexpr int NR = P - IY + 1;  // outputs of the layer: (ix, IY), ix = 0 .. P - IY
  // every lane of the target's group runs to the exchanges below (no early exit)
  const int32_t t = k < a.n_tbox ? a.tbox[k] : -1;
  const bool valid = t >= 0 && t < a.n_box;
  int64_t e0 = 0, e1 = 0;
  if (valid) {
    e0 = a.pair_ptr[k];
    e1 = a.pair_ptr[k + 1];
    e0 = e0 < 0 ? 0 : (e0 > a.n_pair ? a.n_pair : e0);
    e1 = e1 < e0 ? e0 : (e1 > a.n_pair ? a.n_pair : e1);
  }
  double acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = 0.0;
  for (int64_t e = e0 + part; e < e1; e += kSplit) {
    const int32_t s = a.pair_src[e];
    const int32_t tb = a.pair_tab[e];
    if (s < 0 || s >= a.n_box || tb < 0 || tb >= a.n_tab) continue;
    const double* __restrict__ B = a.mpole + (int64_t)s * NC;
    const auto T = tables + (int64_t)(tb - t0) * (2 * C - 1) * SX + IY * SX;
    double b[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) b[q] = B[q];
#pragma unroll
    for (int qy = 0; qy < C && qy <= P; ++qy) {
#pragma unroll
      for (int j = 0; j <= 2 * P - IY - qy; ++j) {
        // table entry (m_x = j, m_y = IY + qy) feeds every (ix, qx) with ix + qx = j
        const double tv = T[qy * SX + j];
#pragma unroll
        for (int ix = 0; ix < NR; ++ix) {
          const int qx = j - ix;
          if (qx >= 0 && qx <= P - qy) acc[ix] = fma(tv, b[kept_pos(P, qx, qy)], acc[ix]);
        }
      }
    }
  }
#pragma unroll
  for (int ix = 0; ix < NR; ++ix)
#pragma unroll
    for (int m = 1; m < kSplit; m <<= 1) acc[ix] += __shfl_xor(acc[ix], m, 64);
  if (!valid || part != 0) return;
  double* out = a.local + (int64_t)t * NC;
#pragma unroll
  for (int ix = 0; ix < NR; ++ix) out[kept_pos(P, ix, IY)] += acc[ix];
}

template <int P, int C, typename TB>
__device__ __forceinline__ void m2l_layers(const M2LArgs2D& a, int64_t k, int part, TB tables, int t0) {
  switch (blockIdx.y) {
    case 0:
      m2l_layer<P, C, 0>(a, k, part, tables, t0);
      break;
    case 1:
      if constexpr (P >= 1) m2l_layer<P, C, 1>(a, k, part, tables, t0);
      break;
    case 2:
      if constexpr (C > 2 && P >= 2) m2l_layer<P, C, 2>(a, k, part, tables, t0);
      break;
    case 3:
      if constexpr (C > 3 && P >= 3) m2l_layer<P, C, 3>(a, k, part, tables, t0);
      break;
    default:
      break;
  }
}

// The 64 targets of a workgroup are consecutive boxes, almost always of one level, whose pairs
// use at most the 40 tables of that level's offsets: the workgroup finds the range of table ids
// its pairs use and, when it is at most kStageTables long, copies those tables into LDS once.
template <int P, int C>
__global__ __launch_bounds__(256) void m2l2d_kernel(M2LArgs2D a) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t k = g / kSplit;  // target; its kSplit lanes are adjacent
  const int part = (int)(g % kSplit);
  if constexpr (stages<P, C>()) {
    constexpr int TSZ = table_size<P, C>();
    __shared__ double stab[kStageTables * TSZ];
    __shared__ int rng[2];
    if (threadIdx.x == 0) {
      rng[0] = 0x7fffffff;
      rng[1] = -1;
    }
    __syncthreads();
    int lo = 0x7fffffff, hi = -1;
    if (k < a.n_tbox) {
      const int32_t t = a.tbox[k];
      if (t >= 0 && t < a.n_box) {
        int64_t e0 = a.pair_ptr[k], e1 = a.pair_ptr[k + 1];
        e0 = e0 < 0 ? 0 : (e0 > a.n_pair ? a.n_pair : e0);
        e1 = e1 < e0 ? e0 : (e1 > a.n_pair ? a.n_pair : e1);
        for (int64_t e = e0 + part; e < e1; e += kSplit) {
          const int32_t tb = a.pair_tab[e];
          if (tb >= 0 && tb < a.n_tab) {
            lo = tb < lo ? tb : lo;
            hi = tb > hi ? tb : hi;
          }
        }
      }
    }
    if (hi >= lo) {
      atomicMin(&rng[0], lo);
      atomicMax(&rng[1], hi);
    }
    __syncthreads();
    const int t0 = rng[0], t1 = rng[1];
    const bool staged = t1 >= t0 && t1 - t0 < kStageTables;  // uniform
    if (staged) {
      const double* src = a.tables + (int64_t)t0 * TSZ;
      for (int i = threadIdx.x; i < (t1 - t0 + 1) * TSZ; i += blockDim.x) stab[i] = src[i];
    }
    __syncthreads();
    if (k >= a.n_tbox) return;  // the same for all lanes of a group, so exchanges stay in step
    if (staged)
      m2l_layers<P, C>(a, k, part, static_cast<const double*>(stab), t0);
    else
      m2l_layers<P, C>(a, k, part, a.tables, 0);
  } else {
    if (k >= a.n_tbox) return;
    m2l_layers<P, C>(a, k, part, a.tables, 0);
  }
}

template <int C, int P>
bool launch_p(const M2LArgs2D& a, int p, hipStream_t s) {
  if constexpr (P > 16) {
    return false;
  } else {
    if (p != P) return launch_p<C, P + 1>(a, p, s);
    const int layers = C < P + 1 ? C : P + 1;
    const dim3 grid((unsigned)((a.n_tbox * kSplit + 255) / 256), (unsigned)layers);
    m2l2d_kernel<P, C><<<grid, 256, 0, s>>>(a);
    return true;
  }
}

}  // namespace

bool launch_m2l2d(const M2LArgs2D& a, int p, int c, hipStream_t s) {
  if (a.n_tbox == 0) return true;
  if (c == 2) return launch_p<2, 0>(a, p, s);
  if (c == 4) return launch_p<4, 0>(a, p, s);
  return false;
}

}  // namespace fmm2d
