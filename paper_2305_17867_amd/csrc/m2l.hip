// Batched compressed M2L (Sec. 4.1, eq. m2l_toeplitz) on the matrix cores of gfx950.
//
//   theta~_t[i] += sum over pairs (t, s):  sum_{q in J} T~_o[i, q] beta~_s[q],
//   T~_o[i, q] = G^(i+q)(d_o) h^|i+q|  (scaled form, Sec. 4.1.1), i, q in J.
//
// The host groups pairs by translation offset o and tiles the target boxes in groups of 16
// (same level and child parity, so that they share almost all offsets).  A tile's entry e is
// one offset o together with the source box of each of the 16 targets at that offset.  For an
// entry the work is the dense product
//   Theta[:, 0:16] += T~_o[J, J] * B,   B[:, col] = beta~ of the source of target col,
// a 16-column GEMM on v_mfma 16x16x4: rows of T~ (i) are split into 16-row tiles, one per
// wavefront; the K loop runs over q in steps of 4.  T~_o is never expanded: because
// T~_o[i, q] depends on i + q only, it is read from the compact derivative grid
// tab[(m_z, m_x, m_y)] staged in LDS at address base(i) + base(q), with
// base(m) = (m_z S + m_x) S + m_y, S = 2p + 1.
//
// Accumulation: FP64 dtypes accumulate in FP64 matrix-core registers.  FP32 dtypes run each
// entry (offset group) as an FP32 product with FP32 accumulation and add the entry's partial
// into FP64 registers, so the sum over the (up to 189 per level) offset groups is FP64.
// Complex dtypes use four real products per K step.  Every output coefficient is owned by
// one workgroup; a tile split over several workgroups writes FP64 partials to scratch and the
// last workgroup to finish (atomic counter) adds them in part order, so results are
// bit-reproducible.
#include "../../include/fmm.h"
#include "common.hpp"
#include "device_util.hpp"
#include "kernels.hpp"

namespace fmm {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename R>
struct MF;
// Operand layouts (both dtypes): lane l supplies A[l & 15][l >> 4] and B[l >> 4][l & 15].
// Result layouts differ: register v of lane l holds C[row(l >> 4, v)][l & 15] with
//   f64 16x16x4: row = 4 v + (l >> 4);   f32 16x16x4: row = 4 (l >> 4) + v.
template <>
struct MF<double> {
  using V = d4;
  static __device__ inline V mma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int kq, int v) { return 4 * v + kq; }
};
template <>
struct MF<float> {
  using V = f4;
  static __device__ inline V mma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int kq, int v) { return 4 * kq + v; }
};

// Shapes instantiated for the persistent multi-batch launch.
#define FMM_M2L_MSHAPES(X) X(2, 2) X(3, 2) X(2, 1) X(3, 1)

// One workgroup owns a tile of NT targets and a contiguous range of its entries (offset
// groups).  Wavefront w owns the RT x CT output tiles (16 x 16 each) of row group w % nrg and
// column group w / nrg.  For every entry the derivative grid (planar re/im, [CW][ts]) and the NT source
// multipoles ([CW][NT][ldb]) are staged in LDS, double buffered: the global loads of entry e+1
// are issued into registers before the products of entry e and written to the other buffer
// after them, one barrier per entry.
//
// K ordering: lane group kq (lanes 16 kq .. 16 kq + 15) takes the contiguous range
// q = kq K4p + ks, ks < K4p (K4p = ceil(Nc/4) rounded up to the vector width), so its B values
// are read from LDS as 128-bit vectors and the table base of q advances incrementally along
// the kept order (m_z, m_x, m_y).  B rows are zero beyond Nc, which makes the padded K steps
// add nothing; padded rows (i >= Nc) read a valid table entry and are never stored.
template <typename R, bool CPLX, int RT, int CT, int PT, int PB, bool DB>
__device__ __forceinline__ void m2l_item(const M2LArgs& a, const M2LItem it) {
  using V = typename MF<R>::V;
  constexpr int CW = CPLX ? 2 : 1;
  const int NT = a.nt;  // 16 x column tiles of the workgroup
  constexpr int VW = 16 / sizeof(R);  // K steps per 128-bit B read
  constexpr bool ACC64 = sizeof(R) == 4;
  typedef R RV __attribute__((ext_vector_type(VW)));
  extern __shared__ __align__(16) char smem_raw[];
  const int ts = a.ts, nc = a.nc, ncp = a.nc_pad, ldb = a.ldb, k4p = a.k4p;
  const int n_tv = CW * ts;
  const int buf_elems = a.buf_elems;  // CW ts rounded up to 4, + CW NT ldb
  R* buf0 = reinterpret_cast<R*>(smem_raw);
  int* sbq = reinterpret_cast<int*>(buf0 + (DB ? 2 : 1) * buf_elems);  // [4 k4p] table base of q
  __shared__ int s_last;

  // the wavefront index is uniform: keep it (and everything derived from it) in scalar
  // registers, so that the row-group / K-range conditions of the inner loop are scalar branches
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nthr = blockDim.x;
  const int rtiles = a.rtiles;  // matrix-core row tiles; rows 16 rtiles .. 16 rtiles + nrem - 1 on the VALU
  const int nrem = a.nrem;
  // wavefront -> (row group, column group, K range): row tiles rg RT + r, column tiles
  // cg CT + c, K steps [s0, s1) of every lane group.  In a launch shared by several batches a
  // workgroup may have more wavefronts than this batch needs; those only help with the staging.
  const int nrg = a.nrg, ncg = NT / (16 * CT), nks = a.nks;
  const int rg = wave % nrg, cg = (wave / nrg) % ncg, kh = wave / (nrg * ncg);
  const bool active = kh < nks;
  const int nsteps = k4p / VW;
  const int s0 = active ? (kh * nsteps) / nks * VW : 0, s1 = active ? ((kh + 1) * nsteps) / nks * VW : 0;
  const int col = lane & 15;
  const int kq = lane >> 4;
  const int tab_off = a.tab_off;  // start of the source tile within a buffer
  const int ncw = nc * CW;

  // zero both buffers' source tiles once: rows are written only for q < Nc afterwards
  for (int k = tid; k < CW * NT * ldb; k += nthr) {
    buf0[tab_off + k] = R(0);
    if constexpr (DB) buf0[buf_elems + tab_off + k] = R(0);
  }
  for (int k = tid; k < 4 * k4p; k += nthr) sbq[k] = k < nc ? a.jbase[k] : 0;

  const R* mp = reinterpret_cast<const R*>(a.mpole);
  const R* tabg = reinterpret_cast<const R*>(a.tab);

  // register prefetch: table elements tid + k nthr; source column js, values rs + k tps
  R pft[PT], pfb[PB];
  const int tps = nthr / NT;
  const int js = tid / tps, rs = tid - js * tps;
  const int us = CPLX ? (rs & 1) : 0;
  const int qs = CPLX ? (rs >> 1) : rs;
  const int qstep = CPLX ? (tps >> 1) : tps;
  const int bdst_off = tab_off + (us * NT + js) * ldb + qs;
  // table and source indices of the next entry to issue, read one entry ahead so that the
  // operand loads of issue() do not wait on them
  int idx_tab = 0, idx_src = -1;
  auto load_idx = [&](int e) {
    idx_tab = a.entry_tab[e];
    idx_src = a.entry_src[(int64_t)e * NT + js];
  };
  auto issue = [&]() {
    const R* gt = tabg + (int64_t)idx_tab * n_tv;
#pragma unroll
    for (int k = 0; k < PT; ++k) {
      const int f = tid + k * nthr;
      if (f < n_tv) pft[k] = gt[f];
    }
    const int src = idx_src;
    const R* gb = mp + (int64_t)(src < 0 ? 0 : src) * ncw + rs;
#pragma unroll
    for (int k = 0; k < PB; ++k) {
      if (rs + k * tps < ncw) pfb[k] = src >= 0 ? gb[k * tps] : R(0);
    }
  };
  auto commit = [&](R* bufp) {
#pragma unroll
    for (int k = 0; k < PT; ++k) {
      const int f = tid + k * nthr;
      if (f < n_tv) bufp[f] = pft[k];
    }
#pragma unroll
    for (int k = 0; k < PB; ++k) {
      if (rs + k * tps < ncw) bufp[bdst_off + k * qstep] = pfb[k];
    }
  };

  V part[RT][CT][CW];
  double acc[RT][CT][CW][4];
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int c = 0; c < CT; ++c)
#pragma unroll
      for (int u = 0; u < CW; ++u) {
        part[r][c][u] = V{};
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[r][c][u][v] = 0.0;
      }
  // table base of this lane's A rows (padded rows use row 0, results discarded)
  int ib[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int i = (rg * RT + r) * 16 + col;
    ib[r] = (i < nc) ? a.jbase[i] : 0;
  }
  const int q0 = kq * k4p;
  // Rows beyond the last full 16-row tile (at most kMaxRem of them) are contracted on the
  // vector ALU by the wavefronts of the last row group, in FP64: a mostly empty 16-row
  // matrix-core tile would cost far more.  Each lane sums its own K steps and columns; the
  // four lane groups are added at the end of the item.
  const bool do_rem = active && nrem > 0 && rg == nrg - 1;
  int ibr[kMaxRem];
  double racc[kMaxRem][CT][CW];
#pragma unroll
  for (int j = 0; j < kMaxRem; ++j) {
    const int i = rtiles * 16 + j;
    ibr[j] = (j < nrem && i < nc) ? a.jbase[i] : 0;
#pragma unroll
    for (int c = 0; c < CT; ++c)
#pragma unroll
      for (int u = 0; u < CW; ++u) racc[j][c][u] = 0.0;
  }

  if (it.e0 < it.e1) {
    load_idx(it.e0);
    issue();
    if (it.e0 + 1 < it.e1) load_idx(it.e0 + 1);
  }
  __syncthreads();  // zero fill done
  if (it.e0 < it.e1) commit(buf0);
  __syncthreads();

  for (int e = it.e0; e < it.e1; ++e) {
    R* cur = DB ? buf0 + ((e - it.e0) & 1) * buf_elems : buf0;
    R* nxt = DB ? buf0 + (((e - it.e0) & 1) ^ 1) * buf_elems : buf0;
    if (e + 1 < it.e1) {
      issue();
      if (e + 2 < it.e1) load_idx(e + 2);
    }
    const R* brow[CT][CW];
#pragma unroll
    for (int c = 0; c < CT; ++c)
#pragma unroll
      for (int u = 0; u < CW; ++u) brow[c][u] = cur + tab_off + (u * NT + (cg * CT + c) * 16 + col) * ldb + q0;
    // K steps of this wavefront.  The operands of a step are read from LDS right before its
    // products: the other wavefronts of the SIMD cover the latency, and single-buffered
    // operands keep the register count low enough for four wavefronts per SIMD.
    typedef int IV __attribute__((ext_vector_type(VW)));
    const int* qrow = sbq + q0;
    const int nr = rtiles - rg * RT;  // row tiles of this wavefront that exist (uniform)
    if (active) {
      for (int ks = s0; ks < s1; ks += VW) {
        const IV qc = *reinterpret_cast<const IV*>(qrow + ks);
        RV bc[CT][CW];
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
          for (int u = 0; u < CW; ++u) bc[c][u] = *reinterpret_cast<const RV*>(brow[c][u] + ks);
        R ac[VW][RT][CW];
#pragma unroll
        for (int v = 0; v < VW; ++v)
#pragma unroll
          for (int r = 0; r < RT; ++r) {
            ac[v][r][0] = cur[ib[r] + qc[v]];
            if constexpr (CPLX) ac[v][r][1] = cur[ts + ib[r] + qc[v]];
          }
#pragma unroll
        for (int v = 0; v < VW; ++v)
#pragma unroll
          for (int r = 0; r < RT; ++r) {
            if (RT > 1 && r >= nr) continue;
            if constexpr (CPLX) {
#pragma unroll
              for (int c = 0; c < CT; ++c) {
                part[r][c][0] = MF<R>::mma(ac[v][r][0], bc[c][0][v], part[r][c][0]);
                part[r][c][0] = MF<R>::mma(-ac[v][r][1], bc[c][1][v], part[r][c][0]);
                part[r][c][1] = MF<R>::mma(ac[v][r][0], bc[c][1][v], part[r][c][1]);
                part[r][c][1] = MF<R>::mma(ac[v][r][1], bc[c][0][v], part[r][c][1]);
              }
            } else {
#pragma unroll
              for (int c = 0; c < CT; ++c) part[r][c][0] = MF<R>::mma(ac[v][r][0], bc[c][0][v], part[r][c][0]);
            }
          }
        if (do_rem) {
#pragma unroll
          for (int v = 0; v < VW; ++v)
#pragma unroll
            for (int j = 0; j < kMaxRem; ++j) {
              if (j >= nrem) continue;
              const double tr = (double)cur[ibr[j] + qc[v]];
              if constexpr (CPLX) {
                const double ti = (double)cur[ts + ibr[j] + qc[v]];
#pragma unroll
                for (int c = 0; c < CT; ++c) {
                  const double br = (double)bc[c][0][v], bi = (double)bc[c][1][v];
                  racc[j][c][0] += tr * br - ti * bi;
                  racc[j][c][1] += tr * bi + ti * br;
                }
              } else {
#pragma unroll
                for (int c = 0; c < CT; ++c) racc[j][c][0] += tr * (double)bc[c][0][v];
              }
            }
        }
      }
    }
    if constexpr (ACC64) {
#pragma unroll
      for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
          for (int u = 0; u < CW; ++u) {
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[r][c][u][v] += (double)part[r][c][u][v];
            part[r][c][u] = V{};
          }
    }
    if constexpr (!DB) __syncthreads();  // single buffer: everyone is done reading it
    if (e + 1 < it.e1) commit(nxt);
    __syncthreads();
  }
  if constexpr (!ACC64) {
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int c = 0; c < CT; ++c)
#pragma unroll
        for (int u = 0; u < CW; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[r][c][u][v] = (double)part[r][c][u][v];
  }

  if (do_rem) {
    // add the four lane groups (K ranges) of every column
#pragma unroll
    for (int j = 0; j < kMaxRem; ++j)
#pragma unroll
      for (int c = 0; c < CT; ++c)
#pragma unroll
        for (int u = 0; u < CW; ++u) {
          racc[j][c][u] += __shfl_xor(racc[j][c][u], 16, 64);
          racc[j][c][u] += __shfl_xor(racc[j][c][u], 32, 64);
        }
  }
  // K splits: the partial sums of wavefronts kh = 1 .. nks-1 are added to those of kh = 0, in
  // that order, through LDS (the staging buffers are free now)
  if (nks > 1) {
    constexpr int NACC = RT * CT * CW * 4 + kMaxRem * CT * CW;
    double* red = reinterpret_cast<double*>(smem_raw);
    const int slot = wave % (nrg * ncg);
    for (int k = 1; k < nks; ++k) {
      __syncthreads();
      constexpr int RB = RT * CT * CW * 4;  // start of the remainder-row sums in a slot
      if (kh == k) {
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
          for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int u = 0; u < CW; ++u)
#pragma unroll
              for (int v = 0; v < 4; ++v)
                red[(slot * NACC + ((r * CT + c) * CW + u) * 4 + v) * 64 + lane] = acc[r][c][u][v];
#pragma unroll
        for (int j = 0; j < kMaxRem; ++j)
#pragma unroll
          for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int u = 0; u < CW; ++u) red[(slot * NACC + RB + (j * CT + c) * CW + u) * 64 + lane] = racc[j][c][u];
      }
      __syncthreads();
      if (kh == 0) {
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
          for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int u = 0; u < CW; ++u)
#pragma unroll
              for (int v = 0; v < 4; ++v)
                acc[r][c][u][v] += red[(slot * NACC + ((r * CT + c) * CW + u) * 4 + v) * 64 + lane];
#pragma unroll
        for (int j = 0; j < kMaxRem; ++j)
#pragma unroll
          for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int u = 0; u < CW; ++u) racc[j][c][u] += red[(slot * NACC + RB + (j * CT + c) * CW + u) * 64 + lane];
      }
    }
  }
  const bool writer = active && kh == 0;

  // result rows of this lane: MF<R>::row(kq, v), column (cg CT + c) 16 + col
  const int nparts = a.tile_nparts[it.tile];
  const int* tg = a.tile_tgt + (int64_t)it.tile * NT;
  if (nparts == 1) {
    if (!writer) return;
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      const int t = tg[(cg * CT + c) * 16 + col];
      if (t < 0) continue;
      R* out = reinterpret_cast<R*>(a.local) + (int64_t)t * nc * CW;
      if (do_rem && kq == 0) {
#pragma unroll
        for (int j = 0; j < kMaxRem; ++j) {
          if (j >= nrem) continue;
          const int i = rtiles * 16 + j;
#pragma unroll
          for (int u = 0; u < CW; ++u) out[i * CW + u] = (R)((double)out[i * CW + u] + racc[j][c][u]);
        }
      }
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        const int rt = rg * RT + r;
        if (rt >= rtiles) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = rt * 16 + MF<R>::row(kq, v);
          if (i < nc) {
#pragma unroll
            for (int u = 0; u < CW; ++u) out[i * CW + u] = (R)((double)out[i * CW + u] + acc[r][c][u][v]);
          }
        }
      }
    }
    return;
  }
  // split tile: FP64 partial to scratch, the last workgroup of the tile adds all parts in order
  double* mine = a.scratch + (int64_t)(a.tile_item0[it.tile] + it.part) * NT * ncp * CW;
#pragma unroll
  for (int c = 0; c < CT; ++c)
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      const int rt = rg * RT + r;
      if (rt >= rtiles || !writer) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = rt * 16 + MF<R>::row(kq, v);
#pragma unroll
        for (int u = 0; u < CW; ++u) mine[(((cg * CT + c) * 16 + col) * ncp + i) * CW + u] = acc[r][c][u][v];
      }
    }
  if (writer && do_rem && kq == 0) {
#pragma unroll
    for (int c = 0; c < CT; ++c)
#pragma unroll
      for (int j = 0; j < kMaxRem; ++j) {
        if (j >= nrem) continue;
        const int i = rtiles * 16 + j;
#pragma unroll
        for (int u = 0; u < CW; ++u) mine[(((cg * CT + c) * 16 + col) * ncp + i) * CW + u] = racc[j][c][u];
      }
  }
  __threadfence();
  __syncthreads();
  if (tid == 0) {
    const int old = atomicAdd(a.counter + it.tile, 1);
    s_last = (old == nparts - 1);
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  // four outputs per thread and pass, the loads of all parts issued before the sums
  const int item0 = a.tile_item0[it.tile];
  const double* __restrict__ parts = a.scratch + (int64_t)item0 * NT * ncp * CW;
  const int64_t pstride = (int64_t)NT * ncp * CW;
  constexpr int U = 4;
  for (int k0 = tid; k0 < NT * nc; k0 += U * nthr) {
    double sr[U], si[U];
    int off[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int k = k0 + j * nthr;
      const int c = k / nc, i = k - c * nc;
      off[j] = k < NT * nc ? (c * ncp + i) * CW : 0;
      sr[j] = si[j] = 0.0;
    }
    for (int pt = 0; pt < nparts; ++pt) {
      const double* ps = parts + pt * pstride;
#pragma unroll
      for (int j = 0; j < U; ++j) {
        sr[j] += ps[off[j]];
        if constexpr (CPLX) si[j] += ps[off[j] + 1];
      }
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int k = k0 + j * nthr;
      if (k >= NT * nc) continue;
      const int c = k / nc, i = k - c * nc;
      const int t = tg[c];
      if (t < 0) continue;
      R* out = reinterpret_cast<R*>(a.local) + (int64_t)t * nc * CW;
      out[i * CW] = (R)((double)out[i * CW] + sr[j]);
      if constexpr (CPLX) out[i * CW + 1] = (R)((double)out[i * CW + 1] + si[j]);
    }
  }
  if (tid == 0) atomicExch(a.counter + it.tile, 0);
}

// Register target: the 2x2 and 3x2 real FP64 tiles with the smallest staging class fit in
// 128 registers, i.e. four wavefronts per SIMD (the compiler would otherwise take a few more).
template <typename R, bool CPLX, int RT, int CT, int PT>
constexpr int m2l_waves_hint() {
  return (sizeof(R) == 8 && !CPLX && PT == kPrefT0 && CT == 2 && (RT == 2 || RT == 3)) ? 4 : 1;
}

template <typename R, bool CPLX, int RT, int CT, int PT, int PB, bool DB>
__global__ __launch_bounds__(kM2LMaxThreads)
__attribute__((amdgpu_waves_per_eu(m2l_waves_hint<R, CPLX, RT, CT, PT>()))) void m2l_kernel(M2LArgs a) {
  m2l_item<R, CPLX, RT, CT, PT, PB, DB>(a, a.items[blockIdx.x]);
}

// Persistent launch over the work items of several batches: workgroup g takes items
// g, g + gridDim.x, ... of the combined list (sorted by decreasing cost on the host); every
// wavefront reaches the end of the list, so the grid drains.
template <typename R, bool CPLX, int RT, int CT, int PT, int PB, bool DB>
__global__ __launch_bounds__(kM2LMaxThreads) void m2l_multi_kernel(M2LMulti m) {
  for (int w = blockIdx.x; w < m.n_work; w += gridDim.x) {
    __syncthreads();
    const int2 wk = m.work[w];
    M2LArgs a = m.args[wk.x];
    a.mpole = m.mpole[wk.x];
    a.local = m.local[wk.x];
    m2l_item<R, CPLX, RT, CT, PT, PB, DB>(a, a.items[wk.y]);
  }
}

template <typename R, bool CPLX, int RT, int CT, int PT, int PB, bool DB>
int launch_multi_cfg(const M2LMulti& m, size_t lds, int waves, int grid, hipStream_t s) {
  auto kern = m2l_multi_kernel<R, CPLX, RT, CT, PT, PB, DB>;
  if (lds > 65536) {
    static size_t granted = 0;
    if (lds > granted) {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(FMM_EUNSUPPORTED, "multi-batch M2L needs too much LDS per workgroup");
      }
      granted = lds;
    }
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3((unsigned)(waves * 64)), lds, s, m);
  FMM_HIP_CHECK(hipGetLastError());
  return FMM_OK;
}

template <typename R, bool CPLX, int RT, int CT, bool DB>
int launch_multi_pf(const M2LMulti& m, int pf, size_t lds, int waves, int grid, hipStream_t s) {
  if (pf == 0) return launch_multi_cfg<R, CPLX, RT, CT, kPrefT0, kPrefB0, DB>(m, lds, waves, grid, s);
  if (pf == 1) return launch_multi_cfg<R, CPLX, RT, CT, kPrefT1, kPrefB1, DB>(m, lds, waves, grid, s);
  return launch_multi_cfg<R, CPLX, RT, CT, kPrefT2, kPrefB2, DB>(m, lds, waves, grid, s);
}

template <typename R, bool CPLX>
int launch_multi_typed(const M2LMulti& m, int rt, int ct, int pf, int nbuf, size_t lds, int waves, int grid,
                       hipStream_t s) {
#define FMM_M2L_MCASE(RT_, CT_)                                                                   \
  if (rt == RT_ && ct == CT_)                                                                     \
    return nbuf == 2 ? launch_multi_pf<R, CPLX, RT_, CT_, true>(m, pf, lds, waves, grid, s)      \
                     : launch_multi_pf<R, CPLX, RT_, CT_, false>(m, pf, lds, waves, grid, s);
  FMM_M2L_MSHAPES(FMM_M2L_MCASE)
#undef FMM_M2L_MCASE
  return fail(FMM_EUNSUPPORTED, "multi-batch M2L shape not instantiated");
}

template <typename R, bool CPLX, int RT, int CT, int PT, int PB, bool DB>
int launch_cfg(const M2LArgs& a, int waves, hipStream_t s) {
  const size_t lds = m2l_lds_bytes(a, sizeof(R), DB ? 2 : 1, RT, CPLX);
  auto kern = m2l_kernel<R, CPLX, RT, CT, PT, PB, DB>;
  if (lds > 65536) {
    static size_t granted = 0;  // per instantiation
    if (lds > granted) {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(FMM_EUNSUPPORTED, "M2L needs " + std::to_string(lds) +
                                          " bytes of LDS per workgroup: " + hipGetErrorString(e));
      }
      granted = lds;
    }
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)a.n_items), dim3((unsigned)(waves * 64)), lds, s, a);
  FMM_HIP_CHECK(hipGetLastError());
  return FMM_OK;
}

template <typename R, bool CPLX, int RT, int CT, bool DB>
int launch_pf(const M2LArgs& a, int pf_class, int waves, hipStream_t s) {
  if (pf_class == 0) return launch_cfg<R, CPLX, RT, CT, kPrefT0, kPrefB0, DB>(a, waves, s);
  if (pf_class == 1) return launch_cfg<R, CPLX, RT, CT, kPrefT1, kPrefB1, DB>(a, waves, s);
  return launch_cfg<R, CPLX, RT, CT, kPrefT2, kPrefB2, DB>(a, waves, s);
}

// Instantiated per-wavefront tile shapes (row tiles RT x column tiles CT).
#define FMM_M2L_SHAPES(X) X(1, 1) X(1, 2) X(2, 1) X(2, 2) X(3, 1) X(3, 2) X(4, 1) X(5, 1)

template <typename R, bool CPLX>
int launch_typed(const M2LArgs& a, int rt, int ct, int pf, int nbuf, int waves, hipStream_t s) {
#define FMM_M2L_CASE(RT_, CT_)                                                        \
  if (rt == RT_ && ct == CT_)                                                         \
    return nbuf == 2 ? launch_pf<R, CPLX, RT_, CT_, true>(a, pf, waves, s)            \
                     : launch_pf<R, CPLX, RT_, CT_, false>(a, pf, waves, s);
  FMM_M2L_SHAPES(FMM_M2L_CASE)
#undef FMM_M2L_CASE
  return fail(FMM_EUNSUPPORTED, "M2L tile shape (rows per wave, column tiles) not instantiated");
}


__global__ void convert_f32_kernel(const double* src, float* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

// Derivative tables [n][ts] (complex interleaved) -> M2L layout [n][CW][ts] (planar) in R.
template <typename R, bool CPLX>
__global__ void m2l_table_layout_kernel(const double* src, R* dst, int64_t n, int ts) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * ts) return;
  const int64_t tb = i / ts, k = i % ts;
  if constexpr (CPLX) {
    dst[(tb * 2 + 0) * ts + k] = (R)src[2 * i];
    dst[(tb * 2 + 1) * ts + k] = (R)src[2 * i + 1];
  } else {
    dst[i] = (R)src[i];
  }
}

}  // namespace

bool m2l_shape_instantiated(int rt, int ct) {
#define FMM_M2L_CASE(RT_, CT_) \
  if (rt == RT_ && ct == CT_) return true;
  FMM_M2L_SHAPES(FMM_M2L_CASE)
#undef FMM_M2L_CASE
  return false;
}

void m2l_shape(M2LArgs& a, size_t real_bytes, bool cplx, int ct_total) {
  const int cw = cplx ? 2 : 1;
  const int vw = (int)(16 / real_bytes);
  const int k4 = (a.nc + 3) / 4;
  a.k4p = (k4 + vw - 1) / vw * vw;
  // row stride: >= 4 k4p, and an odd number of 16-byte units so that the 16 columns of a
  // 128-bit read fall in distinct bank groups
  const int per16 = vw;  // elements per 16 bytes
  int units = (4 * a.k4p + per16 - 1) / per16;
  if ((units & 1) == 0) ++units;
  a.ldb = units * per16;
  a.tab_off = (cw * a.ts + 3) / 4 * 4;
  a.buf_elems = a.tab_off + cw * 16 * ct_total * a.ldb;
  a.nt = 16 * ct_total;
}

size_t m2l_lds_bytes(const M2LArgs& a, size_t real_bytes, int nbuf, int rt, bool cplx) {
  const size_t stage = (size_t)nbuf * a.buf_elems * real_bytes + 4 * (size_t)a.k4p * sizeof(int);
  // K-split reduction: one FP64 accumulator set per (row group, column group) wavefront
  const size_t red = a.nks > 1 ? (size_t)a.nrg * (a.nt / 16) * (cplx ? 2 : 1) * (4 * rt + kMaxRem) * 64 * sizeof(double)
                               : 0;
  return stage > red ? stage : red;
}

int m2l_prefetch_class(const M2LArgs& a, bool cplx, int ct_total, int waves) {
  const int cw = cplx ? 2 : 1, nthr = waves * 64, nt = 16 * ct_total;
  if (nthr % nt) return -1;
  const int tps = nthr / nt;
  if (cplx && (tps & 1)) return -1;
  const int kt = (cw * a.ts + nthr - 1) / nthr, kb = (a.nc * cw + tps - 1) / tps;
  if (kt <= kPrefT0 && kb <= kPrefB0) return 0;
  if (kt <= kPrefT1 && kb <= kPrefB1) return 1;
  if (kt <= kPrefT2 && kb <= kPrefB2) return 2;
  return -1;
}

int launch_m2l(const M2LArgs& a, int dtype, int rows_per_wave, int col_tiles, int pf_class, int nbuf, int waves,
               hipStream_t s) {
  if (a.n_items == 0) return FMM_OK;
  switch (dtype) {
    case FMM_F64: return launch_typed<double, false>(a, rows_per_wave, col_tiles, pf_class, nbuf, waves, s);
    case FMM_F32: return launch_typed<float, false>(a, rows_per_wave, col_tiles, pf_class, nbuf, waves, s);
    case FMM_C128: return launch_typed<double, true>(a, rows_per_wave, col_tiles, pf_class, nbuf, waves, s);
    case FMM_C64: return launch_typed<float, true>(a, rows_per_wave, col_tiles, pf_class, nbuf, waves, s);
  }
  return fail(FMM_EINVAL, "dtype");
}

int launch_m2l_multi(const M2LMulti& m, int dtype, int rows_per_wave, int col_tiles, int pf_class, int nbuf,
                     size_t lds, int waves, int grid, hipStream_t s) {
  if (m.n_work == 0) return FMM_OK;
  switch (dtype) {
    case FMM_F64: return launch_multi_typed<double, false>(m, rows_per_wave, col_tiles, pf_class, nbuf, lds, waves, grid, s);
    case FMM_F32: return launch_multi_typed<float, false>(m, rows_per_wave, col_tiles, pf_class, nbuf, lds, waves, grid, s);
    case FMM_C128: return launch_multi_typed<double, true>(m, rows_per_wave, col_tiles, pf_class, nbuf, lds, waves, grid, s);
    case FMM_C64: return launch_multi_typed<float, true>(m, rows_per_wave, col_tiles, pf_class, nbuf, lds, waves, grid, s);
  }
  return fail(FMM_EINVAL, "dtype");
}

bool m2l_multi_shape_instantiated(int rt, int ct) {
#define FMM_M2L_MCASE(RT_, CT_) \
  if (rt == RT_ && ct == CT_) return true;
  FMM_M2L_MSHAPES(FMM_M2L_MCASE)
#undef FMM_M2L_MCASE
  return false;
}

int launch_m2l_table_layout(const double* src, void* dst, int64_t n, int ts, int dtype, hipStream_t s) {
  const int64_t tot = n * ts;
  if (tot == 0) return FMM_OK;
  dim3 g((unsigned)((tot + 255) / 256)), t(256);
  switch (dtype) {
    case FMM_F64: hipLaunchKernelGGL((m2l_table_layout_kernel<double, false>), g, t, 0, s, src, (double*)dst, n, ts); break;
    case FMM_F32: hipLaunchKernelGGL((m2l_table_layout_kernel<float, false>), g, t, 0, s, src, (float*)dst, n, ts); break;
    case FMM_C128: hipLaunchKernelGGL((m2l_table_layout_kernel<double, true>), g, t, 0, s, src, (double*)dst, n, ts); break;
    case FMM_C64: hipLaunchKernelGGL((m2l_table_layout_kernel<float, true>), g, t, 0, s, src, (float*)dst, n, ts); break;
    default: return fail(FMM_EINVAL, "dtype");
  }
  FMM_HIP_CHECK(hipGetLastError());
  return FMM_OK;
}

int launch_convert_f32(const double* src, float* dst, int64_t n, hipStream_t s) {
  if (n == 0) return FMM_OK;
  hipLaunchKernelGGL(convert_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
  FMM_HIP_CHECK(hipGetLastError());
  return FMM_OK;
}

}  // namespace fmm
