// Batched compressed M2L (Sec. 4.1, eq. m2l_toeplitz), streaming form for the matrix cores.
//
//   theta~_t[i] += sum over pairs (t, s):  sum_{q in J} T~_o[i, q] beta~_s[q],
//   T~_o[i, q] = G^(i+q)(d_o) h^|i+q|   (scaled form, Sec. 4.1.1),  i, q in J.
//
// Work decomposition.  Target boxes are tiled in groups of 16 (one matrix-core column tile)
// that share their offsets; an entry is one offset o of a tile together with the source box
// of each of its 16 targets.  The entries of all tiles, in tile order, are cut into one
// contiguous chunk per workgroup of about equal length, so every workgroup does the same
// amount of work; a tile that straddles a chunk boundary is summed from FP64 partials in
// part order by the last of its workgroups to finish (bit-reproducible).
//
// Inside a workgroup every wavefront streams its own entries (round robin over the chunk)
// and owns a full 16-column accumulator of all Nc output rows: there is no barrier between
// entries.  Per entry a wavefront
//   * writes the entry's compact derivative grid tab[(m_z, m_x, m_y)] (loaded into registers
//     during the previous entry) to its private LDS buffer,
//   * gathers the A operand of the matrix-core products from that grid: T~[i, q] =
//     grid[base(i) + base(q)] with base(m) = (m_z S + m_x) S + m_y, so T~ is never expanded,
//   * takes the B operand (the 16 source multipoles) straight from global memory into
//     registers: lane group g (lanes 16 g .. 16 g + 15) holds the pair q = 8 j + 2 g, q + 1
//     for step j, so the four lane groups read 8 consecutive coefficients of each source;
//     the loads of the next entry are issued into the same registers as soon as a step has
//     consumed them.
// At the end of a workgroup's share of a tile the wavefronts' accumulators are added in a
// fixed tree order through LDS.
//
// Products: v_mfma 16x16x4.  FP64 dtypes accumulate in FP64.  FP32 dtypes run each entry
// (offset group) as an FP32 product with FP32 accumulation (two accumulator sets, one per
// coefficient of a B pair, for more independent products in flight), then add the entry's
// partial into FP64 registers, so the sum over the (up to 189 per level) offset groups is
// FP64.  At most two rows past the last full 16-row tile are contracted on the vector ALU in
// FP64.  Complex dtypes use four real products per K step.
#include "../../include/fmm.h"
#include "common.hpp"
#include "device_util.hpp"
#include "kernels.hpp"

namespace fmm {

namespace {

typedef double sd4 __attribute__((ext_vector_type(4)));
typedef float sf4 __attribute__((ext_vector_type(4)));

// Matrix-core tile of one accumulator set: v_mfma 16x16x4 (FP64 or FP32), a 16-row tile.  Lane
// l supplies A[l & 15][l >> 4] and B[l >> 4][l & 15] (the 16 columns are the 16 targets of a
// tile) and holds C[row(l >> 4, v)][l & 15] in register v:  FP64 row = 4 v + (l >> 4),
// FP32 row = 4 (l >> 4) + v.  (The FP64 4x4x4 product, four independent 4 x 4 x 4 blocks on
// the lane quads, issues faster, but as a 4-row tile it needs one A gather per product and
// measured slower here.)
template <typename R>
struct STile;
template <>
struct STile<double> {
  using V = sd4;
  static constexpr int ROWS = 16, NV = 4;
  static __device__ inline V mma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int arow(int lane) { return lane & 15; }
  static __device__ inline int row(int kq, int v) { return 4 * v + kq; }
};
template <>
struct STile<float> {
  using V = sf4;
  static constexpr int ROWS = 16, NV = 4;
  static __device__ inline V mma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int arow(int lane) { return lane & 15; }
  static __device__ inline int row(int kq, int v) { return 4 * kq + v; }
};

constexpr int n_full_c(int p) { return p < 0 ? 0 : (p + 1) * (p + 2) * (p + 3) / 6; }

// Compile-time shape of one (order, PDE order, dtype) instantiation.
template <typename R, bool CPLX, int P, int C>
struct SShape {
  static constexpr int CW = CPLX ? 2 : 1;
  static constexpr int NC = n_full_c(P) - n_full_c(P - C);      // |J|
  static constexpr int TR = STile<R>::ROWS, NV = STile<R>::NV;
  static constexpr int REM = NC % TR;
  // 16-row tiles: at most two rows past the last full tile go to the vector ALU
  static constexpr bool VALU_ROWS = TR == 16 && NC > 16 && REM >= 1 && REM <= kMaxRem;
  static constexpr int RT = VALU_ROWS ? NC / TR : (NC + TR - 1) / TR;  // matrix-core row tiles
  static constexpr int NREM = VALU_ROWS ? REM : 0;                   // rows on the vector ALU
  // FP32 keeps separate accumulators for the two coefficients of a B step (twice the
  // independent product chains); FP64 has one per 4-row tile
  static constexpr int NSET = sizeof(R) == 4 ? 2 : 1;
  static constexpr int KJ = (NC + 7) / 8;                            // B steps of 8 coefficients
  static constexpr int S = 2 * P + 1, SZ = 2 * C - 1;
  static constexpr int TS = SZ * S * S;                              // grid values per plane
  static constexpr int VEC = 16 / (int)sizeof(R);                    // elements per 128-bit load
  static constexpr int TSP = (CW * TS + 64 * VEC - 1) / (64 * VEC) * (64 * VEC);  // padded table
  static constexpr int NTV = TSP / (64 * VEC);                       // 128-bit table loads per lane
  static constexpr int NACC = RT * CW * NV + NREM * CW;              // FP64 sums per lane
};

template <typename R, int N>
struct RVec {
  typedef R T __attribute__((ext_vector_type(N)));
  // the same vector at element alignment: a source multipole row starts at any element
  typedef R U __attribute__((ext_vector_type(N), aligned(sizeof(R))));
};

template <typename R, bool CPLX, int P, int C>
__device__ __forceinline__ void m2ls_workgroup(const M2LStreamArgs& a) {
  using SH = SShape<R, CPLX, P, C>;
  constexpr int CW = SH::CW, NC = SH::NC, RT = SH::RT, NREM = SH::NREM, KJ = SH::KJ;
  constexpr int TS = SH::TS, TSP = SH::TSP, NTV = SH::NTV, VEC = SH::VEC, NACC = SH::NACC;
  constexpr int TR = SH::TR, NV = SH::NV, NSET = SH::NSET;
  constexpr bool ACC64 = sizeof(R) == 4;
  using TL = STile<R>;
  using V = typename TL::V;
  using BV = typename RVec<R, 2 * CW>::T;  // the lane's pair (q, q + 1) of one B step
  using TV = typename RVec<R, VEC>::T;     // one 128-bit table load
  extern __shared__ __align__(16) char smem_raw[];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int W = blockDim.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  R* const tb = reinterpret_cast<R*>(smem_raw) + wave * TSP;
  int* const sbq = reinterpret_cast<int*>(smem_raw + a.lds_sbq);  // [4][2 KJ] base(q), 0 past Nc
  double* const slots = reinterpret_cast<double*>(smem_raw + a.lds_slot);  // [W][NACC][64] item sums
  // [0] wavefronts arrived at the current item, [1] items done, [2 + w] entries done by wavefront w
  int* const ctl = sbq + 8 * KJ;
  if (tid < 2 + kM2LStreamMaxWaves) ctl[tid] = 0;

  for (int k = tid; k < 8 * KJ; k += blockDim.x) {
    const int g = k / (2 * KJ), jj = k - g * (2 * KJ);
    const int q = 8 * (jj >> 1) + 2 * g + (jj & 1);
    sbq[k] = q < NC ? a.jbase[q] : 0;
  }
  int ib[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int i = TR * r + TL::arow(lane);
    ib[r] = i < NC ? a.jbase[i] : 0;  // padded rows read a valid grid value, never stored
  }
  int ibr[NREM > 0 ? NREM : 1];
#pragma unroll
  for (int j = 0; j < NREM; ++j) ibr[j] = a.jbase[TR * RT + j];
  __syncthreads();

  const R* const mp = reinterpret_cast<const R*>(a.mpole);
  const R* const tabg = reinterpret_cast<const R*>(a.tab);
  const int* const sbq_l = sbq + kq * (2 * KJ);
  const int w0 = a.wg_item[blockIdx.x], w1 = a.wg_item[blockIdx.x + 1];
  int rot = 0;  // round-robin start: continues across the workgroup's items
  int done_entries = 0;  // entries this wavefront has started (all items)

  for (int ii = w0; ii < w1; ++ii) {
    const M2LItem it = a.items[ii];
    const int nent = it.e1 - it.e0;
    double acc[RT][CW][NV];
    double racc[NREM > 0 ? NREM : 1][CW];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int u = 0; u < CW; ++u)
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[r][u][v] = 0.0;
#pragma unroll
    for (int j = 0; j < (NREM > 0 ? NREM : 1); ++j)
#pragma unroll
      for (int u = 0; u < CW; ++u) racc[j][u] = 0.0;
    V vacc[NSET][RT][CW];  // FP64: the accumulators; FP32: one entry's partials
#pragma unroll
    for (int h = 0; h < NSET; ++h)
#pragma unroll
      for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int u = 0; u < CW; ++u) vacc[h][r][u] = V{};

    int first = wave - rot;
    if (first < 0) first += W;
    int e = it.e0 + first;
    TV tv[NTV];
    BV bv[KJ];
    // loads of entry e: table values (lane-contiguous 128-bit pieces) and the lane's B pairs
    auto load_tab = [&](int tab) {
      const TV* g = reinterpret_cast<const TV*>(tabg + (int64_t)tab * TSP) + lane;
#pragma unroll
      for (int k = 0; k < NTV; ++k) tv[k] = g[k * 64];
    };
    auto load_b = [&](const R* src, bool ok, int j) {
      const int q = 8 * j + 2 * kq;
      if (8 * j + 8 <= NC) {
        using BU = typename RVec<R, 2 * CW>::U;
        bv[j] = ok ? BV(*reinterpret_cast<const BU*>(src + q * CW)) : BV{};
      } else {
        BV x{};
        if (ok && q < NC) {
#pragma unroll
          for (int u = 0; u < CW; ++u) x[u] = src[q * CW + u];
          if (q + 1 < NC) {
#pragma unroll
            for (int u = 0; u < CW; ++u) x[CW + u] = src[(q + 1) * CW + u];
          }
        }
        bv[j] = x;
      }
    };
    // table and source indices run two entries ahead of the compute, so that the operand
    // loads of the next entry never wait on them
    int tab1 = 0, src1 = -1;  // entry e + W
    if (e < it.e1) {
      const int tab = a.entry_tab[e];
      const int s = a.entry_src[(int64_t)e * 16 + col];
      if (e + W < it.e1) {
        tab1 = a.entry_tab[e + W];
        src1 = a.entry_src[(int64_t)(e + W) * 16 + col];
      }
      const R* src = mp + (int64_t)(s < 0 ? 0 : s) * NC * CW;
      load_tab(tab);
#pragma unroll
      for (int j = 0; j < KJ; ++j) load_b(src, s >= 0, j);
    }
    for (; e < it.e1; e += W) {
      // the two wavefronts that share a SIMD (w and w + W/2) would otherwise run at very
      // different speeds (the issue arbiter favours the older one) and the younger one would
      // finish alone; the one that is behind takes the higher priority
      if (W >= 8) {
        ++done_entries;
        if (lane == 0) __hip_atomic_store(ctl + 2 + wave, done_entries, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        const int partner = __hip_atomic_load(ctl + 2 + (wave + W / 2) % W, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (__builtin_amdgcn_readfirstlane(partner) < done_entries)
          __builtin_amdgcn_s_setprio(0);
        else
          __builtin_amdgcn_s_setprio(1);
      }
#pragma unroll
      for (int k = 0; k < NTV; ++k) *reinterpret_cast<TV*>(tb + (k * 64 + lane) * VEC) = tv[k];
      const int en = e + W, enn = e + 2 * W;
      const bool more = en < it.e1;
      int tab2 = 0, src2 = -1;
      if (enn < it.e1) {
        tab2 = a.entry_tab[enn];
        src2 = a.entry_src[(int64_t)enn * 16 + col];
      }
      if (more) load_tab(tab1);
      const int sn = src1;
      const R* srcn = mp + (int64_t)(sn < 0 ? 0 : sn) * NC * CW;
      tab1 = tab2;
      src1 = src2;
      int2 qb_next = *reinterpret_cast<const int2*>(sbq_l);
#pragma unroll
      for (int j = 0; j < KJ; ++j) {
        // the table bases of step j + 1 are read while step j runs
        const int2 qb = qb_next;
        if (j + 1 < KJ) qb_next = *reinterpret_cast<const int2*>(sbq_l + 2 * (j + 1));
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          const int qo = v ? qb.y : qb.x;
          (void)qo;
          R ar[RT], ai[RT];
#pragma unroll
          for (int r = 0; r < RT; ++r) {
            ar[r] = tb[ib[r] + qo];
            if constexpr (CPLX) ai[r] = tb[TS + ib[r] + qo];
          }
          const R br = bv[j][v * CW];
          const int h = NSET > 1 ? v : 0;
#pragma unroll
          for (int r = 0; r < RT; ++r) {
            if constexpr (CPLX) {
              const R bi = bv[j][v * CW + 1];
              vacc[h][r][0] = TL::mma(ar[r], br, vacc[h][r][0]);
              vacc[h][r][0] = TL::mma(-ai[r], bi, vacc[h][r][0]);
              vacc[h][r][1] = TL::mma(ar[r], bi, vacc[h][r][1]);
              vacc[h][r][1] = TL::mma(ai[r], br, vacc[h][r][1]);
            } else {
              vacc[h][r][0] = TL::mma(ar[r], br, vacc[h][r][0]);
            }
          }
#pragma unroll
          for (int jr = 0; jr < NREM; ++jr) {
            const double tr = (double)tb[ibr[jr] + qo];
            if constexpr (CPLX) {
              const double ti = (double)tb[TS + ibr[jr] + qo];
              const double xr = (double)br, xi = (double)bv[j][v * CW + 1];
              racc[jr][0] += tr * xr - ti * xi;
              racc[jr][1] += tr * xi + ti * xr;
            } else {
              racc[jr][0] += tr * (double)br;
            }
          }
        }
        if (more) load_b(srcn, sn >= 0, j);
      }
      if constexpr (ACC64) {
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
          for (int u = 0; u < CW; ++u) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
              double x = 0.0;
#pragma unroll
              for (int h = 0; h < NSET; ++h) x += (double)vacc[h][r][u][v];
              acc[r][u][v] += x;
            }
#pragma unroll
            for (int h = 0; h < NSET; ++h) vacc[h][r][u] = V{};
          }
      }
    }
    rot = (rot + nent) % W;
    if constexpr (!ACC64) {
#pragma unroll
      for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int u = 0; u < CW; ++u)
#pragma unroll
          for (int v = 0; v < NV; ++v) acc[r][u][v] = vacc[0][r][u][v];
    }
    // the VALU rows: add the four lane groups (K ranges) of every column
#pragma unroll
    for (int jr = 0; jr < NREM; ++jr)
#pragma unroll
      for (int u = 0; u < CW; ++u) {
        racc[jr][u] += __shfl_xor(racc[jr][u], 16, 64);
        racc[jr][u] += __shfl_xor(racc[jr][u], 32, 64);
      }

    // Hand-off of the item's sums without a barrier: every wavefront stores its sums in its own
    // LDS slot and counts itself in; the last one to arrive adds the slots in wavefront order
    // (a fixed order, so results are bit-reproducible), writes the item out and frees the slots.
    // A wavefront waits before storing only if the previous item's slots are not read yet.
    const int item_no = ii - w0;
    while (__hip_atomic_load(ctl + 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < item_no)
      __builtin_amdgcn_s_sleep(1);
    {
      double* slot = slots + (int64_t)wave * NACC * 64 + lane;
#pragma unroll
      for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int u = 0; u < CW; ++u)
#pragma unroll
          for (int v = 0; v < NV; ++v) slot[((r * CW + u) * NV + v) * 64] = acc[r][u][v];
#pragma unroll
      for (int jr = 0; jr < NREM; ++jr)
#pragma unroll
        for (int u = 0; u < CW; ++u) slot[(RT * CW * NV + jr * CW + u) * 64] = racc[jr][u];
    }
    int arrived = 0;
    if (lane == 0) arrived = __hip_atomic_fetch_add(ctl, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
    arrived = __builtin_amdgcn_readfirstlane(arrived);
    if (arrived != W - 1) continue;  // another wavefront finishes this item

#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int u = 0; u < CW; ++u)
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[r][u][v] = 0.0;
#pragma unroll
    for (int jr = 0; jr < NREM; ++jr)
#pragma unroll
      for (int u = 0; u < CW; ++u) racc[jr][u] = 0.0;
    for (int w = 0; w < W; ++w) {
      const double* slot = slots + (int64_t)w * NACC * 64 + lane;
#pragma unroll
      for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int u = 0; u < CW; ++u)
#pragma unroll
          for (int v = 0; v < NV; ++v) acc[r][u][v] += slot[((r * CW + u) * NV + v) * 64];
#pragma unroll
      for (int jr = 0; jr < NREM; ++jr)
#pragma unroll
        for (int u = 0; u < CW; ++u) racc[jr][u] += slot[(RT * CW * NV + jr * CW + u) * 64];
    }
    if (lane == 0) {
      __hip_atomic_store(ctl, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      __hip_atomic_store(ctl + 1, item_no + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    }

    const int nparts = a.tile_nparts[it.tile];
    const int t = a.tile_tgt[(int64_t)it.tile * 16 + col];
    if (nparts == 1) {
      if (t >= 0) {
        R* out = reinterpret_cast<R*>(a.local) + (int64_t)t * NC * CW;
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const int i = TR * r + TL::row(kq, v);
            if (i < NC) {
#pragma unroll
              for (int u = 0; u < CW; ++u) out[i * CW + u] = (R)((a.overwrite ? 0.0 : (double)out[i * CW + u]) + acc[r][u][v]);
            }
          }
        if (kq == 0) {
#pragma unroll
          for (int jr = 0; jr < NREM; ++jr)
#pragma unroll
            for (int u = 0; u < CW; ++u) {
              const int i = TR * RT + jr;
              out[i * CW + u] = (R)((a.overwrite ? 0.0 : (double)out[i * CW + u]) + racc[jr][u]);
            }
        }
      }
      continue;
    }
    // split tile: the last part of the tile to finish adds the parts in part order.  The others
    // leave their FP64 partials in scratch with device-scope atomic stores; a slot holds the
    // empty pattern (a signalling NaN, which no arithmetic produces) until its value arrives, and
    // the last part reads each value with device-scope atomic loads until none is empty, then
    // empties the slots again.  Coherence of each location is all this needs: no cache
    // write-back or invalidation, and the wait is only for stores already issued.
    constexpr int NCP = (NC + 15) / 16 * 16;
    const int64_t pstride = (int64_t)16 * NCP * CW;
    {
      double* mine = a.scratch + (int64_t)(a.tile_item0[it.tile] + it.part) * pstride;
#pragma unroll
      for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const int i = TR * r + TL::row(kq, v);
          if (i < NC) {
#pragma unroll
            for (int u = 0; u < CW; ++u)
              __hip_atomic_store(mine + (col * NCP + i) * CW + u, acc[r][u][v], __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
          }
        }
      if (kq == 0) {
#pragma unroll
        for (int jr = 0; jr < NREM; ++jr)
#pragma unroll
          for (int u = 0; u < CW; ++u)
            __hip_atomic_store(mine + (col * NCP + TR * RT + jr) * CW + u, racc[jr][u], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    int old = 0;
    if (lane == 0)
      old = __hip_atomic_fetch_add(a.counter + it.tile, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    old = __builtin_amdgcn_readfirstlane(old);
    if (old != nparts - 1) continue;
    // the last part: add all parts in part order, its own from registers, the others from
    // scratch at the same (lane, register) positions (all their loads issued before the sums)
    {
      double tot[RT][CW][NV], totr[NREM > 0 ? NREM : 1][CW];
#pragma unroll
      for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int u = 0; u < CW; ++u)
#pragma unroll
          for (int v = 0; v < NV; ++v) tot[r][u][v] = 0.0;
#pragma unroll
      for (int jr = 0; jr < (NREM > 0 ? NREM : 1); ++jr)
#pragma unroll
        for (int u = 0; u < CW; ++u) totr[jr][u] = 0.0;
      for (int pt = 0; pt < nparts; ++pt) {
        if (pt == it.part) {
#pragma unroll
          for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int u = 0; u < CW; ++u)
#pragma unroll
              for (int v = 0; v < NV; ++v) tot[r][u][v] += acc[r][u][v];
#pragma unroll
          for (int jr = 0; jr < NREM; ++jr)
#pragma unroll
            for (int u = 0; u < CW; ++u) totr[jr][u] += racc[jr][u];
          continue;
        }
        double* ps = a.scratch + (int64_t)(a.tile_item0[it.tile] + pt) * pstride;
        double lr[RT][CW][NV], lrr[NREM > 0 ? NREM : 1][CW];
        bool empty;
        int waits = 0;  // bounded: a slot that never fills gives NaN results, not a hang
        do {
          empty = false;
#pragma unroll
          for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int v = 0; v < NV; ++v) {
              const int i = TR * r + TL::row(kq, v);
#pragma unroll
              for (int u = 0; u < CW; ++u) {
                lr[r][u][v] = i < NC ? __hip_atomic_load(ps + (col * NCP + i) * CW + u, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT)
                                     : 0.0;
                empty |= __builtin_bit_cast(uint64_t, lr[r][u][v]) == kM2LPartialEmpty;
              }
            }
#pragma unroll
          for (int jr = 0; jr < NREM; ++jr)
#pragma unroll
            for (int u = 0; u < CW; ++u) {
              lrr[jr][u] = __hip_atomic_load(ps + (col * NCP + TR * RT + jr) * CW + u, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
              empty |= __builtin_bit_cast(uint64_t, lrr[jr][u]) == kM2LPartialEmpty;
            }
          empty = __builtin_amdgcn_ballot_w64(empty) != 0;
          if (empty) __builtin_amdgcn_s_sleep(2);
        } while (empty && ++waits < kM2LPartialMaxWaits);
        // empty the slot for the next launch (each value was read above by this lane)
        const double none = __builtin_bit_cast(double, kM2LPartialEmpty);
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const int i = TR * r + TL::row(kq, v);
            if (i < NC) {
#pragma unroll
              for (int u = 0; u < CW; ++u)
                __hip_atomic_store(ps + (col * NCP + i) * CW + u, none, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
          }
        if (kq == 0) {
#pragma unroll
          for (int jr = 0; jr < NREM; ++jr)
#pragma unroll
            for (int u = 0; u < CW; ++u)
              __hip_atomic_store(ps + (col * NCP + TR * RT + jr) * CW + u, none, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
        }
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
          for (int u = 0; u < CW; ++u)
#pragma unroll
            for (int v = 0; v < NV; ++v) tot[r][u][v] += lr[r][u][v];
#pragma unroll
        for (int jr = 0; jr < NREM; ++jr)
#pragma unroll
          for (int u = 0; u < CW; ++u) totr[jr][u] += lrr[jr][u];
      }
      if (t >= 0) {
        R* out = reinterpret_cast<R*>(a.local) + (int64_t)t * NC * CW;
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const int i = TR * r + TL::row(kq, v);
            if (i < NC) {
#pragma unroll
              for (int u = 0; u < CW; ++u) out[i * CW + u] = (R)((a.overwrite ? 0.0 : (double)out[i * CW + u]) + tot[r][u][v]);
            }
          }
        if (kq == 0) {
#pragma unroll
          for (int jr = 0; jr < NREM; ++jr)
#pragma unroll
            for (int u = 0; u < CW; ++u) {
              const int i = TR * RT + jr;
              out[i * CW + u] = (R)((a.overwrite ? 0.0 : (double)out[i * CW + u]) + totr[jr][u]);
            }
        }
      }
    }
    if (lane == 0) __hip_atomic_store(a.counter + it.tile, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <typename R, bool CPLX, int P, int C, int MAXT>
__global__ __launch_bounds__(MAXT) void m2l_stream_kernel(M2LStreamArgs a) {
  m2ls_workgroup<R, CPLX, P, C>(a);
}

// Registers a wavefront needs at least: accumulators, the ring of B pairs, the next entry's
// table, the row bases and the A operands of one step in flight.
template <typename R, bool CPLX, int P, int C>
constexpr int stream_min_regs() {
  using SH = SShape<R, CPLX, P, C>;
  constexpr int rw = (int)sizeof(R) / 4;  // registers per element
  return 2 * SH::NACC + (sizeof(R) == 4 ? SH::NSET * SH::RT * SH::CW * 4 : 0) + SH::KJ * 2 * SH::CW * rw +
         SH::NTV * 4 + SH::RT + (CPLX ? 4 : 2) * (SH::RT < 16 ? SH::RT : 16) * SH::CW * rw + 30;
}
// Two wavefronts per SIMD (512 threads) when that need leaves room for scheduling, else one.
template <typename R, bool CPLX, int P, int C>
constexpr int stream_max_threads() {
  return stream_min_regs<R, CPLX, P, C>() <= 200 ? 512 : 256;
}
// Instantiations whose need exceeds what one wavefront can hold use the tiled form.
template <typename R, bool CPLX, int P, int C>
constexpr bool stream_fits() {
  return stream_min_regs<R, CPLX, P, C>() <= 400;
}

template <typename R, bool CPLX, int P, int C>
int launch_stream_cfg(const M2LStreamArgs& a, int waves, size_t lds, hipStream_t s) {
  if constexpr (!stream_fits<R, CPLX, P, C>()) {
    return fail(FMM_EUNSUPPORTED, "streaming M2L: order too high for one wavefront's registers");
  } else {
  constexpr int MAXT = stream_max_threads<R, CPLX, P, C>();
  if (waves * 64 > MAXT) return fail(FMM_EUNSUPPORTED, "streaming M2L: too many wavefronts per workgroup");
  auto kern = m2l_stream_kernel<R, CPLX, P, C, MAXT>;
  if (lds > 65536) {
    static size_t granted = 0;  // per instantiation
    if (lds > granted) {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(FMM_EUNSUPPORTED, "streaming M2L needs " + std::to_string(lds) +
                                          " bytes of LDS per workgroup: " + hipGetErrorString(e));
      }
      granted = lds;
    }
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)a.n_wg), dim3((unsigned)(waves * 64)), lds, s, a);
  FMM_HIP_CHECK(hipGetLastError());
  return FMM_OK;
  }
}

// Instantiated (order, PDE order) pairs: the orders of the Laplace-type kernels (c = 2) and of
// the biharmonic kernel (c = 4) that the workloads use; complex dtypes (Helmholtz, c = 2) up to
// the order whose accumulators and operand registers fit one wavefront.
#define FMM_M2LS_REAL_ORDERS(X) \
  X(2, 2) X(4, 2) X(6, 2) X(8, 2) X(10, 2) X(12, 2) X(6, 4) X(8, 4) X(10, 4)
#define FMM_M2LS_CPLX_ORDERS(X) X(2, 2) X(4, 2) X(6, 2)

template <typename R, bool CPLX>
int launch_stream_typed(const M2LStreamArgs& a, int p, int c, int waves, size_t lds, hipStream_t s) {
#define FMM_M2LS_CASE(P_, C_) \
  if (p == P_ && c == C_) return launch_stream_cfg<R, CPLX, P_, C_>(a, waves, lds, s);
  if constexpr (CPLX) {
    FMM_M2LS_CPLX_ORDERS(FMM_M2LS_CASE)
  } else {
    FMM_M2LS_REAL_ORDERS(FMM_M2LS_CASE)
  }
#undef FMM_M2LS_CASE
  return fail(FMM_EUNSUPPORTED, "streaming M2L not instantiated for this order");
}

template <typename R, bool CPLX>
void stream_shape_typed(int p, int c, M2LStreamShape& sh) {
#define FMM_M2LS_SHAPE(P_, C_)                                     \
  if (p == P_ && c == C_) {                                        \
    using SH = SShape<R, CPLX, P_, C_>;                            \
    sh.ok = stream_fits<R, CPLX, P_, C_>() ? 1 : 0;                \
    sh.tsp = SH::TSP;                                              \
    sh.nacc = SH::NACC;                                            \
    sh.kj = SH::KJ;                                                \
    sh.max_waves = stream_max_threads<R, CPLX, P_, C_>() / 64;     \
    return;                                                        \
  }
  if constexpr (CPLX) {
    FMM_M2LS_CPLX_ORDERS(FMM_M2LS_SHAPE)
  } else {
    FMM_M2LS_REAL_ORDERS(FMM_M2LS_SHAPE)
  }
#undef FMM_M2LS_SHAPE
  sh.ok = 0;
}

template <typename R, bool CPLX>
__global__ void m2ls_table_layout_kernel(const double* src, R* dst, int64_t n, int ts, int tsp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * ts) return;
  const int64_t tb = i / ts, k = i % ts;
  if constexpr (CPLX) {
    dst[tb * tsp + k] = (R)src[2 * i];
    dst[tb * tsp + ts + k] = (R)src[2 * i + 1];
  } else {
    dst[tb * tsp + k] = (R)src[i];
  }
}

__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

int launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
  if (n <= 0) return FMM_OK;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  FMM_HIP_CHECK(hipGetLastError());
  return FMM_OK;
}

int launch_zero_i32(int32_t* p, int64_t n, hipStream_t s) {
  return launch_fill_u32(reinterpret_cast<uint32_t*>(p), n, 0u, s);
}

int launch_m2l_stream_tables(const double* src, void* dst, int64_t n, int ts, int tsp, int dtype, hipStream_t s) {
  const int64_t tot = n * ts;
  if (tot == 0) return FMM_OK;
  dim3 g((unsigned)((tot + 255) / 256)), t(256);
  switch (dtype) {
    case FMM_F64: hipLaunchKernelGGL((m2ls_table_layout_kernel<double, false>), g, t, 0, s, src, (double*)dst, n, ts, tsp); break;
    case FMM_F32: hipLaunchKernelGGL((m2ls_table_layout_kernel<float, false>), g, t, 0, s, src, (float*)dst, n, ts, tsp); break;
    case FMM_C128: hipLaunchKernelGGL((m2ls_table_layout_kernel<double, true>), g, t, 0, s, src, (double*)dst, n, ts, tsp); break;
    case FMM_C64: hipLaunchKernelGGL((m2ls_table_layout_kernel<float, true>), g, t, 0, s, src, (float*)dst, n, ts, tsp); break;
    default: return fail(FMM_EINVAL, "dtype");
  }
  FMM_HIP_CHECK(hipGetLastError());
  return FMM_OK;
}

M2LStreamShape m2l_stream_shape(int p, int c, int dtype) {
  M2LStreamShape sh{};
  switch (dtype) {
    case FMM_F64: stream_shape_typed<double, false>(p, c, sh); break;
    case FMM_F32: stream_shape_typed<float, false>(p, c, sh); break;
    case FMM_C128: stream_shape_typed<double, true>(p, c, sh); break;
    case FMM_C64: stream_shape_typed<float, true>(p, c, sh); break;
    default: break;
  }
  return sh;
}

int launch_m2l_stream(const M2LStreamArgs& a, int p, int c, int dtype, int waves, size_t lds, hipStream_t s) {
  if (a.n_wg == 0) return FMM_OK;
  switch (dtype) {
    case FMM_F64: return launch_stream_typed<double, false>(a, p, c, waves, lds, s);
    case FMM_F32: return launch_stream_typed<float, false>(a, p, c, waves, lds, s);
    case FMM_C128: return launch_stream_typed<double, true>(a, p, c, waves, lds, s);
    case FMM_C64: return launch_stream_typed<float, true>(a, p, c, waves, lds, s);
  }
  return fail(FMM_EINVAL, "dtype");
}

}  // namespace fmm
