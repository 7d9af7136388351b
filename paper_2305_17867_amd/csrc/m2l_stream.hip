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
//   * gathers the A operand of v_mfma 16x16x4 from that grid: T~[i, q] = grid[base(i) +
//     base(q)] with base(m) = (m_z S + m_x) S + m_y, so T~ is never expanded,
//   * takes the B operand (the 16 source multipoles) straight from global memory into
//     registers: lane group g (lanes 16 g .. 16 g + 15) holds the pair q = 8 j + 2 g, q + 1
//     for step j, so the four lane groups read 8 consecutive coefficients of each source;
//     the loads of the next entry are issued into the same registers as soon as a step has
//     consumed them.
// At the end of a workgroup's share of a tile the wavefronts' accumulators are added in a
// fixed tree order through LDS.
//
// Accumulation: FP64 dtypes accumulate in FP64 matrix-core registers.  FP32 dtypes run each
// entry (offset group) as an FP32 product with FP32 accumulation and add the entry's partial
// into FP64 registers, so the sum over the (up to 189 per level) offset groups is FP64.
// Complex dtypes use four real products per K step.  Rows past the last full 16-row tile (at
// most two) are contracted on the vector ALU in FP64.
#include "../../include/fmm.h"
#include "common.hpp"
#include "device_util.hpp"
#include "kernels.hpp"

namespace fmm {

namespace {

typedef double sd4 __attribute__((ext_vector_type(4)));
typedef float sf4 __attribute__((ext_vector_type(4)));

template <typename R>
struct SMF;
// Operand layouts: lane l supplies A[l & 15][l >> 4] and B[l >> 4][l & 15].  Register v of
// lane l holds C[row(l >> 4, v)][l & 15]:  f64: row = 4 v + (l >> 4);  f32: row = 4 (l >> 4) + v.
template <>
struct SMF<double> {
  using V = sd4;
  static __device__ inline V mma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int kq, int v) { return 4 * v + kq; }
};
template <>
struct SMF<float> {
  using V = sf4;
  static __device__ inline V mma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int kq, int v) { return 4 * kq + v; }
};

constexpr int n_full_c(int p) { return p < 0 ? 0 : (p + 1) * (p + 2) * (p + 3) / 6; }

// Compile-time shape of one (order, PDE order, dtype) instantiation.
template <typename R, bool CPLX, int P, int C>
struct SShape {
  static constexpr int CW = CPLX ? 2 : 1;
  static constexpr int NC = n_full_c(P) - n_full_c(P - C);      // |J|
  static constexpr int REM = NC % 16;
  static constexpr bool VALU_ROWS = NC > 16 && REM >= 1 && REM <= kMaxRem;
  static constexpr int RT = VALU_ROWS ? NC / 16 : (NC + 15) / 16;  // matrix-core row tiles
  static constexpr int NREM = VALU_ROWS ? REM : 0;                 // rows on the vector ALU
  static constexpr int KJ = (NC + 7) / 8;                          // B steps of 8 coefficients
  static constexpr int S = 2 * P + 1, SZ = 2 * C - 1;
  static constexpr int TS = SZ * S * S;                            // grid values per plane
  static constexpr int VEC = 16 / (int)sizeof(R);                  // elements per 128-bit load
  static constexpr int TSP = (CW * TS + 64 * VEC - 1) / (64 * VEC) * (64 * VEC);  // padded table
  static constexpr int NTV = TSP / (64 * VEC);                     // 128-bit table loads per lane
  static constexpr int NACC = RT * CW * 4 + NREM * CW;             // FP64 sums per lane
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
  constexpr bool ACC64 = sizeof(R) == 4;
  using V = typename SMF<R>::V;
  using BV = typename RVec<R, 2 * CW>::T;  // the lane's pair (q, q + 1) of one B step
  using TV = typename RVec<R, VEC>::T;     // one 128-bit table load
  extern __shared__ __align__(16) char smem_raw[];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int W = blockDim.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  R* const tb = reinterpret_cast<R*>(smem_raw) + wave * TSP;
  int* const sbq = reinterpret_cast<int*>(smem_raw + a.lds_sbq);  // [4][2 KJ] base(q), 0 past Nc

  for (int k = tid; k < 8 * KJ; k += blockDim.x) {
    const int g = k / (2 * KJ), jj = k - g * (2 * KJ);
    const int q = 8 * (jj >> 1) + 2 * g + (jj & 1);
    sbq[k] = q < NC ? a.jbase[q] : 0;
  }
  int ib[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int i = 16 * r + col;
    ib[r] = i < NC ? a.jbase[i] : 0;  // padded rows read a valid grid value, never stored
  }
  int ibr[NREM > 0 ? NREM : 1];
#pragma unroll
  for (int j = 0; j < NREM; ++j) ibr[j] = a.jbase[16 * RT + j];
  __syncthreads();

  const R* const mp = reinterpret_cast<const R*>(a.mpole);
  const R* const tabg = reinterpret_cast<const R*>(a.tab);
  const int* const sbq_l = sbq + kq * (2 * KJ);
  const int w0 = a.wg_item[blockIdx.x], w1 = a.wg_item[blockIdx.x + 1];
  int rot = 0;  // round-robin start: continues across the workgroup's items

  for (int ii = w0; ii < w1; ++ii) {
    const M2LItem it = a.items[ii];
    const int nent = it.e1 - it.e0;
    double acc[RT][CW][4];
    double racc[NREM > 0 ? NREM : 1][CW];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int u = 0; u < CW; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[r][u][v] = 0.0;
#pragma unroll
    for (int j = 0; j < (NREM > 0 ? NREM : 1); ++j)
#pragma unroll
      for (int u = 0; u < CW; ++u) racc[j][u] = 0.0;
    V vacc[RT][CW];  // FP64: the accumulators; FP32: one entry's partial
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int u = 0; u < CW; ++u) vacc[r][u] = V{};

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
    if (e < it.e1) {
      const int tab = a.entry_tab[e];
      const int s = a.entry_src[(int64_t)e * 16 + col];
      const R* src = mp + (int64_t)(s < 0 ? 0 : s) * NC * CW;
      load_tab(tab);
#pragma unroll
      for (int j = 0; j < KJ; ++j) load_b(src, s >= 0, j);
    }
    for (; e < it.e1; e += W) {
#pragma unroll
      for (int k = 0; k < NTV; ++k) *reinterpret_cast<TV*>(tb + (k * 64 + lane) * VEC) = tv[k];
      const int en = e + W;
      const bool more = en < it.e1;
      int sn = -1;
      if (more) {
        const int tabn = a.entry_tab[en];
        sn = a.entry_src[(int64_t)en * 16 + col];
        load_tab(tabn);
      }
      const R* srcn = mp + (int64_t)(sn < 0 ? 0 : sn) * NC * CW;
#pragma unroll
      for (int j = 0; j < KJ; ++j) {
        const int2 qb = *reinterpret_cast<const int2*>(sbq_l + 2 * j);
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          const int qo = v ? qb.y : qb.x;
          R ar[RT], ai[RT];
#pragma unroll
          for (int r = 0; r < RT; ++r) {
            ar[r] = tb[ib[r] + qo];
            if constexpr (CPLX) ai[r] = tb[TS + ib[r] + qo];
          }
          const R br = bv[j][v * CW];
#pragma unroll
          for (int r = 0; r < RT; ++r) {
            if constexpr (CPLX) {
              const R bi = bv[j][v * CW + 1];
              vacc[r][0] = SMF<R>::mma(ar[r], br, vacc[r][0]);
              vacc[r][0] = SMF<R>::mma(-ai[r], bi, vacc[r][0]);
              vacc[r][1] = SMF<R>::mma(ar[r], bi, vacc[r][1]);
              vacc[r][1] = SMF<R>::mma(ai[r], br, vacc[r][1]);
            } else {
              vacc[r][0] = SMF<R>::mma(ar[r], br, vacc[r][0]);
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
            for (int v = 0; v < 4; ++v) acc[r][u][v] += (double)vacc[r][u][v];
            vacc[r][u] = V{};
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
          for (int v = 0; v < 4; ++v) acc[r][u][v] = vacc[r][u][v];
    }
    // the VALU rows: add the four lane groups (K ranges) of every column
#pragma unroll
    for (int jr = 0; jr < NREM; ++jr)
#pragma unroll
      for (int u = 0; u < CW; ++u) {
        racc[jr][u] += __shfl_xor(racc[jr][u], 16, 64);
        racc[jr][u] += __shfl_xor(racc[jr][u], 32, 64);
      }

    // wavefront sums in a fixed tree order through LDS (the table buffers are free after the
    // barrier): at stride s, wavefront w (w mod 2s == s) hands its sums to wavefront w - s
    double* red = reinterpret_cast<double*>(smem_raw);
    for (int s = 1; s < W; s *= 2) {
      __syncthreads();
      if (wave % (2 * s) == s) {
        double* slot = red + (int64_t)(wave / (2 * s)) * NACC * 64 + lane;
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
          for (int u = 0; u < CW; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) slot[((r * CW + u) * 4 + v) * 64] = acc[r][u][v];
#pragma unroll
        for (int jr = 0; jr < NREM; ++jr)
#pragma unroll
          for (int u = 0; u < CW; ++u) slot[(RT * CW * 4 + jr * CW + u) * 64] = racc[jr][u];
      }
      __syncthreads();
      if (wave % (2 * s) == 0 && wave + s < W) {
        const double* slot = red + (int64_t)(wave / (2 * s)) * NACC * 64 + lane;
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
          for (int u = 0; u < CW; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[r][u][v] += slot[((r * CW + u) * 4 + v) * 64];
#pragma unroll
        for (int jr = 0; jr < NREM; ++jr)
#pragma unroll
          for (int u = 0; u < CW; ++u) racc[jr][u] += slot[(RT * CW * 4 + jr * CW + u) * 64];
      }
    }

    const int nparts = a.tile_nparts[it.tile];
    const int t = a.tile_tgt[(int64_t)it.tile * 16 + col];
    if (nparts == 1) {
      if (wave == 0 && t >= 0) {
        R* out = reinterpret_cast<R*>(a.local) + (int64_t)t * NC * CW;
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = 16 * r + SMF<R>::row(kq, v);
            if (i < NC) {
#pragma unroll
              for (int u = 0; u < CW; ++u) out[i * CW + u] = (R)((double)out[i * CW + u] + acc[r][u][v]);
            }
          }
        if (kq == 0) {
#pragma unroll
          for (int jr = 0; jr < NREM; ++jr)
#pragma unroll
            for (int u = 0; u < CW; ++u) {
              const int i = 16 * RT + jr;
              out[i * CW + u] = (R)((double)out[i * CW + u] + racc[jr][u]);
            }
        }
      }
      __syncthreads();  // the reduction area is reused by the next item's tables
      continue;
    }
    // split tile: FP64 partial to scratch; the last workgroup of the tile adds the parts in order
    constexpr int NCP = (NC + 15) / 16 * 16;
    const int64_t pstride = (int64_t)16 * NCP * CW;
    if (wave == 0) {
      double* mine = a.scratch + (int64_t)(a.tile_item0[it.tile] + it.part) * pstride;
#pragma unroll
      for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * r + SMF<R>::row(kq, v);
#pragma unroll
          for (int u = 0; u < CW; ++u) mine[(col * NCP + i) * CW + u] = acc[r][u][v];
        }
      if (kq == 0) {
#pragma unroll
        for (int jr = 0; jr < NREM; ++jr)
#pragma unroll
          for (int u = 0; u < CW; ++u) mine[(col * NCP + 16 * RT + jr) * CW + u] = racc[jr][u];
      }
      __threadfence();
    }
    __shared__ int s_last;
    __syncthreads();
    if (tid == 0) {
      const int old = atomicAdd(a.counter + it.tile, 1);
      s_last = (old == nparts - 1);
    }
    __syncthreads();
    if (s_last) {
      __threadfence();
      const double* parts = a.scratch + (int64_t)a.tile_item0[it.tile] * pstride;
      for (int k = tid; k < 16 * NC; k += blockDim.x) {
        const int c = k / NC, i = k - c * NC;
        const int tt = a.tile_tgt[(int64_t)it.tile * 16 + c];
        if (tt < 0) continue;
        double sr = 0.0, si = 0.0;
        for (int pt = 0; pt < nparts; ++pt) {
          const double* ps = parts + pt * pstride + (c * NCP + i) * CW;
          sr += ps[0];
          if constexpr (CPLX) si += ps[1];
        }
        R* out = reinterpret_cast<R*>(a.local) + (int64_t)tt * NC * CW;
        out[i * CW] = (R)((double)out[i * CW] + sr);
        if constexpr (CPLX) out[i * CW + 1] = (R)((double)out[i * CW + 1] + si);
      }
      if (tid == 0) atomicExch(a.counter + it.tile, 0);
    }
    __syncthreads();
  }
}

template <typename R, bool CPLX, int P, int C, int MAXT>
__global__ __launch_bounds__(MAXT) void m2l_stream_kernel(M2LStreamArgs a) {
  m2ls_workgroup<R, CPLX, P, C>(a);
}

// Two wavefronts per SIMD (512 threads) when the estimated register need of a wavefront fits
// in 256 registers, else one (256 threads, up to 512 registers).
template <typename R, bool CPLX, int P, int C>
constexpr int stream_max_threads() {
  using SH = SShape<R, CPLX, P, C>;
  constexpr int rw = (int)sizeof(R) / 4;  // registers per element
  constexpr int regs = 2 * SH::NACC + (sizeof(R) == 4 ? SH::RT * SH::CW * 4 : 0) + SH::KJ * 2 * SH::CW * rw +
                       SH::NTV * 4 + 2 * SH::RT * SH::CW * rw + 40;
  return regs <= 240 ? 512 : 256;
}

template <typename R, bool CPLX, int P, int C>
int launch_stream_cfg(const M2LStreamArgs& a, int waves, size_t lds, hipStream_t s) {
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

// Instantiated (order, PDE order) pairs: the orders of the Laplace-type kernels (c = 2) and of
// the biharmonic kernel (c = 4) that the workloads use; complex dtypes (Helmholtz, c = 2) up to
// the order whose accumulators and operand registers fit one wavefront.
#define FMM_M2LS_REAL_ORDERS(X) \
  X(2, 2) X(4, 2) X(6, 2) X(8, 2) X(10, 2) X(12, 2) X(6, 4) X(8, 4) X(10, 4)
#define FMM_M2LS_CPLX_ORDERS(X) X(2, 2) X(4, 2) X(6, 2) X(8, 2)

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
    sh.ok = 1;                                                     \
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

}  // namespace

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
