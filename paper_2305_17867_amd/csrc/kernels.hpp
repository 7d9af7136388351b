// Argument blocks and launchers of the device kernels.  Each launcher validates
// nothing (the C ABI layer has done that) and only enqueues work on `stream`.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fmm {

constexpr int kMaxRecTerms = 6;

// Compression recursion (Sec. 3.1), see RecTerm: for m_z >= c,
//   D_m = sum_k coef[k] * h^hpow[k] * D_{m + d[k]}    (scaled coefficients, level size h).
struct RecArgs {
  int n;
  int dx[kMaxRecTerms], dy[kMaxRecTerms], dz[kMaxRecTerms], hpow[kMaxRecTerms];
  double coef[kMaxRecTerms];
};

struct P2MArgs {
  int64_t n_box;
  const double* center;     // [n_box][3]
  const int32_t* level;     // [n_box]
  const int64_t* range;     // [n_box][2]
  const double* level_h;    // [n_levels]
  int32_t n_levels;
  int64_t n_pts;
  const void* xyz;          // [n_pts][3] real
  const void* w;            // [n_pts] dtype
  void* out;                // [n_box][Nc] dtype
  int32_t nc;
  int32_t c;
  RecArgs rec;
  double xsign;             // X = xsign (c - y) / h  (+1: multipole moments; -1: target moments)
  int32_t ny;               // workgroups per box (contiguous point chunks); > 1 needs part
  double* part;             // [n_box][ny][Nc] (x2 complex) FP64 per-chunk results, summed in chunk order
  // compression beta~ = M~^T alpha~ of each level, sparse rows j < Nc: the entries
  // cmp_ptr[l (Nc + 1) + j] .. cmp_ptr[l (Nc + 1) + j + 1] of cmp_col (full index) / cmp_val
  const int32_t* cmp_ptr;
  const int32_t* cmp_col;
  const double* cmp_val;
};

// Multipole-to-multipole and local-to-local translation between a parent box and its (up
// to eight) children.  Boxes are indices into the box arrays; child[8 k + i] < 0 means none.
struct TransArgs {
  int64_t n_parent;
  const int32_t* parent;    // [n_parent] box index
  const int32_t* child;     // [n_parent][8] box index, < 0: no child
  int64_t n_box;
  const double* center;     // [n_box][3]
  const int32_t* level;     // [n_box]
  const double* level_h;    // [n_levels]
  int32_t n_levels;
  void* coef;               // [n_box][Nc] dtype: multipoles (M2M) or locals (L2L)
  int32_t nc;
  int32_t c;
  RecArgs rec;
  // transposes: the M2M kernel with the translation reversed and the parent accumulated is
  // the transpose of L2L, the L2L kernel with the translation reversed that of M2M
  int32_t transpose;
};

struct L2PArgs {
  int64_t n_box;
  const double* center;
  const int32_t* level;
  const int64_t* range;
  const double* level_h;
  int32_t n_levels;
  int64_t n_pts;
  const void* xyz;          // [n_pts][3] real
  const void* local;        // [n_box][Nc] dtype
  void* pot;                // [n_pts] dtype, accumulated (may be null when grad is set)
  int32_t overwrite;        // 1: the potentials are stored, not added to
  int32_t nc;
  int32_t c;
  RecArgs rec;
  double xsign;             // X = xsign (x - c) / h  (+1: local evaluation; -1: at sources)
  void* grad;               // [n_pts][3] real, accumulated: gscale(x) * d phi / d x (optional)
  const void* gscale;       // [n_pts] real per-point factor of grad (null = 1)
  int64_t chunk;            // points of a box per workgroup chunk (set by the launcher)
  // decompression L~ = M~ theta~ of each level, sparse rows m >= Nc of the full order: entries
  // dec_ptr[l (Nfull + 1) + m] .. dec_ptr[l (Nfull + 1) + m + 1] of dec_col (kept index) / dec_val
  const int32_t* dec_ptr;
  const int32_t* dec_col;
  const double* dec_val;
};

// Compressed P2L and M2P over lists of boxes (fmm_p2l, fmm_m2p): for each k < n_tbox, the
// target box tbox[k] and the boxes list[list_ptr[k] .. list_ptr[k + 1]).
struct PointExpArgs {
  int64_t n_tbox;
  const int32_t* tbox;
  const int32_t* list_ptr;  // [n_tbox + 1], clamped to [0, n_list]
  const int32_t* list;      // [n_list] box ids (ids outside [0, n_box) are skipped)
  int64_t n_list, n_box;
  const double* center;     // [n_box][3]
  const int32_t* level;     // [n_box]
  const int64_t* range;     // [n_box][2] point ranges (targets for M2P, sources for P2L)
  const double* level_h;    // [n_levels]
  int32_t n_levels;
  int64_t n_pts;
  const void* xyz;          // [n_pts][3] real
  const void* w;            // P2L: [n_pts] weights
  const void* mpole;        // M2P: [n_box][Nc]
  void* out;                // M2P: [n_pts] potential; P2L: [n_box][Nc] local (both accumulated)
  const int32_t* jxyz;      // [Nc] kept index m packed as m_x | m_y << 8 | m_z << 16
  int32_t nc, p, c, kernel;
  double param;
};

struct TableArgs {
  int64_t n;
  const double* offset;  // [n][3] units of h
  const double* h;       // [n]
  void* out;             // [n][Sz][S][S] f64 or c128
  int32_t kernel;
  int32_t p2;            // 2p
  int32_t S, Sz;
  double param;
};

// One workgroup's share of a target tile: entries [e0, e1) of tile `tile`, part `part` of
// the tile's `nparts` (nparts > 1 => partial sums go through scratch, last one reduces).
struct M2LItem {
  int32_t tile, e0, e1, part;
};

// M2L launch limits: at most 8 wavefronts per workgroup; per-thread register prefetch of one
// entry in two size classes (table values, source-tile values).
constexpr int kM2LMaxThreads = 512;
constexpr int kMaxRem = 2;  // rows past the last full 16-row tile that go to the VALU instead
constexpr int kPrefT0 = 4, kPrefB0 = 12;
constexpr int kPrefT1 = 8, kPrefB1 = 16;
constexpr int kPrefT2 = 20, kPrefB2 = 24;

struct M2LArgs {
  const M2LItem* items;
  int32_t n_items;
  const int32_t* tile_tgt;     // [n_tiles][16 CT], -1 = empty column
  const int32_t* tile_nparts;  // [n_tiles]
  const int32_t* tile_item0;   // [n_tiles] first item of the tile
  int32_t* counter;            // [n_tiles], zero between launches
  double* scratch;             // [n_items][16 CT][nc_pad] (x2 complex) partials
  const int32_t* entry_tab;    // [n_entries]
  const int32_t* entry_src;    // [n_entries][16 CT], -1 = no source
  const void* tab;             // [n_tab][TS] table values (f64 / f32 / c128 / c64)
  const int32_t* jbase;        // [Nc] base offset of each kept index into a table
  const void* mpole;           // [n_box][Nc]
  void* local;                 // [n_box][Nc]
  int32_t nc, nc_pad;          // nc_pad = rows rounded to 16
  int32_t ts;                  // table size S*S*Sz
  int32_t ldb;                 // LDS row stride of the staged source tile (>= 4 k4p)
  int32_t k4p;                 // K steps per lane group (ceil(nc/4) rounded to the vector width)
  int32_t tab_off;             // offset of the source tile in an LDS buffer (elements)
  int32_t buf_elems;           // elements of one LDS buffer (two buffers)
  int32_t nt;                  // targets per tile (16 x column tiles of the workgroup)
  int32_t rtiles;              // matrix-core row tiles (16 rows each)
  int32_t nrem;                // rows 16 rtiles .. 16 rtiles + nrem - 1 contracted on the VALU
  int32_t nrg;                 // row groups: wavefront w owns row group w % nrg
  int32_t nks;                 // K splits: wavefront w takes K range (w / nrg) / (nt / (16 CT))
};

// Streaming form of the batched M2L: 16-target tiles, entries cut into one contiguous chunk
// per workgroup; workgroup g takes items wg_item[g] .. wg_item[g + 1] - 1 (each a tile and an
// entry range of it).  Split tiles keep FP64 partials in scratch slots tile_item0[tile] + part.
struct M2LStreamArgs {
  const M2LItem* items;        // [n_items]
  const int32_t* wg_item;      // [n_wg + 1]
  int32_t n_wg;
  const int32_t* tile_tgt;     // [n_tiles][16], -1 = empty column
  const int32_t* tile_nparts;  // [n_tiles]
  const int32_t* tile_item0;   // [n_tiles] first partial slot of a split tile
  int32_t* counter;            // [n_tiles], zero between launches
  double* scratch;             // [slots][16][nc rounded to 16] (x2 complex) FP64 partials
  const int32_t* entry_tab;    // [n_entries]
  const int32_t* entry_src;    // [n_entries][16], -1 = no source
  const void* tab;             // [n_tab][tsp] tables in the dtype (complex: re plane, im plane)
  const int32_t* jbase;        // [Nc] base offset of each kept index into a table
  const void* mpole;           // [n_box][Nc]
  void* local;                 // [n_box][Nc]
  int32_t overwrite;           // 1: the targets' rows are stored, not added to
  int32_t lds_slot;            // byte offset of the wavefronts' item-sum slots in LDS
  int32_t lds_sbq;             // byte offset of the q-base table (and two counters) in LDS
};

constexpr int kM2LStreamMaxWaves = 16;

// Compile-time facts of an instantiated streaming shape (ok = 0: not instantiated).
struct M2LStreamShape {
  int32_t ok, tsp, nacc, kj, max_waves;
};

// FFT form of the M2L (eq. convolution_m2l): spectra are Hermitian halves [Sz][S][(S+1)/2].
constexpr int kFftMaxPerThread = 16;  // frequencies per thread in the accumulation (256 threads)

struct FftArgs {
  int32_t S, Sz, nc;
  int64_t n_tab, n_src, n_tgt;
  const double* tab64;      // [n_tab][Sz][S][S] FP64 scaled derivative grids
  void* spec_tab;           // [n_tab][nh] complex R
  void* spec_src;           // [n_box][nh] complex R (rows of listed sources written)
  const int32_t* src_list;  // [n_src] source boxes
  const int32_t* tgt_list;  // [n_tgt] target boxes
  const int32_t* tgt_ptr;   // [n_tgt + 1] CSR into ent_*
  const int32_t* ent_tab;   // table of each (target, source) pair
  const int32_t* ent_src;   // source box of each pair
  const int32_t* jxyz;      // [nc] packed (m_x | m_y << 8 | m_z << 16)
  const double* taupow;     // [2p + 1] tau^k
  double tau;
  const void* mpole;        // [n_box][nc] R
  void* local;              // [n_box][nc] R, accumulated
};

// Persistent launch over several prepared batches (same dtype and launch shape).
constexpr int kM2LMultiMax = 32;
struct M2LMulti {
  const M2LArgs* args;  // [n_batches] device copies (mpole / local pointers replaced below)
  const int2* work;     // [n_work] (batch, item of the batch)
  int32_t n_work;
  const void* mpole[kM2LMultiMax];
  void* local[kM2LMultiMax];
};

struct DirectArgs {
  int64_t n_src, n_tgt;
  const void* src;
  const void* w;
  const void* tgt;
  void* pot;
  int32_t kernel;
  double param;
  int32_t split;  // lanes sharing one target (a power of two <= 64), each taking every split-th source
};

// Near field: for each listed target box, the direct sum over the sources of its neighbour
// boxes (CSR lists), added to the targets' potentials.
struct P2PArgs {
  int64_t n_tbox;
  const int32_t* tbox;       // [n_tbox] target box ids
  const int32_t* nbr_ptr;    // [n_tbox + 1]
  const int32_t* nbr;        // [n_nbr] source box ids
  int64_t n_nbr;
  int64_t n_box;
  const int64_t* tgt_range;  // [n_box][2]
  const int64_t* src_range;  // [n_box][2]
  int64_t n_src, n_tgt;
  const void* src;
  const void* w;
  const void* tgt;
  void* pot;                 // accumulated
  int32_t kernel;
  double param;
};

int launch_tables(const TableArgs& a, bool cplx, hipStream_t s);
int launch_m2p(const PointExpArgs& a, int dtype, hipStream_t s);
int launch_p2l(const PointExpArgs& a, int dtype, hipStream_t s);
int launch_p2p(const P2PArgs& a, int dtype, hipStream_t s);
int launch_p2m(const P2MArgs& a, int p, int dtype, hipStream_t s);
int launch_m2m(const TransArgs& a, int p, int dtype, hipStream_t s);
int launch_l2l(const TransArgs& a, int p, int dtype, hipStream_t s);
int launch_l2p(const L2PArgs& a, int p, int dtype, hipStream_t s);
int launch_m2l(const M2LArgs& a, int dtype, int rows_per_wave, int col_tiles, int pf_class, int nbuf, int waves,
               hipStream_t s);
void m2l_shape(M2LArgs& a, size_t real_bytes, bool cplx, int ct_total);
size_t m2l_lds_bytes(const M2LArgs& a, size_t real_bytes, int nbuf, int rt, bool cplx);
int m2l_prefetch_class(const M2LArgs& a, bool cplx, int ct_total, int waves);
bool m2l_shape_instantiated(int rows_per_wave, int col_tiles_per_wave);
int launch_direct(const DirectArgs& a, int dtype, hipStream_t s);
int launch_fft(const FftArgs& a, int dtype, int which, hipStream_t s);  // 0 tables, 1 sources, 2 targets
size_t fft_lds_bytes(int S, int Sz, size_t real_bytes, bool cplx);
int fft_half_y(int S, bool cplx);  // y frequencies kept per spectrum line
int launch_m2l_multi(const M2LMulti& m, int dtype, int rows_per_wave, int col_tiles, int pf_class, int nbuf,
                     size_t lds, int waves, int grid, hipStream_t s);
bool m2l_multi_shape_instantiated(int rows_per_wave, int col_tiles_per_wave);
int launch_convert_f32(const double* src, float* dst, int64_t n, hipStream_t s);
M2LStreamShape m2l_stream_shape(int p, int c, int dtype);
int launch_m2l_stream(const M2LStreamArgs& a, int p, int c, int dtype, int waves, size_t lds, hipStream_t s);
// FP64 tables [n][ts] (complex interleaved) -> [n][tsp] in the dtype, complex as a re plane then
// an im plane; the padding past CW ts must already be zero.
int launch_m2l_stream_tables(const double* src, void* dst, int64_t n, int ts, int tsp, int dtype, hipStream_t s);
// p[0 .. n-1] = 0 (or v) with a small kernel (capturable, unlike a memset node)
int launch_zero_i32(int32_t* p, int64_t n, hipStream_t s);
int launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);
// An empty slot of the streaming M2L's split-tile partials: a signalling NaN (quiet bit clear,
// payload nonzero), which no floating-point operation returns; both 32-bit halves are the word
// kM2LPartialEmptyWord, so a 32-bit fill writes it.
constexpr uint32_t kM2LPartialEmptyWord = 0x7FF7F7F7u;
constexpr uint64_t kM2LPartialEmpty = ((uint64_t)kM2LPartialEmptyWord << 32) | kM2LPartialEmptyWord;
// Polls of an empty slot before the reader gives up (about 0.2 s): the slot's NaN then reaches
// the output instead of the launch waiting for ever.
constexpr int kM2LPartialMaxWaits = 1 << 22;
int launch_m2l_table_layout(const double* src, void* dst, int64_t n, int ts, int dtype, hipStream_t s);

}  // namespace fmm
