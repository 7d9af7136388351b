// Octree construction and interaction lists on the device (the box hierarchy of Sec. 1 that the
// translation operators run over).  Integer work only: every result is exact.
//
// Points get 60-bit Morton keys (20 bits per axis, x highest within each bit triple); a stable
// radix sort of (key, index) gives the point order; the boxes of level l are the distinct 3l-bit
// key prefixes that occur (adaptive trees: only below boxes holding more than max_leaf points),
// stored level by level in increasing key order.  Lists are built by one thread per box that
// counts, then fills its row at an offset from an exclusive scan; rows that must be sorted by box
// id go through a segmented sort.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstdint>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "common.hpp"

using namespace fmm;

namespace {

constexpr int kAxisBits = 20;  // bits per axis of a point key
constexpr int kTpb = 256;
constexpr int64_t kMaxInt32 = 0x7fffffff;

// ----------------------------------------------------------------------------- keys

__host__ __device__ inline uint64_t spread3(uint64_t v) {
  // move bit b of a 20-bit value to bit 3b, in five shift-and-mask steps
  v &= 0xFFFFFull;
  v = (v | (v << 32)) & 0x1F00000000FFFFull;
  v = (v | (v << 16)) & 0x1F0000FF0000FFull;
  v = (v | (v << 8)) & 0x100F00F00F00F00Full;
  v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

__host__ __device__ inline uint32_t compact3(uint64_t v) {
  // inverse of spread3: bit 3b -> bit b
  v &= 0x1249249249249249ull;
  v = (v ^ (v >> 2)) & 0x10C30C30C30C30C3ull;
  v = (v ^ (v >> 4)) & 0x100F00F00F00F00Full;
  v = (v ^ (v >> 8)) & 0x1F0000FF0000FFull;
  v = (v ^ (v >> 16)) & 0x1F00000000FFFFull;
  v = (v ^ (v >> 32)) & 0x1FFFFFull;
  return (uint32_t)v;
}

__host__ __device__ inline uint64_t morton(int64_t i, int64_t j, int64_t k) {
  return (spread3((uint64_t)i) << 2) | (spread3((uint64_t)j) << 1) | spread3((uint64_t)k);
}

__device__ inline int64_t lower_bound(const uint64_t* a, int64_t n, uint64_t v) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__global__ void point_keys_kernel(int64_t n, const double* __restrict__ xyz, uint64_t* __restrict__ key,
                                  int64_t* __restrict__ idx, int32_t* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t c[3];
  const double scale = (double)(1 << kAxisBits);
  const int64_t top = (1 << kAxisBits) - 1;
  for (int a = 0; a < 3; ++a) {
    const double x = xyz[3 * i + a];
    if (!isfinite(x)) atomicOr(bad, 1);
    const double f = floor(x * scale);
    c[a] = !(f >= 0.0) ? 0 : (f >= (double)top ? top : (int64_t)f);
  }
  key[i] = morton(c[0], c[1], c[2]);
  idx[i] = i;
}

__global__ void gather_points_kernel(int64_t n, const double* __restrict__ xyz, const int64_t* __restrict__ perm,
                                     double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t s = perm[i];
  for (int a = 0; a < 3; ++a) out[3 * i + a] = xyz[3 * s + a];
}

// ----------------------------------------------------------------------------- levels

__global__ void iota_u64_kernel(int64_t n, uint64_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (uint64_t)i;
}

// refine[b] = the box of level lev holds more than max_leaf points and lev < max_depth
__global__ void refine_kernel(int64_t nb, const uint64_t* __restrict__ lkey, int lev, const uint64_t* __restrict__ pkey,
                              int64_t n, int64_t max_leaf, int max_depth, uint8_t* __restrict__ refine) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  int64_t cnt = n;
  if (lev > 0) {
    const int shift = 3 * (kAxisBits - lev);
    cnt = lower_bound(pkey, n, (lkey[b] + 1) << shift) - lower_bound(pkey, n, lkey[b] << shift);
  }
  refine[b] = (cnt > max_leaf && lev < max_depth) ? 1 : 0;
}

// head[i] = 1 where sorted point i starts a new child box (level lev + 1) inside a refined box
__global__ void head_kernel(int64_t n, const uint64_t* __restrict__ pkey, const uint64_t* __restrict__ lkey, int64_t nb,
                            int lev, const uint8_t* __restrict__ refine, int32_t* __restrict__ head) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t pre = pkey[i] >> (3 * (kAxisBits - lev));
  const int64_t pos = lower_bound(lkey, nb, pre);
  const bool in_refined = pos < nb && lkey[pos] == pre && refine[pos];
  const int cs = 3 * (kAxisBits - lev - 1);
  head[i] = (in_refined && (i == 0 || (pkey[i] >> cs) != (pkey[i - 1] >> cs))) ? 1 : 0;
}

__global__ void child_keys_kernel(int64_t n, const uint64_t* __restrict__ pkey, int lev, const int32_t* __restrict__ head,
                                  const int32_t* __restrict__ pos, uint64_t* __restrict__ ckey) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !head[i]) return;
  ckey[pos[i]] = pkey[i] >> (3 * (kAxisBits - lev - 1));
}

struct TreeView {
  int64_t n_box;
  int32_t n_levels;
  const int64_t* ls;  // level_start [n_levels + 1]
  const uint64_t* key;
  const int32_t* level;
  const int32_t* ijk;
  const int64_t* range;
  const uint8_t* leaf;
  const int32_t* parent;
  const int32_t* child0;
};

// level, ijk, centre and point range of every box
__global__ void box_kernel(int64_t n_box, const uint64_t* __restrict__ bkey, const int64_t* __restrict__ ls,
                           int n_levels, const uint64_t* __restrict__ pkey, int64_t n, int32_t* __restrict__ level,
                           int32_t* __restrict__ ijk, double* __restrict__ center, int64_t* __restrict__ range) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_box) return;
  int lev = 0;
  while (lev + 1 < n_levels && ls[lev + 1] <= b) ++lev;
  const uint64_t k = bkey[b];
  int64_t lo = 0, hi = n;
  if (lev > 0) {
    const int shift = 3 * (kAxisBits - lev);
    lo = lower_bound(pkey, n, k << shift);
    hi = lower_bound(pkey, n, (k + 1) << shift);
  }
  const int32_t c[3] = {(int32_t)compact3(k >> 2), (int32_t)compact3(k >> 1), (int32_t)compact3(k)};
  const double h = ldexp(1.0, -lev);
  level[b] = lev;
  for (int a = 0; a < 3; ++a) {
    ijk[3 * b + a] = c[a];
    center[3 * b + a] = ((double)c[a] + 0.5) * h;
  }
  range[2 * b] = lo;
  range[2 * b + 1] = hi;
}

__device__ inline int32_t find_box(const TreeView& t, int lev, int64_t i, int64_t j, int64_t k) {
  const int64_t side = (int64_t)1 << lev;
  if (i < 0 || j < 0 || k < 0 || i >= side || j >= side || k >= side) return -1;
  const int64_t a = t.ls[lev], nb = t.ls[lev + 1] - a;
  const uint64_t key = morton(i, j, k);
  const int64_t p = lower_bound(t.key + a, nb, key);
  return (p < nb && t.key[a + p] == key) ? (int32_t)(a + p) : -1;
}

// parent and first existing child of every box
__global__ void family_kernel(TreeView t, int32_t* __restrict__ parent, int32_t* __restrict__ child0) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= t.n_box) return;
  const int lev = t.level[b];
  const uint64_t k = t.key[b];
  int32_t par = -1, ch = -1;
  if (lev > 0) {
    const int64_t a = t.ls[lev - 1], nb = t.ls[lev] - a;
    par = (int32_t)(a + lower_bound(t.key + a, nb, k >> 3));
  }
  if (!t.leaf[b] && lev + 1 < t.n_levels) {
    const int64_t a = t.ls[lev + 1], nb = t.ls[lev + 2] - a;
    const int64_t p = lower_bound(t.key + a, nb, k << 3);
    if (p < nb && (t.key[a + p] >> 3) == k) ch = (int32_t)(a + p);
  }
  parent[b] = par;
  child0[b] = ch;
}

// ----------------------------------------------------------------------------- list helpers

__device__ inline bool touch(const TreeView& t, int32_t a, int32_t b) {
  // closed cubes of boxes a and b intersect
  const int la = t.level[a], lb = t.level[b];
  const int L = la > lb ? la : lb;
  const int64_t sa = (int64_t)1 << (L - la), sb = (int64_t)1 << (L - lb);
  for (int d = 0; d < 3; ++d) {
    const int64_t lo_a = (int64_t)t.ijk[3 * a + d] << (L - la);
    const int64_t lo_b = (int64_t)t.ijk[3 * b + d] << (L - lb);
    if (lo_a > lo_b + sb || lo_b > lo_a + sa) return false;
  }
  return true;
}

__device__ inline int32_t next_sibling(const TreeView& t, int32_t n) {
  const int lev = t.level[n];
  if ((int64_t)n + 1 >= t.ls[lev + 1]) return -1;
  return (t.key[n + 1] >> 3) == (t.key[n] >> 3) ? n + 1 : -1;
}

// Next box of a depth-first walk under `root` (boxes in octant order) after the subtree of n
// was finished; -1 when the walk is done.
__device__ inline int32_t walk_advance(const TreeView& t, int32_t n, int32_t root) {
  while (n != root) {
    const int32_t s = next_sibling(t, n);
    if (s >= 0) return s;
    n = t.parent[n];
  }
  return -1;
}

template <bool FILL>
__device__ inline void emit(int32_t* out, int64_t& c, int32_t v) {
  if (FILL) out[c] = v;
  ++c;
}

// List 2 of the boxes [b0, n_box): children of the parent's neighbours (parent included) that
// are not adjacent to the box.
template <bool FILL>
__global__ void list2_kernel(TreeView t, int64_t b0, int64_t* __restrict__ count, const int64_t* __restrict__ off,
                             int32_t* __restrict__ tgt, int32_t* __restrict__ src) {
  const int64_t b = b0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= t.n_box) return;
  const int lev = t.level[b];
  const int64_t x = t.ijk[3 * b], y = t.ijk[3 * b + 1], z = t.ijk[3 * b + 2];
  int64_t c = 0;
  const int64_t o = FILL ? off[b - b0] : 0;
  for (int64_t i = 2 * (x >> 1) - 2; i <= 2 * (x >> 1) + 3; ++i)
    for (int64_t j = 2 * (y >> 1) - 2; j <= 2 * (y >> 1) + 3; ++j)
      for (int64_t k = 2 * (z >> 1) - 2; k <= 2 * (z >> 1) + 3; ++k) {
        const int64_t di = i > x ? i - x : x - i, dj = j > y ? j - y : y - j, dk = k > z ? k - z : z - k;
        if (di <= 1 && dj <= 1 && dk <= 1) continue;
        const int32_t s = find_box(t, lev, i, j, k);
        if (s < 0) continue;
        if (FILL) {
          tgt[o + c] = (int32_t)b;
          src[o + c] = s;
        }
        ++c;
      }
  if (!FILL) count[b - b0] = c;
}

// Near lists of the leaves: on the leaf's own level every existing box adjacent to it (itself
// included), on every coarser level the leaves adjacent to its ancestor there; in the order
// level, then offset (di, dj, dk) lexicographic.
template <bool FILL>
__global__ void near_kernel(TreeView t, int64_t n_leaf, const int32_t* __restrict__ leaves, int64_t* __restrict__ count,
                            const int64_t* __restrict__ off, int32_t* __restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_leaf) return;
  const int32_t b = leaves[q];
  const int lb = t.level[b];
  int64_t c = 0;
  int32_t* dst = FILL ? out + off[q] : nullptr;
  for (int lev = 0; lev <= lb; ++lev) {
    const int sh = lb - lev;
    const int64_t x = t.ijk[3 * b] >> sh, y = t.ijk[3 * b + 1] >> sh, z = t.ijk[3 * b + 2] >> sh;
    for (int di = -1; di <= 1; ++di)
      for (int dj = -1; dj <= 1; ++dj)
        for (int dk = -1; dk <= 1; ++dk) {
          const int32_t n = find_box(t, lev, x + di, y + dj, z + dk);
          if (n >= 0 && (lev == lb || t.leaf[n])) emit<FILL>(dst, c, n);
        }
  }
  if (!FILL) count[q] = c;
}

// U and W lists of the leaves: every colleague (same-level box adjacent to the leaf, the leaf
// included) is walked down while its boxes touch the leaf; leaves met that way are U, boxes
// met that do not touch the leaf are W (not descended); coarser leaves adjacent to an ancestor
// that touch the leaf are U.  Unsorted; the rows are sorted afterwards.
template <bool FILL>
__global__ void uw_kernel(TreeView t, int64_t n_leaf, const int32_t* __restrict__ leaves, int64_t* __restrict__ count,
                          const int64_t* __restrict__ off, int32_t* __restrict__ u_out, int32_t* __restrict__ w_out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_leaf) return;
  const int32_t b = leaves[q];
  const int lb = t.level[b];
  int64_t cu = 0, cw = 0;
  int32_t* du = FILL ? u_out + off[2 * q] : nullptr;
  int32_t* dw = FILL ? w_out + off[2 * q + 1] : nullptr;
  const int64_t x = t.ijk[3 * b], y = t.ijk[3 * b + 1], z = t.ijk[3 * b + 2];
  for (int di = -1; di <= 1; ++di)
    for (int dj = -1; dj <= 1; ++dj)
      for (int dk = -1; dk <= 1; ++dk) {
        const int32_t col = find_box(t, lb, x + di, y + dj, z + dk);
        if (col < 0) continue;
        if (t.leaf[col]) {
          emit<FILL>(du, cu, col);
          continue;
        }
        int32_t n = t.child0[col];
        while (n >= 0) {
          if (touch(t, n, b)) {
            if (t.leaf[n]) {
              emit<FILL>(du, cu, n);
            } else {
              n = t.child0[n];
              continue;
            }
          } else {
            emit<FILL>(dw, cw, n);
          }
          n = walk_advance(t, n, col);
        }
      }
  for (int lev = 0; lev < lb; ++lev) {
    const int sh = lb - lev;
    const int64_t ax = x >> sh, ay = y >> sh, az = z >> sh;
    for (int di = -1; di <= 1; ++di)
      for (int dj = -1; dj <= 1; ++dj)
        for (int dk = -1; dk <= 1; ++dk) {
          const int32_t n = find_box(t, lev, ax + di, ay + dj, az + dk);
          if (n >= 0 && t.leaf[n] && touch(t, n, b)) emit<FILL>(du, cu, n);
        }
  }
  if (!FILL) {
    count[2 * q] = cu;
    count[2 * q + 1] = cw;
  }
}

// X list of every box a below the root: leaves coarser than a that touch a's parent but not a.
template <bool FILL>
__global__ void x_kernel(TreeView t, int64_t* __restrict__ count, const int64_t* __restrict__ off,
                         int32_t* __restrict__ out) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= t.n_box) return;
  const int la = t.level[a];
  int64_t c = 0;
  int32_t* dst = FILL ? out + off[a] : nullptr;
  if (la > 0) {
    const int32_t pa = t.parent[a];
    for (int lev = 0; lev < la; ++lev) {
      const int sh = la - lev;
      const int64_t x = t.ijk[3 * a] >> sh, y = t.ijk[3 * a + 1] >> sh, z = t.ijk[3 * a + 2] >> sh;
      for (int di = -1; di <= 1; ++di)
        for (int dj = -1; dj <= 1; ++dj)
          for (int dk = -1; dk <= 1; ++dk) {
            const int32_t n = find_box(t, lev, x + di, y + dj, z + dk);
            if (n >= 0 && t.leaf[n] && touch(t, n, pa) && !touch(t, n, (int32_t)a)) emit<FILL>(dst, c, n);
          }
    }
  }
  if (!FILL) count[a] = c;
}

// Rows whose boxes hold more than max_src points in all are cut: boxes above max_src points are
// replaced by their children (depth first, down to leaves), then the boxes are packed in order
// into entries of at most max_src points (a box above the cap on its own).  count[2r] entries and
// count[2r + 1] list items of row r; the fill pass writes owner, the entry ends and the items.
template <bool FILL>
__global__ void split_kernel(TreeView t, int64_t n_row, const int32_t* __restrict__ row_box,
                             const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ items, int64_t max_src,
                             int64_t* __restrict__ count, const int64_t* __restrict__ off, int32_t* __restrict__ owner,
                             int32_t* __restrict__ ptr, int32_t* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_row) return;
  int64_t ne = 0, ni = 0, run = 0;
  const int64_t e0 = FILL ? off[2 * r] : 0, i0 = FILL ? off[2 * r + 1] : 0;
  const int32_t b = row_box[r];
  for (int64_t s = row_ptr[r]; s < row_ptr[r + 1]; ++s) {
    const int32_t root = items[s];
    int32_t n = root;
    while (n >= 0) {
      const int64_t cnt = t.range[2 * n + 1] - t.range[2 * n];
      if (cnt > max_src && !t.leaf[n]) {
        n = t.child0[n];
        continue;
      }
      if (run > 0 && run + cnt > max_src) {  // close the current entry
        if (FILL) {
          owner[e0 + ne] = b;
          ptr[e0 + ne + 1] = (int32_t)(i0 + ni);
        }
        ++ne;
        run = 0;
      }
      if (FILL) out[i0 + ni] = n;
      ++ni;
      run += cnt;
      n = walk_advance(t, n, root);
    }
  }
  if (FILL) {
    owner[e0 + ne] = b;
    ptr[e0 + ne + 1] = (int32_t)(i0 + ni);
  }
  ++ne;
  if (!FILL) {
    count[2 * r] = ne;
    count[2 * r + 1] = ni;
  }
}

__global__ void leaves_kernel(int64_t n_box, const uint8_t* __restrict__ leaf, const int64_t* __restrict__ pos,
                              int32_t* __restrict__ out) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b < n_box && leaf[b]) out[pos[b]] = (int32_t)b;
}

// rows with at least one item: row ids (box[r] = ids[k]) and their starts
__global__ void compact_rows_kernel(int64_t n, const int32_t* __restrict__ ids, const int64_t* __restrict__ cnt,
                                    const int64_t* __restrict__ off, const int64_t* __restrict__ rpos,
                                    int32_t* __restrict__ box, int32_t* __restrict__ ptr) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n || cnt[k] == 0) return;
  box[rpos[k]] = ids ? ids[k] : (int32_t)k;
  ptr[rpos[k] + 1] = (int32_t)(off[k] + cnt[k]);
}

__global__ void nonzero_kernel(int64_t n, const int64_t* __restrict__ cnt, int64_t stride, int64_t* __restrict__ flag) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) flag[k] = cnt[k * stride] != 0 ? 1 : 0;
}

__global__ void strided_kernel(int64_t n, const int64_t* __restrict__ in, int64_t stride, int64_t* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = in[k * stride];
}

__global__ void interleave_kernel(int64_t n, const int64_t* __restrict__ a, const int64_t* __restrict__ b,
                                  int64_t* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) {
    out[2 * k] = a[k];
    out[2 * k + 1] = b[k];
  }
}

__global__ void to_i32_kernel(int64_t n, const int64_t* __restrict__ in, int32_t* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = (int32_t)in[k];
}

__global__ void leaf_from_refine_kernel(int64_t n, uint8_t* __restrict__ flag) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) flag[k] = flag[k] ? 0 : 1;
}

__global__ void widen_u8_kernel(int64_t n, const uint8_t* __restrict__ in, int64_t* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = in[k];
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + kTpb - 1) / kTpb); }

}  // namespace

// ----------------------------------------------------------------------------- host objects

struct TreeList {
  int64_t n_row = 0, n_item = 0;
  int32_t *box = nullptr, *ptr = nullptr, *item = nullptr;
};

struct fmm_tree_s {
  int64_t n = 0, n_box = 0;
  int32_t n_levels = 0, max_leaf = 0, depth = 0;
  std::vector<int64_t> level_start;
  int64_t* d_ls = nullptr;
  uint64_t* d_pkey = nullptr;
  int64_t* d_perm = nullptr;
  double* d_points = nullptr;
  uint64_t* d_bkey = nullptr;
  int32_t *d_level = nullptr, *d_ijk = nullptr, *d_parent = nullptr, *d_child0 = nullptr;
  double* d_center = nullptr;
  int64_t* d_range = nullptr;
  uint8_t* d_leaf = nullptr;
  int64_t n_leaf = 0;
  int32_t* d_leaves = nullptr;
  // List 2 of all levels, sorted by (target, source); l2_off[l] = first pair of level l
  bool has_l2 = false;
  std::vector<int64_t> l2_off;
  int32_t *d_l2_tgt = nullptr, *d_l2_src = nullptr;
  std::map<std::pair<int, int64_t>, TreeList> lists;  // (kind, max_src) -> rows
  bool alive = true;

  TreeView view() const {
    return TreeView{n_box, n_levels, d_ls, d_bkey, d_level, d_ijk, d_range, d_leaf, d_parent, d_child0};
  }
};

namespace {

void free_list(TreeList& l) {
  (void)hipFree(l.box);
  (void)hipFree(l.ptr);
  (void)hipFree(l.item);
  l = TreeList{};
}

void free_tree(fmm_tree t) {
  void* ptrs[] = {t->d_ls, t->d_pkey, t->d_perm, t->d_points, t->d_bkey, t->d_level, t->d_ijk,
                  t->d_parent, t->d_child0, t->d_center, t->d_range, t->d_leaf, t->d_leaves,
                  t->d_l2_tgt, t->d_l2_src};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (auto& kv : t->lists) free_list(kv.second);
  t->lists.clear();
}

// Device buffers freed on scope exit (temporaries of one call).
struct Scratch {
  std::vector<void*> ptrs;
  ~Scratch() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <typename T>
  int get(T** out, int64_t count) {
    *out = nullptr;
    if (count <= 0) count = 1;
    hipError_t e = hipMalloc((void**)out, (size_t)count * sizeof(T));
    if (e != hipSuccess) return fail(FMM_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    ptrs.push_back(*out);
    return FMM_OK;
  }
};

template <typename T>
int dev_alloc(T** out, int64_t count) {
  *out = nullptr;
  if (count <= 0) count = 1;
  hipError_t e = hipMalloc((void**)out, (size_t)count * sizeof(T));
  if (e != hipSuccess) return fail(FMM_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  return FMM_OK;
}

#define TREE_TRY(x)             \
  do {                          \
    int st_ = (x);              \
    if (st_ != FMM_OK) return st_; \
  } while (0)

// out[0..n] = exclusive sum of in[0..n) (out[n] = total); returns the total on the host
int exclusive_scan(const int64_t* in, int64_t* out, int64_t n, int64_t* total, hipStream_t s) {
  Scratch sc;
  int64_t* tmp_in;
  TREE_TRY(sc.get(&tmp_in, n + 1));
  if (n > 0) FMM_HIP_CHECK(hipMemcpyAsync(tmp_in, in, n * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
  const int64_t zero = 0;
  FMM_HIP_CHECK(hipMemcpyAsync(tmp_in + n, &zero, sizeof(int64_t), hipMemcpyHostToDevice, s));
  size_t bytes = 0;
  FMM_HIP_CHECK(hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, tmp_in, out, n + 1, s));
  void* tmp;
  TREE_TRY(sc.get((char**)&tmp, (int64_t)bytes));
  FMM_HIP_CHECK(hipcub::DeviceScan::ExclusiveSum(tmp, bytes, tmp_in, out, n + 1, s));
  FMM_HIP_CHECK(hipMemcpyAsync(total, out + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  FMM_HIP_CHECK(hipStreamSynchronize(s));
  return FMM_OK;
}

// sort the items of every row (rows given by int64 starts off[0..n_row]) in place
int sort_rows(int32_t* items, int64_t n_item, const int64_t* off, int64_t n_row, hipStream_t s) {
  if (n_item == 0 || n_row == 0) return FMM_OK;
  FMM_REQUIRE(n_item <= kMaxInt32 && n_row <= kMaxInt32, FMM_EUNSUPPORTED, "list too long to sort");
  Scratch sc;
  int32_t *tmp_out, *off32;
  TREE_TRY(sc.get(&tmp_out, n_item));
  TREE_TRY(sc.get(&off32, n_row + 1));
  to_i32_kernel<<<blocks(n_row + 1), kTpb, 0, s>>>(n_row + 1, off, off32);
  size_t bytes = 0;
  FMM_HIP_CHECK(hipcub::DeviceSegmentedSort::SortKeys(nullptr, bytes, items, tmp_out, (int)n_item, (int)n_row,
                                                      off32, off32 + 1, s));
  char* tmp;
  TREE_TRY(sc.get(&tmp, (int64_t)bytes));
  FMM_HIP_CHECK(hipcub::DeviceSegmentedSort::SortKeys(tmp, bytes, items, tmp_out, (int)n_item, (int)n_row, off32,
                                                      off32 + 1, s));
  FMM_HIP_CHECK(hipMemcpyAsync(items, tmp_out, n_item * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  FMM_HIP_CHECK(hipStreamSynchronize(s));
  return FMM_OK;
}

// rows of the ids whose count is nonzero: out.box (ids[k], or k when ids is NULL), out.ptr
int compact_rows(const int32_t* ids, const int64_t* cnt, const int64_t* off, int64_t n, int32_t* items,
                 int64_t n_item, TreeList& out, hipStream_t s) {
  Scratch sc;
  int64_t *flag, *rpos, n_row = 0;
  TREE_TRY(sc.get(&flag, n));
  TREE_TRY(sc.get(&rpos, n + 1));
  if (n > 0) nonzero_kernel<<<blocks(n), kTpb, 0, s>>>(n, cnt, 1, flag);
  TREE_TRY(exclusive_scan(flag, rpos, n, &n_row, s));
  TREE_TRY(dev_alloc(&out.box, n_row));
  TREE_TRY(dev_alloc(&out.ptr, n_row + 1));
  FMM_HIP_CHECK(hipMemsetAsync(out.ptr, 0, sizeof(int32_t), s));
  if (n > 0) compact_rows_kernel<<<blocks(n), kTpb, 0, s>>>(n, ids, cnt, off, rpos, out.box, out.ptr);
  out.n_row = n_row;
  out.n_item = n_item;
  out.item = items;
  FMM_HIP_CHECK(hipStreamSynchronize(s));
  return FMM_OK;
}

// Split rows (box, ptr as int64 starts, items) by max_src into `out` (owner, ptr, items).
int split_rows(const fmm_tree t, int64_t n_row, const int32_t* row_box, const int64_t* row_off, const int32_t* items,
               int64_t max_src, TreeList& out, hipStream_t s) {
  Scratch sc;
  int64_t *cnt, *off, total = 0;
  TREE_TRY(sc.get(&cnt, 2 * n_row));
  TREE_TRY(sc.get(&off, 2 * n_row + 1));
  const TreeView v = t->view();
  if (n_row > 0)
    split_kernel<false><<<blocks(n_row), kTpb, 0, s>>>(v, n_row, row_box, row_off, items, max_src, cnt, nullptr,
                                                      nullptr, nullptr, nullptr);
  // entries and items are scanned separately: off_e[r], off_i[r]
  int64_t *ce, *ci, *oe, *oi, n_ent = 0, n_item = 0;
  TREE_TRY(sc.get(&ce, n_row));
  TREE_TRY(sc.get(&ci, n_row));
  TREE_TRY(sc.get(&oe, n_row + 1));
  TREE_TRY(sc.get(&oi, n_row + 1));
  if (n_row > 0) {
    strided_kernel<<<blocks(n_row), kTpb, 0, s>>>(n_row, cnt, 2, ce);
    strided_kernel<<<blocks(n_row), kTpb, 0, s>>>(n_row, cnt + 1, 2, ci);
  }
  TREE_TRY(exclusive_scan(ce, oe, n_row, &n_ent, s));
  TREE_TRY(exclusive_scan(ci, oi, n_row, &n_item, s));
  FMM_REQUIRE(n_ent <= kMaxInt32 && n_item <= kMaxInt32, FMM_EUNSUPPORTED, "lists exceed 2^31 entries");
  if (n_row > 0) interleave_kernel<<<blocks(n_row), kTpb, 0, s>>>(n_row, oe, oi, off);
  TREE_TRY(dev_alloc(&out.box, n_ent));
  TREE_TRY(dev_alloc(&out.ptr, n_ent + 1));
  TREE_TRY(dev_alloc(&out.item, n_item));
  FMM_HIP_CHECK(hipMemsetAsync(out.ptr, 0, sizeof(int32_t), s));
  if (n_row > 0)
    split_kernel<true><<<blocks(n_row), kTpb, 0, s>>>(v, n_row, row_box, row_off, items, max_src, nullptr, off,
                                                     out.box, out.ptr, out.item);
  out.n_row = n_ent;
  out.n_item = n_item;
  FMM_HIP_CHECK(hipStreamSynchronize(s));
  return FMM_OK;
}

int build_levels_adaptive(fmm_tree t, int64_t max_leaf, int max_depth, std::vector<uint64_t*>& lkeys,
                          std::vector<int64_t>& lcount, std::vector<uint8_t*>& lrefine, hipStream_t s) {
  const int64_t n = t->n;
  Scratch sc;
  int32_t *head = nullptr, *pos = nullptr;
  size_t bytes = 0;
  char* tmp = nullptr;
  if (n > 0) {
    TREE_TRY(sc.get(&head, n));
    TREE_TRY(sc.get(&pos, n));
    FMM_HIP_CHECK(hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, head, pos, n, s));
    TREE_TRY(sc.get(&tmp, (int64_t)bytes));
  }
  uint64_t* root;
  TREE_TRY(dev_alloc(&root, 1));
  lkeys.push_back(root);
  lcount.push_back(1);
  const uint64_t zero = 0;
  FMM_HIP_CHECK(hipMemcpyAsync(root, &zero, sizeof(uint64_t), hipMemcpyHostToDevice, s));
  for (int lev = 0;; ++lev) {
    const int64_t nb = lcount[lev];
    uint8_t* ref;
    TREE_TRY(dev_alloc(&ref, nb));
    lrefine.push_back(ref);
    refine_kernel<<<blocks(nb), kTpb, 0, s>>>(nb, lkeys[lev], lev, t->d_pkey, n, max_leaf, max_depth, ref);
    if (n == 0 || lev >= max_depth) break;
    head_kernel<<<blocks(n), kTpb, 0, s>>>(n, t->d_pkey, lkeys[lev], nb, lev, ref, head);
    FMM_HIP_CHECK(hipcub::DeviceScan::ExclusiveSum(tmp, bytes, head, pos, n, s));
    int32_t last[2];
    FMM_HIP_CHECK(hipMemcpyAsync(&last[0], pos + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    FMM_HIP_CHECK(hipMemcpyAsync(&last[1], head + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    FMM_HIP_CHECK(hipStreamSynchronize(s));
    const int64_t nc = (int64_t)last[0] + last[1];
    if (nc == 0) break;  // no box refined: every box of this level is a leaf
    uint64_t* ck;
    TREE_TRY(dev_alloc(&ck, nc));
    lkeys.push_back(ck);
    lcount.push_back(nc);
    child_keys_kernel<<<blocks(n), kTpb, 0, s>>>(n, t->d_pkey, lev, head, pos, ck);
  }
  return FMM_OK;
}

int check_tree(fmm_tree t) {
  if (!t) return fail(FMM_EINVAL, "tree is NULL");
  if (!t->alive) return fail(FMM_ESTATE, "tree was destroyed");
  return FMM_OK;
}

int build_list2(fmm_tree t, hipStream_t s) {
  if (t->has_l2) return FMM_OK;
  const int64_t b0 = t->n_levels > 2 ? t->level_start[2] : t->n_box;
  const int64_t nt = t->n_box - b0;
  Scratch sc;
  int64_t *cnt, *off, total = 0;
  TREE_TRY(sc.get(&cnt, nt));
  TREE_TRY(sc.get(&off, nt + 1));
  const TreeView v = t->view();
  if (nt > 0) list2_kernel<false><<<blocks(nt), kTpb, 0, s>>>(v, b0, cnt, nullptr, nullptr, nullptr);
  TREE_TRY(exclusive_scan(cnt, off, nt, &total, s));
  FMM_REQUIRE(total <= kMaxInt32, FMM_EUNSUPPORTED, "more than 2^31 List-2 pairs");
  TREE_TRY(dev_alloc(&t->d_l2_tgt, total));
  TREE_TRY(dev_alloc(&t->d_l2_src, total));
  if (nt > 0) list2_kernel<true><<<blocks(nt), kTpb, 0, s>>>(v, b0, nullptr, off, t->d_l2_tgt, t->d_l2_src);
  TREE_TRY(sort_rows(t->d_l2_src, total, off, nt, s));
  // first pair of every level (levels below 2 have none)
  t->l2_off.assign(t->n_levels + 1, 0);
  for (int l = 0; l <= t->n_levels; ++l) {
    const int64_t b = l < t->n_levels ? std::max(t->level_start[l], b0) : t->n_box;
    if (b - b0 >= nt) {
      t->l2_off[l] = total;
    } else {
      FMM_HIP_CHECK(hipMemcpy(&t->l2_off[l], off + (b - b0), sizeof(int64_t), hipMemcpyDeviceToHost));
    }
  }
  t->has_l2 = true;
  return FMM_OK;
}

int build_near(fmm_tree t, TreeList& out, hipStream_t s) {
  const int64_t nl = t->n_leaf;
  Scratch sc;
  int64_t *cnt, *off, total = 0;
  TREE_TRY(sc.get(&cnt, nl));
  TREE_TRY(sc.get(&off, nl + 1));
  const TreeView v = t->view();
  if (nl > 0) near_kernel<false><<<blocks(nl), kTpb, 0, s>>>(v, nl, t->d_leaves, cnt, nullptr, nullptr);
  TREE_TRY(exclusive_scan(cnt, off, nl, &total, s));
  FMM_REQUIRE(total <= kMaxInt32, FMM_EUNSUPPORTED, "near lists exceed 2^31 entries");
  TREE_TRY(dev_alloc(&out.item, total));
  if (nl > 0) near_kernel<true><<<blocks(nl), kTpb, 0, s>>>(v, nl, t->d_leaves, nullptr, off, out.item);
  TREE_TRY(dev_alloc(&out.box, nl));
  TREE_TRY(dev_alloc(&out.ptr, nl + 1));
  if (nl > 0) FMM_HIP_CHECK(hipMemcpyAsync(out.box, t->d_leaves, nl * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  to_i32_kernel<<<blocks(nl + 1), kTpb, 0, s>>>(nl + 1, off, out.ptr);
  out.n_row = nl;
  out.n_item = total;
  FMM_HIP_CHECK(hipStreamSynchronize(s));
  return FMM_OK;
}

int build_uwx(fmm_tree t, TreeList& U, TreeList& Wl, TreeList& X, hipStream_t s) {
  const int64_t nl = t->n_leaf, nb = t->n_box;
  const TreeView v = t->view();
  Scratch sc;
  // U and W: counts interleaved per leaf
  int64_t *cnt, *cu, *cw, *ou, *ow, *off, n_u = 0, n_w = 0;
  TREE_TRY(sc.get(&cnt, 2 * nl));
  TREE_TRY(sc.get(&cu, nl));
  TREE_TRY(sc.get(&cw, nl));
  TREE_TRY(sc.get(&ou, nl + 1));
  TREE_TRY(sc.get(&ow, nl + 1));
  TREE_TRY(sc.get(&off, 2 * nl + 1));
  if (nl > 0) {
    uw_kernel<false><<<blocks(nl), kTpb, 0, s>>>(v, nl, t->d_leaves, cnt, nullptr, nullptr, nullptr);
    strided_kernel<<<blocks(nl), kTpb, 0, s>>>(nl, cnt, 2, cu);
    strided_kernel<<<blocks(nl), kTpb, 0, s>>>(nl, cnt + 1, 2, cw);
  }
  TREE_TRY(exclusive_scan(cu, ou, nl, &n_u, s));
  TREE_TRY(exclusive_scan(cw, ow, nl, &n_w, s));
  FMM_REQUIRE(n_u <= kMaxInt32 && n_w <= kMaxInt32, FMM_EUNSUPPORTED, "lists exceed 2^31 entries");
  int32_t *u_items, *w_items;
  TREE_TRY(dev_alloc(&u_items, n_u));
  TREE_TRY(dev_alloc(&w_items, n_w));
  if (nl > 0) {
    interleave_kernel<<<blocks(nl), kTpb, 0, s>>>(nl, ou, ow, off);
    uw_kernel<true><<<blocks(nl), kTpb, 0, s>>>(v, nl, t->d_leaves, nullptr, off, u_items, w_items);
  }
  int st = sort_rows(u_items, n_u, ou, nl, s);
  if (st == FMM_OK) st = sort_rows(w_items, n_w, ow, nl, s);
  if (st == FMM_OK) st = compact_rows(t->d_leaves, cu, ou, nl, u_items, n_u, U, s);
  if (st == FMM_OK) st = compact_rows(t->d_leaves, cw, ow, nl, w_items, n_w, Wl, s);
  if (st != FMM_OK) {
    if (!U.item) (void)hipFree(u_items);
    if (!Wl.item) (void)hipFree(w_items);
    return st;
  }
  // X: one row per box
  int64_t *cx, *ox, n_x = 0;
  TREE_TRY(sc.get(&cx, nb));
  TREE_TRY(sc.get(&ox, nb + 1));
  if (nb > 0) x_kernel<false><<<blocks(nb), kTpb, 0, s>>>(v, cx, nullptr, nullptr);
  TREE_TRY(exclusive_scan(cx, ox, nb, &n_x, s));
  FMM_REQUIRE(n_x <= kMaxInt32, FMM_EUNSUPPORTED, "lists exceed 2^31 entries");
  int32_t* x_items;
  TREE_TRY(dev_alloc(&x_items, n_x));
  if (nb > 0) x_kernel<true><<<blocks(nb), kTpb, 0, s>>>(v, nullptr, ox, x_items);
  st = sort_rows(x_items, n_x, ox, nb, s);
  if (st == FMM_OK) st = compact_rows(nullptr, cx, ox, nb, x_items, n_x, X, s);
  if (st != FMM_OK && !X.item) (void)hipFree(x_items);
  return st;
}

__global__ void widen_kernel(int64_t n, const int32_t* __restrict__ in, int64_t* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = in[k];
}

// row starts of `l` widened to int64 (the row form split_rows reads)
int row_starts(const TreeList& l, int64_t* out, hipStream_t s) {
  widen_kernel<<<blocks(l.n_row + 1), kTpb, 0, s>>>(l.n_row + 1, l.ptr, out);
  return FMM_OK;
}

// the rows of (kind, max_src), built on first use
int get_list(fmm_tree t, int kind, int64_t max_src, TreeList** out, hipStream_t s) {
  auto key = std::make_pair(kind, max_src);
  auto it = t->lists.find(key);
  if (it != t->lists.end()) {
    *out = &it->second;
    return FMM_OK;
  }
  if (max_src > 0) {
    TreeList* base;
    TREE_TRY(get_list(t, kind, 0, &base, s));
    Scratch sc;
    int64_t* starts;
    TREE_TRY(sc.get(&starts, base->n_row + 1));
    TREE_TRY(row_starts(*base, starts, s));
    TreeList split;
    int st = split_rows(t, base->n_row, base->box, starts, base->item, max_src, split, s);
    if (st != FMM_OK) {
      free_list(split);
      return st;
    }
    *out = &(t->lists[key] = split);
    return FMM_OK;
  }
  if (kind == FMM_LIST_NEAR) {
    TreeList l;
    int st = build_near(t, l, s);
    if (st != FMM_OK) {
      free_list(l);
      return st;
    }
    *out = &(t->lists[key] = l);
    return FMM_OK;
  }
  TreeList U, Wl, X;
  int st = build_uwx(t, U, Wl, X, s);
  if (st != FMM_OK) {
    free_list(U);
    free_list(Wl);
    free_list(X);
    return st;
  }
  t->lists[std::make_pair((int)FMM_LIST_U, (int64_t)0)] = U;
  t->lists[std::make_pair((int)FMM_LIST_W, (int64_t)0)] = Wl;
  t->lists[std::make_pair((int)FMM_LIST_X, (int64_t)0)] = X;
  *out = &t->lists[key];
  return FMM_OK;
}

}  // namespace

extern "C" {

int fmm_tree_build(int64_t n_points, const double* xyz, int32_t max_leaf, int32_t depth, fmm_tree* tree,
                   void* stream) {
  FMM_REQUIRE(tree, FMM_EINVAL, "tree output pointer is NULL");
  *tree = nullptr;
  FMM_REQUIRE(n_points >= 0 && n_points <= kMaxInt32, FMM_EINVAL, "n_points must be in [0, 2^31)");
  FMM_REQUIRE(n_points == 0 || xyz, FMM_EINVAL, "xyz is NULL");
  FMM_REQUIRE(max_leaf >= 0, FMM_EINVAL, "max_leaf < 0");
  if (max_leaf == 0)
    FMM_REQUIRE(depth >= 0 && depth <= FMM_TREE_MAX_UNIFORM_DEPTH, FMM_EINVAL,
                "uniform tree depth must be in [0, FMM_TREE_MAX_UNIFORM_DEPTH]");
  else
    FMM_REQUIRE(depth >= 0 && depth <= FMM_TREE_MAX_DEPTH, FMM_EINVAL, "max_depth must be in [0, FMM_TREE_MAX_DEPTH]");
  hipStream_t s = (hipStream_t)stream;
  auto* t = new fmm_tree_s();
  t->n = n_points;
  t->max_leaf = max_leaf;
  t->depth = depth;
  auto bail = [&](int st) {
    free_tree(t);
    delete t;
    return st;
  };
  const int64_t n = n_points;
  int st;
  {
    Scratch sc;
    uint64_t* key_in;
    int64_t* idx_in;
    int32_t* bad;
    if ((st = sc.get(&key_in, n)) || (st = sc.get(&idx_in, n)) || (st = sc.get(&bad, 1)) ||
        (st = dev_alloc(&t->d_pkey, n)) || (st = dev_alloc(&t->d_perm, n)) || (st = dev_alloc(&t->d_points, 3 * n)))
      return bail(st);
    int32_t h_bad = 0;
    if (hipMemsetAsync(bad, 0, sizeof(int32_t), s) != hipSuccess) return bail(fail(FMM_EHIP, "hipMemsetAsync"));
    if (n > 0) {
      point_keys_kernel<<<blocks(n), kTpb, 0, s>>>(n, xyz, key_in, idx_in, bad);
      size_t bytes = 0;
      if (hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, key_in, t->d_pkey, idx_in, t->d_perm, (int)n, 0,
                                             3 * kAxisBits, s) != hipSuccess)
        return bail(fail(FMM_EHIP, "radix sort"));
      char* tmp;
      if ((st = sc.get(&tmp, (int64_t)bytes))) return bail(st);
      if (hipcub::DeviceRadixSort::SortPairs(tmp, bytes, key_in, t->d_pkey, idx_in, t->d_perm, (int)n, 0,
                                             3 * kAxisBits, s) != hipSuccess)
        return bail(fail(FMM_EHIP, "radix sort"));
      gather_points_kernel<<<blocks(n), kTpb, 0, s>>>(n, xyz, t->d_perm, t->d_points);
    }
    if (hipMemcpyAsync(&h_bad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return bail(fail(FMM_EHIP, std::string("tree build: ") + hipGetErrorString(hipGetLastError())));
    if (h_bad) return bail(fail(FMM_EINVAL, "xyz holds a non-finite coordinate"));
  }
  // boxes of every level: keys (and, adaptive, the refine flags that decide the leaves)
  std::vector<uint64_t*> lkeys;
  std::vector<int64_t> lcount;
  std::vector<uint8_t*> lrefine;
  auto free_levels = [&]() {
    for (auto* p : lkeys) (void)hipFree(p);
    for (auto* p : lrefine) (void)hipFree(p);
  };
  if (max_leaf > 0) {
    st = build_levels_adaptive(t, max_leaf, depth, lkeys, lcount, lrefine, s);
    if (st) {
      free_levels();
      return bail(st);
    }
  } else {
    for (int lev = 0; lev <= depth; ++lev) {
      const int64_t nb = (int64_t)1 << (3 * lev);
      uint64_t* k = nullptr;
      if ((st = dev_alloc(&k, nb))) {
        free_levels();
        return bail(st);
      }
      lkeys.push_back(k);
      lcount.push_back(nb);
      iota_u64_kernel<<<blocks(nb), kTpb, 0, s>>>(nb, k);
    }
  }
  t->n_levels = (int32_t)lkeys.size();
  t->level_start.assign(1, 0);
  for (int64_t c : lcount) t->level_start.push_back(t->level_start.back() + c);
  t->n_box = t->level_start.back();
  if (t->n_box > kMaxInt32) {
    free_levels();
    return bail(fail(FMM_EUNSUPPORTED, "more than 2^31 boxes"));
  }
  const int64_t nb = t->n_box;
  if ((st = dev_alloc(&t->d_ls, t->n_levels + 1)) || (st = dev_alloc(&t->d_bkey, nb)) ||
      (st = dev_alloc(&t->d_level, nb)) || (st = dev_alloc(&t->d_ijk, 3 * nb)) || (st = dev_alloc(&t->d_center, 3 * nb)) ||
      (st = dev_alloc(&t->d_range, 2 * nb)) || (st = dev_alloc(&t->d_leaf, nb)) || (st = dev_alloc(&t->d_parent, nb)) ||
      (st = dev_alloc(&t->d_child0, nb))) {
    free_levels();
    return bail(st);
  }
  bool ok = hipMemcpyAsync(t->d_ls, t->level_start.data(), (t->n_levels + 1) * sizeof(int64_t),
                           hipMemcpyHostToDevice, s) == hipSuccess;
  for (int l = 0; l < t->n_levels && ok; ++l) {
    const int64_t a = t->level_start[l];
    ok = hipMemcpyAsync(t->d_bkey + a, lkeys[l], lcount[l] * sizeof(uint64_t), hipMemcpyDeviceToDevice, s) == hipSuccess;
    if (!ok) break;
    if (max_leaf > 0) {
      // a box is a leaf where it is not refined
      ok = hipMemcpyAsync(t->d_leaf + a, lrefine[l], lcount[l], hipMemcpyDeviceToDevice, s) == hipSuccess;
    } else {
      ok = hipMemsetAsync(t->d_leaf + a, l == depth ? 1 : 0, lcount[l], s) == hipSuccess;
    }
  }
  if (!ok) {
    free_levels();
    return bail(fail(FMM_EHIP, "tree assembly copy failed"));
  }
  if (hipStreamSynchronize(s) != hipSuccess) {
    free_levels();
    return bail(fail(FMM_EHIP, "tree assembly failed"));
  }
  free_levels();
  if (max_leaf > 0) leaf_from_refine_kernel<<<blocks(nb), kTpb, 0, s>>>(nb, t->d_leaf);
  box_kernel<<<blocks(nb), kTpb, 0, s>>>(nb, t->d_bkey, t->d_ls, t->n_levels, t->d_pkey, n, t->d_level, t->d_ijk,
                                         t->d_center, t->d_range);
  family_kernel<<<blocks(nb), kTpb, 0, s>>>(t->view(), t->d_parent, t->d_child0);
  // leaf ids in box order
  {
    Scratch sc;
    int64_t *flag, *pos;
    if ((st = sc.get(&flag, nb)) || (st = sc.get(&pos, nb + 1))) return bail(st);
    widen_u8_kernel<<<blocks(nb), kTpb, 0, s>>>(nb, t->d_leaf, flag);
    if ((st = exclusive_scan(flag, pos, nb, &t->n_leaf, s))) return bail(st);
    if ((st = dev_alloc(&t->d_leaves, t->n_leaf))) return bail(st);
    leaves_kernel<<<blocks(nb), kTpb, 0, s>>>(nb, t->d_leaf, pos, t->d_leaves);
    if (hipStreamSynchronize(s) != hipSuccess) return bail(fail(FMM_EHIP, "tree build failed"));
  }
  *tree = t;
  return FMM_OK;
}

int fmm_tree_size(fmm_tree tree, int64_t* n_box, int32_t* n_levels, int64_t* n_leaf) {
  int st = check_tree(tree);
  if (st) return st;
  if (n_box) *n_box = tree->n_box;
  if (n_levels) *n_levels = tree->n_levels;
  if (n_leaf) *n_leaf = tree->n_leaf;
  return FMM_OK;
}

int fmm_tree_export(fmm_tree tree, int64_t* perm, double* points, int32_t* level, int32_t* ijk, double* center,
                    int64_t* pt_range, uint8_t* is_leaf, int64_t* level_start, void* stream) {
  int st = check_tree(tree);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = tree->n, nb = tree->n_box;
  auto cp = [&](void* dst, const void* src, int64_t bytes) {
    return (dst && bytes > 0) ? hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s) : hipSuccess;
  };
  FMM_HIP_CHECK(cp(perm, tree->d_perm, n * sizeof(int64_t)));
  FMM_HIP_CHECK(cp(points, tree->d_points, 3 * n * sizeof(double)));
  FMM_HIP_CHECK(cp(level, tree->d_level, nb * sizeof(int32_t)));
  FMM_HIP_CHECK(cp(ijk, tree->d_ijk, 3 * nb * sizeof(int32_t)));
  FMM_HIP_CHECK(cp(center, tree->d_center, 3 * nb * sizeof(double)));
  FMM_HIP_CHECK(cp(pt_range, tree->d_range, 2 * nb * sizeof(int64_t)));
  FMM_HIP_CHECK(cp(is_leaf, tree->d_leaf, nb));
  if (level_start) std::copy(tree->level_start.begin(), tree->level_start.end(), level_start);
  return FMM_OK;
}

int fmm_tree_list2(fmm_tree tree, int32_t level_lo, int32_t level_hi, int64_t* n_pair, int32_t* tgt_box,
                   int32_t* src_box, void* stream) {
  int st = check_tree(tree);
  if (st) return st;
  FMM_REQUIRE(n_pair, FMM_EINVAL, "n_pair is NULL");
  FMM_REQUIRE(0 <= level_lo && level_lo <= level_hi && level_hi <= tree->n_levels, FMM_EINVAL,
              "need 0 <= level_lo <= level_hi <= n_levels");
  hipStream_t s = (hipStream_t)stream;
  if ((st = build_list2(tree, s))) return st;
  const int64_t a = tree->l2_off[level_lo], b = tree->l2_off[level_hi];
  *n_pair = b - a;
  if (b > a && tgt_box)
    FMM_HIP_CHECK(hipMemcpyAsync(tgt_box, tree->d_l2_tgt + a, (b - a) * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  if (b > a && src_box)
    FMM_HIP_CHECK(hipMemcpyAsync(src_box, tree->d_l2_src + a, (b - a) * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  return FMM_OK;
}

int fmm_tree_lists(fmm_tree tree, int32_t kind, int64_t max_src, int64_t* n_row, int64_t* n_item, int32_t* box,
                   int32_t* ptr, int32_t* item, void* stream) {
  int st = check_tree(tree);
  if (st) return st;
  FMM_REQUIRE(kind == FMM_LIST_NEAR || kind == FMM_LIST_U || kind == FMM_LIST_W || kind == FMM_LIST_X, FMM_EINVAL,
              "unknown list kind");
  FMM_REQUIRE(max_src >= 0, FMM_EINVAL, "max_src < 0");
  FMM_REQUIRE(max_src == 0 || kind == FMM_LIST_NEAR || kind == FMM_LIST_U, FMM_EINVAL,
              "max_src applies to the near and U lists only");
  FMM_REQUIRE(n_row && n_item, FMM_EINVAL, "n_row or n_item is NULL");
  hipStream_t s = (hipStream_t)stream;
  TreeList* l;
  if ((st = get_list(tree, kind, max_src, &l, s))) return st;
  *n_row = l->n_row;
  *n_item = l->n_item;
  if (box && l->n_row > 0)
    FMM_HIP_CHECK(hipMemcpyAsync(box, l->box, l->n_row * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  if (ptr) FMM_HIP_CHECK(hipMemcpyAsync(ptr, l->ptr, (l->n_row + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  if (item && l->n_item > 0)
    FMM_HIP_CHECK(hipMemcpyAsync(item, l->item, l->n_item * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  return FMM_OK;
}

void fmm_tree_destroy(fmm_tree tree) {
  if (!tree) return;
  free_tree(tree);
  tree->alive = false;
  delete tree;
}

}  // extern "C"
