// C ABI: argument validation, plans, M2L batch preparation and launch wrappers.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <unordered_map>
#include <tuple>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

using namespace fmm;

struct fmm_plan_s {
  fmm_desc desc{};
  int p = 0, c = 2, nc = 0, nfull = 0, S = 1, Sz = 1;
  int n_levels = 0;
  std::vector<double> h;
  std::vector<MIdx> J;
  RecArgs rec{};
  double* d_level_h = nullptr;
  int32_t* d_jbase = nullptr;
  int32_t* d_jxyz = nullptr;
  double* d_p2m_part = nullptr;  // per-chunk P2M results of boxes spread over several workgroups
  // per level: sparse M~^T (compression, rows j < nc) and M~ (decompression, rows m >= nc)
  int32_t *d_cmp_ptr = nullptr, *d_cmp_col = nullptr, *d_dec_ptr = nullptr, *d_dec_col = nullptr;
  double *d_cmp_val = nullptr, *d_dec_val = nullptr;
  bool alive = true;
};

namespace {
constexpr size_t kP2MPartBytes = 16u << 20;  // capacity of fmm_plan_s::d_p2m_part
constexpr int64_t kP2MChunkPoints = 2048;     // points per P2M workgroup for large boxes
constexpr int64_t kP2MMinChunkPoints = 512;   // smallest chunk when boxes are split to fill the GPU
constexpr int64_t kP2MFillGroups = 2048;      // workgroups a P2M launch over few boxes aims for
}  // namespace

// One launch of a multi: a streaming batch on its own (its own tuned shape), or a group of
// tiled batches sharing one tile shape drained by one persistent launch.
struct MultiGroup {
  std::vector<int> idx;  // positions of the group's batches in fmm_multi_s::batches
  bool stream = false;
  int rt = 1, ctw = 1, pf = 0, nbuf = 1, waves = 1, grid = 1;
  size_t lds = 0;
  M2LArgs* d_args = nullptr;
  int2* d_work = nullptr;
  int32_t n_work = 0;
};

struct fmm_multi_s {
  std::vector<fmm_batch> batches;
  int dtype = 0;
  std::vector<MultiGroup> groups;
};

struct fmm_batch_s {
  fmm_plan plan = nullptr;
  int dtype = 0;
  bool adjoint = false;  // prepared by fmm_m2l_prepare_adjoint: pairs reversed, original tables
  bool fft = false;      // prepared by fmm_m2l_prepare_fft
  FftArgs fa{};          // FFT path: device lists and spectra (owned)
  int nc = 0, nc_pad = 0, ts = 0, waves = 1, rows_per_wave = 1, col_tiles = 1, col_groups = 1, k_splits = 1;
  int pf_class = 0, nbuf = 2;
  int64_t lds_bytes = 0;
  M2LArgs shape{};  // ldb, k4p, tab_off, buf_elems, nt, nrg, nks
  int64_t n_pair = 0, n_tab = 0, n_tiles = 0, n_entries = 0, n_items = 0;
  int64_t useful = 0, computed = 0, scratch_bytes = 0;
  void* d_tab = nullptr;
  int32_t* d_tile_tgt = nullptr;
  int32_t* d_tile_nparts = nullptr;
  int32_t* d_tile_item0 = nullptr;
  int32_t* d_counter = nullptr;
  double* d_scratch = nullptr;
  int32_t* d_entry_tab = nullptr;
  int32_t* d_entry_src = nullptr;
  M2LItem* d_items = nullptr;
  int32_t* d_jbase = nullptr;
  std::vector<M2LItem> h_items;  // host copy (work ordering of persistent launches)
  // streaming form (m2l_stream.hip): 16-target tiles, one contiguous entry chunk per workgroup
  bool stream = false;
  int32_t n_wg = 0, c_pde = 2, p = 0, lds_slot = 0, lds_sbq = 0;
  int32_t* d_wg_item = nullptr;
};

namespace {

template <typename T>
int dev_upload(T** dst, const std::vector<T>& v) {
  *dst = nullptr;
  if (v.empty()) return FMM_OK;
  hipError_t e = hipMalloc((void**)dst, v.size() * sizeof(T));
  if (e != hipSuccess) return fail(FMM_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  e = hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(FMM_EHIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
  return FMM_OK;
}

void dev_free(void* p) {
  if (p) (void)hipFree(p);
}

int env_int(const char* name, int dflt) {
  const char* s = std::getenv(name);
  if (!s || !*s) return dflt;
  return std::atoi(s);
}

RecArgs make_rec(const fmm_desc& d) {
  RecArgs r{};
  auto terms = recursion_terms(d.kernel, d.param);
  r.n = (int)terms.size();
  for (int k = 0; k < r.n; ++k) {
    r.dx[k] = terms[k].dx;
    r.dy[k] = terms[k].dy;
    r.dz[k] = terms[k].dz;
    r.hpow[k] = terms[k].hpow;
    r.coef[k] = terms[k].coef;
  }
  return r;
}

uint64_t spread3(uint32_t v) {
  uint64_t x = v & 0x1fffff;
  uint64_t out = 0;
  for (int b = 0; b < 21; ++b) out |= ((x >> b) & 1ull) << (3 * b);
  return out;
}

int check_plan(fmm_plan plan) {
  if (!plan) return fail(FMM_EINVAL, "plan is NULL");
  if (!plan->alive) return fail(FMM_ESTATE, "plan was destroyed");
  return FMM_OK;
}

}  // namespace

extern "C" {

int32_t fmm_abi_version(void) { return FMM_ABI_VERSION; }

const char* fmm_last_error(void) { return last_error().c_str(); }

int fmm_sizes(const fmm_desc* desc, int32_t* n_full_out, int32_t* n_compressed) {
  int st = check_desc(desc);
  if (st) return st;
  const int p = desc->order, c = pde_order(desc->kernel);
  if (n_full_out) *n_full_out = (int32_t)n_full(p);
  if (n_compressed) *n_compressed = (int32_t)(n_full(p) - n_full(p - c));
  return FMM_OK;
}

int fmm_index_table(const fmm_desc* desc, int32_t* mxyz) {
  int st = check_desc(desc);
  if (st) return st;
  FMM_REQUIRE(mxyz, FMM_EINVAL, "mxyz is NULL");
  auto J = kept_set(desc->order, pde_order(desc->kernel));
  for (size_t k = 0; k < J.size(); ++k) {
    mxyz[3 * k] = J[k].x;
    mxyz[3 * k + 1] = J[k].y;
    mxyz[3 * k + 2] = J[k].z;
  }
  return FMM_OK;
}

int fmm_deriv_tables(const fmm_desc* desc, int64_t n, const double* offset, const double* h, void* out,
                     void* stream) {
  int st = check_desc(desc);
  if (st) return st;
  FMM_REQUIRE(n >= 0, FMM_EINVAL, "n < 0");
  if (n == 0) return FMM_OK;
  FMM_REQUIRE(offset && h && out, FMM_EINVAL, "NULL pointer");
  FMM_REQUIRE(n <= (int64_t)0x7fffffff, FMM_EINVAL, "too many tables");
  TableArgs a{};
  a.n = n;
  a.offset = offset;
  a.h = h;
  a.out = out;
  a.kernel = desc->kernel;
  a.p2 = 2 * desc->order;
  a.S = 2 * desc->order + 1;
  a.Sz = 2 * pde_order(desc->kernel) - 1;
  a.param = desc->param;
  return launch_tables(a, desc->kernel == FMM_HELMHOLTZ, (hipStream_t)stream);
}

int fmm_plan_create(const fmm_desc* desc, int32_t n_levels, const double* level_box_size, fmm_plan* out) {
  int st = check_desc(desc);
  if (st) return st;
  FMM_REQUIRE(out, FMM_EINVAL, "plan output pointer is NULL");
  *out = nullptr;
  FMM_REQUIRE(n_levels >= 1 && n_levels <= 64, FMM_EINVAL, "n_levels must be in [1, 64]");
  FMM_REQUIRE(level_box_size, FMM_EINVAL, "level_box_size is NULL");
  for (int l = 0; l < n_levels; ++l)
    FMM_REQUIRE(level_box_size[l] > 0.0 && std::isfinite(level_box_size[l]), FMM_EINVAL,
                "level_box_size must be finite and > 0");
  auto* pl = new fmm_plan_s();
  pl->desc = *desc;
  pl->p = desc->order;
  pl->c = pde_order(desc->kernel);
  pl->J = kept_set(pl->p, pl->c);
  pl->nc = (int)pl->J.size();
  pl->nfull = (int)n_full(pl->p);
  pl->S = 2 * pl->p + 1;
  pl->Sz = 2 * pl->c - 1;
  pl->n_levels = n_levels;
  pl->h.assign(level_box_size, level_box_size + n_levels);
  pl->rec = make_rec(*desc);
  std::vector<int32_t> jb(pl->nc), jx(pl->nc);
  for (int k = 0; k < pl->nc; ++k) {
    jb[k] = (pl->J[k].z * pl->S + pl->J[k].x) * pl->S + pl->J[k].y;
    jx[k] = pl->J[k].x | (pl->J[k].y << 8) | (pl->J[k].z << 16);
  }
  // the compression and decompression of every level as sparse rows (nonzero entries only)
  std::vector<int32_t> cmp_ptr, cmp_col, dec_ptr, dec_col;
  std::vector<double> cmp_val, dec_val;
  {
    const auto terms = recursion_terms(desc->kernel, desc->param);
    const int nf = pl->nfull, nc = pl->nc;
    for (int l = 0; l < n_levels; ++l) {
      const std::vector<double> M = decompression_matrix(pl->p, pl->c, terms, pl->h[l]);
      for (int j = 0; j < nc; ++j) {
        cmp_ptr.push_back((int32_t)cmp_col.size());
        for (int m = 0; m < nf; ++m)
          if (M[(size_t)m * nc + j] != 0.0) {
            cmp_col.push_back(m);
            cmp_val.push_back(M[(size_t)m * nc + j]);
          }
      }
      cmp_ptr.push_back((int32_t)cmp_col.size());
      for (int m = 0; m < nf; ++m) {
        dec_ptr.push_back((int32_t)dec_col.size());
        if (m < nc) continue;  // kept rows are the identity
        for (int j = 0; j < nc; ++j)
          if (M[(size_t)m * nc + j] != 0.0) {
            dec_col.push_back(j);
            dec_val.push_back(M[(size_t)m * nc + j]);
          }
      }
      dec_ptr.push_back((int32_t)dec_col.size());
    }
    if (dec_col.empty()) {  // order below the PDE order: nothing is eliminated
      dec_col.push_back(0);
      dec_val.push_back(0.0);
    }
  }
  if ((st = dev_upload(&pl->d_level_h, pl->h)) || (st = dev_upload(&pl->d_jbase, jb)) ||
      (st = dev_upload(&pl->d_jxyz, jx)) || (st = dev_upload(&pl->d_cmp_ptr, cmp_ptr)) ||
      (st = dev_upload(&pl->d_cmp_col, cmp_col)) || (st = dev_upload(&pl->d_cmp_val, cmp_val)) ||
      (st = dev_upload(&pl->d_dec_ptr, dec_ptr)) || (st = dev_upload(&pl->d_dec_col, dec_col)) ||
      (st = dev_upload(&pl->d_dec_val, dec_val)) ||
      (hipMalloc((void**)&pl->d_p2m_part, kP2MPartBytes) != hipSuccess &&
       (st = fail(FMM_ENOMEM, "hipMalloc of the P2M chunk buffer failed")))) {
    fmm_plan_destroy(pl);
    return st;
  }
  *out = pl;
  return FMM_OK;
}

void fmm_plan_destroy(fmm_plan plan) {
  if (!plan) return;
  plan->alive = false;
  dev_free(plan->d_level_h);
  dev_free(plan->d_jbase);
  dev_free(plan->d_jxyz);
  dev_free(plan->d_p2m_part);
  dev_free(plan->d_cmp_ptr);
  dev_free(plan->d_cmp_col);
  dev_free(plan->d_cmp_val);
  dev_free(plan->d_dec_ptr);
  dev_free(plan->d_dec_col);
  dev_free(plan->d_dec_val);
  delete plan;
}

static int check_box_args(fmm_plan plan, int64_t n_box, const double* center, const int32_t* level,
                          const int64_t* range, int64_t n_pts, const void* xyz, const void* v1, const void* v2) {
  int st = check_plan(plan);
  if (st) return st;
  FMM_REQUIRE(n_box >= 0 && n_box <= (int64_t)0x7fffffff, FMM_EINVAL, "n_box out of range");
  FMM_REQUIRE(n_pts >= 0, FMM_EINVAL, "n_pts < 0");
  if (n_box == 0) return FMM_OK;
  FMM_REQUIRE(center && level && range, FMM_EINVAL, "box arrays must not be NULL");
  FMM_REQUIRE(v1 && v2, FMM_EINVAL, "coefficient / value arrays must not be NULL");
  FMM_REQUIRE(n_pts == 0 || xyz, FMM_EINVAL, "point array is NULL");
  return FMM_OK;
}

// Workgroups per box for P2M: boxes with many points (coarse levels) are split into chunks of
// about kP2MChunkPoints points whose results are added in chunk order, as far as the plan's
// chunk buffer allows.
static void set_p2m_chunks(fmm_plan plan, P2MArgs& a) {
  a.ny = 1;
  a.part = plan->d_p2m_part;
  if (a.n_box <= 0 || !plan->d_p2m_part) return;
  const int64_t per_box = (a.n_pts + a.n_box - 1) / a.n_box;
  int64_t ny = (per_box + kP2MChunkPoints - 1) / kP2MChunkPoints;
  // few boxes (coarse levels): more, smaller chunks, so that the launch has about
  // kP2MFillGroups workgroups, but at least kP2MMinChunkPoints points per chunk
  const int64_t fill = std::min<int64_t>((kP2MFillGroups + a.n_box - 1) / a.n_box,
                                         (per_box + kP2MMinChunkPoints - 1) / kP2MMinChunkPoints);
  ny = std::max<int64_t>(ny, fill);
  const int64_t width = (int64_t)plan->nc * (dtype_complex(plan->desc.dtype) ? 2 : 1);
  ny = std::min<int64_t>(ny, (int64_t)(kP2MPartBytes / sizeof(double)) / (a.n_box * width));
  a.ny = (int32_t)std::max<int64_t>(1, std::min<int64_t>(ny, 1024));
}

int fmm_p2m(fmm_plan plan, int64_t n_box, const double* box_center, const int32_t* box_level,
            const int64_t* pt_range, int64_t n_src, const void* src_xyz, const void* weight, void* mpole,
            void* stream) {
  int st = check_box_args(plan, n_box, box_center, box_level, pt_range, n_src, src_xyz, mpole,
                          n_src ? weight : mpole);
  if (st || n_box == 0) return st;
  P2MArgs a{};
  a.n_box = n_box;
  a.center = box_center;
  a.level = box_level;
  a.range = pt_range;
  a.level_h = plan->d_level_h;
  a.n_levels = plan->n_levels;
  a.n_pts = n_src;
  a.xyz = src_xyz;
  a.w = weight;
  a.out = mpole;
  a.nc = plan->nc;
  a.c = plan->c;
  a.rec = plan->rec;
  a.cmp_ptr = plan->d_cmp_ptr;
  a.cmp_col = plan->d_cmp_col;
  a.cmp_val = plan->d_cmp_val;
  a.xsign = 1.0;
  set_p2m_chunks(plan, a);
  return launch_p2m(a, plan->p, plan->desc.dtype, (hipStream_t)stream);
}

static int trans_args(fmm_plan plan, int64_t n_parent, const int32_t* parent, const int32_t* child, int64_t n_box,
                      const double* box_center, const int32_t* box_level, void* coef, TransArgs& a) {
  int st = check_plan(plan);
  if (st) return st;
  FMM_REQUIRE(n_parent >= 0 && n_parent <= (int64_t)0x7fffffff, FMM_EINVAL, "n_parent out of range");
  FMM_REQUIRE(n_box >= 0 && n_box <= (int64_t)0x7fffffff, FMM_EINVAL, "n_box out of range");
  if (n_parent == 0) return FMM_OK;
  FMM_REQUIRE(parent && child, FMM_EINVAL, "parent / child arrays must not be NULL");
  FMM_REQUIRE(box_center && box_level && coef, FMM_EINVAL, "box arrays must not be NULL");
  a = TransArgs{};
  a.n_parent = n_parent;
  a.parent = parent;
  a.child = child;
  a.n_box = n_box;
  a.center = box_center;
  a.level = box_level;
  a.level_h = plan->d_level_h;
  a.n_levels = plan->n_levels;
  a.coef = coef;
  a.nc = plan->nc;
  a.c = plan->c;
  a.rec = plan->rec;
  return FMM_OK;
}

int fmm_m2m(fmm_plan plan, int64_t n_parent, const int32_t* parent, const int32_t* child, int64_t n_box,
            const double* box_center, const int32_t* box_level, void* mpole, void* stream) {
  TransArgs a{};
  const int st = trans_args(plan, n_parent, parent, child, n_box, box_center, box_level, mpole, a);
  if (st || n_parent == 0) return st;
  return launch_m2m(a, plan->p, plan->desc.dtype, (hipStream_t)stream);
}

int fmm_l2l(fmm_plan plan, int64_t n_parent, const int32_t* parent, const int32_t* child, int64_t n_box,
            const double* box_center, const int32_t* box_level, void* local, void* stream) {
  TransArgs a{};
  const int st = trans_args(plan, n_parent, parent, child, n_box, box_center, box_level, local, a);
  if (st || n_parent == 0) return st;
  return launch_l2l(a, plan->p, plan->desc.dtype, (hipStream_t)stream);
}

int fmm_m2m_adjoint(fmm_plan plan, int64_t n_parent, const int32_t* parent, const int32_t* child, int64_t n_box,
                    const double* box_center, const int32_t* box_level, void* mpole_grad, void* stream) {
  TransArgs a{};
  const int st = trans_args(plan, n_parent, parent, child, n_box, box_center, box_level, mpole_grad, a);
  if (st || n_parent == 0) return st;
  a.transpose = 1;
  return launch_l2l(a, plan->p, plan->desc.dtype, (hipStream_t)stream);
}

int fmm_l2l_adjoint(fmm_plan plan, int64_t n_parent, const int32_t* parent, const int32_t* child, int64_t n_box,
                    const double* box_center, const int32_t* box_level, void* local_grad, void* stream) {
  TransArgs a{};
  const int st = trans_args(plan, n_parent, parent, child, n_box, box_center, box_level, local_grad, a);
  if (st || n_parent == 0) return st;
  a.transpose = 1;
  return launch_m2m(a, plan->p, plan->desc.dtype, (hipStream_t)stream);
}

int fmm_l2p(fmm_plan plan, int64_t n_box, const double* box_center, const int32_t* box_level,
            const int64_t* pt_range, int64_t n_tgt, const void* tgt_xyz, const void* local, void* potential,
            void* stream) {
  return fmm_l2p_ex(plan, n_box, box_center, box_level, pt_range, n_tgt, tgt_xyz, local, potential, FMM_ACCUMULATE,
                    stream);
}

int fmm_l2p_ex(fmm_plan plan, int64_t n_box, const double* box_center, const int32_t* box_level,
               const int64_t* pt_range, int64_t n_tgt, const void* tgt_xyz, const void* local, void* potential,
               int32_t mode, void* stream) {
  FMM_REQUIRE(mode == FMM_ACCUMULATE || mode == FMM_OVERWRITE, FMM_EINVAL, "mode must be FMM_ACCUMULATE or FMM_OVERWRITE");
  int st = check_box_args(plan, n_box, box_center, box_level, pt_range, n_tgt, tgt_xyz, local,
                          n_tgt ? potential : local);
  if (st || n_box == 0) return st;
  L2PArgs a{};
  a.n_box = n_box;
  a.center = box_center;
  a.level = box_level;
  a.range = pt_range;
  a.level_h = plan->d_level_h;
  a.n_levels = plan->n_levels;
  a.n_pts = n_tgt;
  a.xyz = tgt_xyz;
  a.local = local;
  a.pot = potential;
  a.nc = plan->nc;
  a.c = plan->c;
  a.rec = plan->rec;
  a.dec_ptr = plan->d_dec_ptr;
  a.dec_col = plan->d_dec_col;
  a.dec_val = plan->d_dec_val;
  a.xsign = 1.0;
  a.grad = nullptr;
  a.gscale = nullptr;
  a.overwrite = mode == FMM_OVERWRITE ? 1 : 0;
  return launch_l2p(a, plan->p, plan->desc.dtype, (hipStream_t)stream);
}

int fmm_l2p_adjoint(fmm_plan plan, int64_t n_box, const double* box_center, const int32_t* box_level,
                    const int64_t* pt_range, int64_t n_tgt, const void* tgt_xyz, const void* local,
                    const void* potential_grad, void* local_grad, void* tgt_xyz_grad, void* stream) {
  int st = check_box_args(plan, n_box, box_center, box_level, pt_range, n_tgt, tgt_xyz, local_grad,
                          n_tgt ? potential_grad : local_grad);
  if (st || n_box == 0) return st;
  FMM_REQUIRE(!dtype_complex(plan->desc.dtype), FMM_EUNSUPPORTED, "adjoints are implemented for real dtypes");
  FMM_REQUIRE(!tgt_xyz_grad || local, FMM_EINVAL, "target gradients need the local expansions");
  // d L / d theta~ = M~^T (sum_x g(x) X^i / i!), X = (x - c) / h: target moments, then compression
  P2MArgs m{};
  m.n_box = n_box;
  m.center = box_center;
  m.level = box_level;
  m.range = pt_range;
  m.level_h = plan->d_level_h;
  m.n_levels = plan->n_levels;
  m.n_pts = n_tgt;
  m.xyz = tgt_xyz;
  m.w = potential_grad;
  m.out = local_grad;
  m.nc = plan->nc;
  m.c = plan->c;
  m.rec = plan->rec;
  m.cmp_ptr = plan->d_cmp_ptr;
  m.cmp_col = plan->d_cmp_col;
  m.cmp_val = plan->d_cmp_val;
  m.xsign = -1.0;
  set_p2m_chunks(plan, m);
  st = launch_p2m(m, plan->p, plan->desc.dtype, (hipStream_t)stream);
  if (st || !tgt_xyz_grad) return st;
  // d L / d x = g(x) grad phi(x)
  L2PArgs e{};
  e.n_box = n_box;
  e.center = box_center;
  e.level = box_level;
  e.range = pt_range;
  e.level_h = plan->d_level_h;
  e.n_levels = plan->n_levels;
  e.n_pts = n_tgt;
  e.xyz = tgt_xyz;
  e.local = local;
  e.pot = nullptr;
  e.nc = plan->nc;
  e.c = plan->c;
  e.rec = plan->rec;
  e.dec_ptr = plan->d_dec_ptr;
  e.dec_col = plan->d_dec_col;
  e.dec_val = plan->d_dec_val;
  e.xsign = 1.0;
  e.grad = tgt_xyz_grad;
  e.gscale = potential_grad;
  return launch_l2p(e, plan->p, plan->desc.dtype, (hipStream_t)stream);
}

int fmm_p2m_adjoint(fmm_plan plan, int64_t n_box, const double* box_center, const int32_t* box_level,
                    const int64_t* pt_range, int64_t n_src, const void* src_xyz, const void* weight,
                    const void* mpole_grad, void* weight_grad, void* src_xyz_grad, void* stream) {
  int st = check_box_args(plan, n_box, box_center, box_level, pt_range, n_src, src_xyz, mpole_grad, mpole_grad);
  if (st || n_box == 0) return st;
  FMM_REQUIRE(!dtype_complex(plan->desc.dtype), FMM_EUNSUPPORTED, "adjoints are implemented for real dtypes");
  FMM_REQUIRE(weight_grad || src_xyz_grad, FMM_EINVAL, "nothing to compute: both gradients are NULL");
  FMM_REQUIRE(!src_xyz_grad || weight, FMM_EINVAL, "source position gradients need the weights");
  // g = M~ (d L / d beta~); d L / d w_s = sum_q g_q X_s^q / q!, X_s = (c - y_s) / h; d L / d y_s =
  // w_s d/dy of the same polynomial: a decompress-and-evaluate at the sources
  L2PArgs e{};
  e.n_box = n_box;
  e.center = box_center;
  e.level = box_level;
  e.range = pt_range;
  e.level_h = plan->d_level_h;
  e.n_levels = plan->n_levels;
  e.n_pts = n_src;
  e.xyz = src_xyz;
  e.local = mpole_grad;
  e.pot = weight_grad;
  e.nc = plan->nc;
  e.c = plan->c;
  e.rec = plan->rec;
  e.dec_ptr = plan->d_dec_ptr;
  e.dec_col = plan->d_dec_col;
  e.dec_val = plan->d_dec_val;
  e.xsign = -1.0;
  e.grad = src_xyz_grad;
  e.gscale = weight;
  return launch_l2p(e, plan->p, plan->desc.dtype, (hipStream_t)stream);
}

int fmm_direct(const fmm_desc* desc, int64_t n_src, const void* src_xyz, const void* weight, int64_t n_tgt,
               const void* tgt_xyz, void* potential, void* stream) {
  int st = check_desc(desc);
  if (st) return st;
  FMM_REQUIRE(n_src >= 0 && n_tgt >= 0, FMM_EINVAL, "negative size");
  FMM_REQUIRE(n_tgt <= (int64_t)0x7fffffff * 256, FMM_EINVAL, "too many targets");
  if (n_tgt == 0) return FMM_OK;
  FMM_REQUIRE(tgt_xyz && potential, FMM_EINVAL, "NULL target pointer");
  FMM_REQUIRE(n_src == 0 || (src_xyz && weight), FMM_EINVAL, "NULL source pointer");
  DirectArgs a{};
  a.n_src = n_src;
  a.n_tgt = n_tgt;
  a.src = src_xyz;
  a.w = weight;
  a.tgt = tgt_xyz;
  a.pot = potential;
  a.kernel = desc->kernel;
  a.param = desc->param;
  return launch_direct(a, desc->dtype, (hipStream_t)stream);
}

static int point_exp_args(fmm_plan plan, int64_t n_tbox, const int32_t* tbox, const int32_t* list_ptr,
                          int64_t n_list, const int32_t* list, int64_t n_box, const double* box_center,
                          const int32_t* box_level, const int64_t* range, int64_t n_pts, const void* xyz,
                          PointExpArgs& a) {
  int st = check_plan(plan);
  if (st) return st;
  FMM_REQUIRE(n_tbox >= 0 && n_tbox <= (int64_t)0x7fffffff, FMM_EINVAL, "n_tbox out of range");
  FMM_REQUIRE(n_list >= 0 && n_list <= (int64_t)0x7fffffff && n_box >= 0 && n_box <= (int64_t)0x7fffffff &&
                  n_pts >= 0,
              FMM_EINVAL, "negative or too large size");
  if (n_tbox == 0) return FMM_OK;
  FMM_REQUIRE(tbox && list_ptr && (n_list == 0 || list), FMM_EINVAL, "NULL box list");
  FMM_REQUIRE(box_center && box_level && range, FMM_EINVAL, "NULL box arrays");
  FMM_REQUIRE(n_pts == 0 || xyz, FMM_EINVAL, "NULL point array");
  a.n_tbox = n_tbox;
  a.tbox = tbox;
  a.list_ptr = list_ptr;
  a.list = list;
  a.n_list = n_list;
  a.n_box = n_box;
  a.center = box_center;
  a.level = box_level;
  a.range = range;
  a.level_h = plan->d_level_h;
  a.n_levels = plan->n_levels;
  a.n_pts = n_pts;
  a.xyz = xyz;
  a.jxyz = plan->d_jxyz;
  a.nc = plan->nc;
  a.p = plan->p;
  a.c = plan->c;
  a.kernel = plan->desc.kernel;
  a.param = plan->desc.param;
  return FMM_OK;
}

int fmm_m2p(fmm_plan plan, int64_t n_tbox, const int32_t* tbox, const int32_t* list_ptr, int64_t n_list,
            const int32_t* list, int64_t n_box, const double* box_center, const int32_t* box_level,
            const int64_t* tgt_range, int64_t n_tgt, const void* tgt_xyz, const void* mpole, void* potential,
            void* stream) {
  PointExpArgs a{};
  int st = point_exp_args(plan, n_tbox, tbox, list_ptr, n_list, list, n_box, box_center, box_level, tgt_range,
                          n_tgt, tgt_xyz, a);
  if (st || n_tbox == 0) return st;
  FMM_REQUIRE(mpole && (n_tgt == 0 || potential), FMM_EINVAL, "NULL multipole or potential array");
  a.mpole = mpole;
  a.out = potential;
  return launch_m2p(a, plan->desc.dtype, (hipStream_t)stream);
}

int fmm_p2l(fmm_plan plan, int64_t n_tbox, const int32_t* tbox, const int32_t* list_ptr, int64_t n_list,
            const int32_t* list, int64_t n_box, const double* box_center, const int32_t* box_level,
            const int64_t* src_range, int64_t n_src, const void* src_xyz, const void* weight, void* local,
            void* stream) {
  PointExpArgs a{};
  int st = point_exp_args(plan, n_tbox, tbox, list_ptr, n_list, list, n_box, box_center, box_level, src_range,
                          n_src, src_xyz, a);
  if (st || n_tbox == 0) return st;
  FMM_REQUIRE(local && (n_src == 0 || weight), FMM_EINVAL, "NULL local or weight array");
  a.w = weight;
  a.out = local;
  return launch_p2l(a, plan->desc.dtype, (hipStream_t)stream);
}

int fmm_p2p(const fmm_desc* desc, int64_t n_tbox, const int32_t* tbox, const int32_t* nbr_ptr, int64_t n_nbr,
            const int32_t* nbr, int64_t n_box, const int64_t* tgt_range, const int64_t* src_range, int64_t n_src,
            const void* src_xyz, const void* weight, int64_t n_tgt, const void* tgt_xyz, void* potential,
            void* stream) {
  int st = check_desc(desc);
  if (st) return st;
  FMM_REQUIRE(n_tbox >= 0 && n_tbox <= (int64_t)0x7fffffff, FMM_EINVAL, "n_tbox out of range");
  FMM_REQUIRE(n_nbr >= 0 && n_box >= 0 && n_src >= 0 && n_tgt >= 0, FMM_EINVAL, "negative size");
  if (n_tbox == 0) return FMM_OK;
  FMM_REQUIRE(tbox && nbr_ptr && (n_nbr == 0 || nbr), FMM_EINVAL, "NULL box list");
  FMM_REQUIRE(tgt_range && src_range, FMM_EINVAL, "NULL point ranges");
  FMM_REQUIRE(n_tgt == 0 || (tgt_xyz && potential), FMM_EINVAL, "NULL target pointer");
  FMM_REQUIRE(n_src == 0 || (src_xyz && weight), FMM_EINVAL, "NULL source pointer");
  P2PArgs a{};
  a.n_tbox = n_tbox;
  a.tbox = tbox;
  a.nbr_ptr = nbr_ptr;
  a.nbr = nbr;
  a.n_nbr = n_nbr;
  a.n_box = n_box;
  a.tgt_range = tgt_range;
  a.src_range = src_range;
  a.n_src = n_src;
  a.n_tgt = n_tgt;
  a.src = src_xyz;
  a.w = weight;
  a.tgt = tgt_xyz;
  a.pot = potential;
  a.kernel = desc->kernel;
  a.param = desc->param;
  return launch_p2p(a, desc->dtype, (hipStream_t)stream);
}

// ------------------------------------------------------------------------------- M2L batches

int fmm_m2l_prepare(fmm_plan plan, int64_t n_pair, const int32_t* tgt_box, const int32_t* src_box,
                    int64_t n_box, const int32_t* box_ijk, const int32_t* box_level, fmm_batch* out) {
  return fmm_m2l_prepare_ex(plan, n_pair, tgt_box, src_box, n_box, box_ijk, box_level, nullptr, out);
}

static int prepare_impl(fmm_plan plan, int64_t n_pair, const int32_t* tgt_box, const int32_t* src_box,
                        int64_t n_box, const int32_t* box_ijk, const int32_t* box_level,
                        const fmm_m2l_tuning* tuning, bool adjoint, fmm_batch* out);

int fmm_m2l_prepare_ex(fmm_plan plan, int64_t n_pair, const int32_t* tgt_box, const int32_t* src_box,
                       int64_t n_box, const int32_t* box_ijk, const int32_t* box_level,
                       const fmm_m2l_tuning* tuning, fmm_batch* out) {
  return prepare_impl(plan, n_pair, tgt_box, src_box, n_box, box_ijk, box_level, tuning, false, out);
}

int fmm_m2l_prepare_adjoint(fmm_plan plan, int64_t n_pair, const int32_t* tgt_box, const int32_t* src_box,
                            int64_t n_box, const int32_t* box_ijk, const int32_t* box_level,
                            const fmm_m2l_tuning* tuning, fmm_batch* out) {
  FMM_REQUIRE(plan && !dtype_complex(plan->desc.dtype), FMM_EUNSUPPORTED,
              "adjoints are implemented for real dtypes");
  // the transpose runs the same translations with the roles of the boxes swapped
  return prepare_impl(plan, n_pair, src_box, tgt_box, n_box, box_ijk, box_level, tuning, true, out);
}

static int prepare_impl(fmm_plan plan, int64_t n_pair, const int32_t* tgt_box, const int32_t* src_box,
                        int64_t n_box, const int32_t* box_ijk, const int32_t* box_level,
                        const fmm_m2l_tuning* tuning, bool adjoint, fmm_batch* out) {
  int st = check_plan(plan);
  if (st) return st;
  FMM_REQUIRE(out, FMM_EINVAL, "batch output pointer is NULL");
  *out = nullptr;
  FMM_REQUIRE(n_pair >= 0 && n_box >= 0 && n_box <= (int64_t)0x7fffffff, FMM_EINVAL, "bad sizes");
  FMM_REQUIRE(n_pair <= (int64_t)1 << 31, FMM_EINVAL, "too many pairs");
  FMM_REQUIRE(n_pair == 0 || (tgt_box && src_box && box_ijk && box_level), FMM_EINVAL, "NULL host array");
  const int dtype = plan->desc.dtype;
  const bool cplx = dtype_complex(dtype);
  const int CW = cplx ? 2 : 1;

  // 1. validate pairs, group by (level, offset); table ids in order of first appearance
  std::vector<int32_t> tab_of_key((size_t)plan->n_levels * 17 * 289, -1);  // dense over the key range
  std::vector<int64_t> tab_keys;
  std::vector<int32_t> pair_tab(n_pair);
  for (int64_t k = 0; k < n_pair; ++k) {
    const int32_t t = tgt_box[k], s = src_box[k];
    FMM_REQUIRE(t >= 0 && t < n_box && s >= 0 && s < n_box, FMM_EINVAL,
                "pair " + std::to_string(k) + ": box id out of range");
    const int lt = box_level[t], ls = box_level[s];
    FMM_REQUIRE(lt >= 0 && lt < plan->n_levels, FMM_EINVAL, "box level out of range");
    FMM_REQUIRE(lt == ls, FMM_EINVAL, "pair " + std::to_string(k) + ": boxes on different levels");
    // translation offset of the original pair (target - source); for the adjoint the arrays
    // hold the pair reversed, and T~ of the original offset is applied (T~ is symmetric)
    const int sg = adjoint ? -1 : 1;
    const int ox = sg * (box_ijk[3 * t] - box_ijk[3 * s]), oy = sg * (box_ijk[3 * t + 1] - box_ijk[3 * s + 1]),
              oz = sg * (box_ijk[3 * t + 2] - box_ijk[3 * s + 2]);
    FMM_REQUIRE(std::abs(ox) <= 8 && std::abs(oy) <= 8 && std::abs(oz) <= 8, FMM_EINVAL,
                "pair " + std::to_string(k) + ": |offset| > 8");
    FMM_REQUIRE(ox || oy || oz, FMM_EINVAL, "pair " + std::to_string(k) + ": zero offset");
    const int64_t key = ((int64_t)lt * 17 + (ox + 8)) * 289 + (oy + 8) * 17 + (oz + 8);
    int32_t& id = tab_of_key[key];
    if (id < 0) {
      id = (int32_t)tab_keys.size();
      tab_keys.push_back(key);
    }
    pair_tab[k] = id;
  }

  auto* b = new fmm_batch_s();
  b->plan = plan;
  b->dtype = dtype;
  b->adjoint = adjoint;
  b->nc = plan->nc;
  b->nc_pad = (plan->nc + 15) / 16 * 16;
  b->ts = plan->Sz * plan->S * plan->S;
  b->n_pair = n_pair;
  b->n_tab = (int64_t)tab_keys.size();

  // 2. launch shape (see fmm_m2l_tuning): the automatic choice scores every instantiated shape
  //    by row padding, LDS reads per matrix-core product, column fill and occupancy.
  int dev = 0, lds_max = 65536, n_cu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
      lds_max = v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) n_cu = v;
  }
  (void)hipGetLastError();
  // form: the streaming form serves every automatic launch it is instantiated for; the tiled
  // form is chosen explicitly or by giving its tile shape
  const M2LStreamShape ssh = m2l_stream_shape(plan->p, pde_order(plan->desc.kernel), dtype);
  const int form = tuning ? tuning->form : FMM_M2L_FORM_AUTO;
  if (form < FMM_M2L_FORM_AUTO || form > FMM_M2L_FORM_STREAM) {
    delete b;
    return fail(FMM_EINVAL, "unknown M2L form");
  }
  if (form == FMM_M2L_FORM_STREAM && !ssh.ok) {
    delete b;
    return fail(FMM_EUNSUPPORTED, "streaming M2L is not instantiated for this kernel, order and dtype");
  }
  b->stream = ssh.ok && form != FMM_M2L_FORM_TILED &&
              !(form == FMM_M2L_FORM_AUTO && tuning && tuning->rows_per_wave > 0) &&
              env_int("FMM_M2L_STREAM", 1) != 0;
  b->p = plan->p;
  b->c_pde = pde_order(plan->desc.kernel);
  if (b->stream) {
    const int wmax = std::min(ssh.max_waves, kM2LStreamMaxWaves);
    int w = (tuning && tuning->waves > 0) ? tuning->waves : env_int("FMM_M2LS_WAVES", wmax);
    if (w > wmax || w < 1) {
      delete b;
      return fail(FMM_EUNSUPPORTED, "streaming M2L: " + std::to_string(w) + " wavefronts per workgroup (at most " +
                                        std::to_string(wmax) + " for this order and dtype)");
    }
    b->waves = w;
    b->rows_per_wave = (b->nc % 16 >= 1 && b->nc % 16 <= kMaxRem && b->nc > 16) ? b->nc / 16 : (b->nc + 15) / 16;
    b->shape.nrem = (b->nc % 16 >= 1 && b->nc % 16 <= kMaxRem && b->nc > 16) ? b->nc % 16 : 0;
    b->col_tiles = b->col_groups = b->k_splits = 1;
    b->nbuf = 1;
    const size_t rb = real_size(dtype);
    // LDS: the wavefronts' tables, their item-sum slots, the q bases and two counters
    size_t lds = ((size_t)w * ssh.tsp * rb + 15) / 16 * 16;
    b->lds_slot = (int32_t)lds;
    lds += (size_t)w * ssh.nacc * 64 * sizeof(double);
    b->lds_sbq = (int32_t)lds;
    lds += (size_t)8 * ssh.kj * sizeof(int32_t) + (2 + kM2LStreamMaxWaves) * sizeof(int32_t);
    // one workgroup per compute unit: the chunks are equal, so a second resident workgroup on
    // some units would only make those units finish later
    if (env_int("FMM_M2LS_ONE_PER_CU", 1) && lds <= (size_t)lds_max / 2) lds = (size_t)lds_max / 2 + 256;
    if (lds > (size_t)lds_max - 64) {
      if (form == FMM_M2L_FORM_STREAM) {
        delete b;
        return fail(FMM_EUNSUPPORTED, "streaming M2L needs more LDS than a workgroup has");
      }
      b->stream = false;
    } else {
      b->lds_bytes = (int64_t)lds;
    }
  }
  if (!b->stream) {
    // rows past the last full 16-row tile: up to kMaxRem of them are contracted on the VALU
    // instead of a mostly empty matrix-core tile (e.g. 81 = 5 x 16 + 1 at Laplace p = 8)
    int nrem = b->nc % 16;
    const bool valu_rows = b->nc > 16 && nrem >= 1 && nrem <= kMaxRem && env_int("FMM_M2L_VALU_ROWS", 1) != 0;
    const int rtiles = valu_rows ? b->nc / 16 : b->nc_pad / 16;
    if (!valu_rows) nrem = 0;
    const size_t rb = real_size(dtype);
    const size_t cap = (size_t)lds_max - 64;  // room for the kernel's static LDS
    struct Cand {
      int rt, ctw, ncg, nrg, waves, pf, nbuf, nks;
      M2LArgs sh;
      size_t lds;
    };
    auto make = [&](int rt, int ctw, int ncg, int nbuf, int nks, Cand& c) {
      if (rt < 1 || ctw < 1 || ncg < 1 || nks < 1 || nks > 4 || !m2l_shape_instantiated(rt, ctw)) return false;
      const int nrg = (rtiles + rt - 1) / rt;
      const int waves = nrg * ncg * nks;
      if (waves > kM2LMaxThreads / 64 || ncg * ctw > 4) return false;
      c.rt = rt;
      c.ctw = ctw;
      c.ncg = ncg;
      c.nrg = nrg;
      c.waves = waves;
      c.sh = M2LArgs{};
      c.sh.ts = b->ts;
      c.sh.nc = b->nc;
      m2l_shape(c.sh, rb, cplx, ncg * ctw);
      c.sh.nrg = nrg;
      c.sh.nks = nks;
      c.sh.rtiles = rtiles;
      c.sh.nrem = nrem;
      c.nks = nks;
      if (nks > c.sh.k4p / (int)(16 / rb)) return false;  // every K range non-empty
      c.pf = m2l_prefetch_class(c.sh, cplx, ncg * ctw, waves);
      c.nbuf = nbuf;
      c.lds = m2l_lds_bytes(c.sh, rb, nbuf, rt, cplx);
      return c.pf >= 0 && c.lds <= cap;
    };
    Cand best{};
    bool found = false;
    if (tuning && tuning->rows_per_wave > 0) {
      found = make(tuning->rows_per_wave, std::max(1, tuning->col_tiles_per_wave), std::max(1, tuning->col_groups),
                   tuning->lds_buffers == 1 ? 1 : 2, std::max(1, tuning->k_splits), best);
      if (!found) {
        delete b;
        return fail(FMM_EUNSUPPORTED, "requested M2L launch shape is not instantiated or does not fit");
      }
    } else {
      // score: row padding x LDS reads per product x column fill x occupancy (waves per SIMD
      // from LDS and an estimate of the register need)
      double best_score = 1e30;
      for (int rt = 1; rt <= 5; ++rt)
        for (int ctw = 1; ctw <= 2; ++ctw)
          for (int ncg : {1, 2, 4})
            for (int nb : {1, 2})
              for (int nks : {1, 2}) {
              Cand c{};
              if (!make(rt, ctw, ncg, nb, nks, c)) continue;
              const double pad = (double)(c.nrg * rt) / rtiles;
              const double reads = (double)(rt + ctw) / (rt * ctw);
              const int nt = 16 * ncg * ctw;
              const double fill = nt <= 16 ? 1.0 : (nt <= 32 ? 1.04 : 1.10);
              const int wg_lds = (int)std::max<size_t>(1, (size_t)lds_max / std::max<size_t>(c.lds, 1));
              const int vgpr = 40 + rt * ctw * (cplx ? 2 : 1) * (int)(rb == 8 ? 8 : 4) * (rb == 4 ? 2 : 1) +
                               (c.pf == 0 ? 24 : c.pf == 1 ? 48 : 88) * (int)(rb / 4);
              const int waves_simd_reg = std::max(1, 512 / std::max(64, vgpr));
              const int wgs = std::max(1, std::min(wg_lds, (4 * waves_simd_reg) / c.waves));
              const double per_simd = (double)(wgs * c.waves) / 4.0;
              const double occ = per_simd >= 3.0 ? 1.0 : per_simd >= 2.0 ? 1.1 : (per_simd >= 1.0 ? 1.5 : 2.0);
              const double sync = (nb == 1 ? 1.0 : 1.08) * (1.0 + 0.02 * (nks - 1));
              const double score = pad * (0.5 + 0.5 * reads) * fill * occ * sync;
              if (score < best_score) {
                best_score = score;
                best = c;
                found = true;
              }
            }
      if (!found) {
        delete b;
        return fail(FMM_EUNSUPPORTED, "M2L tile does not fit in LDS / registers for this order and dtype");
      }
    }
    b->rows_per_wave = best.rt;
    b->col_tiles = best.ctw;
    b->col_groups = best.ncg;
    b->k_splits = best.nks;
    b->waves = best.waves;
    b->pf_class = best.pf;
    b->nbuf = best.nbuf;
    b->shape = best.sh;
    b->lds_bytes = (int64_t)best.lds;
  }
  const int NT = b->stream ? 16 : 16 * b->col_tiles * b->col_groups;


  // 3. target tiles: same level and child parity, then the same set of offsets (signature) where
  //    possible, then Morton order of the parent; NT targets per tile
  // box id -> position among the targets (dense over the box ids)
  std::vector<int32_t> tpos(n_box, -1);
  std::vector<int32_t> targets;
  for (int64_t k = 0; k < n_pair; ++k)
    if (tpos[tgt_box[k]] < 0) {
      tpos[tgt_box[k]] = 0;
      targets.push_back(tgt_box[k]);
    }
  std::sort(targets.begin(), targets.end());
  for (size_t k = 0; k < targets.size(); ++k) tpos[targets[k]] = (int32_t)k;
  std::vector<std::vector<int32_t>> sig(targets.size());
  for (int64_t k = 0; k < n_pair; ++k) sig[tpos[tgt_box[k]]].push_back(pair_tab[k]);
  auto geo = [&](int32_t t) {
    const int x = box_ijk[3 * t], y = box_ijk[3 * t + 1], z = box_ijk[3 * t + 2];
    const uint64_t par = (uint64_t)((x & 1) << 2 | (y & 1) << 1 | (z & 1));
    const uint64_t mort = (spread3((uint32_t)(x >> 1)) << 2) | (spread3((uint32_t)(y >> 1)) << 1) |
                          spread3((uint32_t)(z >> 1));
    return std::make_tuple(box_level[t], par, mort, t);
  };
  std::sort(targets.begin(), targets.end(), [&](int32_t a, int32_t c) { return geo(a) < geo(c); });
  std::map<std::vector<int32_t>, int32_t> sig_id;
  std::vector<int32_t> tsig(targets.size());
  for (int32_t t : targets) {
    auto& v = sig[tpos[t]];
    std::sort(v.begin(), v.end());
    auto it2 = sig_id.emplace(v, (int32_t)sig_id.size()).first;
    tsig[tpos[t]] = it2->second;
  }
  std::stable_sort(targets.begin(), targets.end(), [&](int32_t a, int32_t c) {
    auto ga = geo(a), gc = geo(c);
    if (std::get<0>(ga) != std::get<0>(gc)) return std::get<0>(ga) < std::get<0>(gc);
    if (std::get<1>(ga) != std::get<1>(gc)) return std::get<1>(ga) < std::get<1>(gc);
    return tsig[tpos[a]] < tsig[tpos[c]];
  });
  std::vector<int32_t> tile_tgt;
  std::vector<int32_t> slot_of(n_box, -1);  // target -> tile * NT + col
  {
    int col = NT;
    int64_t prev_group = -1;
    for (int32_t t : targets) {
      auto k = geo(t);
      const int64_t group = (int64_t)std::get<0>(k) * 8 + (int64_t)std::get<1>(k);
      if (col == NT || group != prev_group) {
        tile_tgt.resize(tile_tgt.size() + NT, -1);
        col = 0;
        prev_group = group;
      }
      const int32_t tile = (int32_t)(tile_tgt.size() / NT - 1);
      tile_tgt[tile * NT + col] = t;
      slot_of[t] = tile * NT + col;
      ++col;
    }
  }
  const int64_t n_tiles = (int64_t)tile_tgt.size() / NT;
  b->n_tiles = n_tiles;

  // 4. entries: (tile, table) -> NT sources
  struct PE {
    int32_t tile, tab, col, src;
  };
  std::vector<PE> pe(n_pair);
  for (int64_t k = 0; k < n_pair; ++k) {
    const int32_t sl = slot_of[tgt_box[k]];
    pe[k] = {sl / NT, pair_tab[k], sl % NT, src_box[k]};
  }
  // order by (tile, tab, col): three stable counting passes, least significant key first
  {
    std::vector<PE> tmp(n_pair);
    auto pass = [&](std::vector<PE>& in, std::vector<PE>& out, int64_t n_keys, auto key) {
      std::vector<int64_t> pos(n_keys + 1, 0);
      for (const PE& x : in) ++pos[key(x) + 1];
      for (int64_t i = 0; i < n_keys; ++i) pos[i + 1] += pos[i];
      for (const PE& x : in) out[pos[key(x)]++] = x;
    };
    pass(pe, tmp, NT, [](const PE& x) { return (int64_t)x.col; });
    pass(tmp, pe, b->n_tab, [](const PE& x) { return (int64_t)x.tab; });
    pass(pe, tmp, n_tiles, [](const PE& x) { return (int64_t)x.tile; });
    pe.swap(tmp);
  }
  std::vector<int32_t> entry_tab, entry_src, tile_e0(n_tiles + 1, 0);
  for (int64_t k = 0; k < n_pair; ++k) {
    if (k > 0 && pe[k].tile == pe[k - 1].tile && pe[k].tab == pe[k - 1].tab && pe[k].col == pe[k - 1].col)
    {
      delete b;
      return fail(FMM_EINVAL, "duplicate pair (same target and offset twice)");
    }
    if (k == 0 || pe[k].tile != pe[k - 1].tile || pe[k].tab != pe[k - 1].tab) {
      entry_tab.push_back(pe[k].tab);
      entry_src.resize(entry_src.size() + NT, -1);
      tile_e0[pe[k].tile + 1] = (int32_t)entry_tab.size();
    }
    entry_src[(entry_tab.size() - 1) * NT + pe[k].col] = pe[k].src;
  }
  for (int64_t t = 1; t <= n_tiles; ++t) tile_e0[t] = std::max(tile_e0[t], tile_e0[t - 1]);
  b->n_entries = (int64_t)entry_tab.size();
  auto bail = [&](int s) {
    fmm_batch_destroy(b);
    return s;
  };
  b->useful = n_pair;
  b->computed = b->n_entries * NT;

  // 5. work items.  Streaming form: the entries (already in tile order) are cut into n_wg
  //    contiguous chunks of equal length; a chunk's share of each tile it touches is one item.
  std::vector<int32_t> wg_item;
  std::vector<M2LItem> items;
  std::vector<int32_t> tile_nparts(n_tiles), tile_item0(n_tiles);
  if (b->stream) {
    const int64_t E = b->n_entries;
    int n_wg = (tuning && tuning->workgroups > 0) ? tuning->workgroups : std::max(1, env_int("FMM_M2LS_WG", n_cu));
    n_wg = (int)std::max<int64_t>(1, std::min<int64_t>(n_wg, (E + 2 * b->waves - 1) / (2 * b->waves)));
    std::vector<int64_t> cut(n_wg + 1);
    for (int g = 0; g <= n_wg; ++g) cut[g] = E * g / n_wg;
    std::vector<std::vector<M2LItem>> chunk(n_wg);
    std::vector<int32_t> nparts(n_tiles, 0);
    int64_t t = 0;
    for (int g = 0; g < n_wg; ++g) {
      while (t < n_tiles && tile_e0[t + 1] <= cut[g]) ++t;
      for (int64_t u = t; u < n_tiles && tile_e0[u] < cut[g + 1]; ++u) {
        const int32_t e0 = (int32_t)std::max<int64_t>(tile_e0[u], cut[g]);
        const int32_t e1 = (int32_t)std::min<int64_t>(tile_e0[u + 1], cut[g + 1]);
        if (e0 >= e1) continue;
        chunk[g].push_back({(int32_t)u, e0, e1, nparts[u]++});
      }
    }
    int64_t slots = 0;
    for (int64_t u = 0; u < n_tiles; ++u) {
      tile_nparts[u] = std::max(1, nparts[u]);
      tile_item0[u] = nparts[u] > 1 ? (int32_t)slots : 0;
      if (nparts[u] > 1) slots += nparts[u];
    }
    // workgroup g runs on XCD g mod 8: give XCD x the chunks x m .. x m + m - 1 (m = n_wg / 8),
    // neighbouring tiles sharing their sources and tables in that XCD's L2
    std::vector<int> chunk_of(n_wg);
    for (int g = 0; g < n_wg; ++g) chunk_of[g] = (n_wg % 8 == 0) ? (g % 8) * (n_wg / 8) + g / 8 : g;
    wg_item.push_back(0);
    for (int g = 0; g < n_wg; ++g) {
      for (const M2LItem& it : chunk[chunk_of[g]]) items.push_back(it);
      wg_item.push_back((int32_t)items.size());
    }
    b->n_wg = n_wg;
    b->n_items = (int64_t)items.size();
    b->scratch_bytes = slots * 16 * b->nc_pad * CW * (int64_t)sizeof(double);
  }
  int target_items = (tuning && tuning->target_items > 0) ? tuning->target_items : 4 * n_cu;
  target_items = std::max(1, env_int("FMM_M2L_ITEMS", target_items));
  const int min_entries = std::max(1, env_int("FMM_M2L_MIN_ENTRIES", 8));
  int64_t split_items = 0;
  // parts of about equal cost: every item gets about n_entries / target_items entries (at
  // least min_entries), so that the workgroups of one launch finish together
  const double per_item = std::max<double>(min_entries, (double)b->n_entries / target_items);
  for (int64_t t = 0; t < n_tiles && !b->stream; ++t) {
    const int ne = tile_e0[t + 1] - tile_e0[t];
    int np = (int)std::lround(ne / per_item);
    np = std::max(1, std::min(np, ne));
    tile_nparts[t] = np;
    tile_item0[t] = (int32_t)items.size();
    for (int k = 0; k < np; ++k) {
      const int e0 = tile_e0[t] + (int)((int64_t)ne * k / np), e1 = tile_e0[t] + (int)((int64_t)ne * (k + 1) / np);
      items.push_back({(int32_t)t, e0, e1, k});
    }
    if (np > 1) split_items = (int64_t)items.size();
  }
  if (!b->stream) b->n_items = (int64_t)items.size();
  // launch order: part-major within each group below; partial sums keep their slot
  // tile_item0[tile] + part whatever the order
  if (!b->stream)
    std::stable_sort(items.begin(), items.end(),
                     [](const M2LItem& x, const M2LItem& y) { return x.part < y.part; });
  if (n_tiles >= 8 && !b->stream) {
    // XCD-contiguous order: the tiles are cut into 8 contiguous ranges (neighbouring targets,
    // hence shared sources and tables in one XCD's L2); position i of the launch takes the next
    // item of range i % 8
    std::vector<std::vector<M2LItem>> grp(8);
    for (const M2LItem& it : items) grp[std::min<int64_t>(7, (int64_t)it.tile * 8 / n_tiles)].push_back(it);
    std::vector<size_t> pos(8, 0);
    std::vector<M2LItem> out;
    out.reserve(items.size());
    while (out.size() < items.size())
      for (int x = 0; x < 8; ++x)
        if (pos[x] < grp[x].size()) out.push_back(grp[x][pos[x]++]);
    items.swap(out);
  }
  // partials are indexed by item id; allocate for every item up to the last split tile
  if (!b->stream) b->scratch_bytes = split_items * NT * b->nc_pad * CW * (int64_t)sizeof(double);

  // 6. derivative tables (FP64) for every (level, offset), then the M2L layout in the dtype
  std::vector<double> off(3 * b->n_tab), hs(b->n_tab);
  for (int64_t k = 0; k < b->n_tab; ++k) {
    const int64_t key = tab_keys[k];
    const int oz = (int)(key % 17) - 8, oy = (int)((key / 17) % 17) - 8, ox = (int)((key / 289) % 17) - 8;
    const int lev = (int)(key / (289 * 17));
    off[3 * k] = ox;
    off[3 * k + 1] = oy;
    off[3 * k + 2] = oz;
    hs[k] = plan->h[lev];
  }
  double *d_off = nullptr, *d_h = nullptr, *d_tab64 = nullptr;
  if ((st = dev_upload(&d_off, off)) || (st = dev_upload(&d_h, hs))) {
    dev_free(d_off);
    dev_free(d_h);
    return bail(st);
  }
  const size_t tab_vals = (size_t)b->n_tab * b->ts * CW;
  const size_t tab_dev = b->stream ? (size_t)b->n_tab * ssh.tsp : tab_vals;  // padded rows (streaming)
  if (tab_vals) {
    if (hipMalloc((void**)&d_tab64, tab_vals * sizeof(double)) != hipSuccess ||
        hipMalloc(&b->d_tab, tab_dev * real_size(dtype)) != hipSuccess ||
        (b->stream && hipMemset(b->d_tab, 0, tab_dev * real_size(dtype)) != hipSuccess)) {
      dev_free(d_off);
      dev_free(d_h);
      dev_free(d_tab64);
      return bail(fail(FMM_ENOMEM, "table allocation failed"));
    }
    st = fmm_deriv_tables(&plan->desc, b->n_tab, d_off, d_h, d_tab64, nullptr);
    if (!st)
      st = b->stream ? launch_m2l_stream_tables(d_tab64, b->d_tab, b->n_tab, b->ts, ssh.tsp, dtype, nullptr)
                     : launch_m2l_table_layout(d_tab64, b->d_tab, b->n_tab, b->ts, dtype, nullptr);
    hipError_t e = hipDeviceSynchronize();
    dev_free(d_off);
    dev_free(d_h);
    dev_free(d_tab64);
    if (st) return bail(st);
    if (e != hipSuccess) return bail(fail(FMM_EHIP, std::string("table generation: ") + hipGetErrorString(e)));
  } else {
    dev_free(d_off);
    dev_free(d_h);
  }

  std::vector<int32_t> zeros(n_tiles, 0);
  if ((st = dev_upload(&b->d_tile_tgt, tile_tgt)) || (st = dev_upload(&b->d_tile_nparts, tile_nparts)) ||
      (st = dev_upload(&b->d_tile_item0, tile_item0)) || (st = dev_upload(&b->d_counter, zeros)) ||
      (st = dev_upload(&b->d_entry_tab, entry_tab)) || (st = dev_upload(&b->d_entry_src, entry_src)) ||
      (st = dev_upload(&b->d_items, items)) || (st = dev_upload(&b->d_wg_item, wg_item)))
    return bail(st);
  b->h_items = items;
  b->d_jbase = plan->d_jbase;
  if (b->scratch_bytes) {
    if (hipMalloc((void**)&b->d_scratch, b->scratch_bytes) != hipSuccess)
      return bail(fail(FMM_ENOMEM, "scratch allocation failed"));
    if (b->stream) {  // every partial slot starts empty (the kernel leaves it empty again)
      st = launch_fill_u32(reinterpret_cast<uint32_t*>(b->d_scratch), b->scratch_bytes / 4, kM2LPartialEmptyWord,
                           nullptr);
      hipError_t e = hipDeviceSynchronize();
      if (st) return bail(st);
      if (e != hipSuccess) return bail(fail(FMM_EHIP, std::string("scratch fill: ") + hipGetErrorString(e)));
    }
  }
  *out = b;
  return FMM_OK;
}

int fmm_m2l_prepare_fft(fmm_plan plan, int64_t n_pair, const int32_t* tgt_box, const int32_t* src_box,
                        int64_t n_box, const int32_t* box_ijk, const int32_t* box_level, fmm_batch* out) {
  int st = check_plan(plan);
  if (st) return st;
  FMM_REQUIRE(out, FMM_EINVAL, "batch output pointer is NULL");
  *out = nullptr;
  const int dtype = plan->desc.dtype;
  const bool cplx = dtype_complex(dtype);
  FMM_REQUIRE(n_pair >= 0 && n_box >= 0 && n_box <= (int64_t)0x7fffffff && n_pair <= (int64_t)0x7fffffff,
              FMM_EINVAL, "bad sizes");
  FMM_REQUIRE(n_pair == 0 || (tgt_box && src_box && box_ijk && box_level), FMM_EINVAL, "NULL host array");
  const int S = plan->S, Sz = plan->Sz, Hy = fft_half_y(S, cplx), nh = Sz * S * Hy;
  FMM_REQUIRE((nh + 255) / 256 <= kFftMaxPerThread, FMM_EUNSUPPORTED, "order too high for the FFT M2L path");
  int dev = 0, lds_max = 65536;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0) lds_max = v;
  }
  (void)hipGetLastError();
  FMM_REQUIRE(fft_lds_bytes(S, Sz, real_size(dtype), cplx) <= (size_t)lds_max, FMM_EUNSUPPORTED,
              "FFT M2L working set exceeds LDS for this order");
  // (level, offset) tables and per-target pair lists
  std::unordered_map<int64_t, int32_t> tab_of_key;
  std::vector<int64_t> tab_keys;
  std::vector<std::tuple<int32_t, int32_t, int32_t>> pe(n_pair);  // target, table, source
  for (int64_t k = 0; k < n_pair; ++k) {
    const int32_t t = tgt_box[k], s = src_box[k];
    FMM_REQUIRE(t >= 0 && t < n_box && s >= 0 && s < n_box, FMM_EINVAL, "box id out of range");
    const int lt = box_level[t];
    FMM_REQUIRE(lt >= 0 && lt < plan->n_levels && lt == box_level[s], FMM_EINVAL, "bad box levels");
    const int ox = box_ijk[3 * t] - box_ijk[3 * s], oy = box_ijk[3 * t + 1] - box_ijk[3 * s + 1],
              oz = box_ijk[3 * t + 2] - box_ijk[3 * s + 2];
    FMM_REQUIRE(std::abs(ox) <= 8 && std::abs(oy) <= 8 && std::abs(oz) <= 8 && (ox || oy || oz), FMM_EINVAL,
                "offset zero or larger than 8");
    const int64_t key = ((int64_t)lt * 17 + (ox + 8)) * 289 + (oy + 8) * 17 + (oz + 8);
    auto it = tab_of_key.find(key);
    if (it == tab_of_key.end()) {
      it = tab_of_key.emplace(key, (int32_t)tab_keys.size()).first;
      tab_keys.push_back(key);
    }
    pe[k] = {t, it->second, s};
  }
  std::sort(pe.begin(), pe.end());
  std::vector<int32_t> tgt_list, tgt_ptr{0}, ent_tab, ent_src, src_list(src_box, src_box + n_pair);
  for (int64_t k = 0; k < n_pair; ++k) {
    if (k == 0 || std::get<0>(pe[k]) != std::get<0>(pe[k - 1])) {
      if (k > 0) tgt_ptr.push_back((int32_t)k);
      tgt_list.push_back(std::get<0>(pe[k]));
    }
    ent_tab.push_back(std::get<1>(pe[k]));
    ent_src.push_back(std::get<2>(pe[k]));
  }
  if (n_pair) tgt_ptr.push_back((int32_t)n_pair);
  std::sort(src_list.begin(), src_list.end());
  src_list.erase(std::unique(src_list.begin(), src_list.end()), src_list.end());

  auto* b = new fmm_batch_s();
  b->plan = plan;
  b->dtype = dtype;
  b->fft = true;
  b->nc = plan->nc;
  b->n_pair = n_pair;
  b->n_tab = (int64_t)tab_keys.size();
  b->n_tiles = (int64_t)tgt_list.size();
  b->n_entries = n_pair;
  b->n_items = (int64_t)tgt_list.size();
  b->useful = b->computed = n_pair;
  FftArgs& a = b->fa;
  a.S = S;
  a.Sz = Sz;
  a.nc = plan->nc;
  a.n_tab = b->n_tab;
  a.n_src = (int64_t)src_list.size();
  a.n_tgt = (int64_t)tgt_list.size();
  a.jxyz = plan->d_jxyz;
  a.tau = std::max(1.0, plan->p / 4.0);
  std::vector<double> tp(2 * plan->p + 1);
  for (int k = 0; k <= 2 * plan->p; ++k) tp[k] = std::pow(a.tau, k);
  std::vector<double> off(3 * b->n_tab), hs(b->n_tab);
  for (int64_t k = 0; k < b->n_tab; ++k) {
    const int64_t key = tab_keys[k];
    off[3 * k] = (int)((key / 289) % 17) - 8;
    off[3 * k + 1] = (int)((key / 17) % 17) - 8;
    off[3 * k + 2] = (int)(key % 17) - 8;
    hs[k] = plan->h[(int)(key / (289 * 17))];
  }
  auto bail = [&](int s) {
    fmm_batch_destroy(b);
    return s;
  };
  double *d_off = nullptr, *d_h = nullptr, *d_tp = nullptr;
  int32_t *d_sl = nullptr, *d_tl = nullptr, *d_tp2 = nullptr, *d_et = nullptr, *d_es = nullptr;
  if ((st = dev_upload(&d_tp, tp)) || (st = dev_upload(&d_sl, src_list)) || (st = dev_upload(&d_tl, tgt_list)) ||
      (st = dev_upload(&d_tp2, tgt_ptr)) || (st = dev_upload(&d_et, ent_tab)) || (st = dev_upload(&d_es, ent_src)))
    return bail(st);
  a.taupow = d_tp;
  a.src_list = d_sl;
  a.tgt_list = d_tl;
  a.tgt_ptr = d_tp2;
  a.ent_tab = d_et;
  a.ent_src = d_es;
  const size_t cb = 2 * real_size(dtype);
  double* d_tab64 = nullptr;
  if (b->n_tab) {
    if ((st = dev_upload(&d_off, off)) || (st = dev_upload(&d_h, hs))) {
      dev_free(d_off);
      dev_free(d_h);
      return bail(st);
    }
    if (hipMalloc((void**)&d_tab64, (size_t)b->n_tab * Sz * S * S * sizeof(double) * (cplx ? 2 : 1)) != hipSuccess ||
        hipMalloc(&a.spec_tab, (size_t)b->n_tab * nh * cb) != hipSuccess) {
      dev_free(d_off);
      dev_free(d_h);
      dev_free(d_tab64);
      return bail(fail(FMM_ENOMEM, "FFT table allocation failed"));
    }
    a.tab64 = d_tab64;
    st = fmm_deriv_tables(&plan->desc, b->n_tab, d_off, d_h, d_tab64, nullptr);
    if (!st) st = launch_fft(a, dtype, 0, nullptr);
    hipError_t e = hipDeviceSynchronize();
    dev_free(d_off);
    dev_free(d_h);
    if (st) return bail(st);
    if (e != hipSuccess) return bail(fail(FMM_EHIP, std::string("FFT table spectra: ") + hipGetErrorString(e)));
  }
  if (n_box && hipMalloc(&a.spec_src, (size_t)n_box * nh * cb) != hipSuccess)
    return bail(fail(FMM_ENOMEM, "FFT spectra allocation failed"));
  b->scratch_bytes = (int64_t)n_box * nh * cb;
  *out = b;
  return FMM_OK;
}

void fmm_batch_destroy(fmm_batch b) {
  if (!b) return;
  if (b->fft) {
    dev_free((void*)b->fa.tab64);
    dev_free(b->fa.spec_tab);
    dev_free(b->fa.spec_src);
    dev_free((void*)b->fa.src_list);
    dev_free((void*)b->fa.tgt_list);
    dev_free((void*)b->fa.tgt_ptr);
    dev_free((void*)b->fa.ent_tab);
    dev_free((void*)b->fa.ent_src);
    dev_free((void*)b->fa.taupow);
  }
  dev_free(b->d_tab);
  dev_free(b->d_tile_tgt);
  dev_free(b->d_tile_nparts);
  dev_free(b->d_tile_item0);
  dev_free(b->d_counter);
  dev_free(b->d_scratch);
  dev_free(b->d_entry_tab);
  dev_free(b->d_entry_src);
  dev_free(b->d_items);
  dev_free(b->d_wg_item);
  delete b;
}

int fmm_batch_info(fmm_batch b, int64_t* info, int32_t n_info) {
  FMM_REQUIRE(b, FMM_EINVAL, "batch is NULL");
  FMM_REQUIRE(info || n_info == 0, FMM_EINVAL, "info is NULL");
  const int64_t v[] = {b->n_pair,        b->n_tab,     b->n_tiles, b->n_entries,  b->n_items,
                       b->useful,        b->computed,  b->nc,      b->nc_pad,     b->scratch_bytes,
                       b->rows_per_wave, b->col_tiles, b->waves,   b->col_groups, b->lds_bytes,
                       b->nbuf,          b->k_splits,  b->shape.nrem, (int64_t)b->stream,
                       b->n_wg};
  for (int k = 0; k < n_info && k < (int)(sizeof(v) / sizeof(v[0])); ++k) info[k] = v[k];
  return FMM_OK;
}

static M2LStreamArgs m2l_stream_args(fmm_batch b, const void* mpole, void* local) {
  M2LStreamArgs a{};
  a.items = b->d_items;
  a.wg_item = b->d_wg_item;
  a.n_wg = b->n_wg;
  a.tile_tgt = b->d_tile_tgt;
  a.tile_nparts = b->d_tile_nparts;
  a.tile_item0 = b->d_tile_item0;
  a.counter = b->d_counter;
  a.scratch = b->d_scratch;
  a.entry_tab = b->d_entry_tab;
  a.entry_src = b->d_entry_src;
  a.tab = b->d_tab;
  a.jbase = b->d_jbase;
  a.mpole = mpole;
  a.local = local;
  a.lds_slot = b->lds_slot;
  a.lds_sbq = b->lds_sbq;
  return a;
}

static M2LArgs m2l_args(fmm_batch b, const void* mpole, void* local) {
  M2LArgs a{};
  a.items = b->d_items;
  a.n_items = (int32_t)b->n_items;
  a.tile_tgt = b->d_tile_tgt;
  a.tile_nparts = b->d_tile_nparts;
  a.tile_item0 = b->d_tile_item0;
  a.counter = b->d_counter;
  a.scratch = b->d_scratch;
  a.entry_tab = b->d_entry_tab;
  a.entry_src = b->d_entry_src;
  a.tab = b->d_tab;
  a.jbase = b->d_jbase;
  a.mpole = mpole;
  a.local = local;
  a.nc = b->nc;
  a.nc_pad = b->nc_pad;
  a.ts = b->ts;
  a.ldb = b->shape.ldb;
  a.k4p = b->shape.k4p;
  a.tab_off = b->shape.tab_off;
  a.buf_elems = b->shape.buf_elems;
  a.nt = b->shape.nt;
  a.nrg = b->shape.nrg;
  a.rtiles = b->shape.rtiles;
  a.nrem = b->shape.nrem;
  a.nks = b->shape.nks;
  return a;
}

static int m2l_launch(fmm_batch b, const void* in, void* out, void* stream);
static M2LStreamArgs m2l_stream_args(fmm_batch b, const void* mpole, void* local);

int fmm_m2l_batched(fmm_batch b, const void* mpole, void* local, void* stream) {
  FMM_REQUIRE(b, FMM_EINVAL, "batch is NULL");
  FMM_REQUIRE(!b->adjoint, FMM_ESTATE, "batch was prepared for the adjoint; use fmm_m2l_batched_adjoint");
  return m2l_launch(b, mpole, local, stream);
}

int fmm_m2l_batched_ex(fmm_batch b, const void* mpole, void* local, int32_t mode, void* stream) {
  FMM_REQUIRE(b, FMM_EINVAL, "batch is NULL");
  FMM_REQUIRE(mode == FMM_ACCUMULATE || mode == FMM_OVERWRITE, FMM_EINVAL, "mode must be FMM_ACCUMULATE or FMM_OVERWRITE");
  FMM_REQUIRE(!b->adjoint, FMM_ESTATE, "batch was prepared for the adjoint; use fmm_m2l_batched_adjoint");
  if (mode == FMM_ACCUMULATE) return m2l_launch(b, mpole, local, stream);
  FMM_REQUIRE(b->plan && b->plan->alive, FMM_ESTATE, "the batch's plan was destroyed");
  FMM_REQUIRE(b->stream && !b->fft, FMM_EUNSUPPORTED, "FMM_OVERWRITE needs a streaming-form batch");
  if (b->n_items == 0) return FMM_OK;
  FMM_REQUIRE(mpole && local, FMM_EINVAL, "NULL coefficient array");
  M2LStreamArgs a = m2l_stream_args(b, mpole, local);
  a.overwrite = 1;
  return launch_m2l_stream(a, b->p, b->c_pde, b->dtype, b->waves, (size_t)b->lds_bytes, (hipStream_t)stream);
}

int fmm_m2l_batched_adjoint(fmm_batch b, const void* local_grad, void* mpole_grad, void* stream) {
  FMM_REQUIRE(b, FMM_EINVAL, "batch is NULL");
  FMM_REQUIRE(b->adjoint, FMM_ESTATE, "batch was not prepared with fmm_m2l_prepare_adjoint");
  return m2l_launch(b, local_grad, mpole_grad, stream);
}

static int m2l_launch(fmm_batch b, const void* mpole, void* local, void* stream) {
  FMM_REQUIRE(b->plan && b->plan->alive, FMM_ESTATE, "the batch's plan was destroyed");
  if (b->fft) {
    if (b->n_pair == 0) return FMM_OK;
    FMM_REQUIRE(mpole && local, FMM_EINVAL, "NULL coefficient array");
    FftArgs a = b->fa;
    a.mpole = mpole;
    a.local = local;
    int st = launch_fft(a, b->dtype, 1, (hipStream_t)stream);
    if (st) return st;
    return launch_fft(a, b->dtype, 2, (hipStream_t)stream);
  }
  if (b->n_items == 0) return FMM_OK;
  FMM_REQUIRE(mpole && local, FMM_EINVAL, "NULL coefficient array");
  if (b->stream) return launch_m2l_stream(m2l_stream_args(b, mpole, local), b->p, b->c_pde, b->dtype, b->waves,
                                          (size_t)b->lds_bytes, (hipStream_t)stream);
  return launch_m2l(m2l_args(b, mpole, local), b->dtype, b->rows_per_wave, b->col_tiles, b->pf_class, b->nbuf,
                    b->waves, (hipStream_t)stream);
}

static M2LArgs m2l_args(fmm_batch b, const void* mpole, void* local);

// ---- fmm_m2l_batched_static: the split-tile partials and part counters of an M2L launch in a
// fixed device array instead of the batch's own scratch, for callers that cannot allocate.
namespace {
constexpr size_t kStaticScratchBytes = 16u << 20;
constexpr int kMaxDevices = 64;
// Host code must not use this name as a device address: its address on a device comes from
// hipGetSymbolAddress (static_scratch below), once per device.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int static_scratch(void** out) {
  int dev = 0;
  FMM_HIP_CHECK(hipGetDevice(&dev));
  FMM_REQUIRE(dev >= 0 && dev < kMaxDevices, FMM_EUNSUPPORTED, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(FMM_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return FMM_OK;
}
}  // namespace

int fmm_m2l_batched_static(fmm_batch b, const void* mpole, void* local, void* stream) {
  FMM_REQUIRE(b, FMM_EINVAL, "batch is NULL");
  FMM_REQUIRE(b->plan && b->plan->alive, FMM_ESTATE, "the batch's plan was destroyed");
  FMM_REQUIRE(!b->adjoint, FMM_ESTATE, "batch was prepared for the adjoint");
  FMM_REQUIRE(!b->fft, FMM_EUNSUPPORTED, "the FFT form keeps its spectra in the batch; use fmm_m2l_batched");
  if (b->n_items == 0) return FMM_OK;
  FMM_REQUIRE(mpole && local, FMM_EINVAL, "NULL coefficient array");
  const size_t part_bytes = ((size_t)b->scratch_bytes + 255) / 256 * 256;
  const size_t need = part_bytes + (size_t)b->n_tiles * sizeof(int32_t);
  FMM_REQUIRE(need <= kStaticScratchBytes, FMM_EUNSUPPORTED,
              "this batch needs " + std::to_string(need) + " bytes of scratch; the static array holds " +
                  std::to_string(kStaticScratchBytes) + " (use fmm_m2l_batched)");
  void* base = nullptr;
  int st = static_scratch(&base);
  if (st) return st;
  double* part = reinterpret_cast<double*>(base);
  int32_t* counter = reinterpret_cast<int32_t*>(static_cast<unsigned char*>(base) + part_bytes);
  // the part counters must start at zero (and, for the streaming form, the partial slots
  // empty); the array keeps whatever the last call left there
  st = launch_zero_i32(counter, b->n_tiles, (hipStream_t)stream);
  if (st) return st;
  if (b->stream) {
    st = launch_fill_u32(reinterpret_cast<uint32_t*>(part), b->scratch_bytes / 4, kM2LPartialEmptyWord,
                         (hipStream_t)stream);
    if (st) return st;
    M2LStreamArgs a = m2l_stream_args(b, mpole, local);
    a.scratch = part;
    a.counter = counter;
    return launch_m2l_stream(a, b->p, b->c_pde, b->dtype, b->waves, (size_t)b->lds_bytes, (hipStream_t)stream);
  }
  M2LArgs a = m2l_args(b, mpole, local);
  a.scratch = part;
  a.counter = counter;
  return launch_m2l(a, b->dtype, b->rows_per_wave, b->col_tiles, b->pf_class, b->nbuf, b->waves,
                    (hipStream_t)stream);
}

// Persistent launch state of a group of tiled batches sharing one tile shape: work items of all
// its batches ordered by decreasing cost, the workgroup sized for the largest wavefront count.
static int multi_group_prepare(fmm_multi m, MultiGroup& g, int n_cu) {
  const fmm_batch b0 = m->batches[g.idx[0]];
  if (!m2l_multi_shape_instantiated(b0->rows_per_wave, b0->col_tiles))
    return fail(FMM_EUNSUPPORTED, "tiled launch shape not instantiated for multi-batch launches");
  g.rt = b0->rows_per_wave;
  g.ctw = b0->col_tiles;
  g.nbuf = b0->nbuf;
  std::vector<M2LArgs> args(g.idx.size());
  struct Wk {
    double cost;
    int2 w;
  };
  std::vector<Wk> work;
  for (size_t k = 0; k < g.idx.size(); ++k) {
    const fmm_batch b = m->batches[g.idx[k]];
    g.waves = std::max(g.waves, b->waves);
    g.pf = std::max(g.pf, b->pf_class);
    g.lds = std::max(g.lds, (size_t)b->lds_bytes);
    args[k] = m2l_args(b, nullptr, nullptr);
    for (size_t i = 0; i < b->h_items.size(); ++i) {
      const M2LItem& it = b->h_items[i];
      const double cost = (double)(it.e1 - it.e0) * b->nc_pad * b->shape.k4p * b->shape.nt;
      work.push_back({cost, int2{(int)k, (int)i}});
    }
  }
  // the shared workgroup has the largest wave count; every batch's staging must divide evenly
  for (int k : g.idx) {
    const fmm_batch b = m->batches[k];
    const int nthr = g.waves * 64;
    if (nthr % b->shape.nt || (dtype_complex(m->dtype) && ((nthr / b->shape.nt) & 1)))
      return fail(FMM_EUNSUPPORTED, "batch tile size does not divide the shared workgroup");
  }
  std::stable_sort(work.begin(), work.end(), [](const Wk& a, const Wk& c) { return a.cost > c.cost; });
  std::vector<int2> wl(work.size());
  for (size_t i = 0; i < work.size(); ++i) wl[i] = work[i].w;
  g.n_work = (int32_t)wl.size();
  g.grid = std::max(1, std::min<int>(g.n_work, 2 * n_cu));
  int st;
  if ((st = dev_upload(&g.d_args, args)) || (st = dev_upload(&g.d_work, wl))) return st;
  return FMM_OK;
}

int fmm_m2l_multi_prepare(int32_t n, const fmm_batch* batches, fmm_multi* out) {
  FMM_REQUIRE(out, FMM_EINVAL, "output pointer is NULL");
  *out = nullptr;
  FMM_REQUIRE(n >= 1 && n <= kM2LMultiMax, FMM_EINVAL, "number of batches must be in [1, 32]");
  FMM_REQUIRE(batches, FMM_EINVAL, "batches is NULL");
  const fmm_batch b0 = batches[0];
  FMM_REQUIRE(b0, FMM_EINVAL, "NULL batch");
  for (int k = 0; k < n; ++k) {
    const fmm_batch b = batches[k];
    FMM_REQUIRE(b && b->plan && b->plan->alive, FMM_EINVAL, "NULL or stale batch");
    FMM_REQUIRE(!b->fft && !b->adjoint, FMM_EINVAL, "FFT and adjoint batches cannot join a multi launch");
    FMM_REQUIRE(b->dtype == b0->dtype, FMM_EINVAL, "batches must share one dtype");
    for (int j = 0; j < k; ++j)  // split tiles keep their partials in the batch's own scratch
      FMM_REQUIRE(batches[j] != b, FMM_EINVAL, "a batch may appear only once in a multi launch");
  }
  auto* m = new fmm_multi_s();
  m->batches.assign(batches, batches + n);
  m->dtype = b0->dtype;
  // streaming batches launch on their own; tiled batches are grouped by tile shape, in order of
  // first appearance
  for (int k = 0; k < n; ++k) {
    const fmm_batch b = batches[k];
    if (b->stream) {
      MultiGroup g;
      g.stream = true;
      g.idx.push_back(k);
      m->groups.push_back(g);
      continue;
    }
    MultiGroup* hit = nullptr;
    for (MultiGroup& g : m->groups) {
      const fmm_batch f = batches[g.idx[0]];
      if (!g.stream && f->rows_per_wave == b->rows_per_wave && f->col_tiles == b->col_tiles && f->nbuf == b->nbuf)
        hit = &g;
    }
    if (hit) {
      hit->idx.push_back(k);
    } else {
      MultiGroup g;
      g.idx.push_back(k);
      m->groups.push_back(g);
    }
  }
  int dev = 0, n_cu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) n_cu = v;
  }
  (void)hipGetLastError();
  for (MultiGroup& g : m->groups) {
    if (g.stream) continue;
    if (int st = multi_group_prepare(m, g, n_cu)) {
      fmm_m2l_multi_destroy(m);
      return st;
    }
  }
  *out = m;
  return FMM_OK;
}

int fmm_m2l_multi_launch(fmm_multi m, const void* const* mpole, void* const* local, void* stream) {
  FMM_REQUIRE(m, FMM_EINVAL, "multi is NULL");
  FMM_REQUIRE(mpole && local, FMM_EINVAL, "NULL pointer arrays");
  for (size_t k = 0; k < m->batches.size(); ++k) {
    FMM_REQUIRE(m->batches[k]->plan && m->batches[k]->plan->alive, FMM_ESTATE, "a batch's plan was destroyed");
    FMM_REQUIRE(mpole[k] && local[k], FMM_EINVAL, "NULL coefficient array");
  }
  for (const MultiGroup& g : m->groups) {
    if (g.stream) {
      const int k = g.idx[0];
      if (int st = m2l_launch(m->batches[k], mpole[k], local[k], stream)) return st;
      continue;
    }
    if (g.n_work == 0) continue;
    M2LMulti a{};
    a.args = g.d_args;
    a.work = g.d_work;
    a.n_work = g.n_work;
    for (size_t k = 0; k < g.idx.size(); ++k) {
      a.mpole[k] = mpole[g.idx[k]];
      a.local[k] = local[g.idx[k]];
    }
    if (int st = launch_m2l_multi(a, m->dtype, g.rt, g.ctw, g.pf, g.nbuf, g.lds, g.waves, g.grid,
                                  (hipStream_t)stream))
      return st;
  }
  return FMM_OK;
}

void fmm_m2l_multi_destroy(fmm_multi m) {
  if (!m) return;
  for (MultiGroup& g : m->groups) {
    dev_free(g.d_args);
    dev_free(g.d_work);
  }
  delete m;
}

int fmm_m2l_batched_multi(int32_t n, const fmm_batch* batches, const void* const* mpole, void* const* local,
                          void* stream) {
  FMM_REQUIRE(n >= 0, FMM_EINVAL, "n < 0");
  if (n == 0) return FMM_OK;
  FMM_REQUIRE(batches && mpole && local, FMM_EINVAL, "NULL array");
  for (int k = 0; k < n; ++k) {
    FMM_REQUIRE(batches[k], FMM_EINVAL, "NULL batch");
    FMM_REQUIRE(batches[k]->dtype == batches[0]->dtype, FMM_EINVAL, "batches must share one dtype");
    FMM_REQUIRE(!batches[k]->adjoint, FMM_ESTATE, "adjoint batch passed to fmm_m2l_batched_multi");
    FMM_REQUIRE(!batches[k]->fft, FMM_EINVAL, "FFT batch passed to fmm_m2l_batched_multi");
  }
  for (int k = 0; k < n; ++k) {
    int st = fmm_m2l_batched(batches[k], mpole[k], local[k], stream);
    if (st) return st;
  }
  return FMM_OK;
}

}  // extern "C"
