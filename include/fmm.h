/*
 * fmm.h -- C ABI of the MI355X (gfx950) library for the PDE-compressed
 * Cartesian-Taylor FMM translation operators of Fernando & Kloeckner,
 * "Automatic Synthesis of Low-Complexity Translation Operators for the Fast
 * Multipole Method" (arXiv 2305.17867).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Pointers are device pointers unless marked [host].  The caller owns every
 * buffer it passes; the library never frees or retains caller memory.  Launch
 * entry points enqueue kernels on `stream` (a hipStream_t passed as void*,
 * NULL = the default stream), return at once, never allocate device memory and
 * never synchronise, so they may be captured into a HIP graph.  The set-up and
 * tear-down calls allocate, free or synchronise: fmm_plan_create, the
 * fmm_m2l_prepare* calls (_ex, _fft, _adjoint), fmm_m2l_multi_prepare, the
 * fmm_tree_* calls and the fmm_*_destroy calls.
 *
 * Every entry point returns an fmm_status.  Arguments are validated on the host
 * before anything is enqueued; on a non-OK status nothing was enqueued and
 * fmm_last_error() returns a thread-local message.  Device-side index values
 * (box point ranges, box ids in prepared batches) cannot be checked on the host
 * without a synchronisation; kernels clamp point ranges to [0, n_points] so a
 * bad range never reads or writes out of bounds.
 *
 * Kernels G (3-D, r = |x|), each obeying a constant-coefficient elliptic PDE
 * (Sec. 4.1, Property 1):
 *   FMM_LAPLACE    1/(4 pi r)            Delta G = 0
 *   FMM_HELMHOLTZ  exp(i k r)/(4 pi r)   (Delta + k^2) G = 0,  param = k
 *   FMM_YUKAWA     exp(-l r)/(4 pi r)    (Delta - l^2) G = 0,  param = l
 *   FMM_BIHARMONIC r                     Delta^2 G = 0
 *
 * Dtypes.  FMM_F64: points, weights, coefficients and potentials float64.
 * FMM_F32: points float32, weights/coefficients/potentials float32; M2L runs as
 * FP32 matrix-core products with each offset group's partial sum accumulated in
 * FP64, derivative tables are generated in FP64 and rounded once.  FMM_C128 /
 * FMM_C64: as F64 / F32 with complex weights, coefficients and potentials,
 * interleaved (re, im) like C99 double complex.  Helmholtz needs a complex
 * dtype; the other kernels need a real one.  Box centres are always float64.
 *
 * Expansions (Secs. 2, 3.3, 3.4, 4.1).  With J = {m : |m| <= p, m_z < c} (c = PDE
 * order; the compressed axis is z, Lemma max_prod_nice) a multipole about centre
 * c1 is stored as beta = M^T alpha, alpha_q = sum_y w(y) (c1 - y)^q / q!
 * (eqs. mpole, define_beta_multipole), and a local about c2 as the kept derivatives
 * theta_i, i in J (eqs. stored_local_coeffs, compressed-local-form: no factorial).
 * Both are stored in the scaled form of Sec. 4.1.1 with t = 1/h, h the box size
 * of the box's level:  beta~_q = beta_q / h^|q|,  theta~_i = theta_i * h^|i|.
 * Coefficient arrays are [n_box][Nc] (Nc = |J|), entries in the order that
 * fmm_index_table returns: lexicographic in (m_z, m_x, m_y), m_y fastest.
 */
#ifndef FMM_H
#define FMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FMM_ABI_VERSION 2
#define FMM_MAX_ORDER 16

typedef enum {
  FMM_OK = 0,
  FMM_EINVAL = -1,       /* invalid argument (null pointer, size, range, mismatch) */
  FMM_EUNSUPPORTED = -2, /* valid but not supported (kernel/dtype pair, order) */
  FMM_EHIP = -3,         /* a HIP runtime call failed */
  FMM_ENOMEM = -4,       /* device or host allocation failed */
  FMM_ESTATE = -5        /* object in the wrong state (e.g. destroyed plan) */
} fmm_status;

typedef enum {
  FMM_LAPLACE = 0,
  FMM_HELMHOLTZ = 1,
  FMM_YUKAWA = 2,
  FMM_BIHARMONIC = 3,
  FMM_LAPLACE2D = 4,   /* 2-D log r; only the fmm2d_* calls take it */
  FMM_BIHARMONIC2D = 5 /* 2-D r^2 log r; only the fmm2d_* calls take it */
} fmm_kernel;
typedef enum { FMM_F64 = 0, FMM_F32 = 1, FMM_C128 = 2, FMM_C64 = 3 } fmm_dtype;

typedef struct {
  int32_t kernel; /* fmm_kernel */
  int32_t order;  /* expansion order p, 0 <= p <= FMM_MAX_ORDER */
  int32_t dtype;  /* fmm_dtype */
  int32_t flags;  /* must be 0 */
  double param;   /* Helmholtz k or Yukawa lambda (> 0); ignored otherwise */
} fmm_desc;

typedef struct fmm_plan_s* fmm_plan;   /* per (kernel, p, dtype, level sizes): index and
                                          recursion tables in device memory */
typedef struct fmm_batch_s* fmm_batch; /* a prepared M2L batch: derivative tables and
                                          target-tile work lists in device memory */
typedef struct fmm_multi_s* fmm_multi; /* several batches drained by one persistent launch */

/* ABI version (FMM_ABI_VERSION). */
int32_t fmm_abi_version(void);

/* Thread-local description of the last non-OK status returned on this thread. */
const char* fmm_last_error(void);

/* Sizes of the full Taylor set M(p) (N(p) = C(p+3,3), reading of eq. np-count) and of
 * the kept set J (|J| = N(p) - N(p-c), Sec. 3.1).  Host only; no GPU needed.
 * n_full, n_compressed: [host] outputs, either may be NULL. */
int fmm_sizes(const fmm_desc* desc, int32_t* n_full, int32_t* n_compressed);

/* Multi-indices of the stored coefficients, in storage order (Lemma max_prod_nice: J =
 * {m : m_z < c}).  mxyz: [host] output [Nc][3] (m_x, m_y, m_z).  Host only. */
int fmm_index_table(const fmm_desc* desc, int32_t* mxyz);

/* Derivative tables G^(m)(h * o) * h^|m| (the scaled table of Sec. 4.1.1 with t = 1/h) for
 * |m| <= 2p and m_z <= 2(c-1): every derivative the compressed M2L of eq. m2l_toeplitz
 * reads.  Generated in FP64 whatever desc->dtype says (Taylor-coefficient recurrences; for
 * Laplace the recurrence of eq. deriv_laplace_3d is the same relation).
 *   n       number of tables
 *   offset  [n][3] float64: translation vector in units of h (c_target - c_source) / h;
 *           must be nonzero
 *   h       [n] float64 > 0 box sizes
 *   out     [n][2c-1][2p+1][2p+1] float64 (complex128 for Helmholtz), index
 *           (m_z, m_x, m_y); entries with |m| > 2p are set to zero.  OVERWRITTEN. */
int fmm_deriv_tables(const fmm_desc* desc, int64_t n, const double* offset, const double* h,
                     void* out, void* stream);

/* Create a plan.  level_box_size [host][n_levels]: h of each tree level (> 0).  Allocates
 * and synchronises (not capturable). */
int fmm_plan_create(const fmm_desc* desc, int32_t n_levels, const double* level_box_size,
                    fmm_plan* plan);
void fmm_plan_destroy(fmm_plan plan);

/* Compressed P2M (Sec. 3.4): for each box b < n_box, the scaled compressed multipole
 * beta~ = (M^T alpha)/h^|q| of the sources src[pt_range[b][0] : pt_range[b][1]] about
 * box_center[b], h = level_box_size[box_level[b]].
 *   box_center [n_box][3] f64; box_level [n_box] i32; pt_range [n_box][2] i64
 *   src_xyz    [n_src][3] real dtype; weight [n_src] dtype
 *   mpole      [n_box][Nc] dtype, OVERWRITTEN
 * Boxes with many points are spread over several workgroups whose results go through a
 * buffer owned by the plan and are added in a fixed order, so P2M calls (and fmm_l2p_adjoint
 * calls) of one plan must not run at the same time on different streams. */
int fmm_p2m(fmm_plan plan, int64_t n_box, const double* box_center, const int32_t* box_level,
            const int64_t* pt_range, int64_t n_src, const void* src_xyz, const void* weight,
            void* mpole, void* stream);

/* Compressed L2P (Sec. 3.3, eq. compressed-local-form): for each box b, decompress its
 * scaled local, apply 1/i!, and add phi(x) = sum_i ([M theta]_i / i!) (x - c)^i to every
 * target x in tgt[pt_range[b][0] : pt_range[b][1]].
 *   tgt_xyz [n_tgt][3] real dtype; local [n_box][Nc] dtype
 *   potential [n_tgt] dtype, ACCUMULATED.  The point ranges of the boxes of one call must
 *   be disjoint (apply tree levels in separate calls). */
int fmm_l2p(fmm_plan plan, int64_t n_box, const double* box_center, const int32_t* box_level,
            const int64_t* pt_range, int64_t n_tgt, const void* tgt_xyz, const void* local,
            void* potential, void* stream);

/* Output modes of the _ex calls: add to the output (as the plain calls do), or store into it
 * (BLAS beta = 0: the old values are neither read nor needed, so the caller need not clear
 * them). */
enum { FMM_ACCUMULATE = 0, FMM_OVERWRITE = 1 };

/* fmm_l2p with an output mode.  FMM_OVERWRITE: potential[x] = the local expansion's value for
 * every target x of the call's boxes (ranges of one call must be disjoint); other entries are
 * left unchanged. */
int fmm_l2p_ex(fmm_plan plan, int64_t n_box, const double* box_center, const int32_t* box_level,
               const int64_t* pt_range, int64_t n_tgt, const void* tgt_xyz, const void* local, void* potential,
               int32_t mode, void* stream);

/* Compressed M2M (Sec. 4.3, eq. define_psi): for each k < n_parent, the scaled compressed
 * multipole of box parent[k] becomes psi~ = M^T T E beta~ summed over its children: each
 * child's kept coefficients are embedded with zeros elsewhere (E), translated to the parent
 * centre with the binomial formula of eq. mpole_translated_full_coeffs (T) and compressed
 * at the parent's box size (M^T).  Exact for Laplace and biharmonic; for Helmholtz and
 * Yukawa the translated expansion differs from the parent's own P2M at truncation level.
 *   parent     [n_parent] i32 box indices; entries outside [0, n_box) are skipped
 *   child      [n_parent][8] i32 box indices; entries outside [0, n_box) mean "no child"
 *   box_center [n_box][3] f64; box_level [n_box] i32 (scaled by the level's box size)
 *   mpole      [n_box][Nc] dtype: read at the children, OVERWRITTEN at the parents (zero
 *              for a parent without children).
 * A box must not be both a parent and a child in one call (apply levels in separate calls,
 * children first). */
int fmm_m2m(fmm_plan plan, int64_t n_parent, const int32_t* parent, const int32_t* child, int64_t n_box,
            const double* box_center, const int32_t* box_level, void* mpole, void* stream);

/* Compressed L2L (Sec. 4.2, eq. l2l-expr in derivative form): for each k < n_parent the
 * scaled compressed local of box parent[k] is decompressed (M), translated to the centre of
 * each of its children and the kept entries are added to the child's local.  Exact for
 * Laplace and biharmonic (the local polynomial satisfies the PDE); truncation-level
 * differences for Helmholtz and Yukawa.
 *   parent, child, box_center, box_level as for fmm_m2m
 *   local      [n_box][Nc] dtype: read at the parents, ACCUMULATED at the children.
 * A box must appear at most once as a child and not also as a parent in one call. */
int fmm_l2l(fmm_plan plan, int64_t n_parent, const int32_t* parent, const int32_t* child, int64_t n_box,
            const double* box_center, const int32_t* box_level, void* local, void* stream);

/* Compressed M2P (Sec. 3.5, eq. multipole_eval_beta): multipoles evaluated directly at targets
 * (the W list of an adaptive tree).  For each k < n_tbox and every target x of box tbox[k],
 *   potential[x] += sum over the boxes s of list[list_ptr[k] : list_ptr[k+1]] of
 *                   sum_{q in J} mpole[s][q] G^(q)(x - c_s) h_s^|q|
 * (the scaled multipoles of fmm_p2m, h_s the size of s's level).  The derivatives at each
 * target are computed on the kept set only (m_z < c, |m| <= p) by the FP64 recurrences of
 * fmm_deriv_tables; the sums are FP64, rounded to the dtype when added.
 *   tbox [n_tbox] i32 box ids, each at most once (its targets are written by one workgroup);
 *   list_ptr [n_tbox + 1] i32 CSR pointers into list [n_list] i32 box ids (pointers clamped to
 *   [0, n_list]; ids outside [0, n_box) skipped)
 *   box_center [n_box][3] f64, box_level [n_box] i32, tgt_range [n_box][2] i64 target ranges
 *   tgt_xyz [n_tgt][3] real dtype; mpole [n_box][Nc] dtype; potential [n_tgt] dtype, ACCUMULATED.
 * Deterministic. */
int fmm_m2p(fmm_plan plan, int64_t n_tbox, const int32_t* tbox, const int32_t* list_ptr, int64_t n_list,
            const int32_t* list, int64_t n_box, const double* box_center, const int32_t* box_level,
            const int64_t* tgt_range, int64_t n_tgt, const void* tgt_xyz, const void* mpole, void* potential,
            void* stream);

/* Compressed P2L (Sec. 3.2, eq. stored_local_coeffs, with the density): source points formed
 * directly into local expansions (the X list of an adaptive tree).  For each k < n_tbox,
 *   local[t][j] += sum over the boxes s of list[list_ptr[k] : list_ptr[k+1]] and their sources y
 *                  of w(y) G^(j)(c_t - y) h_t^|j|,   t = tbox[k], j in J
 * (the scaled derivative-form local of fmm_m2l_batched, h_t the size of t's level; fmm_l2p
 * evaluates it).  Derivatives as in fmm_m2p.  Arguments as fmm_m2p with src_range [n_box][2] i64
 * source ranges, src_xyz [n_src][3] real dtype, weight [n_src] dtype, and local [n_box][Nc]
 * dtype, ACCUMULATED; each target box at most once.  Deterministic. */
int fmm_p2l(fmm_plan plan, int64_t n_tbox, const int32_t* tbox, const int32_t* list_ptr, int64_t n_list,
            const int32_t* list, int64_t n_box, const double* box_center, const int32_t* box_level,
            const int64_t* src_range, int64_t n_src, const void* src_xyz, const void* weight, void* local,
            void* stream);

/* Near field (P2P): eq. (1) restricted to neighbour boxes.  For each k < n_tbox and every
 * target x of box tbox[k], phi(x) += sum_y G(x - y) w(y) over the sources y of the boxes
 * nbr[nbr_ptr[k] : nbr_ptr[k+1]] (terms with x == y skipped).  With the far field of the
 * interaction lists this completes the FMM potential.
 *   tbox [n_tbox] i32 box ids; nbr_ptr [n_tbox + 1] i32 CSR pointers into nbr [n_nbr] i32
 *   box ids (ranges are clamped to [0, n_nbr]; ids outside [0, n_box) are skipped)
 *   tgt_range, src_range [n_box][2] i64 point ranges of every box into tgt / src
 *   src_xyz [n_src][3] real dtype; weight [n_src] dtype; tgt_xyz [n_tgt][3] real dtype
 *   potential [n_tgt] dtype, ACCUMULATED with atomic adds.  A target box may appear several
 *   times, each with its own source list (a long list split so that its parts run in
 *   parallel); the order in which the parts are added is then not fixed, so such results can
 *   differ in the last bits from run to run.  A box listed once is added by one workgroup. */
int fmm_p2p(const fmm_desc* desc, int64_t n_tbox, const int32_t* tbox, const int32_t* nbr_ptr, int64_t n_nbr,
            const int32_t* nbr, int64_t n_box, const int64_t* tgt_range, const int64_t* src_range, int64_t n_src,
            const void* src_xyz, const void* weight, int64_t n_tgt, const void* tgt_xyz, void* potential,
            void* stream);

/* Transposes of fmm_m2m and fmm_l2l for gradients (derived from the same passages).
 * fmm_m2m_adjoint: mpole_grad read at the parents, ACCUMULATED at the children:
 *   grad beta~_child += (M^T T E)^T grad psi~_parent.
 * fmm_l2l_adjoint: local_grad read at the children, ACCUMULATED at the parents:
 *   grad theta~_parent += sum over children of (L2L)^T grad theta~_child.
 * Arguments and restrictions as for fmm_m2m / fmm_l2l. */
int fmm_m2m_adjoint(fmm_plan plan, int64_t n_parent, const int32_t* parent, const int32_t* child, int64_t n_box,
                    const double* box_center, const int32_t* box_level, void* mpole_grad, void* stream);
int fmm_l2l_adjoint(fmm_plan plan, int64_t n_parent, const int32_t* parent, const int32_t* child, int64_t n_box,
                    const double* box_center, const int32_t* box_level, void* local_grad, void* stream);

/* Prepare a batched M2L (Sec. 4.1, eq. m2l_toeplitz) over n_pair (target box, source box)
 * pairs, all [host]:
 *   tgt_box, src_box [n_pair] i32 in [0, n_box); both boxes of a pair on the same level
 *   box_ijk   [n_box][3] i32 integer grid coordinates of each box on its level
 *   box_level [n_box] i32 in [0, n_levels)
 * The translation vector of a pair is (ijk_t - ijk_s) * h_level; it must be nonzero and
 * |ijk_t - ijk_s|_inf <= 8.  Pairs are grouped by (level, offset), one FP64 derivative
 * table per group is generated on the GPU, and targets are tiled so that every output
 * coefficient is owned by one workgroup.  Allocates and synchronises (not capturable). */
int fmm_m2l_prepare(fmm_plan plan, int64_t n_pair, const int32_t* tgt_box, const int32_t* src_box,
                    int64_t n_box, const int32_t* box_ijk, const int32_t* box_level,
                    fmm_batch* batch);
void fmm_batch_destroy(fmm_batch batch);

/* Launch shape of a prepared M2L batch.  Two forms compute the same sums:
 *
 * Streaming form (FMM_M2L_FORM_STREAM): targets are tiled in groups of 16; the (tile, offset)
 * entries of all tiles are cut into `workgroups` contiguous chunks of equal length, one per
 * workgroup of `waves` wavefronts; every wavefront streams its own entries with its own staged
 * derivative table and owns all Nc output rows of its 16 targets (no barrier between entries);
 * a tile cut by a chunk boundary is summed from FP64 partials in part order.  Instantiated for
 * the Laplace-type kernels at p = 2, 4, ..., 12 (real dtypes; complex up to p = 6) and the
 * biharmonic kernel at p = 6, 8 (and 10 in FP32).
 *
 * Tiled form (FMM_M2L_FORM_TILED): a workgroup owns a tile of 16 * col_groups *
 * col_tiles_per_wave target boxes; each of its wavefronts computes rows_per_wave x
 * col_tiles_per_wave output tiles of 16 x 16 coefficients on the matrix cores, and there are
 * ceil(ceil(Nc / 16) / rows_per_wave) * col_groups * k_splits wavefronts (at most 8): with
 * k_splits > 1 the contraction index of every product is cut into k_splits ranges taken by
 * different wavefronts, whose FP64 partial sums are added in a fixed order at the end of the
 * workgroup's work (more wavefronts share one staged offset group).  Tiles are split into parts
 * (partials summed in a fixed order) so that one launch has about target_items workgroups.
 *
 * form 0 (automatic): the streaming form where it is instantiated and fits, else the tiled
 * form; rows_per_wave > 0 with form 0 selects the tiled form.  Zero fields are chosen
 * automatically (k_splits 0 means 1 when rows_per_wave is given). */
#define FMM_M2L_FORM_AUTO 0
#define FMM_M2L_FORM_TILED 1
#define FMM_M2L_FORM_STREAM 2
typedef struct {
  int32_t rows_per_wave;      /* 1..5 (tiled) */
  int32_t col_tiles_per_wave; /* 1..2 (tiled) */
  int32_t col_groups;         /* 1, 2 or 4 (tiled) */
  int32_t target_items;       /* >= 1 (tiled) */
  int32_t lds_buffers;        /* 1: stage one offset group at a time; 2: double buffered (tiled) */
  int32_t k_splits;           /* 1..4 (tiled) */
  int32_t form;               /* FMM_M2L_FORM_* */
  int32_t waves;              /* wavefronts per workgroup, 1..16 (streaming; 0 = the most that fit) */
  int32_t workgroups;         /* chunks = workgroups of one launch (streaming; 0 = compute units) */
} fmm_m2l_tuning;

/* fmm_m2l_prepare with an explicit launch shape (tuning may be NULL: automatic).  An
 * unsupported or unfitting shape returns FMM_EUNSUPPORTED. */
int fmm_m2l_prepare_ex(fmm_plan plan, int64_t n_pair, const int32_t* tgt_box, const int32_t* src_box,
                       int64_t n_box, const int32_t* box_ijk, const int32_t* box_level,
                       const fmm_m2l_tuning* tuning, fmm_batch* batch);

/* Prepare the FFT form of the batched M2L (eq. convolution_m2l): per table and per source box a
 * 3-D DFT of size (2c-1) x (2p+1) x (2p+1) (real dtypes: Hermitian half kept; complex dtypes:
 * full spectrum), per target box the sum of spectral products over its pairs and one inverse
 * DFT; the inputs are rescaled by tau = max(1, p/4) (Sec. 4.1.1) for accuracy.
 * fmm_m2l_batched then computes the same result as the matrix-core path (to the FFT's rounding
 * error, which grows with p).  FMM_EUNSUPPORTED when the working set exceeds the LDS of a
 * workgroup (high orders); same pair arguments as fmm_m2l_prepare.  Allocates the spectra of
 * all n_box boxes. */
int fmm_m2l_prepare_fft(fmm_plan plan, int64_t n_pair, const int32_t* tgt_box, const int32_t* src_box,
                        int64_t n_box, const int32_t* box_ijk, const int32_t* box_level, fmm_batch* batch);

/* fmm_m2l_batched without any allocation or library scratch, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the FP64 partial sums of tiles split over several workgroups and the per-tile part
 * counters live in one fixed device array of 16 MiB per device (held until the process ends)
 * instead of the batch's scratch.  Same arguments and results as fmm_m2l_batched (bit-identical
 * for the same batch and inputs).  A batch whose partials and counters need more than 16 MiB
 * gets FMM_EUNSUPPORTED; FFT batches get FMM_EUNSUPPORTED, adjoint batches FMM_ESTATE.  The
 * counters (and the partial slots, which the streaming form needs empty) are reset by a small
 * kernel on `stream` at every call.  All calls on one device
 * share the array: calls that can overlap in time on one device (different streams without
 * ordering) race and give wrong results. */
int fmm_m2l_batched_static(fmm_batch batch, const void* mpole, void* local, void* stream);

/* Statistics of a prepared batch, written to info[0 .. n_info-1] ([host]):
 * 0 n_pair, 1 n_tables, 2 n_tiles, 3 n_entries (tile x offset groups), 4 n_items (workgroups
 * of one launch), 5 useful pair-columns, 6 computed pair-columns (incl. padding), 7 Nc,
 * 8 rows padded to a multiple of 16, 9 scratch bytes, 10 row tiles per wavefront,
 * 11 column tiles per wavefront, 12 wavefronts per workgroup, 13 column groups,
 * 14 LDS bytes per workgroup, 15 LDS buffers, 16 K splits, 17 rows contracted on the vector
 * ALU (at most 2 rows past the last full 16-row tile), 18 1 for the streaming form, 19 its
 * workgroups per launch. */
int fmm_batch_info(fmm_batch batch, int64_t* info, int32_t n_info);

/* Batched M2L (Sec. 4.1, eq. m2l_toeplitz, in the scaled form of Sec. 4.1.1): local[t] +=
 * sum over pairs (t, s) of T(c_t - c_s) mpole[s], T[i,q] = G^(i+q) h^|i+q| for i, q in J.
 * mpole [n_box][Nc] dtype; local [n_box][Nc] dtype, ACCUMULATED.  Deterministic: every output
 * is summed in a fixed order. */
int fmm_m2l_batched(fmm_batch batch, const void* mpole, void* local, void* stream);

/* fmm_m2l_batched with an output mode (FMM_ACCUMULATE, FMM_OVERWRITE above).  FMM_OVERWRITE:
 * local[t] = M2L(mpole) for every target box t of the batch, other rows unchanged; only for a
 * streaming-form batch (FMM_EUNSUPPORTED for the tiled and FFT forms).  Same results bit for
 * bit as accumulating into zeroed rows.  Allocates nothing; capturable. */
int fmm_m2l_batched_ex(fmm_batch batch, const void* mpole, void* local, int32_t mode, void* stream);

/* Several prepared batches launched one after another on `stream` (same dtype).  batches,
 * mpole, local: [host] arrays of n pointers.  For a single persistent launch see below. */
int fmm_m2l_batched_multi(int32_t n, const fmm_batch* batches, const void* const* mpole,
                          void* const* local, void* stream);

/* Up to 32 prepared forward batches of one dtype (kernels, orders, levels and interaction lists
 * may differ; each batch at most once) enqueued by one call, each keeping its own launch shape
 * (the batching of uneven lists and mixed orders of Sec. 5's workloads, as one capturable unit):
 *   - a streaming-form batch runs its own launch, in the wavefront count and workgroup count it
 *     was prepared with (its instantiation is specific to its kernel and order);
 *   - tiled-form batches that share a tile shape (rows and column tiles per wavefront, LDS
 *     buffers) are drained by one persistent launch: work items of all of them ordered by
 *     decreasing cost and taken round-robin by a grid of at most twice the compute units, the
 *     workgroup sized for the largest wavefront count.
 * Launches are enqueued in the order of the batches' first appearance.  Allocates (not
 * capturable). */
int fmm_m2l_multi_prepare(int32_t n, const fmm_batch* batches, fmm_multi* multi);

/* Enqueue the launches: local[k] += M2L_k(mpole[k]) for every batch k.  mpole, local: [host]
 * arrays of the batches' device coefficient arrays.  Results are bit-identical to
 * fmm_m2l_batched of each batch.  Allocates nothing; capturable. */
int fmm_m2l_multi_launch(fmm_multi multi, const void* const* mpole, void* const* local, void* stream);
void fmm_m2l_multi_destroy(fmm_multi multi);

/* ---- Adjoints (real dtypes).  For a loss L with d L / d phi = potential_grad at the targets,
 * these apply the transposes of L2P, M2L and P2M in the scaled coefficient convention above,
 * so that a backward pass  L2P^T -> M2L^T -> P2M^T  gives d L / d (weights, source positions,
 * target positions) of the discrete FMM map.  Complex dtypes return FMM_EUNSUPPORTED. ---- */

/* Transpose of fmm_l2p.  local_grad[b] = M~^T (sum_x g(x) X^i / i!), X = (x - c)/h, over the
 * targets of box b ([n_box][Nc], OVERWRITTEN); if tgt_xyz_grad is not NULL, also
 * tgt_xyz_grad[x] += g(x) * grad phi(x) ([n_tgt][3], ACCUMULATED; needs `local`, the forward
 * local expansions).  g = potential_grad [n_tgt]. */
int fmm_l2p_adjoint(fmm_plan plan, int64_t n_box, const double* box_center, const int32_t* box_level,
                    const int64_t* pt_range, int64_t n_tgt, const void* tgt_xyz, const void* local,
                    const void* potential_grad, void* local_grad, void* tgt_xyz_grad, void* stream);

/* Prepare the transpose of a batched M2L over the same pairs (same arguments as
 * fmm_m2l_prepare_ex).  Because T~[i, q] = G^(i+q) is symmetric, the transpose applies the same
 * tables with target and source exchanged. */
int fmm_m2l_prepare_adjoint(fmm_plan plan, int64_t n_pair, const int32_t* tgt_box, const int32_t* src_box,
                            int64_t n_box, const int32_t* box_ijk, const int32_t* box_level,
                            const fmm_m2l_tuning* tuning, fmm_batch* batch);

/* mpole_grad[s] += sum over pairs (t, s) of T~(c_t - c_s) local_grad[t]  ([n_box][Nc],
 * ACCUMULATED).  batch must come from fmm_m2l_prepare_adjoint. */
int fmm_m2l_batched_adjoint(fmm_batch batch, const void* local_grad, void* mpole_grad, void* stream);

/* Transpose of fmm_p2m.  With g = M~ mpole_grad[b] (decompression), for every source s of box b:
 * weight_grad[s] += sum_q g_q X_s^q / q!  and  src_xyz_grad[s] += w_s d/dy_s of that sum,
 * X_s = (c - y_s)/h.  Either output may be NULL (src_xyz_grad needs `weight`).  Point ranges of
 * one call must be disjoint. */
int fmm_p2m_adjoint(fmm_plan plan, int64_t n_box, const double* box_center, const int32_t* box_level,
                    const int64_t* pt_range, int64_t n_src, const void* src_xyz, const void* weight,
                    const void* mpole_grad, void* weight_grad, void* src_xyz_grad, void* stream);

/* Direct sum eq. (1): potential[x] = sum_y G(x - y) weight[y], terms with x == y skipped.
 *   src_xyz [n_src][3], tgt_xyz [n_tgt][3] real dtype; weight [n_src] dtype;
 *   potential [n_tgt] dtype, OVERWRITTEN. */
int fmm_direct(const fmm_desc* desc, int64_t n_src, const void* src_xyz, const void* weight,
               int64_t n_tgt, const void* tgt_xyz, void* potential, void* stream);

/* ---- Two dimensions (Sec. 4.4, Laplace 2D and Biharmonic 2D): G = log r (FMM_LAPLACE2D,
 * Delta G = 0 away from 0, c = 2) and G = r^2 log r (FMM_BIHARMONIC2D, Delta^2 G = 0, c = 4),
 * FMM_F64 only, orders 0..FMM_MAX_ORDER.  desc->param is ignored.
 *
 * Expansions as in 3-D with d = 2: M(p) = {(a, b) : a + b <= p}, kept set J = {(a, b) : b < c}
 * (y is the compressed axis), |J| = 2p + 1 for c = 2 and 4p - 2 for c = 4 (p >= 3).  Stored
 * coefficient order: by b, then a (a fastest).  Multipoles and locals are stored scaled by
 * their box size h: beta~_q = beta_q / h^|q|, theta~_i = theta_i h^|i|.  Points are [n][2]
 * float64, box centres [n_box][2] float64, box sizes box_h [n_box] float64 > 0. ---- */

/* N(p) = (p+1)(p+2)/2 and |J|.  Host only. */
int fmm2d_sizes(const fmm_desc* desc, int32_t* n_full, int32_t* n_compressed);

/* J in storage order: mxy [host][Nc][2] (a, b).  Host only. */
int fmm2d_index_table(const fmm_desc* desc, int32_t* mxy);

/* Scaled derivative tables G^(a,b)(h o) h^(a+b) for a + b <= 2p, b <= 2(c-1): every derivative
 * the 2-D M2L reads.  From the paper's recurrences in x (eqs. deriv_laplace_2d,
 * deriv_biharmonic_2d, with the y terms -2 m y G(n, m-1) - m(m-1) G(n, m-2) of their general
 * form) started from closed-form low-order values, evaluated at o and scaled exactly in h.
 *   offset [n][2] f64: translation vector in units of h, nonzero;  h [n] f64 > 0
 *   out [n][2c-1][2p+1] f64, index (b, a); entries a + b > 2p zero.  OVERWRITTEN. */
int fmm2d_deriv_tables(const fmm_desc* desc, int64_t n, const double* offset, const double* h, double* out,
                       void* stream);

/* 2-D P2M: mpole[k] += M^T alpha~ for the sources of pt_range[k] about box_center[k], alpha~_q =
 * sum_y w ((c - y)/h)^q / q! (eqs. mpole, define_beta_multipole).  mpole [n_box][Nc]
 * ACCUMULATED (zero it first for the multipoles alone); ranges clamped to [0, n_src].  A box's
 * points are taken in chunks of 256 by ceil(max_src_per_box / 256) workgroups, whose compressed
 * sums are added atomically (in no fixed order when a box has more than 256 points); every
 * point is summed whatever max_src_per_box says. */
int fmm2d_p2m(const fmm_desc* desc, int64_t n_box, const double* box_center, const double* box_h,
              const int64_t* pt_range, int64_t n_src, const double* src_xy, const double* weight, double* mpole,
              int32_t max_src_per_box, void* stream);

/* 2-D M2L (eq. m2l_toeplitz for d = 2): for k < n_tbox and every pair e in
 * [pair_ptr[k], pair_ptr[k+1]): local[tbox[k]] += T~(tables[pair_tab[e]]) mpole[pair_src[e]],
 * theta~_i += sum_{q in J} T~_(i+q) beta~_q.  Tables come from fmm2d_deriv_tables at the pair's
 * offset (c_t - c_s)/h and h.  Target boxes of one call must be distinct; pair ranges are
 * clamped to [0, n_pair] and pairs with ids outside [0, n_box) or [0, n_tab) skipped.
 * Allocates nothing; capturable. */
int fmm2d_m2l(const fmm_desc* desc, int64_t n_tbox, const int32_t* tbox, const int32_t* pair_ptr, int64_t n_pair,
              const int32_t* pair_src, const int32_t* pair_tab, int64_t n_tab, const double* tables, int64_t n_box,
              const double* mpole, double* local, void* stream);

/* 2-D L2P: potential[x] += sum_{m in M(p)} (M theta~[k])_m ((x - c)/h)^m / m! for the targets of
 * pt_range[k] (eq. compressed-local-form).  Ranges of one call must be disjoint.  A box's targets
 * are taken in chunks of 256 by ceil(max_tgt_per_box / 256) workgroups (every target is
 * evaluated whatever max_tgt_per_box says). */
int fmm2d_l2p(const fmm_desc* desc, int64_t n_box, const double* box_center, const double* box_h,
              const int64_t* pt_range, int64_t n_tgt, const double* tgt_xy, const double* local, double* potential,
              int32_t max_tgt_per_box, void* stream);

/* 2-D compressed M2M (Sec. 4.3, eq. define_psi for d = 2): mpole[parent[k]] = sum over the
 * children child[k][0..3] (ids outside [0, n_box) mean "no child") of M^T T E beta~_child, the
 * child's kept coefficients embedded in M(p), translated to the parent's centre by the binomial
 * sums of eq. mpole_translated_full_coeffs and compressed; rescaled between the children's
 * and the parent's box sizes.  OVERWRITTEN at the parents (zero without children).  Exact for
 * both 2-D kernels (their PDEs are homogeneous).  A box must not be both a parent and a child
 * in one call. */
int fmm2d_m2m(const fmm_desc* desc, int64_t n_parent, const int32_t* parent, const int32_t* child, int64_t n_box,
              const double* box_center, const double* box_h, double* mpole, void* stream);

/* 2-D compressed L2L (Sec. 4.2, eq. l2l-expr for d = 2): local[child[k][o]] += the kept part of
 * the parent's decompressed local re-expanded about the child's centre.  ACCUMULATED at the
 * children.  Children of one call must be distinct and must not be parents in the call. */
int fmm2d_l2l(const fmm_desc* desc, int64_t n_parent, const int32_t* parent, const int32_t* child, int64_t n_box,
              const double* box_center, const double* box_h, double* local, void* stream);

/* 2-D direct sum (eq. (1)): potential[x] = sum_y G(x - y) w_y, x == y skipped.  OVERWRITTEN. */
int fmm2d_direct(const fmm_desc* desc, int64_t n_src, const double* src_xy, const double* weight, int64_t n_tgt,
                 const double* tgt_xy, double* potential, void* stream);

/* 2-D near field: potential[targets of tbox[k]] += direct sum over the sources of the boxes
 * nbr[nbr_ptr[k] : nbr_ptr[k+1]] (x == y skipped).  Target boxes of one call must be distinct;
 * list ranges are clamped to [0, n_nbr] and ids outside [0, n_box) skipped.  max_tgt_per_box
 * sets the launch width (ceil(max / 64) wavefronts per box); every target is computed whatever
 * its value. */
int fmm2d_p2p(const fmm_desc* desc, int64_t n_tbox, const int32_t* tbox, const int32_t* nbr_ptr, int64_t n_nbr,
              const int32_t* nbr, int64_t n_box, const int64_t* tgt_range, const int64_t* src_range, int64_t n_src,
              const double* src_xy, const double* weight, int64_t n_tgt, const double* tgt_xy, double* potential,
              int32_t max_tgt_per_box, void* stream);

/* ---- Octree and interaction lists on the device (the box hierarchy of Sec. 1 over which
 * the operators above run; the adaptive lists of the classical adaptive FMM).  Integer work:
 * every result is exact and equals what a host builder of the same definitions gives.
 *
 * Box order: level by level (level 0 = the unit cube [0,1)^3), within a level by increasing
 * Morton key of the box's integer coordinates ijk (bits interleaved, x highest within each
 * triple).  Every box's points are one contiguous range of the sorted points.
 *
 * All fmm_tree_* calls allocate and synchronise `stream` (set-up calls; not capturable). ---- */

typedef struct fmm_tree_s* fmm_tree;

#define FMM_TREE_MAX_DEPTH 20         /* key bits per axis */
#define FMM_TREE_MAX_UNIFORM_DEPTH 10 /* every box of every level is stored */

/* Build a tree over n_points points xyz [n_points][3] float64 (device), coordinates in [0, 1)
 * (values outside are clamped into the boundary boxes; a non-finite coordinate is FMM_EINVAL).
 * Each point gets the Morton key of floor(x * 2^20) (per axis, clamped to [0, 2^20 - 1]); points
 * are sorted by key, ties kept in input order (a stable sort).
 *   max_leaf == 0: uniform tree, all 8^l boxes of every level l <= depth (empty ones
 *                  included), leaves = the boxes of level `depth` (<= FMM_TREE_MAX_UNIFORM_DEPTH);
 *   max_leaf  > 0: adaptive tree: a box is refined when it holds more than max_leaf points and
 *                  its level is below depth (<= FMM_TREE_MAX_DEPTH); children holding no point
 *                  are not created; unrefined boxes are leaves. */
int fmm_tree_build(int64_t n_points, const double* xyz, int32_t max_leaf, int32_t depth, fmm_tree* tree,
                   void* stream);

/* Sizes: boxes, levels, leaves.  Any output may be NULL; all [host]. */
int fmm_tree_size(fmm_tree tree, int64_t* n_box, int32_t* n_levels, int64_t* n_leaf);

/* Copy the tree out; every output is optional (NULL skips it).
 *   perm [n_points] i64: input index of each sorted point;  points [n_points][3] f64: sorted
 *   level [n_box] i32;  ijk [n_box][3] i32;  center [n_box][3] f64 = (ijk + 1/2) 2^-level
 *   pt_range [n_box][2] i64: [begin, end) into the sorted points;  is_leaf [n_box] u8
 *   level_start [host][n_levels + 1] i64: first box of each level. */
int fmm_tree_export(fmm_tree tree, int64_t* perm, double* points, int32_t* level, int32_t* ijk, double* center,
                    int64_t* pt_range, uint8_t* is_leaf, int64_t* level_start, void* stream);

/* List-2 (well separated, Sec. 1) pairs of the target boxes on levels [level_lo, level_hi): the
 * children of the parent's neighbours (parent included) that are not adjacent to the target,
 * sorted by (target, source).  *n_pair [host] receives the count; tgt_box, src_box [n_pair] i32
 * are written when not NULL (call once with NULL to size them). */
int fmm_tree_list2(fmm_tree tree, int32_t level_lo, int32_t level_hi, int64_t* n_pair, int32_t* tgt_box,
                   int32_t* src_box, void* stream);

enum {
  FMM_LIST_NEAR = 0, /* per leaf b: existing boxes of b's level adjacent to b (b included), then
                        on every coarser level the leaves adjacent to b's ancestor there; in the
                        order (level, offset (di, dj, dk) lexicographic).  With List 2 of every
                        level each (target leaf, source leaf) pair is counted exactly once. */
  FMM_LIST_U = 1,    /* per leaf b: the leaves whose closed cube touches b's (b included); sorted */
  FMM_LIST_W = 2,    /* per leaf b with any: boxes not touching b whose parent touches b, below
                        b's colleagues (multipoles evaluated at b's targets, M2P); sorted */
  FMM_LIST_X = 3     /* per box a with any: leaves coarser than a that touch a's parent but not a
                        (their sources form a's local expansion, P2L); sorted */
};

/* Rows of the lists of `kind` in CSR form: box [n_row] i32 (the row's box), ptr [n_row + 1] i32,
 * item [n_item] i32.  U, W and X with the List-2 pairs count every leaf pair exactly once.
 * max_src > 0 (NEAR and U only): a row whose boxes hold more than max_src points in all is cut
 * into several rows of the same box: boxes above max_src points are replaced by their children
 * (depth first, octant order, down to leaves) and the boxes are packed in order into rows of at
 * most max_src points (a box above the cap alone).  *n_row, *n_item [host] receive the sizes;
 * box, ptr, item are written when not NULL.  Lists are built on first use and kept by the tree. */
int fmm_tree_lists(fmm_tree tree, int32_t kind, int64_t max_src, int64_t* n_row, int64_t* n_item, int32_t* box,
                   int32_t* ptr, int32_t* item, void* stream);

void fmm_tree_destroy(fmm_tree tree);

#ifdef __cplusplus
}
#endif

#endif /* FMM_H */
