// Shared host-side helpers: status handling, index sets and the kernel/PDE
// descriptors used by the plan and by every launch wrapper.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/fmm.h"

namespace fmm {

void set_error(const std::string& msg);
const std::string& last_error();
int fail(int status, const std::string& msg);

#define FMM_HIP_CHECK(call)                                                              \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return ::fmm::fail(FMM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));   \
  } while (0)

#define FMM_REQUIRE(cond, status, msg)                     \
  do {                                                     \
    if (!(cond)) return ::fmm::fail((status), (msg));      \
  } while (0)

struct MIdx {
  int x, y, z;
};

inline int pde_order(int kernel) { return kernel == FMM_BIHARMONIC ? 4 : 2; }
inline bool dtype_complex(int dt) { return dt == FMM_C128 || dt == FMM_C64; }
inline bool dtype_single(int dt) { return dt == FMM_F32 || dt == FMM_C64; }
inline size_t real_size(int dt) { return dtype_single(dt) ? 4 : 8; }
inline size_t value_size(int dt) { return real_size(dt) * (dtype_complex(dt) ? 2 : 1); }
inline int64_t n_full(int p) { return p < 0 ? 0 : (int64_t)(p + 1) * (p + 2) * (p + 3) / 6; }

// Validates a descriptor; returns FMM_OK or a status (error message set).
int check_desc(const fmm_desc* d);

// Kept multi-indices J = {|m| <= p, m_z < c} in storage order: (m_z, m_x, m_y) lexicographic.
std::vector<MIdx> kept_set(int p, int c);

// Full set M(p) in the library's internal order: (m_z, m_x, m_y) lexicographic.
std::vector<MIdx> full_set(int p);

// One term of the compression recursion (Sec. 3.1 / Thm. mult_decompression): for an index
// m with m_z >= c,  D_m = sum_terms coef * D_{m - c e_z + xi},  coef = -a_xi / a_{c e_z};
// `lev_dep` marks the term whose coefficient scales with the level (h^(c - |xi|) != 1).
struct RecTerm {
  int dx, dy, dz;  // xi - c e_z
  double coef;     // unscaled -a_xi / a_t
  int hpow;        // c - |xi|: the scaled coefficient is coef * h^hpow
};
std::vector<RecTerm> recursion_terms(int kernel, double param);

// The scaled decompression matrix M~ of one tree level (box size h): [nfull][nc] row-major.
std::vector<double> decompression_matrix(int p, int c, const std::vector<RecTerm>& terms, double h);

}  // namespace fmm
