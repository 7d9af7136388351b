// Host-side core: error state, descriptor validation, index sets and the
// compression recursion derived from the PDE coefficients.
#include <cmath>
#include <cstring>
#include <string>

#include "common.hpp"

namespace fmm {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

const std::string& last_error() { return g_last_error; }

int fail(int status, const std::string& msg) {
  g_last_error = msg;
  return status;
}

int check_desc(const fmm_desc* d) {
  if (!d) return fail(FMM_EINVAL, "desc is NULL");
  if (d->kernel < FMM_LAPLACE || d->kernel > FMM_BIHARMONIC)
    return fail(FMM_EINVAL, "unknown kernel " + std::to_string(d->kernel));
  if (d->dtype < FMM_F64 || d->dtype > FMM_C64)
    return fail(FMM_EINVAL, "unknown dtype " + std::to_string(d->dtype));
  if (d->order < 0 || d->order > FMM_MAX_ORDER)
    return fail(FMM_EUNSUPPORTED, "order " + std::to_string(d->order) + " outside [0, " +
                                      std::to_string(FMM_MAX_ORDER) + "]");
  if (d->flags != 0) return fail(FMM_EINVAL, "flags must be 0");
  const bool cplx = dtype_complex(d->dtype);
  if (d->kernel == FMM_HELMHOLTZ && !cplx)
    return fail(FMM_EUNSUPPORTED, "Helmholtz needs a complex dtype (FMM_C128 or FMM_C64)");
  if (d->kernel != FMM_HELMHOLTZ && cplx)
    return fail(FMM_EUNSUPPORTED, "real kernels need a real dtype (FMM_F64 or FMM_F32)");
  if ((d->kernel == FMM_HELMHOLTZ || d->kernel == FMM_YUKAWA) &&
      !(d->param > 0.0 && std::isfinite(d->param)))
    return fail(FMM_EINVAL, "kernel parameter must be finite and > 0");
  return FMM_OK;
}

std::vector<MIdx> kept_set(int p, int c) {
  std::vector<MIdx> out;
  for (int z = 0; z <= p && z < c; ++z)
    for (int x = 0; x <= p - z; ++x)
      for (int y = 0; y <= p - z - x; ++y) out.push_back({x, y, z});
  return out;
}

std::vector<MIdx> full_set(int p) {
  std::vector<MIdx> out;
  for (int z = 0; z <= p; ++z)
    for (int x = 0; x <= p - z; ++x)
      for (int y = 0; y <= p - z - x; ++y) out.push_back({x, y, z});
  return out;
}

// PDE coefficients a_xi of L = sum a_xi d^xi; t = c e_z has a_t = 1 for all four kernels
// (Property 1 holds with k = z).
std::vector<RecTerm> recursion_terms(int kernel, double param) {
  struct A {
    int x, y, z;
    double a;
  };
  std::vector<A> a;
  int c = pde_order(kernel);
  if (kernel == FMM_BIHARMONIC) {
    a = {{4, 0, 0, 1.0}, {0, 4, 0, 1.0}, {2, 2, 0, 2.0}, {2, 0, 2, 2.0}, {0, 2, 2, 2.0}};
  } else {
    a = {{2, 0, 0, 1.0}, {0, 2, 0, 1.0}};
    if (kernel == FMM_HELMHOLTZ) a.push_back({0, 0, 0, param * param});
    if (kernel == FMM_YUKAWA) a.push_back({0, 0, 0, -param * param});
  }
  std::vector<RecTerm> out;
  for (const auto& t : a) out.push_back({t.x, t.y, t.z - c, -t.a, c - (t.x + t.y + t.z)});
  return out;
}

// M~ of one level: L = M~ theta for every full index m and kept index j, by the recursion with
// its coefficients scaled by h^hpow (the forward substitution of Thm. mult_decompression, levels
// of m_z ascending) run on the unit vectors of the kept set.  Row-major [nfull][nc].
std::vector<double> decompression_matrix(int p, int c, const std::vector<RecTerm>& terms, double h) {
  const int nf = (int)n_full(p);
  const int nc = (int)kept_set(p, c).size();
  auto index = [p](int x, int y, int z) {  // position in the full order (m_z, m_x, m_y)
    const int s = (int)(n_full(p) - n_full(p - z));
    return s + x * (p - z + 1) - x * (x - 1) / 2 + y;
  };
  std::vector<double> M((size_t)nf * nc, 0.0);
  for (int j = 0; j < nc; ++j) M[(size_t)j * nc + j] = 1.0;
  std::vector<double> cf(terms.size());
  for (size_t t = 0; t < terms.size(); ++t) cf[t] = terms[t].coef * std::pow(h, terms[t].hpow);
  const std::vector<MIdx> full = full_set(p);
  for (int m = nc; m < nf; ++m) {  // the eliminated indices in full order: m_z ascending
    const MIdx& q = full[m];
    double* row = &M[(size_t)m * nc];
    for (size_t t = 0; t < terms.size(); ++t) {
      const int n = index(q.x + terms[t].dx, q.y + terms[t].dy, q.z + terms[t].dz);
      const double* src = &M[(size_t)n * nc];
      for (int j = 0; j < nc; ++j) row[j] += cf[t] * src[j];
    }
  }
  return M;
}

}  // namespace fmm
