// Compressed 2-D M2M and L2L (Secs. 4.2-4.3 for d = 2) as products in the ring of kept
// coefficients.
//
// A compressed expansion of order p is a polynomial in (d_x, d_y) of degree <= p reduced modulo
// the PDE's symbol (d_x^2 + d_y^2)^(c/2), stored by its kept coefficients (powers of d_y below c).
// Reduction is a ring homomorphism and the symbol is homogeneous, so for both kernels:
//
//   M2M: the parent's moments are sum_y w exp((c_p - y).grad) = exp(D.grad) times the child's,
//        D = c_p - c_c; compressed, beta_p = R(D) * beta_c, where R(D) = the kept moments of D
//        (kept_moments) and * is the product of reduced polynomials truncated at degree p.  This
//        equals embedding beta_c in M(p), translating it by the binomial sums of eq.
//        mpole_translated_full_coeffs and compressing the sum (eq. define_psi), up to rounding.
//   L2L: a local evaluates as phi(x) = <theta, R(x - c)>; with x - c_p = (x - c_c) + d,
//        d = c_c - c_p, R(x - c_p) = R(d) * R(x - c_c), so theta_c is theta_p through the
//        transpose of the product by R(d): the kept part of the parent's polynomial re-expanded
//        about the child (eq. l2l-expr), exact, as the re-expansion of a polynomial is.
//
// In the stored scaled forms (beta~ = beta / h^|q|, theta~ = theta h^|i|): L2L takes d in units of
// h_p and gives the child's degree k the factor (h_c / h_p)^k; M2M takes D in units of h_c, which
// gives every term the same factor (h_c / h_p)^n of its output degree n (R is homogeneous).  The
// product of kept entries of d_y-powers b1 and b2 has power b1 + b2 <= 2c - 2; the powers
// c .. 2c - 2 are reduced by the symbol: d_y^2 = -d_x^2 (c = 2); d_y^4 = -d_x^4 - 2 d_x^2 d_y^2,
// d_y^5 = -d_x^4 d_y - 2 d_x^2 d_y^3, d_y^6 = 2 d_x^6 + 3 d_x^4 d_y^2 (c = 4).  For c = 2 this is
// the product of complex polynomials.
//
// One lane per (parent, child slot): 16 parents per wavefront; M2M adds the four lanes' sums of
// each output degree by lane exchanges.  A lane loops over its output degree and the shift's
// degree m, advancing R(D)_m by one moment_step per m, with c accumulators; the other operand
// (the child's multipole, the parent's local) sits in the lane's own LDS row, read at run-time
// indices.  Fully unrolled, the four nested loops outgrow the registers at c = 4, p >= 8.
#include "two_d.hpp"

namespace fmm2d {
namespace {

// storage position of d_x^(n - b) d_y^b (n may be a run-time value)
template <int P>
__device__ __forceinline__ int kp(int n, int b) { return kept_pos(P, n - b, b); }

// acc[.] += v * (d_y^B reduced), for one output degree (B a compile-time constant)
template <int C, int B>
__device__ __forceinline__ void add_reduced(double* acc, double v) {
  if constexpr (B < C) {
    acc[B] += v;
  } else if constexpr (C == 2) {
    acc[0] -= v;
  } else if constexpr (B == 4) {
    acc[0] -= v;
    acc[2] = fma(-2.0, v, acc[2]);
  } else if constexpr (B == 5) {
    acc[1] -= v;
    acc[3] = fma(-2.0, v, acc[3]);
  } else {
    acc[0] = fma(2.0, v, acc[0]);
    acc[2] = fma(3.0, v, acc[2]);
  }
}

// <t, d_x^(n - B) d_y^B reduced> for the kept coefficients t (LDS row) at degree n
template <int P, int C, int B>
__device__ __forceinline__ double get_reduced(const double* t, int n) {
  if constexpr (B < C) {
    return t[kp<P>(n, B)];
  } else if constexpr (C == 2) {
    return -t[kp<P>(n, 0)];
  } else if constexpr (B == 4) {
    return fma(-2.0, t[kp<P>(n, 2)], -t[kp<P>(n, 0)]);
  } else if constexpr (B == 5) {
    return fma(-2.0, t[kp<P>(n, 3)], -t[kp<P>(n, 1)]);
  } else {
    return fma(3.0, t[kp<P>(n, 2)], 2.0 * t[kp<P>(n, 0)]);
  }
}

template <int C, int B1, int B2>
__device__ __forceinline__ void m2m_terms(double* acc, const double* e, const double* f, int m, int k) {
  if constexpr (B2 < C) {
    if (B1 <= m && B2 <= k) add_reduced<C, B1 + B2>(acc, e[B1] * f[B2]);
    m2m_terms<C, B1, B2 + 1>(acc, e, f, m, k);
  } else if constexpr (B1 + 1 < C) {
    m2m_terms<C, B1 + 1, 0>(acc, e, f, m, k);
  }
}

template <int P, int C, int B1, int B2>
__device__ __forceinline__ void l2l_terms(double* acc, const double* e, const double* t, int m, int k) {
  if constexpr (B2 < C) {
    if (B1 <= m && B2 <= k) acc[B2] = fma(e[B1], get_reduced<P, C, B1 + B2>(t, k + m), acc[B2]);
    l2l_terms<P, C, B1, B2 + 1>(acc, e, t, m, k);
  } else if constexpr (B1 + 1 < C) {
    l2l_terms<P, C, B1 + 1, 0>(acc, e, t, m, k);
  }
}

template <int P, int C>
__global__ __launch_bounds__(64) void m2m2d_ring_kernel(ShiftArgs2D a) {
  constexpr int NC = n_kept(P, C);
  constexpr int S = NC | 1;  // odd row stride: the lanes' rows fall in different banks
  __shared__ double rows[64 * S];
  const int64_t g = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const int64_t k0 = g >> 2;
  const int o = (int)(g & 3);
  int par = -1, ch = -1;
  if (k0 < a.n_parent) {
    par = a.parent[k0];
    if (par < 0 || par >= a.n_box) par = -1;
    if (par >= 0) {
      ch = a.child[4 * k0 + o];
      if (ch < 0 || ch >= a.n_box) ch = -1;
    }
  }
  double* F = rows + threadIdx.x * S;  // this lane's row only: no barrier
  double X = 0.0, Y = 0.0, s = 0.0;
  if (ch >= 0) {
    const double hc = a.box_h[ch], ihc = 1.0 / hc;
    s = hc / a.box_h[par];
    X = (a.center[2 * par] - a.center[2 * ch]) * ihc;
    Y = (a.center[2 * par + 1] - a.center[2 * ch + 1]) * ihc;
    const double* src = a.coef + (int64_t)ch * NC;
    for (int j = 0; j < NC; ++j) F[j] = src[j];
  } else {
    for (int j = 0; j < NC; ++j) F[j] = 0.0;
  }
  double* dst = par >= 0 ? a.coef + (int64_t)par * NC : nullptr;
  double sn = 1.0;  // (h_c / h_p)^n
  for (int n = 0; n <= P; ++n) {
    double acc[C];
#pragma unroll
    for (int b = 0; b < C; ++b) acc[b] = 0.0;
    double e[C];  // R(D)_m, m = 0, 1, ..., n
    e[0] = 1.0;
#pragma unroll
    for (int b = 1; b < C; ++b) e[b] = 0.0;
    for (int m = 0; m <= n; ++m) {
      if (m > 0) moment_step<C>(e, X, Y, 1.0 / m);
      double f[C];
      const int k = n - m;
#pragma unroll
      for (int b = 0; b < C; ++b) {
        f[b] = 0.0;
        if (b <= k) f[b] = F[kp<P>(k, b)];
      }
      m2m_terms<C, 0, 0>(acc, e, f, m, k);
    }
#pragma unroll
    for (int b = 0; b < C; ++b) {
      acc[b] *= sn;
      acc[b] += __shfl_xor(acc[b], 1, 64);  // the four lanes of a parent are adjacent
      acc[b] += __shfl_xor(acc[b], 2, 64);
    }
    if (dst) {
#pragma unroll
      for (int b = 0; b < C; ++b)
        if (b == o && b <= n) dst[kp<P>(n, b)] = acc[b];
    }
    sn *= s;
  }
}

template <int P, int C>
__global__ __launch_bounds__(64) void l2l2d_ring_kernel(ShiftArgs2D a) {
  constexpr int NC = n_kept(P, C);
  constexpr int S = NC | 1;
  __shared__ double rows[64 * S];
  const int64_t g = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const int64_t k0 = g >> 2;
  const int o = (int)(g & 3);
  if (k0 >= a.n_parent) return;  // no exchanges below
  const int par = a.parent[k0];
  if (par < 0 || par >= a.n_box) return;
  const int ch = a.child[4 * k0 + o];
  if (ch < 0 || ch >= a.n_box) return;
  const double ihp = 1.0 / a.box_h[par], s = a.box_h[ch] * ihp;
  const double X = (a.center[2 * ch] - a.center[2 * par]) * ihp;
  const double Y = (a.center[2 * ch + 1] - a.center[2 * par + 1]) * ihp;
  double* T = rows + threadIdx.x * S;  // this lane's copy of the parent's local
  const double* src = a.coef + (int64_t)par * NC;
  for (int j = 0; j < NC; ++j) T[j] = src[j];
  double* dst = a.coef + (int64_t)ch * NC;
  double sk = 1.0;  // (h_c / h_p)^k
  for (int k = 0; k <= P; ++k) {
    double acc[C];
#pragma unroll
    for (int b = 0; b < C; ++b) acc[b] = 0.0;
    double e[C];
    e[0] = 1.0;
#pragma unroll
    for (int b = 1; b < C; ++b) e[b] = 0.0;
    for (int m = 0; m <= P - k; ++m) {
      if (m > 0) moment_step<C>(e, X, Y, 1.0 / m);
      l2l_terms<P, C, 0, 0>(acc, e, T, m, k);
    }
#pragma unroll
    for (int b = 0; b < C; ++b)
      if (b <= k) dst[kp<P>(k, b)] += acc[b] * sk;
    sk *= s;
  }
}

template <int C, int P>
bool launch_p(const ShiftArgs2D& a, bool l2l, int p, hipStream_t s) {
  if constexpr (P > 16) {
    return false;
  } else {
    if (p != P) return launch_p<C, P + 1>(a, l2l, p, s);
    const unsigned grid = (unsigned)((a.n_parent * 4 + 63) / 64);
    if (l2l)
      l2l2d_ring_kernel<P, C><<<grid, 64, 0, s>>>(a);
    else
      m2m2d_ring_kernel<P, C><<<grid, 64, 0, s>>>(a);
    return true;
  }
}

}  // namespace

bool launch_shift2d(const ShiftArgs2D& a, bool l2l, int p, int c, hipStream_t s) {
  if (a.n_parent == 0) return true;
  if (c == 2) return launch_p<2, 0>(a, l2l, p, s);
  if (c == 4) return launch_p<4, 0>(a, l2l, p, s);
  return false;
}

}  // namespace fmm2d
