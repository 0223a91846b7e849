// Host-side scalar work of the Zolotarev sign iteration (Sec. 5.2, Alg. 8).
//
// Coefficients of the scaled Zolotarev function hat Z_{2r+1}(x; l):
//   c_i = l^2 sn^2(u_i; l') / cn^2(u_i; l'),  u_i = i K'/(2r+1),  l' = sqrt(1 - l^2),
//   K' = K(l')                                                     (Eq:Compcis)
//   hat C = prod_j (1 + c_{2j-1}) / (1 + c_{2j})                   (Eq:hatZ)
//   a_j = - prod_k (c_{2j-1} - c_{2k}) / prod_{k!=j} (c_{2j-1} - c_{2k-1})
//                                       (Eq:ZPartialFrac2, as the partial-fraction residue)
//   l_next = hat Z(l; l)                                            (Alg. 8)
// sn, cn and K' come from the arithmetic-geometric mean with descending Landen
// transformations (Abramowitz & Stegun 16.4 and 17.6).  The AGM is started from
// b_0 = l itself, the complementary modulus of l', so the parameter 1 - l^2 never
// has to be formed.  The back-recurrence evaluates asin close to +-1 when l is tiny,
// which amplifies rounding by about 1/sqrt(l): for l >= 1e-4 (amplification <= 100)
// the x87 extended format (64-bit significand, rounding 5.4e-20) keeps the result far
// below double rounding and runs on the hardware; smaller l use IEEE quadruple
// precision (113-bit significand, software).  Both round to double once at the end.
// This file is host-only C++ (compiled by the host compiler, linked to libquadmath).
#include <quadmath.h>

#include <cmath>
#include <limits>

#include "zolo_host.h"

namespace ps {

namespace {
// the elementary functions of each working format
struct Ext {
  using T = long double;
  static T sqrt_(T x) { return sqrtl(x); }
  static T abs_(T x) { return fabsl(x); }
  static T asin_(T x) { return asinl(x); }
  static T sin_(T x) { return sinl(x); }
  static T tan_(T x) { return tanl(x); }
  static T ldexp_(T x, int e) { return ldexpl(x, e); }
  static T pi() { return 3.141592653589793238462643383279502884L; }
  static T eps() { return std::numeric_limits<long double>::epsilon(); }
};
struct Quad {
  using T = __float128;
  static T sqrt_(T x) { return sqrtq(x); }
  static T abs_(T x) { return fabsq(x); }
  static T asin_(T x) { return asinq(x); }
  static T sin_(T x) { return sinq(x); }
  static T tan_(T x) { return tanq(x); }
  static T ldexp_(T x, int e) { return ldexpq(x, e); }
  static T pi() { return M_PIq; }
  static T eps() { return FLT128_EPSILON; }
};

// (sn/cn)^2 at u_i = i K'/(2r+1), i = 1..r (the upper half follows from the reflection
// c_i c_{2r+1-i} = l^2), for modulus k' whose complementary modulus is l
template <class F>
void sc_values(double ell_d, int r, typename F::T* sc2) {
  using T = typename F::T;
  const T ell = ell_d;
  T a[64], c[64];
  T an = 1, bn = ell, cn = F::sqrt_((1 - ell) * (1 + ell));
  int N = 0;
  a[0] = an;
  c[0] = cn;
  while (F::abs_(cn) > 4 * F::eps() * an && N < 60) {
    const T a1 = (an + bn) / 2;
    const T b1 = F::sqrt_(an * bn);
    const T c1 = (an - bn) / 2;
    an = a1;
    bn = b1;
    cn = c1;
    ++N;
    a[N] = an;
    c[N] = cn;
  }
  // K' = pi / (2 a_N);  phi_N = 2^N a_N u_i = 2^(N-1) i pi / (2r+1)
  for (int i = 1; i <= r; ++i) {
    T phi = F::ldexp_(F::pi() * (T)i / (T)(2 * r + 1), N - 1);
    for (int n = N; n >= 1; --n) phi = (phi + F::asin_(c[n] / a[n] * F::sin_(phi))) / 2;
    const T t = F::tan_(phi);
    sc2[i - 1] = t * t;
  }
}

template <class F>
void coefficients(double ell_in, int r, ZoloHost* out) {
  using T = typename F::T;
  const T ell = ell_in;
  T sc2[16];
  sc_values<F>(ell_in, r, sc2);
  T c[16];
  for (int i = 0; i < r; ++i) c[i] = ell * ell * sc2[i];
  for (int i = r + 1; i <= 2 * r; ++i) c[i - 1] = ell * ell / c[2 * r - i];
  T chat = 1, zl = ell;
  for (int j = 0; j < r; ++j) {
    chat *= (1 + c[2 * j]) / (1 + c[2 * j + 1]);
    zl *= (ell * ell + c[2 * j + 1]) / (ell * ell + c[2 * j]);
  }
  zl *= chat;
  for (int j = 0; j < r; ++j) {
    T num = 1, den = 1;
    for (int k = 0; k < r; ++k) {
      num *= c[2 * j] - c[2 * k + 1];
      if (k != j) den *= c[2 * j] - c[2 * k];
    }
    out->a[j] = (double)(-num / den);
  }
  for (int i = 0; i < 2 * r; ++i) out->c[i] = (double)c[i];
  out->chat = (double)chat;
  out->ell_next = (double)zl;
}
}  // namespace

int zolotarev_host(double ell_in, int r, ZoloHost* out) {
  if (!(ell_in > 0.0) || !(ell_in < 1.0) || r < 1 || r > 8 || !out) return -1;
  if (ell_in >= 1e-4)
    coefficients<Ext>(ell_in, r, out);
  else
    coefficients<Quad>(ell_in, r, out);
  out->r = r;
  out->ell = ell_in;
  return 0;
}

// Extreme eigenvalues of the symmetric tridiagonal T = B^T B of an upper bidiagonal
// B (diagonal d[0..n-1], superdiagonal e[0..n-2]), by Sturm-sequence bisection.
namespace {
using lx = long double;

int sturm_count(const lx* td, const lx* te2, int n, lx x) {
  int cnt = 0;
  lx q = 1.0L;
  for (int i = 0; i < n; ++i) {
    q = td[i] - x - (i > 0 ? te2[i - 1] / q : 0.0L);
    if (q == 0.0L) q = -std::numeric_limits<lx>::min();
    if (q < 0) ++cnt;
  }
  return cnt;
}
}  // namespace

void bidiag_extreme_sv(const double* d, const double* e, int n, double* smax, double* smin) {
  lx td[128], te2[128];
  if (n > 128) n = 128;
  for (int i = 0; i < n; ++i) {
    const lx di = d[i], ei = (i > 0) ? e[i - 1] : 0.0;
    td[i] = di * di + ei * ei;  // (B^T B)_{ii} = d_i^2 + e_{i-1}^2
    if (i + 1 < n) {
      const lx off = (lx)d[i] * e[i];  // (B^T B)_{i,i+1} = d_i e_i
      te2[i] = off * off;
    }
  }
  lx hi = 0.0L;
  for (int i = 0; i < n; ++i) {
    const lx rad = (i > 0 ? std::sqrt(te2[i - 1]) : 0.0L) + (i + 1 < n ? std::sqrt(te2[i]) : 0.0L);
    hi = std::fmax(hi, td[i] + rad);
  }
  auto kth = [&](int k) {  // k-th smallest eigenvalue (0-based)
    lx lo = 0.0L, up = hi * (1.0L + 1e-12L) + 1e-300L;
    for (int it = 0; it < 200; ++it) {
      const lx mid = 0.5L * (lo + up);
      if (sturm_count(td, te2, n, mid) > k) up = mid; else lo = mid;
      if (up - lo <= 1e-19L * up) break;
    }
    return 0.5L * (lo + up);
  };
  *smax = (double)std::sqrt(kth(n - 1));
  *smin = (double)std::sqrt(std::fmax(kth(0), 0.0L));
}

}  // namespace ps
