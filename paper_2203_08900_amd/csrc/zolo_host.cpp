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
// which amplifies rounding by about 1/sqrt(l), so the whole computation runs in
// IEEE quadruple precision (113-bit significand) and is rounded to double once.
// This file is host-only C++ (compiled by the host compiler, linked to libquadmath).
#include <quadmath.h>

#include <cmath>
#include <limits>

#include "zolo_host.h"

namespace ps {

namespace {
using ld = __float128;
const ld kPi = M_PIq;

// tan(phi_0) for u = i K'/(2r+1) with modulus k' whose complementary modulus is l
void sc_values(ld ell, int r, ld* sc2 /* 2r values: (sn/cn)^2 at u_1..u_2r */) {
  ld a[64], c[64];
  ld an = 1, bn = ell, cn = sqrtq((1 - ell) * (1 + ell));
  int N = 0;
  a[0] = an;
  c[0] = cn;
  while (fabsq(cn) > 4 * FLT128_EPSILON * an && N < 60) {
    const ld a1 = (an + bn) / 2;
    const ld b1 = sqrtq(an * bn);
    const ld c1 = (an - bn) / 2;
    an = a1;
    bn = b1;
    cn = c1;
    ++N;
    a[N] = an;
    c[N] = cn;
  }
  // K' = pi / (2 a_N);  phi_N = 2^N a_N u_i = 2^(N-1) i pi / (2r+1)
  for (int i = 1; i <= 2 * r; ++i) {
    ld phi = ldexpq(kPi * (ld)i / (ld)(2 * r + 1), N - 1);
    for (int n = N; n >= 1; --n) phi = (phi + asinq(c[n] / a[n] * sinq(phi))) / 2;
    const ld t = tanq(phi);
    sc2[i - 1] = t * t;
  }
}
}  // namespace

int zolotarev_host(double ell_in, int r, ZoloHost* out) {
  if (!(ell_in > 0.0) || !(ell_in < 1.0) || r < 1 || r > 8 || !out) return -1;
  const ld ell = ell_in;
  ld sc2[16];
  sc_values(ell, r, sc2);
  ld c[16];
  for (int i = 0; i < 2 * r; ++i) c[i] = ell * ell * sc2[i];
  // the reflection c_i c_{2r+1-i} = l^2 holds exactly; use it for the upper half,
  // where cn is small and tan(phi_0) is least accurate
  for (int i = r + 1; i <= 2 * r; ++i) c[i - 1] = ell * ell / c[2 * r - i];
  ld chat = 1, zl = ell;
  for (int j = 0; j < r; ++j) {
    chat *= (1 + c[2 * j]) / (1 + c[2 * j + 1]);
    zl *= (ell * ell + c[2 * j + 1]) / (ell * ell + c[2 * j]);
  }
  zl *= chat;
  for (int j = 0; j < r; ++j) {
    ld num = 1, den = 1;
    for (int k = 0; k < r; ++k) {
      num *= c[2 * j] - c[2 * k + 1];
      if (k != j) den *= c[2 * j] - c[2 * k];
    }
    out->a[j] = (double)(-num / den);
  }
  out->r = r;
  out->ell = ell_in;
  for (int i = 0; i < 2 * r; ++i) out->c[i] = (double)c[i];
  out->chat = (double)chat;
  out->ell_next = (double)zl;
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
