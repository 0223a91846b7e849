// Host-side scalar routines of the Zolotarev iteration (no device code).
#pragma once

namespace ps {

struct ZoloHost {
  int r;
  double ell;
  double c[16];    // c_1..c_2r
  double a[8];     // a_1..a_r
  double chat;
  double ell_next;
};

// Coefficients of hat Z_{2r+1}(x; ell), 0 < ell < 1, 1 <= r <= 8.  Returns 0 or -1.
int zolotarev_host(double ell, int r, ZoloHost* out);

// Largest and smallest singular value of the upper bidiagonal matrix with diagonal
// d[0..n-1] and superdiagonal e[0..n-2].
void bidiag_extreme_sv(const double* d, const double* e, int n, double* smax, double* smin);

}  // namespace ps
