// Batched FP64 Cholesky factorization with the inverse factor, Z = R^T R, W = R^{-1}.
//
// Blocked right-looking algorithm over 64 x 64 diagonal blocks.  Per block step k:
//   1. one workgroup per matrix factors the diagonal block in LDS (unscaled
//      elimination, one barrier per pivot) and inverts it (row sweep);
//   2. one grouped GEMM launch: the panel R(k, k+1:) = R_kk^{-T} Z(k, k+1:) and the
//      product U = R(0:k, k) R_kk^{-1} needed for the new block column of W;
//   3. one grouped GEMM launch: the symmetric trailing update
//      Z(k+1:, k+1:) -= R(k, k+1:)^T R(k, k+1:) and W(0:k, k) = -W(0:k, 0:k) U.
// The batch index runs over independent matrices (the r shifted Gram matrices of a
// Zolotarev step, or A+B and A-B), so every launch covers all of them at once.
#include "ps_internal.h"

namespace ps {

namespace {
constexpr int NB = kNb;
constexpr int NTD = 256;
}

__global__ __launch_bounds__(NTD) void potrf_diag_kernel(double* z, long long sz, double* w,
                                                         long long sw, int ld, int k0,
                                                         int* info) {
  __shared__ double a[NB][NB + 1];
  __shared__ double wl[NB][NB + 1];
  __shared__ double red[4][NB];
  __shared__ double dg[NB];
  const int b = blockIdx.x;
  double* Z = z + b * sz + k0 + (long long)k0 * ld;
  double* W = w + b * sw + k0 + (long long)k0 * ld;
  const int tid = threadIdx.x;

  for (int e = tid; e < NB * NB; e += NTD) {
    const int i = e % NB, j = e / NB;
    a[i][j] = (i <= j) ? Z[i + (long long)j * ld] : 0.0;
    wl[i][j] = 0.0;
  }
  __syncthreads();

  // unscaled elimination on the upper triangle: after step k row k holds u(k, :)
  bool bad = false;
  for (int k = 0; k < NB; ++k) {
    const double piv = a[k][k];
    if (!(piv > 0.0)) bad = true;
    const int n = NB - 1 - k;
    const double inv = (piv > 0.0) ? 1.0 / piv : 0.0;
    for (int e = tid; e < n * n; e += NTD) {
      const int i = k + 1 + e % n, j = k + 1 + e / n;
      if (i <= j) a[i][j] -= a[k][i] * a[k][j] * inv;
    }
    __syncthreads();
  }
  if (bad && tid == 0) atomicOr(info, 1 << (b < 30 ? b : 30));

  if (tid < NB) dg[tid] = sqrt(fmax(a[tid][tid], 0.0));
  __syncthreads();
  for (int e = tid; e < NB * NB; e += NTD) {
    const int i = e % NB, j = e / NB;
    if (i <= j) a[i][j] = (dg[i] > 0.0) ? a[i][j] / dg[i] : 0.0;  // R(i, j) = u(i, j)/sqrt(u(i, i))
  }
  __syncthreads();

  // W = R^{-1}: rows from the bottom, W(i, j) = (delta_ij - sum_{i<l<=j} R(i,l) W(l,j)) / R(i,i)
  const int jj = tid & (NB - 1), q = tid >> 6;
  for (int i = NB - 1; i >= 0; --i) {
    double part = 0.0;
    if (jj >= i)
      for (int l = i + 1 + q; l <= jj; l += 4) part += a[i][l] * wl[l][jj];
    red[q][jj] = part;
    __syncthreads();
    if (q == 0 && jj >= i) {
      const double s = red[0][jj] + red[1][jj] + red[2][jj] + red[3][jj];
      const double rii = a[i][i];
      wl[i][jj] = (rii != 0.0) ? (((i == jj) ? 1.0 : 0.0) - s) / rii : 0.0;
    }
    __syncthreads();
  }

  for (int e = tid; e < NB * NB; e += NTD) {
    const int i = e % NB, j = e / NB;
    Z[i + (long long)j * ld] = (i <= j) ? a[i][j] : 0.0;
    W[i + (long long)j * ld] = (i <= j) ? wl[i][j] : 0.0;
  }
}

void potrf_inv_f64(hipStream_t s, double* z, long long sz, double* w, long long sw,
                   double* tmp, int mp, int batch, int* info) {
  if (mp % NB) throw HipError{hipErrorInvalidValue, "potrf_inv_f64: size not a multiple of 64"};
  for (int b = 0; b < batch; ++b) fill_zero(s, w + b * sw, (size_t)mp * mp);
  const long long st = (long long)mp * NB;
  const int nbk = mp / NB;
  for (int k = 0; k < nbk; ++k) {
    const int k0 = k * NB;
    const int rest = mp - k0 - NB;
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(batch), dim3(NTD), 0, s, z, sz, w, sw, mp, k0,
                       info);
    PS_HIP(hipGetLastError());

    GemmProblem ga[2];
    int na = 0;
    double* wkk = w + k0 + (long long)k0 * mp;
    if (rest > 0) {
      double* zr = z + k0 + (long long)(k0 + NB) * mp;
      GemmProblem p = gemm_problem(NB, rest, NB, wkk, mp, 1, zr, mp, 0, zr, mp, 1.0, 0.0,
                                   nullptr, 0, kALower);
      p.nb1 = batch;
      p.sA[0] = sw;
      p.sB[0] = sz;
      p.sC[0] = sz;
      p.sD[0] = sz;
      ga[na++] = p;
    }
    if (k0 > 0) {
      GemmProblem p = gemm_problem(k0, NB, NB, z + (long long)k0 * mp, mp, 0, wkk, mp, 0, tmp,
                                   mp, 1.0, 0.0, nullptr, 0, kBUpper);
      p.nb1 = batch;
      p.sA[0] = sz;
      p.sB[0] = sw;
      p.sC[0] = st;
      p.sD[0] = st;
      ga[na++] = p;
    }
    if (na) gemm_f64(s, ga, na);

    GemmProblem gb[2];
    int nbp = 0;
    if (rest > 0) {
      double* zr = z + k0 + (long long)(k0 + NB) * mp;
      double* zt = z + (k0 + NB) + (long long)(k0 + NB) * mp;
      GemmProblem p = gemm_problem(rest, rest, NB, zr, mp, 1, zr, mp, 0, zt, mp, -1.0, 1.0, zt,
                                   mp, kOutUpper);
      p.nb1 = batch;
      p.sA[0] = sz;
      p.sB[0] = sz;
      p.sC[0] = sz;
      p.sD[0] = sz;
      gb[nbp++] = p;
    }
    if (k0 > 0) {
      GemmProblem p = gemm_problem(k0, NB, k0, w, mp, 0, tmp, mp, 0, w + (long long)k0 * mp, mp,
                                   -1.0, 0.0, nullptr, 0, kAUpper);
      p.nb1 = batch;
      p.sA[0] = sw;
      p.sB[0] = st;
      p.sC[0] = sw;
      p.sD[0] = sw;
      gb[nbp++] = p;
    }
    if (nbp) gemm_f64(s, gb, nbp);
  }
}

}  // namespace ps
