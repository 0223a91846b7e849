// Batched FP64 Cholesky factorization with the inverse factor, Z = R^T R, W = R^{-1}.
//
// Blocked right-looking algorithm over 64 x 64 diagonal blocks.  Per block step k:
//   1. one workgroup per matrix factors the diagonal block and inverts it;
//   2. the panel R(k, k+1:) = R_kk^{-T} Z(k, k+1:) (GEMM with the inverted block);
//   3. the symmetric trailing update Z(k+1:, k+1:) -= R(k, k+1:)^T R(k, k+1:).
// The full inverse factor W = R^{-1} is then assembled from the inverted diagonal
// blocks by recursive doubling, one pair of GEMM launches per level.  The batch index
// runs over independent matrices (the r shifted Gram matrices of a Zolotarev step, or
// A+B and A-B), so every launch covers all of them at once.
#include "ps_internal.h"

namespace ps {

namespace {
constexpr int NB = kNb;
constexpr int NTD = 256;
}

// Factor and invert one 64 x 64 diagonal block per workgroup.  Thread (bi, bj) of a
// 16 x 16 grid owns the 4 x 4 register block rows 4bi.., columns 4bj.. (only blocks
// with bi <= bj carry data).  Elimination is right-looking and unscaled: at pivot k
// the owners of row k publish u(k, :) to LDS (double-buffered), one barrier, then
// every thread applies u(i, j) -= u(k, i) u(k, j) / u(k, k) to its rows i > k.
// R(i, j) = u(i, j) / sqrt(u(i, i)).  The inverse W = R^{-1} runs the same rank-1
// pattern from the bottom row up: W(l, :) /= R(l, l), then W(i, :) -= R(i, l) W(l, :)
// for i < l, with column l of R and row l of W read from LDS.
__global__ __launch_bounds__(NTD) void potrf_diag_kernel(double* z, long long sz, double* w,
                                                         long long sw, int ld, int k0,
                                                         int* info) {
  __shared__ double prow[2][NB];
  __shared__ double rfull[NB][NB + 1];   // R, filled after the factorization
  __shared__ double dgs[NB];
  const int b = blockIdx.x;
  double* Z = z + b * sz + k0 + (long long)k0 * ld;
  double* W = w + b * sw + k0 + (long long)k0 * ld;
  const int tid = threadIdx.x;
  const int bi = tid & 15, bj = tid >> 4;          // block row, block column
  const int r0 = 4 * bi, c0 = 4 * bj;
  const bool active = bi <= bj;
  double v[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int i = r0 + x, j = c0 + y;
      v[x][y] = (active && i <= j) ? Z[i + (long long)j * ld] : 0.0;
    }
  // publish row 0
  if (bi == 0)
#pragma unroll
    for (int y = 0; y < 4; ++y) prow[0][c0 + y] = v[0][y];
  __syncthreads();
  bool bad = false;
  for (int k = 0; k < NB; ++k) {
    const int cur = k & 1;
    const double piv = prow[cur][k];
    if (!(piv > 0.0)) bad = true;
    const double inv = (piv > 0.0) ? 1.0 / piv : 0.0;
    if (active && r0 + 3 > k) {
      double ui[4], uj[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) ui[x] = prow[cur][r0 + x] * inv;
#pragma unroll
      for (int y = 0; y < 4; ++y) uj[y] = prow[cur][c0 + y];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
          if (r0 + x > k && r0 + x <= c0 + y) v[x][y] -= ui[x] * uj[y];
    }
    // owners of row k+1 publish it (already updated by this step)
    if (k + 1 < NB && active && (k + 1) / 4 == bi) {
      const int x = (k + 1) & 3;
#pragma unroll
      for (int xx = 0; xx < 4; ++xx)
        if (xx == x)
#pragma unroll
          for (int y = 0; y < 4; ++y) prow[cur ^ 1][c0 + y] = v[xx][y];
    }
    __syncthreads();
  }
  if (bad && tid == 0) atomicOr(info, 1 << (b < 30 ? b : 30));

  // diagonal: u(i, i) sits in the diagonal blocks
  if (bi == bj)
#pragma unroll
    for (int x = 0; x < 4; ++x) dgs[r0 + x] = sqrt(fmax(v[x][x], 0.0));
  __syncthreads();
  // R = u / sqrt(u_ii), stored to LDS (full, zero below the diagonal)
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const double d = dgs[r0 + x];
    const double sc = d > 0.0 ? 1.0 / d : 0.0;
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int i = r0 + x, j = c0 + y;
      const double rv = (active && i <= j) ? v[x][y] * sc : 0.0;
      v[x][y] = rv;
      rfull[i][j] = rv;
    }
  }
  // write R
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) Z[(r0 + x) + (long long)(c0 + y) * ld] = v[x][y];
  // W = I, then rank-1 updates from the bottom row up
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) v[x][y] = (r0 + x == c0 + y) ? 1.0 : 0.0;
  __syncthreads();
  for (int l = NB - 1; l >= 0; --l) {
    const int cur = l & 1;
    const double rll = rfull[l][l];
    const double rinv = rll != 0.0 ? 1.0 / rll : 0.0;
    // owners of row l scale it (its updates from rows > l are complete) and publish
    if (l / 4 == bi) {
      const int x = l & 3;
#pragma unroll
      for (int xx = 0; xx < 4; ++xx)
        if (xx == x)
#pragma unroll
          for (int y = 0; y < 4; ++y) {
            v[xx][y] *= rinv;
            prow[cur][c0 + y] = v[xx][y];
          }
    }
    __syncthreads();
    if (r0 < l) {
      double rc[4], wl[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) rc[x] = rfull[r0 + x][l];
#pragma unroll
      for (int y = 0; y < 4; ++y) wl[y] = prow[cur][c0 + y];
#pragma unroll
      for (int x = 0; x < 4; ++x)
        if (r0 + x < l)
#pragma unroll
          for (int y = 0; y < 4; ++y) v[x][y] -= rc[x] * wl[y];
    }
  }
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int i = r0 + x, j = c0 + y;
      W[i + (long long)j * ld] = (i <= j) ? v[x][y] : 0.0;
    }
}

void potrf_inv_f64(hipStream_t s, double* z, long long sz, double* w, long long sw,
                   double* /*tmp*/, int mp, int batch, int* info) {
  zero_lower(s, w, mp, sw, batch);  // the diagonal blocks and W12 blocks cover the rest
  if (mp % NB) throw HipError{hipErrorInvalidValue, "potrf_inv_f64: size not a multiple of 64"};
  const int nbk = mp / NB;
  // ---- blocked right-looking Cholesky; the diagonal kernel also inverts R_kk
  for (int k = 0; k < nbk; ++k) {
    const int k0 = k * NB;
    const int rest = mp - k0 - NB;
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(batch), dim3(NTD), 0, s, z, sz, w, sw, mp, k0,
                       info);
    PS_HIP(hipGetLastError());
    if (rest <= 0) break;
    double* wkk = w + k0 + (long long)k0 * mp;
    double* zr = z + k0 + (long long)(k0 + NB) * mp;
    double* zt = z + (k0 + NB) + (long long)(k0 + NB) * mp;
    // panel R(k, k+1:) = R_kk^{-T} Z(k, k+1:), in place (each tile reads its own columns)
    GemmProblem pp = gemm_problem(NB, rest, NB, wkk, mp, 1, zr, mp, 0, zr, mp, 1.0, 0.0, nullptr,
                                  0, kALower);
    pp.nb1 = batch;
    pp.sA[0] = sw;
    pp.sB[0] = sz;
    pp.sC[0] = sz;
    pp.sD[0] = sz;
    gemm_f64(s, pp);
    // trailing update Z(k+1:, k+1:) -= R(k, k+1:)^T R(k, k+1:)  (upper triangle)
    GemmProblem pt = gemm_problem(rest, rest, NB, zr, mp, 1, zr, mp, 0, zt, mp, -1.0, 1.0, zt, mp,
                                  kOutUpper);
    pt.nb1 = batch;
    pt.sA[0] = sz;
    pt.sB[0] = sz;
    pt.sC[0] = sz;
    pt.sD[0] = sz;
    gemm_f64(s, pt);
  }
  // ---- W = R^{-1} by recursive doubling over the block diagonal: at level S every
  // diagonal block of size S is already inverted, and for each pair of neighbours
  //   W12 = -W11 R12 W22.
  // T = R12 W22 is kept transposed in the (still unused) strictly lower block W21 and
  // cleared right after use: the triangle-aware GEMMs of the next levels read whole
  // diagonal tiles of W11 and W22 and rely on zeros below the diagonal.
  for (int S = NB; S < mp; S *= 2) {
    const int full = mp / (2 * S);               // pairs whose right block has size S
    const int rem = mp - full * 2 * S;           // leftover rows after the full pairs
    const long long pstride = (long long)2 * S * (mp + 1);
    GemmProblem t1[2], t2[2];
    int n1 = 0;
    auto add_pair = [&](long long off, int sr, int nb2) {
      double* w11 = w + off;
      double* w22 = w + off + (long long)S * (mp + 1);
      double* w21 = w + off + S;                  // rows right, cols left (sr x S)
      double* w12 = w + off + (long long)S * mp;  // rows left, cols right (S x sr)
      const double* r12 = z + off + (long long)S * mp;
      GemmProblem a = gemm_problem(sr, S, sr, w22, mp, 1, r12, mp, 1, w21, mp, 1.0, 0.0, nullptr,
                                   0, kALower);
      GemmProblem b = gemm_problem(S, sr, S, w11, mp, 0, w21, mp, 1, w12, mp, -1.0, 0.0, nullptr,
                                   0, kAUpper);
      for (GemmProblem* q : {&a, &b}) {
        q->nb1 = batch;
        q->sA[0] = (q == &a) ? sw : sw;
        q->sB[0] = (q == &a) ? sz : sw;
        q->sC[0] = sw;
        q->sD[0] = sw;
        q->nb2 = nb2;
        q->sA[1] = q->sB[1] = q->sC[1] = q->sD[1] = pstride;
      }
      t1[n1] = a;
      t2[n1] = b;
      ++n1;
    };
    if (full > 0) add_pair(0, S, full);
    if (rem > S) add_pair((long long)full * pstride, rem - S, 1);
    if (n1) {
      gemm_f64(s, t1, n1);
      gemm_f64(s, t2, n1);
      for (int q = 0; q < n1; ++q)
        zero_block(s, const_cast<double*>(t2[q].B), t2[q].N, t2[q].K, mp, batch, sw, t2[q].nb2,
                   pstride);
    }
  }
}

}  // namespace ps
