// Batched Cholesky factorization with the inverse factor, Z = R^T R, W = R^{-1}, in FP64
// or FP32 (one template).
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
// 16 x 16 grid owns the 4 x 4 register block rows 4bi.., columns 4bj.. (blocks with
// bi <= bj carry data).  Factorization, blocked by 4 pivots (kb = 0..15):
//   1. thread (kb, kb) factors its block D = R_d^T R_d and inverts R_d, in registers;
//   2. threads (kb, bj > kb) form the panel R(kb, bj) = R_d^{-T} U(kb, bj);
//   3. every thread with kb < bi <= bj applies U(bi, bj) -= R(kb, bi)^T R(kb, bj).
// The inverse W = R^{-1} is built bottom-up by block rows: W(lb, :) = R_d(lb)^{-1} B(lb, :)
// followed by B(bi, :) -= R(bi, lb) W(lb, :) for bi < lb, with B initialized to I.
// Two barriers per 4 pivots in the factorization, one per 4 rows in the inverse.
namespace {
// 1/sqrt(x) and 1/x from the hardware approximations, each refined by two Newton
// steps (y <- y (3 - x y^2)/2 and y <- y (2 - x y)), which brings the approximations
// to full double precision; x > 0 is checked by the caller.
__device__ inline double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  y = y * (1.5 - 0.5 * x * y * y);
  return y;
}
__device__ inline double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(y, fma(-x, y, 1.0), y);
  y = fma(y, fma(-x, y, 1.0), y);
  return y;
}

template <class T>
__device__ inline void chol4(T d[4][4], T w[4][4], bool& bad) {
  // upper Cholesky of the 4 x 4 block d (upper triangle used) and w = R_d^{-1}
  T rinv[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const T piv = d[p][p];
    if (!(piv > T(0))) bad = true;
    const T ri = piv > T(0) ? (T)rsqrt_nr((double)piv) : T(0);
    rinv[p] = ri;
    d[p][p] = piv * ri;
#pragma unroll
    for (int y = p + 1; y < 4; ++y) d[p][y] *= ri;
#pragma unroll
    for (int x = p + 1; x < 4; ++x)
#pragma unroll
      for (int y = x; y < 4; ++y) d[x][y] -= d[p][x] * d[p][y];
  }
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < x; ++y) d[x][y] = T(0);
  // w = R_d^{-1}: columns by back substitution with the reciprocal diagonal
#pragma unroll
  for (int y = 0; y < 4; ++y) {
#pragma unroll
    for (int x = 3; x >= 0; --x) {
      T acc = (x == y) ? T(1) : T(0);
#pragma unroll
      for (int q = x + 1; q < 4; ++q) acc -= d[x][q] * w[q][y];
      w[x][y] = (x <= y) ? acc * rinv[x] : T(0);
    }
  }
}
}  // namespace

template <class T>
__global__ __launch_bounds__(NTD) void potrf_diag_kernel(T* z, long long sz, T* w, long long sw,
                                                         int ld, int k0, int* info) {
  __shared__ T panel[4][NB];        // R(kb, :) of the current block row
  __shared__ T wd[NB / 4][4][4];    // R_d^{-1} of every diagonal block
  __shared__ T rfull[NB][NB + 1];   // R after the factorization
  __shared__ T wrow[2][4][NB];      // published block row of W
  const int b = blockIdx.x;
  T* Z = z + b * sz + k0 + (long long)k0 * ld;
  T* W = w + b * sw + k0 + (long long)k0 * ld;
  const int tid = threadIdx.x;
  const int bi = tid & 15, bj = tid >> 4;
  const int r0 = 4 * bi, c0 = 4 * bj;
  const bool active = bi <= bj;
  T v[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int i = r0 + x, j = c0 + y;
      v[x][y] = (active && i <= j) ? Z[i + (long long)j * ld] : T(0);
    }
  bool bad = false;
  for (int kb = 0; kb < NB / 4; ++kb) {
    // 1. diagonal block
    if (bi == kb && bj == kb) {
      T wl[4][4];
      chol4(v, wl, bad);
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) wd[kb][x][y] = wl[x][y];
    }
    __syncthreads();
    // 2. panel blocks of block row kb (the panel buffer is free: every reader of the
    // previous one has passed the barrier above)
    if (bi == kb && bj == kb) {
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) panel[x][c0 + y] = v[x][y];
    }
    if (bi == kb && bj > kb) {
      T r[4][4];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
          T acc = T(0);
#pragma unroll
          for (int p = 0; p <= x; ++p) acc += wd[kb][p][x] * v[p][y];
          r[x][y] = acc;
        }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
          v[x][y] = r[x][y];
          panel[x][c0 + y] = r[x][y];
        }
    }
    __syncthreads();
    // 3. trailing update
    if (active && bi > kb) {
      T ra[4][4], rb[4][4];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
          ra[p][y] = panel[p][r0 + y];
          rb[p][y] = panel[p][c0 + y];
        }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
          T acc = v[x][y];
#pragma unroll
          for (int p = 0; p < 4; ++p) acc -= ra[p][x] * rb[p][y];
          v[x][y] = acc;
        }
    }
    // the next step's diagonal thread works in its own registers and on wd[kb + 1];
    // the panel buffer is rewritten only after the next step's first barrier
  }
  if (bad) atomicOr(info, 1 << (b < 30 ? b : 30));
  // R out (zero below the diagonal) and into LDS
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int i = r0 + x, j = c0 + y;
      const T rv = (active && i <= j) ? v[x][y] : T(0);
      v[x][y] = rv;
      rfull[i][j] = rv;
      Z[i + (long long)j * ld] = rv;
    }
  // W: B = I, bottom-up block rows
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) v[x][y] = (r0 + x == c0 + y) ? T(1) : T(0);
  __syncthreads();
  for (int lb = NB / 4 - 1; lb >= 0; --lb) {
    const int buf = lb & 1;
    if (bi == lb && bj >= lb) {
      T t[4][4];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
          T acc = T(0);
#pragma unroll
          for (int p = x; p < 4; ++p) acc += wd[lb][x][p] * v[p][y];
          t[x][y] = acc;
        }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
          v[x][y] = t[x][y];
          wrow[buf][x][c0 + y] = t[x][y];
        }
    }
    __syncthreads();
    if (bi < lb && bj >= lb) {
      T rc[4][4], wr[4][4];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int p = 0; p < 4; ++p) rc[x][p] = rfull[r0 + x][4 * lb + p];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int y = 0; y < 4; ++y) wr[p][y] = wrow[buf][p][c0 + y];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
          T acc = v[x][y];
#pragma unroll
          for (int p = 0; p < 4; ++p) acc -= rc[x][p] * wr[p][y];
          v[x][y] = acc;
        }
    }
  }
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int i = r0 + x, j = c0 + y;
      W[i + (long long)j * ld] = (active && i <= j) ? v[x][y] : T(0);
    }
}

inline void gemm_t(hipStream_t s, const GemmProblem* p, int n) { gemm_f64(s, p, n); }
inline void gemm_t(hipStream_t s, const GemmProblemF* p, int n) { gemm_f32(s, p, n); }

template <class T>
void potrf_inv_t(hipStream_t s, T* z, long long sz, T* w, long long sw, int mp, int batch,
                 int* info, bool inverse = true) {
  zero_lower(s, w, mp, sw, batch);  // the diagonal blocks and W12 blocks cover the rest
  if (mp % NB) throw HipError{hipErrorInvalidValue, "potrf_inv_f64: size not a multiple of 64"};
  const int nbk = mp / NB;
  // ---- blocked right-looking Cholesky; the diagonal kernel also inverts R_kk
  for (int k = 0; k < nbk; ++k) {
    const int k0 = k * NB;
    const int rest = mp - k0 - NB;
    hipLaunchKernelGGL(potrf_diag_kernel<T>, dim3(batch), dim3(NTD), 0, s, z, sz, w, sw, mp, k0,
                       info);
    PS_HIP(hipGetLastError());
    if (rest <= 0) break;
    T* wkk = w + k0 + (long long)k0 * mp;
    T* zr = z + k0 + (long long)(k0 + NB) * mp;
    T* zt = z + (k0 + NB) + (long long)(k0 + NB) * mp;
    // panel R(k, k+1:) = R_kk^{-T} Z(k, k+1:), in place (each tile reads its own columns)
    GemmProblemT<T> pp = gemm_problem(NB, rest, NB, wkk, mp, 1, zr, mp, 0, zr, mp, 1.0, 0.0, nullptr,
                                  0, kALower);
    pp.nb1 = batch;
    pp.sA[0] = sw;
    pp.sB[0] = sz;
    pp.sC[0] = sz;
    pp.sD[0] = sz;
    gemm_t(s, &pp, 1);
    // trailing update Z(k+1:, k+1:) -= R(k, k+1:)^T R(k, k+1:)  (upper triangle)
    GemmProblemT<T> pt = gemm_problem(rest, rest, NB, zr, mp, 1, zr, mp, 0, zt, mp, -1.0, 1.0, zt, mp,
                                  kOutUpper);
    pt.nb1 = batch;
    pt.sA[0] = sz;
    pt.sB[0] = sz;
    pt.sC[0] = sz;
    pt.sD[0] = sz;
    gemm_t(s, &pt, 1);
  }
  if (!inverse) return;   // W then holds only the inverted diagonal blocks
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
    GemmProblemT<T> t1[2], t2[2];
    int n1 = 0;
    auto add_pair = [&](long long off, int sr, int nb2) {
      T* w11 = w + off;
      T* w22 = w + off + (long long)S * (mp + 1);
      T* w21 = w + off + S;                  // rows right, cols left (sr x S)
      T* w12 = w + off + (long long)S * mp;  // rows left, cols right (S x sr)
      const T* r12 = z + off + (long long)S * mp;
      GemmProblemT<T> a = gemm_problem(sr, S, sr, w22, mp, 1, r12, mp, 1, w21, mp, 1.0, 0.0, nullptr,
                                   0, kALower);
      GemmProblemT<T> b = gemm_problem(S, sr, S, w11, mp, 0, w21, mp, 1, w12, mp, -1.0, 0.0, nullptr,
                                   0, kAUpper);
      for (GemmProblemT<T>* q : {&a, &b}) {
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
      gemm_t(s, t1, n1);
      gemm_t(s, t2, n1);
      for (int q = 0; q < n1; ++q)
        zero_block(s, const_cast<T*>(t2[q].B), t2[q].N, t2[q].K, mp, batch, sw, t2[q].nb2,
                   pstride);
    }
  }
}

void potrf_inv_f64(hipStream_t s, double* z, long long sz, double* w, long long sw,
                   double* /*tmp*/, int mp, int batch, int* info, bool inverse) {
  potrf_inv_t(s, z, sz, w, sw, mp, batch, info, inverse);
}

void potrf_inv_f32(hipStream_t s, float* z, long long sz, float* w, long long sw, int mp,
                   int batch, int* info) {
  potrf_inv_t(s, z, sz, w, sw, mp, batch, info);
}

}  // namespace ps
