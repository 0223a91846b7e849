// Factor and invert one 64 x 64 SPD diagonal block inside a workgroup: Z_kk = R^T R
// (upper R) and W_kk = R^{-1}, from a copy of the block staged in LDS.
//
// Work split: thread (bi, bj) of a 16 x 16 grid (threads 0..255) owns the 4 x 4
// register block at rows 4bi.., columns 4bj.. (blocks with bi <= bj carry data).
// Factorization, blocked by 4 pivots (kb = 0..15):
//   1. thread (kb, kb) factors its block D = R_d^T R_d and inverts R_d, in registers;
//   2. threads (kb, bj > kb) form the panel R(kb, bj) = R_d^{-T} U(kb, bj);
//   3. every thread with kb < bi <= bj applies U(bi, bj) -= R(kb, bi)^T R(kb, bj).
// The inverse W = R^{-1} is built bottom-up by block rows: W(lb, :) = R_d(lb)^{-1} B(lb, :)
// followed by B(bi, :) -= R(bi, lb) W(lb, :) for bi < lb, with B initialized to I.
// Two barriers per 4 pivots in the factorization, one per 4 rows in the inverse.
#pragma once

#include <hip/hip_runtime.h>

namespace ps {
namespace blk {

constexpr int kB = 64;          // block edge
constexpr int kThreads = 256;   // threads that carry data; others only join the barriers
// LDS layout in elements of T: panel [4][64] (also the first W row buffer) | wd [16][4][4]
// | staged block / R [64][65] | second W row buffer [4][64]
constexpr int kPanel = 0;
constexpr int kWd = 4 * kB;
constexpr int kStage = kWd + 16 * 16;
constexpr int kLdS = kB + 1;
constexpr int kWrow1 = kStage + kB * kLdS;
constexpr int kLdsElems = kWrow1 + 4 * kB;

// 1/sqrt(x) from the hardware approximation refined by two Newton steps
// (y <- y (3 - x y^2) / 2), which brings it to full double precision; x > 0 is checked
// by the caller.
__device__ inline double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  y = y * (1.5 - 0.5 * x * y * y);
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

// The block's upper triangle is staged in lds[kStage + i * kLdS + j] (entry (i, j),
// i <= j) and a barrier has passed since.  Stores R (zero below the diagonal) at Z and
// R^{-1} at W (leading dimension ld for both) and sets bit `bit` of *info on a
// non-positive pivot.  Every thread of the workgroup must call this.
template <class T>
__device__ void factor_invert_block(T* lds, T* Z, T* W, long long ld, int* info, int bit) {
  auto panel = reinterpret_cast<T(*)[kB]>(lds + kPanel);
  auto wd = reinterpret_cast<T(*)[4][4]>(lds + kWd);
  T* stage = lds + kStage;
  T* wrow[2] = {lds + kPanel, lds + kWrow1};   // [4][kB] each
  const int tid = threadIdx.x;
  const bool live = tid < kThreads;
  const int bi = tid & 15, bj = (tid >> 4) & 15;
  const int r0 = 4 * bi, c0 = 4 * bj;
  const bool active = live && bi <= bj;
  T v[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int i = r0 + x, j = c0 + y;
      v[x][y] = (active && i <= j) ? stage[i * kLdS + j] : T(0);
    }
  bool bad = false;
  for (int kb = 0; kb < kB / 4; ++kb) {
    // 1. diagonal block
    if (live && bi == kb && bj == kb) {
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
    if (live && bi == kb && bj == kb) {
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) panel[x][c0 + y] = v[x][y];
    }
    if (live && bi == kb && bj > kb) {
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
  if (bad) atomicOr(info, 1 << bit);
  // R out (zero below the diagonal) and into the staging area, which nobody reads any
  // more (its only reads were the initial loads above, before the barriers)
  if (live) {
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) {
        const int i = r0 + x, j = c0 + y;
        const T rv = (active && i <= j) ? v[x][y] : T(0);
        v[x][y] = rv;
        stage[i * kLdS + j] = rv;
        Z[i + (long long)j * ld] = rv;
      }
  }
  // W: B = I, bottom-up block rows
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) v[x][y] = (r0 + x == c0 + y) ? T(1) : T(0);
  __syncthreads();
  for (int lb = kB / 4 - 1; lb >= 0; --lb) {
    T* wr_buf = wrow[lb & 1];
    if (live && bi == lb && bj >= lb) {
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
          wr_buf[x * kB + c0 + y] = t[x][y];
        }
    }
    __syncthreads();
    if (live && bi < lb && bj >= lb) {
      T rc[4][4], wr[4][4];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int p = 0; p < 4; ++p) rc[x][p] = stage[(r0 + x) * kLdS + 4 * lb + p];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int y = 0; y < 4; ++y) wr[p][y] = wr_buf[p * kB + c0 + y];
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
  if (live) {
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) {
        const int i = r0 + x, j = c0 + y;
        W[i + (long long)j * ld] = (active && i <= j) ? v[x][y] : T(0);
      }
  }
}

}  // namespace blk
}  // namespace ps
