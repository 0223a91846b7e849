// Factor and invert one 64 x 64 SPD diagonal block inside a workgroup: Z_kk = R^T R
// (upper R) and W_kk = R^{-1}, from a copy of the block staged in LDS.
//
// Work split: thread (bi, bj) of a 16 x 16 grid (threads 0..255, bi = tid / 16) owns the
// 4 x 4 register block at rows 4bi.., columns 4bj.. (blocks with bi <= bj carry data).
// Factorization, blocked by 4 pivots (kb = 0..15):
//   1. thread (kb, kb) factors its block D = R_d^T R_d and inverts R_d, in registers;
//   2. threads (kb, bj > kb), in the same wave, form the panel R(kb, bj) = R_d^{-T} U(kb, bj)
//      with R_d^{-1} read from the diagonal lane's registers;
//   3. every thread with kb < bi <= bj applies U(bi, bj) -= R(kb, bi)^T R(kb, bj).
// One barrier per 4 pivots.  The inverse W = R^{-1} is then assembled from the inverted
// 4 x 4 diagonal blocks by recursive doubling, W12 = -W11 (R12 W22) for neighbouring
// diagonal blocks of size 4, 8 (scalar FMAs, one thread per entry), 16 and 32 (matrix
// cores, one wave per 16 x 16 tile): eight barrier-separated phases instead of sixteen
// dependent block rows.
#pragma once

#include <hip/hip_runtime.h>

namespace ps {
namespace blk {

constexpr int kB = 64;          // block edge
constexpr int kThreads = 256;   // threads that carry data; others only join the barriers
// LDS layout in elements of T: panel [2][4][64] | wd [16][4][4] | staged block, then R,
// row-major [64][65] | W = R^{-1}, row-major [64][65] | products of the doubling [32][33]
constexpr int kPanel = 0;
constexpr int kWd = 2 * 4 * kB;
constexpr int kStage = kWd + 16 * 16;
constexpr int kLdS = kB + 1;
constexpr int kWl = kStage + kB * kLdS;
constexpr int kTmp = kWl + kB * kLdS;
constexpr int kLdT = 33;
constexpr int kLdsElems = kTmp + 32 * kLdT;

typedef double dv4 __attribute__((ext_vector_type(4)));
typedef float fv4 __attribute__((ext_vector_type(4)));
// 16 x 16 x 4 matrix-core step per element type (layouts checked on the device: lane l
// supplies A(l%16, l/16) and B(l/16, l%16); accumulator element v of lane l is
// D(4v + l/16, l%16) in FP64 and D(4(l/16) + v, l%16) in FP32)
template <class T>
struct BlkMfma;
template <>
struct BlkMfma<double> {
  using acc_t = dv4;
  __device__ static acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lk, int v) { return lk + 4 * v; }
};
template <>
struct BlkMfma<float> {
  using acc_t = fv4;
  __device__ static acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lk, int v) { return 4 * lk + v; }
};

// One wave: the 16 x 16 product A[0:16, 0:K] B[0:K, 0:16] of row-major LDS operands
// (leading dimensions lda, ldb), returned in the accumulator layout.
template <class T>
__device__ inline typename BlkMfma<T>::acc_t tile_mm(const T* A, int lda, const T* B, int ldb,
                                                     int K) {
  const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
  typename BlkMfma<T>::acc_t acc = {0, 0, 0, 0};
  for (int k = 0; k < K; k += 4)
    acc = BlkMfma<T>::step(A[li * lda + k + lk], B[(k + lk) * ldb + li], acc);
  return acc;
}

// Same with A given transposed: A(i, k) = At[k * ldat + i].
template <class T>
__device__ inline typename BlkMfma<T>::acc_t tile_mm_ta(const T* At, int ldat, const T* B, int ldb,
                                                        int K) {
  const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
  typename BlkMfma<T>::acc_t acc = {0, 0, 0, 0};
  for (int k = 0; k < K; k += 4)
    acc = BlkMfma<T>::step(At[(k + lk) * ldat + li], B[(k + lk) * ldb + li], acc);
  return acc;
}

// Store -acc of tile_mm into a row-major LDS array.
template <class T>
__device__ inline void tile_store_neg(const typename BlkMfma<T>::acc_t& acc, T* D, int ldd) {
  const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
#pragma unroll
  for (int v = 0; v < 4; ++v) D[BlkMfma<T>::row(lk, v) * ldd + li] = -acc[v];
}
template <class T>
__device__ inline void tile_store(const typename BlkMfma<T>::acc_t& acc, T* D, int ldd) {
  const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
#pragma unroll
  for (int v = 0; v < 4; ++v) D[BlkMfma<T>::row(lk, v) * ldd + li] = acc[v];
}

// 1/sqrt(x) from the hardware approximation refined by two Newton steps
// (y <- y (3 - x y^2) / 2), which brings it to full double precision; x > 0 is checked
// by the caller.
__device__ inline double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  y = y * (1.5 - 0.5 * x * y * y);
  return y;
}

// Value of x in lane `src` of the wave (src wave-uniform), through scalar registers.
__device__ inline double bcast(double x, int src) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline float bcast(float x, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), src));
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
// R^{-1} at W (leading dimension ld for both; only with `store`) and sets bit `bit` of
// *info on a non-positive pivot.  R stays in the staging area and R^{-1} in
// lds[kWl + i * kLdS + j]; after the final barrier inside, only the W stores remain, so
// the caller may reuse the staging area at once.  Every thread of the workgroup must
// call this (at least 256).
template <class T>
__device__ __forceinline__ void factor_invert_block(T* lds, T* Z, T* W, long long ld, int* info,
                                                    int bit, bool store) {
  auto panels = reinterpret_cast<T(*)[4][kB]>(lds + kPanel);
  auto wd = reinterpret_cast<T(*)[4][4]>(lds + kWd);
  T* stage = lds + kStage;
  T* Wl = lds + kWl;
  T* tmp = lds + kTmp;
  const int tid = threadIdx.x;
  const bool live = tid < kThreads;
  // block row bi lives in one wave (rows 4w..4w+3 in wave w), so a pivot block and its
  // panel are formed without a workgroup barrier between them
  const int bi = (tid >> 4) & 15, bj = tid & 15;
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
  const int wave = tid >> 6;
  for (int kb = 0; kb < kB / 4; ++kb) {
    auto panel = panels[kb & 1];
    // 1. the diagonal block, in one lane; 2. the panel blocks of block row kb, in the
    // other lanes of the same wave, which take R_d^{-1} from that lane's registers
    T wl[4][4];
    if (live && bi == kb && bj == kb) chol4(v, wl, bad);
    if (wave == (kb >> 2)) {
      const int src = (kb * 16 + kb) & 63;
      T w[4][4];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int x = p; x < 4; ++x) w[p][x] = bcast(wl[p][x], src);
      if (live && bi == kb && bj > kb) {
        T r[4][4];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) {
            T acc = T(0);
#pragma unroll
            for (int p = 0; p <= x; ++p) acc += w[p][x] * v[p][y];
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
    }
    // one barrier per step: the panel buffers alternate, and a wave can only start
    // writing the buffer of step kb + 2 after every wave passed the barrier of step
    // kb + 1, i.e. finished reading it in step kb
    __syncthreads();
    // the diagonal lane keeps R_d^{-1} for the inverse, off the critical path
    if (live && bi == kb && bj == kb) {
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) wd[kb][x][y] = wl[x][y];
    }
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
        if (store) Z[i + (long long)j * ld] = rv;
      }
  }
  // ---- W = R^{-1} by recursive doubling (R now in stage, zero below the diagonal)
  for (int e = tid; e < kB * kLdS; e += blockDim.x) Wl[e] = T(0);
  __syncthreads();
  if (tid < kThreads) {
    const int I = tid >> 4, x = (tid >> 2) & 3, y = tid & 3;
    Wl[(4 * I + x) * kLdS + 4 * I + y] = wd[I][x][y];
  }
  __syncthreads();
  // sizes 4 and 8: one thread per entry of W12 (8 pairs of 4 x 4, then 4 pairs of 8 x 8)
#pragma unroll
  for (int S = 4; S <= 8; S *= 2) {
    const int per = S * S;                 // entries per pair
    const int g = tid / per, x = (tid % per) / S, y = tid % S;
    const bool on = tid < (kB / (2 * S)) * per;
    const int L0 = 2 * S * g, R0 = L0 + S;
    if (on) {
      T acc = T(0);
#pragma unroll
      for (int k = 0; k < S; ++k) acc += stage[(L0 + x) * kLdS + R0 + k] * Wl[(R0 + k) * kLdS + R0 + y];
      tmp[g * per + x * S + y] = acc;      // T = R12 W22
    }
    __syncthreads();
    if (on) {
      T acc = T(0);
#pragma unroll
      for (int k = 0; k < S; ++k) acc += Wl[(L0 + x) * kLdS + L0 + k] * tmp[g * per + k * S + y];
      Wl[(L0 + x) * kLdS + R0 + y] = -acc;  // W12 = -W11 T
    }
    __syncthreads();
  }
  // size 16: waves 0 and 1 take one pair each
  if (wave < 2) {
    const int L0 = 32 * wave, R0 = L0 + 16;
    T* tw = tmp + wave * 16 * 17;
    tile_store(tile_mm(stage + L0 * kLdS + R0, kLdS, Wl + R0 * kLdS + R0, kLdS, 16), tw, 17);
  }
  __syncthreads();
  if (wave < 2) {
    const int L0 = 32 * wave, R0 = L0 + 16;
    const T* tw = tmp + wave * 16 * 17;
    tile_store_neg(tile_mm(Wl + L0 * kLdS + L0, kLdS, tw, 17, 16), Wl + L0 * kLdS + R0, kLdS);
  }
  __syncthreads();
  // size 32: one 16 x 16 tile of W12 (rows 0..31, columns 32..63) per wave
  const int ti = wave & 1, tj = (wave >> 1) & 1;
  if (wave < 4)
    tile_store(tile_mm(stage + 16 * ti * kLdS + 32, kLdS, Wl + 32 * kLdS + 32 + 16 * tj, kLdS, 32),
               tmp + 16 * ti * kLdT + 16 * tj, kLdT);
  __syncthreads();
  if (wave < 4)
    tile_store_neg(tile_mm(Wl + 16 * ti * kLdS, kLdS, tmp + 16 * tj, kLdT, 32),
                   Wl + 16 * ti * kLdS + 32 + 16 * tj, kLdS);
  __syncthreads();
  if (store) {
    for (int e = tid; e < kB * kB; e += blockDim.x) {
      const int i = e % kB, j = e / kB;
      W[i + (long long)j * ld] = Wl[i * kLdS + j];
    }
  }
}

}  // namespace blk
}  // namespace ps
