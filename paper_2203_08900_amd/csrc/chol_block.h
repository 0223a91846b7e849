// Factor and invert one 64 x 64 SPD diagonal block inside a workgroup: Z_kk = R^T R
// (upper R) and W_kk = R^{-1}, from a copy of the block staged in LDS.
//
// The factorization is a chain of 64 dependent pivots, so its time is the length of
// that chain times the cost of one link.  Wave 0 runs the chain alone, one block row of
// four pivots per step, one lane per column: it applies the previous step's rank-4
// update to its block row, gathers the 4 x 4 diagonal block through LDS, factors it in
// every lane at once (no broadcast of the result), and forms its own column of the
// panel R(k, k+1:) by forward substitution.  The other three waves hold the trailing
// matrix as 16 x 16 matrix-core tiles in registers and apply each panel to them (one
// rank-4 step per tile) as soon as it is written, handing a block row to wave 0 one step
// before it needs it.  One barrier per step.
//
// W = R^{-1} follows by recursive doubling, W12 = -W11 (R12 W22).  The inverses of the
// 16 x 16 diagonal blocks (levels 4, 8 and 16, one wave each, no workgroup barrier) and
// the first pair of level 32 run in the trailing waves' idle time as soon as their rows
// of R are final; after the last step only the last 16 x 16 block, the second pair of
// level 32 and level 64 remain.
#pragma once

#include <hip/hip_runtime.h>

namespace ps {
namespace blk {

constexpr int kB = 64;          // block edge
constexpr int kThreads = 256;   // threads that carry data; others only join the barriers
// LDS layout in elements of T: small scratch [512] (the gathered diagonal block, the
// reciprocal pivots, per-wave products of the 8-level) | [256] unused | staged block,
// then R, row-major [64][65] | W = R^{-1}, row-major [64][65] | products of the
// doubling [32][33]
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

// The same with the depth K fixed at compile time (the operand loads are issued ahead of
// the matrix-core steps).
template <class T, int K>
__device__ inline typename BlkMfma<T>::acc_t tile_mm_k(const T* A, int lda, const T* B, int ldb) {
  const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
  T a[K / 4], b[K / 4];
#pragma unroll
  for (int s = 0; s < K / 4; ++s) {
    a[s] = A[li * lda + 4 * s + lk];
    b[s] = B[(4 * s + lk) * ldb + li];
  }
  typename BlkMfma<T>::acc_t acc = {0, 0, 0, 0};
#pragma unroll
  for (int s = 0; s < K / 4; ++s) acc = BlkMfma<T>::step(a[s], b[s], acc);
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

// tile_mm_ta with the depth K fixed at compile time (operand loads ahead of the steps).
template <class T, int K>
__device__ inline typename BlkMfma<T>::acc_t tile_mm_ta_k(const T* At, int ldat, const T* B, int ldb) {
  const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
  T a[K / 4], b[K / 4];
#pragma unroll
  for (int s = 0; s < K / 4; ++s) {
    a[s] = At[(4 * s + lk) * ldat + li];
    b[s] = B[(4 * s + lk) * ldb + li];
  }
  typename BlkMfma<T>::acc_t acc = {0, 0, 0, 0};
#pragma unroll
  for (int s = 0; s < K / 4; ++s) acc = BlkMfma<T>::step(a[s], b[s], acc);
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

// 1/sqrt(x) to full double precision: the hardware estimate (about 24 correct bits) and
// one third-order correction y (1 + e/2 + 3e^2/8) with e = 1 - x y^2, whose error is
// O(e^3).  x > 0 is checked by the caller.
__device__ inline double rsqrt_full(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double t = x * y;
  const double e = __builtin_fma(-t, y, 1.0);
  const double g = __builtin_fma(e, 0.375, 0.5);
  return __builtin_fma(y * e, g, y);
}

// Order this wave's LDS writes before its later LDS reads (the lanes of a wave run in
// lockstep, so no workgroup barrier is needed for data the same wave wrote).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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

// One part of the inverse of the 16 x 16 diagonal block at offset o, W_oo = R_oo^{-1}
// (row-major R in S, W in Wl, reciprocal pivots in rinv), run by one whole wave.  Parts
// in order, each after the previous one is visible: 0, the four 4 x 4 diagonal inverses
// (one column per lane) and zeros in the 4 x 4 blocks below the diagonal; 1, level 8 (one
// entry of each 4 x 4 W12 per lane); 2 and 3, level 16 (T = R12 W22 into the scratch tw
// of 64 elements, then W12 = -W11 T).
template <class T>
__device__ inline void inv16_part(const T* S, T* Wl, const T* rinv, T* tw, int o, int part) {
  const int lane = threadIdx.x & 63;
  if (part == 0) {
    if (lane < 16) {
      const int c = o + 4 * (lane >> 2), y = lane & 3;
      T ri[4], r[4][4], wv[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        ri[x] = rinv[c + x];
#pragma unroll
        for (int z = x + 1; z < 4; ++z) r[x][z] = S[(c + x) * kLdS + c + z];
      }
      wv[3] = y == 3 ? ri[3] : T(0);
#pragma unroll
      for (int x = 2; x >= 0; --x) {
        T acc = T(0);
#pragma unroll
        for (int z = x + 1; z < 4; ++z) acc += r[x][z] * wv[z];
        wv[x] = x < y ? -ri[x] * acc : (x == y ? ri[x] : T(0));
      }
#pragma unroll
      for (int x = 0; x < 4; ++x) Wl[(c + x) * kLdS + c + y] = wv[x];
    } else {
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        const int e = lane - 16 + 48 * m, blkno = e >> 4, pos = e & 15;
        const int i4 = blkno < 1 ? 1 : (blkno < 3 ? 2 : 3);
        const int j4 = blkno < 1 ? 0 : (blkno < 3 ? blkno - 1 : blkno - 3);
        Wl[(o + 4 * i4 + (pos >> 2)) * kLdS + o + 4 * j4 + (pos & 3)] = T(0);
      }
    }
  } else if (part == 1) {
    if (lane < 32) {
      const int b = o + 8 * (lane >> 4), x = (lane >> 2) & 3, y = lane & 3;
      T t[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        T acc = T(0);
#pragma unroll
        for (int m = 0; m < 4; ++m) acc += S[(b + k) * kLdS + b + 4 + m] * Wl[(b + 4 + m) * kLdS + b + 4 + y];
        t[k] = acc;
      }
      T acc = T(0);
#pragma unroll
      for (int k = 0; k < 4; ++k) acc += Wl[(b + x) * kLdS + b + k] * t[k];
      Wl[(b + x) * kLdS + b + 4 + y] = -acc;
    }
  } else {
    const int x = lane >> 3, y = lane & 7;
    T acc = T(0);
    if (part == 2) {
#pragma unroll
      for (int m = 0; m < 8; ++m) acc += S[(o + x) * kLdS + o + 8 + m] * Wl[(o + 8 + m) * kLdS + o + 8 + y];
      tw[lane] = acc;
    } else {
#pragma unroll
      for (int k = 0; k < 8; ++k) acc += Wl[(o + x) * kLdS + o + k] * tw[k * 8 + y];
      Wl[(o + x) * kLdS + o + 8 + y] = -acc;
    }
  }
}

// Level 32 for the pair of 16 x 16 blocks at b and b + 16 (one wave; tt: 16 x 17 scratch):
// W(b, b + 16) = -W(b, b) (R(b, b + 16) W(b + 16, b + 16)).
template <class T>
__device__ inline void inv32_pair(const T* S, T* Wl, T* tt, int b) {
  tile_store(tile_mm_k<T, 16>(S + b * kLdS + b + 16, kLdS, Wl + (b + 16) * kLdS + b + 16, kLdS), tt, 17);
  wave_sync();
  tile_store_neg(tile_mm_k<T, 16>(Wl + b * kLdS + b, kLdS, tt, 17), Wl + b * kLdS + b + 16, kLdS);
}

// Column j (lane j of the calling wave) of row block rb of R, four rows, from S to Z;
// zero below the diagonal.  Rows 4 rb.. of one column are contiguous in Z.
template <class T>
__device__ inline void store_r_rows(const T* S, T* Z, long long ld, int rb) {
  const int j = threadIdx.x & 63, r0 = 4 * rb;
  T val[4];
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const T sv = S[(r0 + x) * kLdS + j];
    val[x] = j >= r0 + x ? sv : T(0);
  }
#pragma unroll
  for (int x = 0; x < 4; ++x) Z[r0 + x + (long long)j * ld] = val[x];
}

// The block's upper triangle is staged in lds[kStage + i * kLdS + j] (entry (i, j),
// i <= j; the lower triangle is ignored) and a barrier has passed since.  Stores R (zero
// below the diagonal) at Z and R^{-1} at W (leading dimension ld for both; only with
// `store`) and sets bit `bit` of *info on a non-positive pivot.  R^{-1} stays in
// lds[kWl + i * kLdS + j] with zeros below the diagonal; the staging area holds R above
// the diagonal and is free for the caller after the final barrier inside, after which
// only the W stores remain.  Every thread of the workgroup must call this (at least 256).
// Inverse pieces run by the trailing waves during the factorization, as (step, wave,
// code): code = 4 * block + part for part p of the 16 x 16 diagonal block `block`
// (inv16_part), 12 for level 32 of blocks 0 and 1.  A block's parts start once its rows of
// R are final (block b after step 4 b + 3) and go to waves with few tiles at that step.
constexpr unsigned char kInvPieces[][3] = {
    {4, 1, 0},  {5, 2, 1},  {6, 3, 2},  {7, 1, 3},  {8, 1, 4},  {9, 3, 5},  {10, 1, 6},
    {11, 3, 7}, {12, 1, 12}, {12, 3, 8}, {13, 3, 9}, {14, 1, 10}, {15, 3, 11}};
// The code per step for one wave, four bits per step (15: none).
constexpr unsigned long long inv_schedule(int wave) {
  unsigned long long m = ~0ull;
  for (const auto& pc : kInvPieces)
    if (pc[1] == wave) m = (m & ~(15ull << (4 * pc[0]))) | ((unsigned long long)pc[2] << (4 * pc[0]));
  return m;
}

template <class T>
__device__ __forceinline__ void factor_invert_block(T* lds, T* Z, T* W, long long ld, int* info,
                                                    int bit, bool store) {
  T* const S = lds + kStage;     // A, then R, row-major
  T* const Wl = lds + kWl;       // R^{-1}, row-major
  T* const rinv = lds + kPanel;  // 1 / R(i, i), i = 0..63
  T* const tw = rinv + 64;       // level-16 scratch, 64 per 16 x 16 block
  T* const tmp = lds + kTmp;
  const int tid = threadIdx.x;
  // (the wave index in a scalar register, so that every role test is a scalar branch)
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  constexpr int kSteps = kB / 4;
  // Wave 0 and the trailing waves run separate loops with one barrier per step each.
  if (wave == 0) {
    bool bad = false;
    for (int kb = 0; kb < kSteps; ++kb) {
      const int c0 = 4 * kb, j = lane;
      // block row kb of column j, with the update by panel kb - 1 (the trailing waves
      // applied the earlier panels)
      T a[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) a[x] = S[(c0 + x) * kLdS + j];
      if (kb > 0) {
        const T* P = S + (c0 - 4) * kLdS;
        T pc[4], u[4][4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          pc[p] = P[p * kLdS + j];
#pragma unroll
          for (int x = 0; x < 4; ++x) u[p][x] = P[p * kLdS + c0 + x];
        }
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
          for (int x = 0; x < 4; ++x) a[x] -= u[p][x] * pc[p];
      }
      // the diagonal block to every lane (lanes c0.. hold its columns), its factor R_d
      // (rows r[p][p..3]) and reciprocal pivots, in every lane
      T d[4][4];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int z = x; z < 4; ++z) d[x][z] = bcast(a[x], c0 + z);
      T r[4][4], ri[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const T piv = d[p][p];
        if (!(piv > T(0))) bad = true;
        const T rp = piv > T(0) ? (T)rsqrt_full((double)piv) : T(0);
        ri[p] = rp;
        r[p][p] = piv * rp;
#pragma unroll
        for (int z = p + 1; z < 4; ++z) r[p][z] = d[p][z] * rp;
#pragma unroll
        for (int x = p + 1; x < 4; ++x)
#pragma unroll
          for (int z = x; z < 4; ++z) d[x][z] -= r[p][x] * r[p][z];
      }
      // column j of R(k, :) = R_d^{-T} A(k, :) by forward substitution (in the diagonal
      // block's columns the same recurrence reproduces R_d above the diagonal; below it
      // the entries are zero; columns left of the block are not written)
      T R[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        T v = a[p];
#pragma unroll
        for (int z = 0; z < p; ++z) v -= r[z][p] * R[z];
        R[p] = v * ri[p];
      }
      if (j >= c0) {
        const int y = j - c0;
#pragma unroll
        for (int x = 0; x < 4; ++x) S[(c0 + x) * kLdS + j] = (y < 4 && x > y) ? T(0) : R[x];
      }
      if (j == 0) {
#pragma unroll
        for (int p = 0; p < 4; ++p) rinv[c0 + p] = ri[p];
      }
      __syncthreads();
    }
    if (bad && lane == 0) atomicOr(info, 1 << bit);
  } else if (wave < 4) {
    // The trailing matrix as the ten 16 x 16 tiles (ti, tj), ti <= tj, three or four per
    // wave so that every step has at most two live tiles per wave once tile row 0 is done
    // (tile row ti takes panels up to step 4 ti + 2).  Byte e of tl: ti * 4 + tj.  Every
    // tile takes a matrix-core step each step, with zero operands once it is done, so
    // that the accumulators are never updated conditionally.
    using Acc = typename BlkMfma<T>::acc_t;
    const int li = lane & 15, lk = lane >> 4;
    const int tl = wave == 1 ? 0x03000a05 : (wave == 2 ? 0x02010f06 : 0x02020b07);
    const int ntl = wave == 1 ? 4 : 3;
    constexpr unsigned long long kSched1 = inv_schedule(1), kSched2 = inv_schedule(2),
                                 kSched3 = inv_schedule(3);
    const unsigned long long sched = wave == 1 ? kSched1 : (wave == 2 ? kSched2 : kSched3);
    Acc acc[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int code = (tl >> (8 * e)) & 0xff, r0 = 16 * (code >> 2), q0 = 16 * (code & 3);
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[e][v] = S[(r0 + BlkMfma<T>::row(lk, v)) * kLdS + q0 + li];
    }
    // zeros in W's six 16 x 16 blocks below the diagonal (8 per lane of waves 1..3)
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int e = tid - 64 + 192 * m, blkno = e >> 8, pos = e & 255;
      const int i16 = blkno < 1 ? 1 : (blkno < 3 ? 2 : 3);
      const int j16 = blkno < 1 ? 0 : (blkno < 3 ? blkno - 1 : blkno - 3);
      Wl[(16 * i16 + (pos >> 4)) * kLdS + 16 * j16 + (pos & 15)] = T(0);
    }
    __syncthreads();
    for (int kb = 1; kb < kSteps; ++kb) {
      const int c0 = 4 * kb;
      // the rank-4 update by panel kb - 1: A(i, k) = -R(c0 - 4 + k, r0 + i),
      // B(k, j) = R(c0 - 4 + k, q0 + j)
      const T* P = S + (c0 - 4 + lk) * kLdS;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int code = (tl >> (8 * e)) & 0xff, ti = code >> 2;
        const int r0 = 16 * ti, q0 = 16 * (code & 3);
        const bool live = e < ntl && kb <= 4 * ti + 2;
        const T pa = P[r0 + li], pb = P[q0 + li];
        acc[e] = BlkMfma<T>::step(live ? -pa : T(0), live ? pb : T(0), acc[e]);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int code = (tl >> (8 * e)) & 0xff, ti = code >> 2;
        const int r0 = 16 * ti, q0 = 16 * (code & 3);
        // block row kb + 1 is wave 0's in the next step: accumulator element vs of every
        // lane in FP64 (rows lk + 4v), all four elements of the lanes lk == vs in FP32
        // (rows 4 lk + v)
        const int vs = kb + 1 - 4 * ti;
        if (e < ntl && vs >= 0 && vs < 4) {
          if constexpr (sizeof(T) == 8) {
            const T val = vs == 0 ? acc[e][0] : (vs == 1 ? acc[e][1] : (vs == 2 ? acc[e][2] : acc[e][3]));
            S[(r0 + lk + 4 * vs) * kLdS + q0 + li] = val;
          } else if (lk == vs) {
#pragma unroll
            for (int v = 0; v < 4; ++v) S[(r0 + 4 * lk + v) * kLdS + q0 + li] = acc[e][v];
          }
        }
      }
      // row block kb - 1 of R is final
      if (wave == 2 && store) store_r_rows(S, Z, ld, kb - 1);
      const int pc = (int)((sched >> (4 * kb)) & 15);
      if (pc == 12)
        inv32_pair(S, Wl, tmp, 0);
      else if (pc != 15)
        inv16_part(S, Wl, rinv, tw + 64 * (pc >> 2), 16 * (pc >> 2), pc & 3);
      __syncthreads();
    }
  } else {
    for (int kb = 0; kb < kSteps; ++kb) __syncthreads();
  }

  // ---- the rest of W = R^{-1}: the last 16 x 16 block (wave 0), then level 32 for the
  // second pair and level 64; the last row block of R goes out meanwhile
  if (wave == 0) {
#pragma unroll
    for (int part = 0; part < 4; ++part) {
      inv16_part(S, Wl, rinv, tw + 64 * 3, 48, part);
      wave_sync();
    }
  } else if (wave == 2 && store) {
    store_r_rows(S, Z, ld, kB / 4 - 1);
  }
  __syncthreads();
  if (wave == 1) inv32_pair(S, Wl, tmp + 16 * 17, 32);
  __syncthreads();
  // level 64: one 16 x 16 tile (ti, tj) of the 32 x 32 W12 per wave, skipping the zero
  // blocks of the triangular factors
  const int ti = wave & 1, tj = (wave >> 1) & 1;
  if (wave < 4) {
    const T* a = S + 16 * ti * kLdS + 32;
    const T* b = Wl + 32 * kLdS + 32 + 16 * tj;
    tile_store(tj ? tile_mm_k<T, 32>(a, kLdS, b, kLdS) : tile_mm_k<T, 16>(a, kLdS, b, kLdS),
               tmp + 16 * ti * kLdT + 16 * tj, kLdT);
  }
  __syncthreads();
  if (wave < 4) {
    const T* a = Wl + 16 * ti * kLdS + 16 * ti;
    const T* b = tmp + 16 * ti * kLdT + 16 * tj;
    tile_store_neg(ti ? tile_mm_k<T, 16>(a, kLdS, b, kLdT) : tile_mm_k<T, 32>(a, kLdS, b, kLdT),
                   Wl + 16 * ti * kLdS + 32 + 16 * tj, kLdS);
  }
  __syncthreads();
  // (all LDS reads ahead of the global stores, which may not be reordered past them)
  if (store && tid < kThreads) {
    T val[kB * kB / kThreads];
#pragma unroll
    for (int m = 0; m < kB * kB / kThreads; ++m) {
      const int e = tid + kThreads * m, i = e % kB, j = e / kB;
      val[m] = Wl[i * kLdS + j];
    }
#pragma unroll
    for (int m = 0; m < kB * kB / kThreads; ++m) {
      const int e = tid + kThreads * m, i = e % kB, j = e / kB;
      W[i + (long long)j * ld] = val[m];
    }
  }
}

}  // namespace blk
}  // namespace ps
