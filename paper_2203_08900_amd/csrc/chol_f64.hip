// Batched Cholesky factorization with the inverse factor, Z = R^T R, W = R^{-1}, in FP64
// or FP32 (one template).
//
// Blocked right-looking algorithm over 64 x 64 diagonal blocks with a look-ahead of one
// block row.  Per block step k:
//   1. a small GEMM applies panel k to block row k+1;
//   2. one launch factors and inverts diagonal block k+1 and forms its panel
//      R(k+1, k+2:) = R^{-T} Z(k+1, k+2:) (each panel tile's workgroup factors the block
//      itself) while its other workgroups apply panel k to the rows below block row k+1.
// The full inverse factor W = R^{-1} is then assembled from the inverted diagonal
// blocks by recursive doubling, one pair of GEMM launches per level.  The batch index
// runs over independent matrices (the r shifted Gram matrices of a Zolotarev step, or
// A+B and A-B), so every launch covers all of them at once.
#include "chol_block.h"
#include "gemm_tile.h"
#include "ps_internal.h"

namespace ps {

namespace {
constexpr int NB = kNb;
constexpr int NTD = 256;
}

// One step of the blocked factorization, diagonal block and panel together.  Every
// workgroup (ntiles per matrix) factors and inverts the 64 x 64 diagonal block at k0 in
// LDS (the same arithmetic in each, so all agree; tile 0 stores R_kk^{-1} and R_kk) and
// then forms its 64-column tile of the panel R(k, k+1:) = R_kk^{-T} Z(k, k+1:) on the
// matrix cores, in place.  The redundant factorizations run side by side on otherwise
// idle compute units; what they save is a dependent launch per step.
template <class T>
__device__ void diag_panel(T* lds, int bid, T* z, long long sz, T* w, long long sw, int ld, int k0,
                           int rest, int ntiles, int* info) {
  const int b = bid / ntiles, t = bid - b * ntiles;
  T* Z = z + b * sz + k0 + (long long)k0 * ld;
  T* W = w + b * sw + k0 + (long long)k0 * ld;
  constexpr int Q = NB * NB / NTD;
  // all loads in flight at once, then into LDS (the lower triangle is staged too and
  // ignored)
  T val[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int e = threadIdx.x + q * NTD;
    val[q] = Z[e % NB + (long long)(e / NB) * ld];
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int e = threadIdx.x + q * NTD;
    lds[blk::kStage + (e % NB) * blk::kLdS + e / NB] = val[q];
  }
  __syncthreads();
  // The other workgroups of this matrix may still be reading the diagonal block, so
  // tile 0 leaves it untouched: R_kk goes to the (unused, zero) block below W_kk and
  // moves into place in the next step's launch, which also clears that block; the last
  // step (a single workgroup) writes it directly.
  if (t == 0 && k0 > 0) {
    T* src = W - (long long)NB * ld;              // block (k, k-1) of W
    T* dst = Z - NB - (long long)NB * ld;         // block (k-1, k-1) of Z
    for (int e = threadIdx.x; e < NB * NB; e += NTD) {
      const long long o = e % NB + (long long)(e / NB) * ld;
      dst[o] = src[o];
      src[o] = T(0);
    }
  }
  blk::factor_invert_block(lds, rest > 0 ? W + NB : Z, W, ld, info, b < 30 ? b : 30, t == 0);
  if (rest <= 0) return;
  // panel tile t: rows k0.., columns k0 + 64 + 64t.., staged where R was
  T* Zt = Z + (long long)(NB + NB * t) * ld;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int e = threadIdx.x + q * NTD;
    val[q] = Zt[e % NB + (long long)(e / NB) * ld];
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int e = threadIdx.x + q * NTD;
    lds[blk::kStage + (e % NB) * blk::kLdS + e / NB] = val[q];
  }
  __syncthreads();
  // wave w: rows 16w.. of the tile, four 16-column tiles, P = W_kk^T Z_tile
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
  const T* Wl = lds + blk::kWl;
  const T* St = lds + blk::kStage;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const auto acc = blk::tile_mm_ta(Wl + 16 * wave, blk::kLdS, St + 16 * c, blk::kLdS, NB);
#pragma unroll
    for (int v = 0; v < 4; ++v)
      Zt[(16 * wave + blk::BlkMfma<T>::row(lk, v)) + (long long)(16 * c + li) * ld] = acc[v];
  }
}

// One launch of the factorization: workgroups below ndiag run diag_panel for the block
// at k0; the others are tiles of the trailing update `tp` that the step before k0 still
// owes to the rows below block row k0 (look-ahead: the row block at k0 was updated
// first, by a launch of its own, so its diagonal block and panel need not wait for the
// whole trailing update).  The two roles touch disjoint parts of Z.
template <class T>
__global__ __launch_bounds__(NTD) void chol_step_kernel(T* z, long long sz, T* w, long long sw,
                                                        int ld, int k0, int rest, int ntiles,
                                                        int* info, GemmProblemT<T> tp, int ndiag) {
  constexpr int kAB = 2 * GemmLds<64, 64>::ASZ + 2 * GemmLds<64, 64>::BSZ;
  __shared__ T lds[blk::kLdsElems > kAB ? blk::kLdsElems : kAB];
  if ((int)blockIdx.x < ndiag)
    diag_panel(lds, blockIdx.x, z, sz, w, sw, ld, k0, rest, ntiles, info);
  else
    gemm_tile<T, 64, 64, 2, 2, 1, 0>(tp, blockIdx.x - ndiag, lds);
}

inline void gemm_t(hipStream_t s, const GemmProblem* p, int n) { gemm_f64(s, p, n); }
inline void gemm_t(hipStream_t s, const GemmProblemF* p, int n) { gemm_f32(s, p, n); }

template <class T>
void potrf_inv_t(hipStream_t s, T* z, long long sz, T* w, long long sw, int mp, int batch,
                 int* info, bool inverse = true) {
  zero_lower(s, w, mp, sw, batch);  // the diagonal blocks and W12 blocks cover the rest
  if (mp % NB) throw HipError{hipErrorInvalidValue, "potrf_inv_f64: size not a multiple of 64"};
  const int nbk = mp / NB;
  // ---- blocked right-looking Cholesky with a look-ahead of one block row:
  //   C_0 = diagonal block and panel of block row 0;
  //   for k = 0, 1, ...:  A_k = update of block row k+1 by panel k (one small GEMM);
  //                       C_{k+1} = diagonal block and panel of block row k+1, together
  //                       with the update by panel k of the rows below block row k+1.
  // Per step the chain waits for A_k and C_{k+1}; the bulk of the trailing update runs
  // beside the next diagonal factorization instead of before it.
  auto step = [&](int k0, const GemmProblemT<T>* tp) {
    const int rest = mp - k0 - NB;
    const int nt = rest > 0 ? rest / NB : 1;
    const int ndiag = batch * nt;
    GemmProblemT<T> t{};
    int ntrail = 0;
    if (tp) {
      t = *tp;
      t.tm = t.M / 64;
      t.tn = t.N / 64;
      t.tiles = t.tm * (t.tm + 1) / 2;   // upper-triangular output
      t.tiles_per_batch = t.tiles;
      t.tile_begin = 0;
      ntrail = t.tiles * batch;
    }
    hipLaunchKernelGGL(chol_step_kernel<T>, dim3(ndiag + ntrail), dim3(NTD), 0, s, z, sz, w, sw,
                       mp, k0, rest, nt, info, t, ndiag);
    PS_HIP(hipGetLastError());
  };
  step(0, nullptr);
  for (int k = 0; k + 1 < nbk; ++k) {
    const int k0 = k * NB;
    const int rest = mp - k0 - NB;   // > 0
    T* zr = z + k0 + (long long)(k0 + NB) * mp;          // R(k, k+1:)
    T* zn = z + (k0 + NB) + (long long)(k0 + NB) * mp;   // Z(k+1, k+1:)
    // A_k: Z(k+1, k+1:) -= R(k, k+1)^T R(k, k+1:)
    GemmProblemT<T> pa = gemm_problem(NB, rest, NB, zr, mp, 1, zr, mp, 0, zn, mp, -1.0, 1.0, zn, mp, 0);
    pa.nb1 = batch;
    pa.sA[0] = sz;
    pa.sB[0] = sz;
    pa.sC[0] = sz;
    pa.sD[0] = sz;
    gemm_t(s, &pa, 1);
    // C_{k+1} with the rest of the trailing update of step k:
    // Z(k+2:, k+2:) -= R(k, k+2:)^T R(k, k+2:)  (upper triangle)
    if (rest > NB) {
      T* zr2 = zr + (long long)NB * mp;
      T* zt2 = zn + NB + (long long)NB * mp;
      GemmProblemT<T> pt = gemm_problem(rest - NB, rest - NB, NB, zr2, mp, 1, zr2, mp, 0, zt2, mp,
                                        -1.0, 1.0, zt2, mp, kOutUpper);
      pt.nb1 = batch;
      pt.sA[0] = sz;
      pt.sB[0] = sz;
      pt.sC[0] = sz;
      pt.sD[0] = sz;
      step(k0 + NB, &pt);
    } else {
      step(k0 + NB, nullptr);
    }
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
