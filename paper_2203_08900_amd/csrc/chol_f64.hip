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
#include "chol_block.h"
#include "ps_internal.h"

namespace ps {

namespace {
constexpr int NB = kNb;
constexpr int NTD = 256;
}

// Factor and invert one 64 x 64 diagonal block per workgroup.
template <class T>
__global__ __launch_bounds__(NTD) void potrf_diag_kernel(T* z, long long sz, T* w, long long sw,
                                                         int ld, int k0, int* info) {
  __shared__ T lds[blk::kLdsElems];
  const int b = blockIdx.x;
  T* Z = z + b * sz + k0 + (long long)k0 * ld;
  T* W = w + b * sw + k0 + (long long)k0 * ld;
  // all loads in flight at once, then into LDS (the lower triangle is staged too and
  // ignored)
  T val[NB * NB / NTD];
#pragma unroll
  for (int q = 0; q < NB * NB / NTD; ++q) {
    const int e = threadIdx.x + q * NTD;
    val[q] = Z[e % NB + (long long)(e / NB) * ld];
  }
#pragma unroll
  for (int q = 0; q < NB * NB / NTD; ++q) {
    const int e = threadIdx.x + q * NTD;
    lds[blk::kStage + (e % NB) * blk::kLdS + e / NB] = val[q];
  }
  __syncthreads();
  blk::factor_invert_block(lds, Z, W, ld, info, b < 30 ? b : 30);
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
