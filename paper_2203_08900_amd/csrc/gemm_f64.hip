// FP64 GEMM on CDNA4 matrix cores (v_mfma_f64_16x16x4_f64).
//
// One workgroup of 4 waves computes a 64 x 64 tile of D = alpha op(A) op(B) + beta C;
// each wave owns a 32 x 32 quadrant as 2 x 2 MFMA 16x16 fragments.  K advances in
// steps of 16 through two LDS buffers (one barrier per step): the next step's
// global loads are issued into registers before the MFMAs of the current step.
//
// LDS layouts are chosen per operand so that global loads are coalesced along the
// contiguous dimension and the fragment reads hit distinct banks:
//   op(A) = A   : [k][i], stride 64+16 doubles   (A read down columns)
//   op(A) = A^T : [i][k], stride 16+1  doubles   (A read along columns = op rows)
//   op(B) = B   : [j][k], stride 16+1
//   op(B) = B^T : [k][j], stride 64+16
// Structure flags restrict the K loop of each tile to the non-zero band of
// triangular operands and restrict/mirror the stored output for symmetric results.
#include "ps_internal.h"

namespace ps {

typedef double d4 __attribute__((ext_vector_type(4)));

struct GemmGroup {
  int count;
  GemmProblem p[kMaxGroup];
};

namespace {

constexpr int BM = 64, BN = 64, BK = 16, WM = 2, WN = 2;
constexpr int NT = WM * WN * 64;
constexpr int FM = BM / (WM * 16), FN = BN / (WN * 16);
constexpr int LDKM = BM + 16;   // [k][i] stride
constexpr int LDIK = BK + 1;    // [i][k] stride
constexpr int ASZ = (BK * LDKM > BM * LDIK) ? BK * LDKM : BM * LDIK;
constexpr int BSZ = (BK * (BN + 16) > BN * LDIK) ? BK * (BN + 16) : BN * LDIK;
constexpr int APT = BM * BK / NT;
constexpr int BPT = BN * BK / NT;

__device__ inline void tri_index(int t, int& hi, int& lo) {
  // t enumerates pairs (lo <= hi) row by row of hi: t = hi*(hi+1)/2 + lo
  int h = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while ((h + 1) * (h + 2) / 2 <= t) ++h;
  while (h * (h + 1) / 2 > t) --h;
  hi = h;
  lo = t - h * (h + 1) / 2;
}

}  // namespace

__global__ __launch_bounds__(NT) void gemm_f64_kernel(GemmGroup g) {
  __shared__ double As[2][ASZ];
  __shared__ double Bs[2][BSZ];

  const int bid = blockIdx.x;
  int pi = 0;
  while (pi + 1 < g.count && bid >= g.p[pi + 1].tile_begin) ++pi;
  const GemmProblem& P = g.p[pi];

  const int local = bid - P.tile_begin;
  const int z = local / P.tiles_per_batch;
  const int t = local - z * P.tiles_per_batch;
  int I, J;
  if (P.flags & kOutUpper) {
    tri_index(t, J, I);
  } else if (P.flags & kOutLower) {
    tri_index(t, I, J);
  } else {
    I = t % P.tm;
    J = t / P.tm;
  }
  const int z1 = z % P.nb1, z2 = z / P.nb1;
  const double* __restrict__ A = P.A + z1 * P.sA[0] + z2 * P.sA[1];
  const double* __restrict__ B = P.B + z1 * P.sB[0] + z2 * P.sB[1];
  double* D = P.D + z1 * P.sD[0] + z2 * P.sD[1];
  const double* C = P.C ? P.C + z1 * P.sC[0] + z2 * P.sC[1] : nullptr;

  const int i0 = I * BM, j0 = J * BN;
  const int flags = P.flags;
  const int segK = P.kseg > 0 ? P.kseg : P.K;
  const int nseg = P.kseg > 0 ? P.nseg : 1;
  int kb = 0, ke = segK;
  if (flags & kAUpper) kb = max(kb, i0);
  if (flags & kBLower) kb = max(kb, j0);
  if (flags & kALower) ke = min(ke, i0 + BM);
  if (flags & kBUpper) ke = min(ke, j0 + BN);
  kb = kb / BK * BK;
  ke = min(segK, (ke + BK - 1) / BK * BK);
  const int per = ke > kb ? (ke - kb) / BK : 0;
  const int nkt = per * nseg;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int li = lane & 15, lk = lane >> 4;
  const int tA = P.tA, tB = P.tB;
  const long long lda = P.lda, ldb = P.ldb;

  d4 acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

  double ra[APT], rb[BPT];

  auto load = [&](int kt) {
    const int s = kt / per;
    const int k0 = s * segK + kb + (kt - s * per) * BK;
    const double sc = P.kseg > 0 ? P.kscale[s] : 1.0;
#pragma unroll
    for (int p = 0; p < APT; ++p) {
      const int idx = tid + p * NT;
      if (!tA) {
        const int i = idx % BM, k = idx / BM;
        ra[p] = A[(i0 + i) + (long long)(k0 + k) * lda] * sc;
      } else {
        const int k = idx % BK, i = idx / BK;
        ra[p] = A[(k0 + k) + (long long)(i0 + i) * lda] * sc;
      }
    }
#pragma unroll
    for (int p = 0; p < BPT; ++p) {
      const int idx = tid + p * NT;
      if (!tB) {
        const int k = idx % BK, j = idx / BK;
        rb[p] = B[(k0 + k) + (long long)(j0 + j) * ldb];
      } else {
        const int j = idx % BN, k = idx / BN;
        rb[p] = B[(j0 + j) + (long long)(k0 + k) * ldb];
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int p = 0; p < APT; ++p) {
      const int idx = tid + p * NT;
      if (!tA) {
        const int i = idx % BM, k = idx / BM;
        As[buf][k * LDKM + i] = ra[p];
      } else {
        const int k = idx % BK, i = idx / BK;
        As[buf][i * LDIK + k] = ra[p];
      }
    }
#pragma unroll
    for (int p = 0; p < BPT; ++p) {
      const int idx = tid + p * NT;
      if (!tB) {
        const int k = idx % BK, j = idx / BK;
        Bs[buf][j * LDIK + k] = rb[p];
      } else {
        const int j = idx % BN, k = idx / BN;
        Bs[buf][k * (BN + 16) + j] = rb[p];
      }
    }
  };

  if (nkt > 0) {
    load(0);
    store(0);
    __syncthreads();
    for (int kt = 0; kt < nkt; ++kt) {
      const int buf = kt & 1;
      if (kt + 1 < nkt) load(kt + 1);
#pragma unroll
      for (int kk = 0; kk < BK / 4; ++kk) {
        const int k = kk * 4 + lk;
        double av[FM], bv[FN];
#pragma unroll
        for (int a = 0; a < FM; ++a) {
          const int i = wm * FM * 16 + a * 16 + li;
          av[a] = !tA ? As[buf][k * LDKM + i] : As[buf][i * LDIK + k];
        }
#pragma unroll
        for (int b = 0; b < FN; ++b) {
          const int j = wn * FN * 16 + b * 16 + li;
          bv[b] = !tB ? Bs[buf][j * LDIK + k] : Bs[buf][k * (BN + 16) + j];
        }
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
          for (int b = 0; b < FN; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
      }
      if (kt + 1 < nkt) store(buf ^ 1);
      __syncthreads();
    }
  }

  const double alpha = P.alpha, beta = P.beta;
  const long long ldc = P.ldc, ldd = P.ldd;
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + wm * FM * 16 + a * 16 + lk + 4 * v;  // D(4v + lane/16, lane%16)
        const int j = j0 + wn * FN * 16 + b * 16 + li;
        if ((flags & kOutUpper) && i > j) continue;
        if ((flags & kOutLower) && i < j) continue;
        double val = alpha * acc[a][b][v];
        if (beta != 0.0) val += beta * C[i + j * ldc];
        D[i + j * ldd] = val;
        if ((flags & kMirror) && i != j) D[j + i * ldd] = val;
      }
}

GemmProblem gemm_problem(int M, int N, int K, const double* A, int lda, int tA,
                         const double* B, int ldb, int tB, double* D, int ldd, double alpha,
                         double beta, const double* C, int ldc, int flags) {
  GemmProblem p{};
  p.A = A;
  p.B = B;
  p.C = C ? C : D;
  p.D = D;
  p.M = M;
  p.N = N;
  p.K = K;
  p.lda = lda;
  p.ldb = ldb;
  p.ldc = C ? ldc : ldd;
  p.ldd = ldd;
  p.tA = tA;
  p.tB = tB;
  p.flags = flags;
  p.nb1 = 1;
  p.nb2 = 1;
  p.kseg = 0;
  p.nseg = 1;
  p.alpha = alpha;
  p.beta = beta;
  return p;
}

void gemm_f64(hipStream_t s, const GemmProblem* probs, int count) {
  GemmGroup g{};
  int total = 0;
  for (int q = 0; q < count; ++q) {
    GemmProblem p = probs[q];
    if (p.M <= 0 || p.N <= 0 || p.nb1 <= 0 || p.nb2 <= 0) continue;
    if (p.M % BM || p.N % BN || p.K % BK || (p.kseg > 0 && p.kseg % BK))
      throw HipError{hipErrorInvalidValue, "gemm_f64: dimensions must be multiples of the tile"};
    if ((p.flags & (kOutUpper | kOutLower)) && p.M != p.N)
      throw HipError{hipErrorInvalidValue, "gemm_f64: triangular output needs M == N"};
    if (p.kseg > 0 && (p.nseg < 1 || p.nseg > kMaxSeg || p.kseg * p.nseg != p.K))
      throw HipError{hipErrorInvalidValue, "gemm_f64: bad K segmentation"};
    p.tm = p.M / BM;
    p.tn = p.N / BN;
    p.tiles_per_batch = (p.flags & (kOutUpper | kOutLower)) ? p.tm * (p.tm + 1) / 2 : p.tm * p.tn;
    p.tile_begin = total;
    total += p.tiles_per_batch * p.nb1 * p.nb2;
    g.p[g.count++] = p;
  }
  if (total == 0) return;
  hipLaunchKernelGGL(gemm_f64_kernel, dim3(total), dim3(NT), 0, s, g);
  PS_HIP(hipGetLastError());
}

}  // namespace ps
