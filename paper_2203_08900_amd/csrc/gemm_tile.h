// One output tile of a GEMM on CDNA4 matrix cores: FP64 (v_mfma_f64_16x16x4_f64) and
// FP32 (v_mfma_f32_16x16x4_f32).  Used by the grouped GEMM kernel and by the Cholesky
// step kernel, whose trailing-update workgroups run it.
//
// A workgroup computes a BM x BN tile of D = alpha op(A) op(B) + beta C; its waves
// own (BM/WM) x (BN/WN) sub-tiles as MFMA 16x16 fragments.  Two shapes: 128 x 128 with
// 16 waves of 32 x 32 (16 flops per byte loaded, four waves per SIMD) for problems whose
// tiles fill the chip, and 64 x 64 with 4 waves of 32 x 32 for the others.  A group of up to four
// independent problems (any operand transposes) shares one launch, so that problems
// whose tile counts alone would leave compute units idle fill the machine together.
// K advances in steps of 16 through two LDS buffers (one barrier per step); the global
// loads run two steps ahead of the MFMAs, through two register slots.
//
// LDS layouts per operand keep global loads coalesced along the contiguous
// dimension and fragment reads on distinct banks:
//   op(A) = A   : [k][i], stride BM+16       op(A) = A^T : [i][k], stride 16+1
//   op(B) = B   : [j][k], stride 16+1        op(B) = B^T : [k][j], stride BN+16
// Structure flags restrict each tile's K loop to the non-zero band of triangular
// operands and restrict / mirror the stored output of symmetric results.  Split-K
// writes per-split partial tiles that a second kernel sums in a fixed order.
//
// MFMA f64 16x16x4 register layout (checked on the device): A operand lane l holds
// A(l%16, l/16), B operand lane l holds B(l/16, l%16), accumulator element v of
// lane l is D(4v + l/16, l%16).
#pragma once

#include "ps_internal.h"

namespace ps {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Matrix-core step and accumulator layout per element type (checked on the device):
// both take A(l%16, l/16) and B(l/16, l%16) from lane l; accumulator element v of
// lane l is D(4v + l/16, l%16) for FP64 and D(4(l/16) + v, l%16) for FP32.
template <class T>
struct Mfma;
template <>
struct Mfma<double> {
  using acc_t = d4;
  __device__ static acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lk, int v) { return lk + 4 * v; }
};
template <>
struct Mfma<float> {
  using acc_t = f4;
  __device__ static acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lk, int v) { return 4 * lk + v; }
};

namespace {

constexpr int BK = 16;
constexpr int LDIK = BK + 1;

__device__ inline void tri_index(int t, int& hi, int& lo) {
  // t enumerates pairs (lo <= hi) row by row of hi: t = hi*(hi+1)/2 + lo
  int h = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while ((h + 1) * (h + 2) / 2 <= t) ++h;
  while (h * (h + 1) / 2 > t) --h;
  hi = h;
  lo = t - h * (h + 1) / 2;
}

}  // namespace

template <int BM, int BN>
struct GemmLds {
  static constexpr int LDKM = BM + 16;
  static constexpr int LDKN = BN + 16;
  static constexpr int ASZ = (BK * LDKM > BM * LDIK) ? BK * LDKM : BM * LDIK;
  static constexpr int BSZ = (BK * LDKN > BN * LDIK) ? BK * LDKN : BN * LDIK;
};

// One output tile of problem P (logical tile index bid within the launch).
// kUseC = false: the caller guarantees beta = 0 (no C operand), which frees the
// registers of the C prefetch.
template <class T, int BM, int BN, int WM, int WN, int TA, int TB, bool kUseC = true>
__device__ __forceinline__ void gemm_tile(const GemmProblemT<T>& P, int bid, T* smem) {
  auto As = reinterpret_cast<T(*)[GemmLds<BM, BN>::ASZ]>(smem);
  auto Bs = reinterpret_cast<T(*)[GemmLds<BM, BN>::BSZ]>(smem + 2 * GemmLds<BM, BN>::ASZ);
  constexpr int NT = WM * WN * 64;
  constexpr int FM = BM / (WM * 16), FN = BN / (WN * 16);
  constexpr int LDKM = GemmLds<BM, BN>::LDKM;
  constexpr int LDKN = GemmLds<BM, BN>::LDKN;
  constexpr int APT = BM * BK / NT;
  constexpr int BPT = BN * BK / NT;
  const int local = bid - P.tile_begin;
  // Triangular operands make the K extent differ from tile to tile.  Such problems (with
  // a full output) are launched without the XCD remap (dispatch is round-robin over the
  // XCDs) and enumerate their tiles longest first, batch entries interleaved, so the
  // long tiles start in the first wave of workgroups and the short ones fill in behind
  // them.  Triangular outputs keep the remap: their columns-ascending order already puts
  // the long tiles of the usual lower-K-bound operands first.
  const int tri_ops = (P.flags & (kOutUpper | kOutLower))
                          ? 0
                          : P.flags & (kAUpper | kALower | kBUpper | kBLower);
  const int nbat = P.nb1 * P.nb2;
  int z, tz;
  if (tri_ops) {
    z = local % nbat;
    tz = local / nbat;
  } else {
    z = local / P.tiles_per_batch;
    tz = local - z * P.tiles_per_batch;
  }
  const int ks = tz / P.tiles;          // split index
  const int t = tz - ks * P.tiles;
  int I, J;
  if (P.flags & kOutUpper) {
    tri_index(t, J, I);                 // columns J ascending
  } else if (P.flags & kOutLower) {
    tri_index(t, I, J);
  } else if (tri_ops == kAUpper) {      // K from i0: rows ascending
    I = t / P.tn;
    J = t - I * P.tn;
  } else if (tri_ops == kALower) {      // K to i0 + BM: rows descending
    I = t / P.tn;
    J = t - I * P.tn;
    I = P.tm - 1 - I;
  } else if (tri_ops == kBUpper) {      // K to j0 + BN: columns descending
    J = t / P.tm;
    I = t - J * P.tm;
    J = P.tn - 1 - J;
  } else if ((tri_ops == (kAUpper | kBLower) || tri_ops == (kALower | kBUpper)) && P.tm == P.tn) {
    // K from max(i0, j0) (resp. to min(i0, j0) + 128): shells of equal max(I, J),
    // innermost first (resp. mirrored through the far corner)
    int sh = (int)sqrtf((float)t);
    while (sh * sh > t) --sh;
    while ((sh + 1) * (sh + 1) <= t) ++sh;
    const int r = t - sh * sh;
    if (r <= sh) {
      I = sh;
      J = r;
    } else {
      I = r - sh - 1;
      J = sh;
    }
    if (tri_ops == (kALower | kBUpper)) {
      I = P.tm - 1 - I;
      J = P.tn - 1 - J;
    }
  } else {
    I = t % P.tm;
    J = t / P.tm;
  }
  const int z1 = z % P.nb1, z2 = z / P.nb1;
  const T* __restrict__ A = P.A + z1 * P.sA[0] + z2 * P.sA[1];
  const T* __restrict__ B = P.B + z1 * P.sB[0] + z2 * P.sB[1];
  T* D = P.D + z1 * P.sD[0] + z2 * P.sD[1];
  const T* C = P.C ? P.C + z1 * P.sC[0] + z2 * P.sC[1] : nullptr;

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
  const int nkt_all = per * nseg;
  const int kt_begin = (int)((long long)nkt_all * ks / P.ksplit);
  const int kt_end = (int)((long long)nkt_all * (ks + 1) / P.ksplit);

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int li = lane & 15, lk = lane >> 4;
  constexpr int tA = TA, tB = TB;
  const long long lda = P.lda, ldb = P.ldb;

  using acc_t = typename Mfma<T>::acc_t;
  acc_t acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

  // Two register slots for the global loads of the next two K steps: the loads of step
  // kt + 2 are issued before the matrix-core work of step kt and land in LDS only after
  // that of step kt + 1, so two steps of compute cover their latency (a single step of
  // a 64 x 64 tile is shorter than a trip to memory).
  T ra0[APT], rb0[BPT], ra1[APT], rb1[BPT];
  double rsc0 = 1.0, rsc1 = 1.0;   // segment scale of the A values in each slot

  auto load = [&](int kt, T* ra, T* rb, double& rsc) {
    const int s = kt / per;
    const int k0 = s * segK + kb + (kt - s * per) * BK;
    rsc = P.kseg > 0 ? (P.kscale_b ? P.kscale_b[z * P.nseg + s] : P.kscale[s]) : 1.0;
#pragma unroll
    for (int p = 0; p < APT; ++p) {
      const int idx = tid + p * NT;
      if (!tA) {
        const int i = idx % BM, k = idx / BM;
        ra[p] = A[(i0 + i) + (long long)(k0 + k) * lda];
      } else {
        const int k = idx % BK, i = idx / BK;
        ra[p] = A[(k0 + k) + (long long)(i0 + i) * lda];
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
  auto store = [&](int buf, const T* ra, const T* rb, double rsc) {
#pragma unroll
    for (int p = 0; p < APT; ++p) {
      const int idx = tid + p * NT;
      const T v = P.kseg > 0 ? (T)((double)ra[p] * rsc) : ra[p];
      if (!tA) {
        const int i = idx % BM, k = idx / BM;
        As[buf][k * LDKM + i] = v;
      } else {
        const int k = idx % BK, i = idx / BK;
        As[buf][i * LDIK + k] = v;
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
        Bs[buf][k * LDKN + j] = rb[p];
      }
    }
  };
  auto compute = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int k = kk * 4 + lk;
      T av[FM], bv[FN];
#pragma unroll
      for (int a = 0; a < FM; ++a) {
        const int i = wm * FM * 16 + a * 16 + li;
        av[a] = !tA ? As[buf][k * LDKM + i] : As[buf][i * LDIK + k];
      }
#pragma unroll
      for (int b = 0; b < FN; ++b) {
        const int j = wn * FN * 16 + b * 16 + li;
        bv[b] = !tB ? Bs[buf][j * LDIK + k] : Bs[buf][k * LDKN + j];
      }
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = Mfma<T>::step(av[a], bv[b], acc[a][b]);
    }
  };

  // 64 x 64 tiles (short-K trailing updates of the factorizations among them) load their
  // C values before the K loop, so that trip to memory overlaps the loop instead of
  // following it; the large tiles keep their registers for occupancy and prefetch C
  // row by row in the epilogue.
  constexpr bool kEarlyC = (BM == 64) && kUseC;
  T cpre[kEarlyC ? FM : 1][FN][4];
  if (kEarlyC && (P.beta_b ? P.beta_b[z] : P.beta) != 0.0) {
#pragma unroll
    for (int a = 0; a < (kEarlyC ? FM : 1); ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = i0 + wm * FM * 16 + a * 16 + Mfma<T>::row(lk, v);
          const int j = j0 + wn * FN * 16 + b * 16 + li;
          cpre[a][b][v] = C[i + j * (long long)P.ldc];
        }
  }

  // Steps alternate between (LDS buffer 0, slot 0 refilled) and (buffer 1, slot 1): the
  // store after a step's compute writes the other buffer, whose readers finished before
  // the previous barrier, from the slot loaded one step earlier.
  const int nkt = kt_end - kt_begin;
  if (nkt > 0) {
    load(kt_begin, ra0, rb0, rsc0);
    if (nkt > 1) load(kt_begin + 1, ra1, rb1, rsc1);
    store(0, ra0, rb0, rsc0);
    __syncthreads();
    for (int it = 0; it < nkt; it += 2) {
      if (it + 2 < nkt) load(kt_begin + it + 2, ra0, rb0, rsc0);
      compute(0);
      if (it + 1 < nkt) store(1, ra1, rb1, rsc1);
      __syncthreads();
      if (it + 1 >= nkt) break;
      if (it + 3 < nkt) load(kt_begin + it + 3, ra1, rb1, rsc1);
      compute(1);
      if (it + 2 < nkt) store(0, ra0, rb0, rsc0);
      __syncthreads();
    }
  }

  const double alpha = P.alpha_b ? P.alpha_b[z] : P.alpha;
  const double beta = kUseC ? (P.beta_b ? P.beta_b[z] : P.beta) : 0.0;
  if (P.ksplit > 1) {
    // partial tile of split ks (batch extent is 1 for split problems)
    T* W = P.ws + (long long)ks * P.M * P.N;
    const long long M = P.M;
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = i0 + wm * FM * 16 + a * 16 + Mfma<T>::row(lk, v);
          const int j = j0 + wn * FN * 16 + b * 16 + li;
          W[i + j * M] = (T)(alpha * acc[a][b][v]);
        }
    return;
  }
  const long long ldc = P.ldc, ldd = P.ldd;
  // C may be D itself (in-place updates), so the compiler cannot move a C load above an
  // earlier D store: loaded one by one, every element would wait a full memory latency.
  // The C values of fragment row a + 1 are therefore loaded before the stores of row a
  // (they are other elements, so the order is safe whether or not C aliases D).
  T cur[FN][4], nxt[FN][4];
  auto load_c = [&](int a, T (*dst)[4]) {
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + wm * FM * 16 + a * 16 + Mfma<T>::row(lk, v);
        const int j = j0 + wn * FN * 16 + b * 16 + li;
        dst[b][v] = C[i + j * ldc];
      }
  };
  if (!kEarlyC && beta != 0.0) load_c(0, cur);
#pragma unroll
  for (int a = 0; a < FM; ++a) {
    if (!kEarlyC && beta != 0.0 && a + 1 < FM) load_c(a + 1, nxt);
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + wm * FM * 16 + a * 16 + Mfma<T>::row(lk, v);
        const int j = j0 + wn * FN * 16 + b * 16 + li;
        if ((flags & kOutUpper) && i > j) continue;
        if ((flags & kOutLower) && i < j) continue;
        double val = alpha * acc[a][b][v];
        if (beta != 0.0)
          val += beta * (double)(kEarlyC ? cpre[kEarlyC ? a : 0][b][v] : cur[b][v]);
        D[i + j * ldd] = (T)val;
        if ((flags & kMirror) && i != j) D[j + i * ldd] = (T)val;
      }
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) cur[b][v] = nxt[b][v];
  }
}

}  // namespace ps
