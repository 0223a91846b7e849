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
// K advances in steps of 32 through two LDS buffers (one barrier per step); the global
// loads run two steps ahead of the MFMAs, through two register slots.  Every global
// access is a 16-byte vector along the operand's contiguous dimension (all operands,
// leading dimensions and batch strides are 16-byte aligned; the launcher checks), and
// the epilogue goes through LDS so that C, D, the mirrored stores and split-K partial
// tiles move as coalesced vectors too.
//
// LDS layouts per operand keep global loads coalesced along the contiguous
// dimension and fragment reads on distinct banks:
//   op(A) = A   : [k][i], stride BM+16       op(A) = A^T : [i][k], stride 32+1
//   op(B) = B   : [j][k], stride 32+1        op(B) = B^T : [k][j], stride BN+16
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

constexpr int BK = 32;
constexpr int LDIK = BK + 1;

__host__ __device__ inline void tri_index(int t, int& hi, int& lo) {
  // t enumerates pairs (lo <= hi) row by row of hi: t = hi*(hi+1)/2 + lo
  int h = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while ((h + 1) * (h + 2) / 2 <= t) ++h;
  while (h * (h + 1) / 2 > t) --h;
  hi = h;
  lo = t - h * (h + 1) / 2;
}

}  // namespace

// 16-byte vector of T
template <class T>
struct VecT {
  static constexpr int VW = 16 / sizeof(T);
  typedef T type __attribute__((ext_vector_type(16 / sizeof(T))));
};

template <int BM, int BN>
struct GemmLds {
  static constexpr int LDKM = BM + 16;
  static constexpr int LDKN = BN + 16;
  static constexpr int ASZ = (BK * LDKM > BM * LDIK) ? BK * LDKM : BM * LDIK;
  static constexpr int BSZ = (BK * LDKN > BN * LDIK) ? BK * LDKN : BN * LDIK;
};

// Tile (I, J) of logical tile t of a problem (batch and split indices removed).
// Triangular operands make the K extent differ from tile to tile.  Such problems (with
// a full output) enumerate their tiles longest first, so the long tiles start in the
// first wave of workgroups and the short ones fill in behind them; triangular outputs
// go by columns ascending, which already puts the long tiles of the usual lower-K-bound
// operands first (their launches are mostly a single round of workgroups, where the
// start order only moves tiles between the XCDs' caches).
template <int BM, int BN, class Prob>
__host__ __device__ inline void tile_coords(const Prob& P, int t, int& I, int& J) {
  const int tri_ops = (P.flags & (kOutUpper | kOutLower))
                          ? 0
                          : P.flags & (kAUpper | kALower | kBUpper | kBLower);
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
  } else if ((tri_ops == (kAUpper | kBUpper) || tri_ops == (kALower | kBLower)) && P.tm == P.tn) {
    // K from i0 to j0 + BN (resp. from j0 to i0 + BM): diagonals of the nonzero triangle,
    // the far corner first (longest K), then the empty tiles of the other triangle
    const int T = P.tm, ntri = T * (T + 1) / 2;
    if (t < ntri) {
      int e, r;
      tri_index(t, e, r);   // diagonal e from the far corner, position r along it
      I = r;
      J = r + (T - 1 - e);
    } else {
      int a, b;
      tri_index(t - ntri, a, b);   // strictly below the diagonal: (a + 1, b)
      I = a + 1;
      J = b;
    }
    if (tri_ops == (kALower | kBLower)) {
      const int x = I;
      I = J;
      J = x;
    }
  } else {
    I = t % P.tm;
    J = t / P.tm;
  }
}

// The K band of tile (I, J) within each K segment: [kb, kb + per BK); the tile takes
// per * nseg steps of BK in all.
template <int BM, int BN, class Prob>
__host__ __device__ inline int tile_band(const Prob& P, int I, int J, int& kb) {
  const int segK = P.kseg > 0 ? P.kseg : P.K;
  const int i0 = I * BM, j0 = J * BN;
  int b = 0, e = segK;
  if (P.flags & kAUpper) b = b > i0 ? b : i0;
  if (P.flags & kBLower) b = b > j0 ? b : j0;
  if (P.flags & kALower) e = e < i0 + BM ? e : i0 + BM;
  if (P.flags & kBUpper) e = e < j0 + BN ? e : j0 + BN;
  b = b / BK * BK;
  e = (e + BK - 1) / BK * BK;
  e = e < segK ? e : segK;
  kb = b;
  return e > b ? (e - b) / BK : 0;
}

// The epilogue of tile (I, J) of batch entry z, from the product op(A) op(B) held in LDS
// at Ds as [j][i] (row length BM + VW): D = alpha Ds + beta C with the output triangle
// and mirror conventions.  The tile moves between LDS and memory as coalesced vectors:
// vector q of a thread holds rows [VW (e % (BM/VW)), + VW) of column e / (BM/VW),
// e = tid + q NT (cpre: those C vectors loaded beforehand when use_pre and NC covers
// them).  C may be D itself
// (in-place updates): every element is read and written by one thread, in that order.
// Ends on a barrier when it writes the mirror.
template <class T, int BM, int BN, int NT, int NC>
__device__ __forceinline__ void tile_epilogue(const GemmProblemT<T>& P, int z, int I, int J, T* Ds,
                                              double alpha, double beta, bool use_pre,
                                              const typename VecT<T>::type (&cpre)[NC]) {
  constexpr int VW = VecT<T>::VW;
  using vec_t = typename VecT<T>::type;
  constexpr int LDD = BM + VW;
  constexpr int OV = BM * BN / (VW * NT);
  const int tid = threadIdx.x;
  const int z1 = z % P.nb1, z2 = z / P.nb1;
  T* D = P.D + z1 * P.sD[0] + z2 * P.sD[1];
  const T* C = P.C ? P.C + z1 * P.sC[0] + z2 * P.sC[1] : nullptr;
  const long long ldc = P.ldc, ldd = P.ldd;
  const int i0 = I * BM, j0 = J * BN;
  const int flags = P.flags;
  const bool up = flags & kOutUpper, lo = flags & kOutLower, mir = flags & kMirror;
#pragma unroll
  for (int q = 0; q < OV; ++q) {
    const int e = tid + q * NT, iv = e % (BM / VW), j = e / (BM / VW);
    const int i = i0 + VW * iv, jj = j0 + j;
    vec_t cv;
    if (beta != 0.0) {
      if (NC == OV && use_pre)
        cv = cpre[NC == OV ? q : 0];
      else
        cv = *reinterpret_cast<const vec_t*>(C + i + (long long)jj * ldc);
    }
    vec_t out;
    bool all = true;
#pragma unroll
    for (int u = 0; u < VW; ++u) {
      double val = alpha * (double)Ds[j * LDD + VW * iv + u];
      if (beta != 0.0) val += beta * (double)cv[u];
      out[u] = (T)val;
      all = all && !((up && i + u > jj) || (lo && i + u < jj));
    }
    if (mir) {
#pragma unroll
      for (int u = 0; u < VW; ++u) Ds[j * LDD + VW * iv + u] = out[u];
    }
    if (all) {
      *reinterpret_cast<vec_t*>(D + i + (long long)jj * ldd) = out;
    } else {
#pragma unroll
      for (int u = 0; u < VW; ++u)
        if (!((up && i + u > jj) || (lo && i + u < jj))) D[i + u + (long long)jj * ldd] = out[u];
    }
  }
  if (!mir) return;
  // D(j, i) = D(i, j) for the stored entries off the diagonal, as vectors along j
  __syncthreads();
#pragma unroll
  for (int q = 0; q < OV; ++q) {
    const int e = tid + q * NT, jv = e % (BN / VW), il = e / (BN / VW);
    const int ii = i0 + il, jb = j0 + VW * jv;
    vec_t out;
    bool any = false, all = true;
#pragma unroll
    for (int u = 0; u < VW; ++u) {
      const int jj = jb + u;
      const bool st = up ? ii < jj : (lo ? ii > jj : ii != jj);
      out[u] = Ds[(VW * jv + u) * LDD + il];
      any = any || st;
      all = all && st;
    }
    if (all) {
      *reinterpret_cast<vec_t*>(D + jb + (long long)ii * ldd) = out;
    } else if (any) {
#pragma unroll
      for (int u = 0; u < VW; ++u) {
        const int jj = jb + u;
        if (up ? ii < jj : (lo ? ii > jj : ii != jj)) D[jj + (long long)ii * ldd] = out[u];
      }
    }
  }
  __syncthreads();
}

// K steps [kt_begin, kt_end) of tile (I, J) of batch entry z.  Output: part non-null, the
// partial tile alpha * (its product) to part as [j][i] with row length BM; otherwise
// with a uniform split-K (P.ksplit > 1) the partial tile of split ks to P.ws (M x N
// per split); otherwise the epilogue.  kUseC = false: the caller guarantees beta = 0
// (no C operand), which frees the registers of the C prefetch.  LDS is free again when
// this returns (its last accesses are behind a barrier).
template <class T, int BM, int BN, int WM, int WN, int TA, int TB, bool kUseC>
__device__ __forceinline__ void gemm_tile_run(const GemmProblemT<T>& P, int z, int I, int J,
                                              int kt_begin, int kt_end, int ks, T* part,
                                              T* smem) {
  auto As = reinterpret_cast<T(*)[GemmLds<BM, BN>::ASZ]>(smem);
  auto Bs = reinterpret_cast<T(*)[GemmLds<BM, BN>::BSZ]>(smem + 2 * GemmLds<BM, BN>::ASZ);
  constexpr int NT = WM * WN * 64;
  constexpr int FM = BM / (WM * 16), FN = BN / (WN * 16);
  constexpr int LDKM = GemmLds<BM, BN>::LDKM;
  constexpr int LDKN = GemmLds<BM, BN>::LDKN;
  constexpr int VW = VecT<T>::VW;               // elements per 16-byte access
  using vec_t = typename VecT<T>::type;
  constexpr int AV = BM * BK / (VW * NT);       // operand vectors per thread and K step
  constexpr int BV = BN * BK / (VW * NT);
  static_assert(AV * VW * NT == BM * BK && BV * VW * NT == BN * BK, "tile / thread mismatch");
  const int z1 = z % P.nb1, z2 = z / P.nb1;
  const T* __restrict__ A = P.A + z1 * P.sA[0] + z2 * P.sA[1];
  const T* __restrict__ B = P.B + z1 * P.sB[0] + z2 * P.sB[1];
  const T* C = P.C ? P.C + z1 * P.sC[0] + z2 * P.sC[1] : nullptr;
  const int i0 = I * BM, j0 = J * BN;
  const int segK = P.kseg > 0 ? P.kseg : P.K;
  int kb;
  const int per = tile_band<BM, BN>(P, I, J, kb);

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

  // Register slots for the global loads of the next K steps: small tiles keep two (the
  // loads of step kt + 2 are issued before the matrix-core work of step kt, so two steps
  // of compute cover their latency); the large tiles, whose 16 waves leave 128 registers
  // each and whose step is four times longer, keep one.  Vector p of a thread:
  // op(A) = A takes VW consecutive rows i of one column k, op(A) = A^T VW consecutive k
  // of one row i (likewise for B).
  constexpr int kSlots = BM == 128 ? 1 : 2;
  vec_t ra0[AV], rb0[BV], ra1[kSlots == 2 ? AV : 1], rb1[kSlots == 2 ? BV : 1];
  double rsc0 = 1.0, rsc1 = 1.0;   // segment scale of the A values in each slot

  auto load = [&](int kt, vec_t* ra, vec_t* rb, double& rsc) {
    const int s = kt / per;
    const int k0 = s * segK + kb + (kt - s * per) * BK;
    rsc = P.kseg > 0 ? (P.kscale_b ? P.kscale_b[z * P.nseg + s] : P.kscale[s]) : 1.0;
#pragma unroll
    for (int p = 0; p < AV; ++p) {
      const int idx = tid + p * NT;
      if (!tA) {
        const int iv = idx % (BM / VW), k = idx / (BM / VW);
        ra[p] = *reinterpret_cast<const vec_t*>(A + (i0 + VW * iv) + (long long)(k0 + k) * lda);
      } else {
        const int kv = idx % (BK / VW), i = idx / (BK / VW);
        ra[p] = *reinterpret_cast<const vec_t*>(A + (k0 + VW * kv) + (long long)(i0 + i) * lda);
      }
    }
#pragma unroll
    for (int p = 0; p < BV; ++p) {
      const int idx = tid + p * NT;
      if (!tB) {
        const int kv = idx % (BK / VW), j = idx / (BK / VW);
        rb[p] = *reinterpret_cast<const vec_t*>(B + (k0 + VW * kv) + (long long)(j0 + j) * ldb);
      } else {
        const int jv = idx % (BN / VW), k = idx / (BN / VW);
        rb[p] = *reinterpret_cast<const vec_t*>(B + (j0 + VW * jv) + (long long)(k0 + k) * ldb);
      }
    }
  };
  auto store = [&](int buf, const vec_t* ra, const vec_t* rb, double rsc) {
#pragma unroll
    for (int p = 0; p < AV; ++p) {
      const int idx = tid + p * NT;
      vec_t v = ra[p];
      if (P.kseg > 0) {
#pragma unroll
        for (int u = 0; u < VW; ++u) v[u] = (T)((double)v[u] * rsc);
      }
      if (!tA) {
        const int iv = idx % (BM / VW), k = idx / (BM / VW);
        *reinterpret_cast<vec_t*>(&As[buf][k * LDKM + VW * iv]) = v;
      } else {
        const int kv = idx % (BK / VW), i = idx / (BK / VW);
#pragma unroll
        for (int u = 0; u < VW; ++u) As[buf][i * LDIK + VW * kv + u] = v[u];
      }
    }
#pragma unroll
    for (int p = 0; p < BV; ++p) {
      const int idx = tid + p * NT;
      if (!tB) {
        const int kv = idx % (BK / VW), j = idx / (BK / VW);
#pragma unroll
        for (int u = 0; u < VW; ++u) Bs[buf][j * LDIK + VW * kv + u] = rb[p][u];
      } else {
        const int jv = idx % (BN / VW), k = idx / (BN / VW);
        *reinterpret_cast<vec_t*>(&Bs[buf][k * LDKN + VW * jv]) = rb[p];
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

  // 64 x 64 tiles load their C values before the K loop, so that trip to memory overlaps
  // the loop instead of following it; the large tiles keep their registers for occupancy
  // and read C in the epilogue.
  constexpr int LDD = BM + VW;
  constexpr int OV = BM * BN / (VW * NT);
  static_assert(BN * LDD <= 2 * (GemmLds<BM, BN>::ASZ + GemmLds<BM, BN>::BSZ), "output tile LDS");
  constexpr bool kEarlyC = (BM == 64) && kUseC;
  const double beta_z = kUseC ? (P.beta_b ? P.beta_b[z] : P.beta) : 0.0;
  const bool early = kEarlyC && beta_z != 0.0 && P.ksplit <= 1 && !part;
  vec_t cpre[kEarlyC ? OV : 1];
  if (early) {
#pragma unroll
    for (int q = 0; q < (kEarlyC ? OV : 1); ++q) {
      const int e = tid + q * NT, iv = e % (BM / VW), j = e / (BM / VW);
      cpre[q] = *reinterpret_cast<const vec_t*>(C + (i0 + VW * iv) + (long long)(j0 + j) * P.ldc);
    }
  }

  // Steps alternate between (LDS buffer 0, slot 0 refilled) and (buffer 1, slot 1): the
  // store after a step's compute writes the other buffer, whose readers finished before
  // the previous barrier, from the slot loaded one step earlier.
  const int nkt = kt_end - kt_begin;
  if (nkt > 0 && kSlots == 2) {
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
  } else if (nkt > 0) {
    // one slot: the loads of step kt + 1 are issued before the work of step kt and stored
    // into the other LDS buffer after it
    load(kt_begin, ra0, rb0, rsc0);
    store(0, ra0, rb0, rsc0);
    __syncthreads();
    for (int it = 0; it < nkt; ++it) {
      if (it + 1 < nkt) load(kt_begin + it + 1, ra0, rb0, rsc0);
      compute(it & 1);
      if (it + 1 < nkt) store((it + 1) & 1, ra0, rb0, rsc0);
      __syncthreads();
    }
  }

  const double alpha = P.alpha_b ? P.alpha_b[z] : P.alpha;
  // the product to LDS (the operand buffers are free: the K loop ended on a barrier)
  T* Ds = smem;
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        Ds[(wn * FN * 16 + b * 16 + li) * LDD + wm * FM * 16 + a * 16 + Mfma<T>::row(lk, v)] =
            acc[a][b][v];
  __syncthreads();
  if (part || P.ksplit > 1) {
    // a partial tile alpha op(A) op(B): compact [j][i] for part, the split's M x N slot
    // otherwise (batch extent 1 for split problems)
    T* W = part ? part : P.ws + (long long)ks * P.M * P.N + i0 + (long long)j0 * P.M;
    const long long ldw = part ? BM : P.M;
#pragma unroll
    for (int q = 0; q < OV; ++q) {
      const int e = tid + q * NT, iv = e % (BM / VW), j = e / (BM / VW);
      vec_t x;
#pragma unroll
      for (int u = 0; u < VW; ++u) x[u] = (T)(alpha * (double)Ds[j * LDD + VW * iv + u]);
      *reinterpret_cast<vec_t*>(W + VW * iv + j * ldw) = x;
    }
    __syncthreads();
    return;
  }
  tile_epilogue<T, BM, BN, NT>(P, z, I, J, Ds, alpha, beta_z, early, cpre);
  __syncthreads();
}

// One output tile of problem P (logical tile index bid within the launch), with the
// uniform split-K of P.ksplit.
template <class T, int BM, int BN, int WM, int WN, int TA, int TB, bool kUseC = true>
__device__ __forceinline__ void gemm_tile(const GemmProblemT<T>& P, int bid, T* smem) {
  const int local = bid - P.tile_begin;
  // Triangular operands with a full output are launched without the XCD remap (dispatch
  // is round-robin over the XCDs), batch entries interleaved.
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
  tile_coords<BM, BN>(P, t, I, J);
  int kb;
  const int nseg = P.kseg > 0 ? P.nseg : 1;
  const int nkt_all = tile_band<BM, BN>(P, I, J, kb) * nseg;
  const int kt_begin = (int)((long long)nkt_all * ks / P.ksplit);
  const int kt_end = (int)((long long)nkt_all * (ks + 1) / P.ksplit);
  gemm_tile_run<T, BM, BN, WM, WN, TA, TB, kUseC>(P, z, I, J, kt_begin, kt_end, ks, nullptr, smem);
}

}  // namespace ps
