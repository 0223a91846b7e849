// Grouped, batched GEMM on CDNA4 matrix cores (FP64 and FP32): the launcher, the
// split-K reduction and the algorithmic flop count.  The tile itself (layouts, K loop,
// epilogue) is in gemm_tile.h.
#include "gemm_tile.h"
#include "ps_internal.h"

#include <type_traits>

namespace ps {

template <class T>
struct GemmGroup {
  int count;
  int remap;   // nonzero: spread consecutive tiles over one XCD (8 XCDs, round-robin dispatch)
  int total;
  GemmProblemT<T> p[kMaxGroup];
};

// The operand transposes are per problem, so one launch covers a group of problems
// with different transposes (each workgroup branches once, uniformly).
template <class T, int BM, int BN, int WM, int WN, bool kUseC>
__global__ __launch_bounds__(WM * WN * 64) void gemm_mfma_kernel(GemmGroup<T> g) {
  __shared__ __attribute__((aligned(16))) T smem[2 * GemmLds<BM, BN>::ASZ + 2 * GemmLds<BM, BN>::BSZ];
  int bid = blockIdx.x;
  if (g.remap) {
    // dispatch is round-robin over 8 XCDs: block b runs on XCD b % 8.  Give XCD x the
    // contiguous range of logical tiles [x * total/8, (x+1) * total/8).
    const int per = g.total >> 3;
    bid = (bid & 7) * per + (bid >> 3);
  }
  int pi = 0;
  while (pi + 1 < g.count && bid >= g.p[pi + 1].tile_begin) ++pi;
  const GemmProblemT<T>& P = g.p[pi];
  const int v = P.tA * 2 + P.tB;
  if (v == 0)
    gemm_tile<T, BM, BN, WM, WN, 0, 0, kUseC>(P, bid, smem);
  else if (v == 1)
    gemm_tile<T, BM, BN, WM, WN, 0, 1, kUseC>(P, bid, smem);
  else if (v == 2)
    gemm_tile<T, BM, BN, WM, WN, 1, 0, kUseC>(P, bid, smem);
  else
    gemm_tile<T, BM, BN, WM, WN, 1, 1, kUseC>(P, bid, smem);
}

// D = sum_s partial_s + beta C with the triangle / mirror conventions of the GEMM
template <class T>
__global__ void gemm_split_reduce_kernel(GemmProblemT<T> P) {
  const long long M = P.M, N = P.N;
  const long long n = M * N;
  const long long MN = M * N;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % M), j = (int)(e / M);
    if ((P.flags & kOutUpper) && i > j) continue;
    if ((P.flags & kOutLower) && i < j) continue;
    double val = 0.0;
    for (int s = 0; s < P.ksplit; ++s) val += P.ws[s * MN + e];
    if (P.beta != 0.0) val += P.beta * P.C[i + (long long)j * P.ldc];
    P.D[i + (long long)j * P.ldd] = (T)val;
    if ((P.flags & kMirror) && i != j) P.D[j + (long long)i * P.ldd] = (T)val;
  }
}

template <class T>
GemmProblemT<T> make_problem(int M, int N, int K, const T* A, int lda, int tA, const T* B, int ldb,
                             int tB, T* D, int ldd, double alpha, double beta, const T* C, int ldc,
                             int flags) {
  GemmProblemT<T> p{};
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
  p.ksplit = 1;
  p.alpha = alpha;
  p.beta = beta;
  p.ws = nullptr;
  return p;
}

GemmProblem gemm_problem(int M, int N, int K, const double* A, int lda, int tA, const double* B,
                         int ldb, int tB, double* D, int ldd, double alpha, double beta,
                         const double* C, int ldc, int flags) {
  return make_problem<double>(M, N, K, A, lda, tA, B, ldb, tB, D, ldd, alpha, beta, C, ldc, flags);
}

GemmProblemF gemm_problem(int M, int N, int K, const float* A, int lda, int tA, const float* B,
                          int ldb, int tB, float* D, int ldd, double alpha, double beta,
                          const float* C, int ldc, int flags) {
  return make_problem<float>(M, N, K, A, lda, tA, B, ldb, tB, D, ldd, alpha, beta, C, ldc, flags);
}

namespace {
thread_local KernelRecorder* g_rec = nullptr;   // per host thread (batched calls use several)

template <class T, int BM, int BN, int WM, int WN>
void launch_group(hipStream_t s, const GemmProblemT<T>* probs, int count) {
  GemmGroup<T> g{};
  int total = 0;
  for (int q = 0; q < count; ++q) {
    GemmProblemT<T> p = probs[q];
    if (p.M <= 0 || p.N <= 0 || p.nb1 <= 0 || p.nb2 <= 0) continue;
    p.tm = p.M / BM;
    p.tn = p.N / BN;
    p.tiles = (p.flags & (kOutUpper | kOutLower)) ? p.tm * (p.tm + 1) / 2 : p.tm * p.tn;
    p.tiles_per_batch = p.tiles * p.ksplit;
    p.tile_begin = total;
    total += p.tiles_per_batch * p.nb1 * p.nb2;
    g.p[g.count++] = p;
  }
  if (total == 0) return;
  g.total = total;
  bool tri_ops = false;
  for (int q = 0; q < g.count; ++q)
    tri_ops = tri_ops || ((g.p[q].flags & (kAUpper | kALower | kBUpper | kBLower)) &&
                          !(g.p[q].flags & (kOutUpper | kOutLower)));
  g.remap = (!tri_ops && total % 8 == 0 && total >= 64) ? 1 : 0;
  // without any C operand (beta = 0 everywhere, or split-K partials) the tiles use the
  // variant that keeps no C registers
  bool use_c = false;
  for (int q = 0; q < g.count; ++q)
    use_c = use_c || (g.p[q].ksplit <= 1 && (g.p[q].beta_b || g.p[q].beta != 0.0));
  const int slot = krec_begin(s);
  if (use_c)
    hipLaunchKernelGGL((gemm_mfma_kernel<T, BM, BN, WM, WN, true>), dim3(total),
                       dim3(WM * WN * 64), 0, s, g);
  else
    hipLaunchKernelGGL((gemm_mfma_kernel<T, BM, BN, WM, WN, false>), dim3(total),
                       dim3(WM * WN * 64), 0, s, g);
  PS_HIP(hipGetLastError());
  for (int q = 0; q < g.count; ++q) {
    const GemmProblemT<T>& p = g.p[q];
    if (p.ksplit > 1) {
      const long long n = (long long)p.M * p.N;
      const unsigned nb = (unsigned)std::min<long long>((n + 255) / 256, 8192);
      hipLaunchKernelGGL(gemm_split_reduce_kernel<T>, dim3(nb), dim3(256), 0, s, p);
      PS_HIP(hipGetLastError());
    }
  }
  if (slot >= 0) {   // the window covers the split-K reductions
    double f = 0.0;
    for (int q = 0; q < g.count; ++q) f += gemm_algorithmic_flops(g.p[q]);
    const int cls = std::is_same<T, float>::value ? kKcGemm32 : (BM == 128 ? kKcGemm128 : kKcGemm64);
    krec_end(s, slot, cls, f);
  }
}

}  // namespace

void kernel_set_recorder(KernelRecorder* r) { g_rec = r; }
KernelRecorder* kernel_recorder() { return g_rec; }

int krec_begin(hipStream_t s) {
  if (!g_rec || g_rec->n >= g_rec->cap) return -1;
  const int slot = g_rec->n++;
  PS_HIP(hipEventRecord(g_rec->ev[2 * slot], s));
  return slot;
}

void krec_end(hipStream_t s, int slot, int cls, double flops, int launches) {
  if (!g_rec || slot < 0) return;
  PS_HIP(hipEventRecord(g_rec->ev[2 * slot + 1], s));
  g_rec->cls[slot] = cls;
  g_rec->flops[slot] = flops;
  if (g_rec->nl) g_rec->nl[slot] = launches;
}

// 2 x (number of structurally non-zero products) over the stored output entries.  For
// each output (i, j) the K range is the intersection of the non-zero bands of op(A) row
// i and op(B) column j within every segment; the unstored triangle is not counted.
template <class T>
double gemm_algorithmic_flops(const GemmProblemT<T>& p) {
  const long long M = p.M, N = p.N;
  const long long segK = p.kseg > 0 ? p.kseg : p.K;
  const long long nseg = p.kseg > 0 ? p.nseg : 1;
  auto kb_a = [&](long long i) { return (p.flags & kAUpper) ? i : 0LL; };
  auto ke_a = [&](long long i) { return (p.flags & kALower) ? std::min(segK, i + 1) : segK; };
  auto kb_b = [&](long long j) { return (p.flags & kBLower) ? j : 0LL; };
  auto ke_b = [&](long long j) { return (p.flags & kBUpper) ? std::min(segK, j + 1) : segK; };
  const bool a_dep = p.flags & (kAUpper | kALower);
  const bool b_dep = p.flags & (kBUpper | kBLower);
  const bool tri = p.flags & (kOutUpper | kOutLower);
  double total = 0.0;
  if (!a_dep && !b_dep && !tri) {
    total = (double)M * N * segK;
  } else {
    // sum over i of sum over the stored j of max(0, ke - kb); O(M * N) only when both
    // operands or the output triangle couple i and j, done in closed form per row
    for (long long i = 0; i < M; ++i) {
      long long jlo = 0, jhi = N;   // stored columns [jlo, jhi)
      if (p.flags & kOutUpper) jlo = i;
      if (p.flags & kOutLower) jhi = std::min(N, i + 1);
      if (!b_dep) {
        const long long len = std::max(0LL, ke_a(i) - kb_a(i));
        total += (double)len * std::max(0LL, jhi - jlo);
      } else {
        // B's band depends on j: lower (k >= j) or upper (k <= j); sum the piecewise
        // linear length over j in [jlo, jhi) in closed form
        const long long a0 = kb_a(i), a1 = ke_a(i);
        auto sum_range = [](long long lo, long long hi, long long c0, long long c1) {
          // sum over j in [lo, hi) of (c0 + c1 * j)
          if (hi <= lo) return 0.0;
          const double n = (double)(hi - lo);
          return n * c0 + c1 * (double)(lo + hi - 1) * n / 2.0;
        };
        if (p.flags & kBLower) {
          // len = a1 - max(a0, j) for j < a1
          const long long hi = std::min(jhi, a1);
          total += sum_range(jlo, std::min(hi, a0), a1 - a0, 0);
          total += sum_range(std::max(jlo, a0), hi, a1, -1);
        } else {
          // kBUpper: len = min(a1, j + 1) - a0 for j + 1 > a0
          const long long lo = std::max(jlo, a0);
          total += sum_range(lo, std::min(jhi, a1), 1 - a0, 1);
          total += sum_range(std::max(lo, a1), jhi, a1 - a0, 0);
        }
      }
    }
  }
  return 2.0 * total * nseg * p.nb1 * p.nb2;
}

template <class T>
void gemm_any(hipStream_t s, const GemmProblemT<T>* probs, int count) {
  bool big = true;
  long long tiles128 = 0;
  int live = 0;
  for (int q = 0; q < count; ++q) {
    const GemmProblemT<T>& p = probs[q];
    if (p.M <= 0 || p.N <= 0 || p.nb1 <= 0 || p.nb2 <= 0) continue;
    ++live;
    if (p.M % 64 || p.N % 64 || p.K % BK || (p.kseg > 0 && p.kseg % BK))
      throw HipError{hipErrorInvalidValue, "gemm_f64: dimensions must be multiples of the tile"};
    if ((p.flags & (kOutUpper | kOutLower)) && p.M != p.N)
      throw HipError{hipErrorInvalidValue, "gemm_f64: triangular output needs M == N"};
    if (p.kseg > 0 && (p.nseg < 1 || p.nseg > kMaxSeg || p.kseg * p.nseg != p.K))
      throw HipError{hipErrorInvalidValue, "gemm_f64: bad K segmentation"};
    if (p.ksplit < 1 || (p.ksplit > 1 && (p.nb1 * p.nb2 != 1 || !p.ws)))
      throw HipError{hipErrorInvalidValue, "gemm_f64: bad split-K setup"};
    if (p.ksplit > 1 && (p.alpha_b || p.beta_b))
      throw HipError{hipErrorInvalidValue, "gemm_f64: per-entry scalars with split-K"};
    // the tiles move every operand as 16-byte vectors
    constexpr long long vw = 16 / sizeof(T);
    auto al = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) % 16) == 0; };
    bool ok = al(p.A) && al(p.B) && al(p.D) && (!p.C || al(p.C)) && (!p.ws || al(p.ws)) &&
              p.lda % vw == 0 && p.ldb % vw == 0 && p.ldc % vw == 0 && p.ldd % vw == 0;
    for (int d = 0; d < 2; ++d)
      ok = ok && p.sA[d] % vw == 0 && p.sB[d] % vw == 0 && p.sC[d] % vw == 0 && p.sD[d] % vw == 0;
    if (!ok) throw HipError{hipErrorInvalidValue, "gemm: operands not 16-byte aligned"};
    if (p.M % 128 || p.N % 128 || std::min(p.M, p.N) < 512) big = false;
    const long long tm = p.M / 128, tn = p.N / 128;
    tiles128 += ((p.flags & (kOutUpper | kOutLower)) ? tm * (tm + 1) / 2 : tm * tn) *
                p.ksplit * p.nb1 * p.nb2;
  }
  if (!live) return;
  // triangular operands with a full output: the K extents of the tiles differ by up to
  // the whole K, and while there are few large tiles per compute unit one with the
  // longest K bounds the launch; small tiles spread that work four times finer.  Two
  // triangular operands (K from max(i0, j0), or up to min) skew it most.
  int skew = 0;
  for (int q = 0; q < count; ++q) {
    const int f = probs[q].flags;
    if (f & (kOutUpper | kOutLower)) continue;
    const int na = (f & (kAUpper | kALower)) ? 1 : 0, nb = (f & (kBUpper | kBLower)) ? 1 : 0;
    skew = std::max(skew, na + nb);
  }
  const long long skew_max = skew == 2 ? 2048 : (skew == 1 ? 512 : 0);
  if (big && tiles128 >= 256 && tiles128 >= skew_max)
    launch_group<T, 128, 128, 4, 4>(s, probs, count);
  else
    launch_group<T, 64, 64, 2, 2>(s, probs, count);
}

template double gemm_algorithmic_flops<double>(const GemmProblem&);
template double gemm_algorithmic_flops<float>(const GemmProblemF&);

void gemm_f64(hipStream_t s, const GemmProblem* probs, int count) { gemm_any(s, probs, count); }
void gemm_f32(hipStream_t s, const GemmProblemF* probs, int count) { gemm_any(s, probs, count); }

}  // namespace ps
