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
  int group;   // > 0: XCD x runs groups of `group` consecutive logical tiles (see the kernel)
  int total;
  GemmProblemT<T> p[kMaxGroup];
};

// The operand transposes are per problem, so one launch covers a group of problems
// with different transposes (each workgroup branches once, uniformly).
template <class T, int BM, int BN, int WM, int WN, bool kUseC>
__global__ __launch_bounds__(WM * WN * 64) void gemm_mfma_kernel(GemmGroup<T> g) {
  __shared__ __attribute__((aligned(16))) T smem[2 * GemmLds<BM, BN>::ASZ + 2 * GemmLds<BM, BN>::BSZ];
  int bid = blockIdx.x;
  if (g.group > 0) {
    // dispatch is round-robin over 8 XCDs: block b runs on XCD b % 8 as that XCD's
    // (b / 8)-th block.  Deal the logical tiles to the XCDs in groups of g.group
    // consecutive ones (group total / 8: XCD x takes [x * total/8, (x+1) * total/8));
    // blocks past the last whole round of groups keep their own index.
    const int gs = g.group, full = g.total / (8 * gs) * (8 * gs);
    if (bid < full) {
      const int x = bid & 7, q = bid >> 3;
      bid = ((q / gs) * 8 + x) * gs + q % gs;
    }
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

// Stream-K schedule for single problems whose tiles cannot share the machine evenly
// (symmetric outputs, triangular operands, fewer tiles than compute units): the K steps
// of all tiles, in tile order, are cut into gridDim.x equal ranges, one per workgroup.
// A workgroup finishes the tiles its range covers whole; of a tile it covers in part it
// writes alpha times the partial product to its slot (2w for the first tile of its
// range, 2w + 1 for the last).  The reduction then sums, per tile, the slots of the
// workgroups that covered it, in workgroup order (deterministic), and applies the
// epilogue; no workgroup waits for another.
template <class T, int BM, int BN, int WM, int WN, int TA, int TB, bool kUseC>
__global__ __launch_bounds__(WM * WN * 64) void gemm_streamk_kernel(GemmProblemT<T> P, long long U,
                                                                    T* slots) {
  __shared__ __attribute__((aligned(16))) T smem[2 * GemmLds<BM, BN>::ASZ + 2 * GemmLds<BM, BN>::BSZ];
  const int w = blockIdx.x, nw = gridDim.x;
  const long long u0 = U * w / nw, u1 = U * (w + 1) / nw;
  const int nseg = P.kseg > 0 ? P.nseg : 1;
  long long c = 0;
  for (int t = 0; t < P.tiles && c < u1; ++t) {
    int I, J, kb;
    tile_coords<BM, BN>(P, t, I, J);
    const long long n = (long long)tile_band<BM, BN>(P, I, J, kb) * nseg;
    if (n > 0 && c + n > u0) {
      const int a = (int)((u0 > c ? u0 : c) - c), b = (int)((u1 < c + n ? u1 : c + n) - c);
      T* part = (a == 0 && b == n) ? nullptr
                                   : slots + (long long)(u0 >= c ? 2 * w : 2 * w + 1) * BM * BN;
      gemm_tile_run<T, BM, BN, WM, WN, TA, TB, kUseC>(P, 0, I, J, a, b, 0, part, smem);
    }
    c += n;
  }
}

// One tile per workgroup: tiles that one workgroup finished are skipped; the others are
// the sum of their partial tiles (none for a tile with no K steps) plus beta C.
template <class T, int BM, int BN, int NT>
__global__ __launch_bounds__(NT) void gemm_streamk_reduce_kernel(GemmProblemT<T> P, long long U,
                                                                 const T* slots, int nwg) {
  constexpr int VW = VecT<T>::VW;
  using vec_t = typename VecT<T>::type;
  constexpr int LDD = BM + VW;
  constexpr int OV = BM * BN / (VW * NT);
  __shared__ __attribute__((aligned(16))) T Ds[BN * LDD];
  const int t = blockIdx.x;
  const int nseg = P.kseg > 0 ? P.nseg : 1;
  // K steps before this tile, counted by the threads together
  long long part_c = 0;
  for (int tt = threadIdx.x; tt < t; tt += blockDim.x) {
    int I, J, kb;
    tile_coords<BM, BN>(P, tt, I, J);
    part_c += (long long)tile_band<BM, BN>(P, I, J, kb) * nseg;
  }
  __shared__ long long red[NT / 64];
  for (int off = 32; off > 0; off >>= 1) part_c += __shfl_down(part_c, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part_c;
  __syncthreads();
  long long c = 0;
  for (int i = 0; i < NT / 64; ++i) c += red[i];
  int I, J, kb;
  tile_coords<BM, BN>(P, t, I, J);
  const long long n = (long long)tile_band<BM, BN>(P, I, J, kb) * nseg;
  auto owner = [&](long long x) {
    long long w = x * nwg / U;
    while (w + 1 < nwg && U * (w + 1) / nwg <= x) ++w;
    while (w > 0 && U * w / nwg > x) --w;
    return (int)w;
  };
  int wf = 0, wl = -1;
  if (n > 0) {
    wf = owner(c);
    wl = owner(c + n - 1);
    if (wf == wl) return;   // finished by one workgroup
  }
  const int tid = threadIdx.x;
#pragma unroll
  for (int qv = 0; qv < OV; ++qv) {
    const int e = tid + qv * NT, iv = e % (BM / VW), j = e / (BM / VW);
    double sum[VW];
#pragma unroll
    for (int u = 0; u < VW; ++u) sum[u] = 0.0;
    for (int w = wf; w <= wl; ++w) {
      const int slot = (U * w / nwg >= c) ? 2 * w : 2 * w + 1;
      const vec_t x = *reinterpret_cast<const vec_t*>(slots + (long long)slot * BM * BN + VW * iv + (long long)j * BM);
#pragma unroll
      for (int u = 0; u < VW; ++u) sum[u] += (double)x[u];
    }
#pragma unroll
    for (int u = 0; u < VW; ++u) Ds[j * LDD + VW * iv + u] = (T)sum[u];
  }
  __syncthreads();
  const vec_t none[1] = {};
  tile_epilogue<T, BM, BN, NT>(P, 0, I, J, Ds, 1.0, P.beta, false, none);
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
thread_local const GemmTuneTable* g_tune = nullptr;
thread_local const GemmChoice* g_force = nullptr;
thread_local GemmLog* g_log = nullptr;

// FNV-1a over the launch's problem shapes
template <class T>
unsigned long long launch_key(const GemmProblemT<T>* probs, int count) {
  unsigned long long h = 1469598103934665603ull;
  auto mix = [&](long long v) {
    for (int b = 0; b < 8; ++b) {
      h ^= (unsigned long long)((v >> (8 * b)) & 0xff);
      h *= 1099511628211ull;
    }
  };
  mix(sizeof(T));
  mix(count);
  for (int q = 0; q < count; ++q) {
    const GemmProblemT<T>& p = probs[q];
    for (long long v : {(long long)p.M, (long long)p.N, (long long)p.K, (long long)p.flags,
                        (long long)p.tA, (long long)p.tB, (long long)p.nb1, (long long)p.nb2,
                        (long long)p.kseg, (long long)p.nseg, (long long)p.ksplit,
                        (long long)(p.alpha_b != nullptr), (long long)(p.beta_b != nullptr),
                        (long long)(p.beta != 0.0), (long long)(p.ws_slots > 0)})
      mix(v);
  }
  return h;
}

void log_launch(const GemmProblemT<double>* probs, int count, unsigned long long key) {
  g_log->keys.push_back(key);
  g_log->p64.emplace_back(probs, probs + count);
  g_log->p32.emplace_back();
}
void log_launch(const GemmProblemT<float>* probs, int count, unsigned long long key) {
  g_log->keys.push_back(key);
  g_log->p64.emplace_back();
  g_log->p32.emplace_back(probs, probs + count);
}

// Whether the one-range-per-XCD placement (XCD x runs logical tiles [x * total/8,
// (x+1) * total/8)) gives every XCD within 10 % of the mean number of K steps.  Only for
// launches whose batch entries are laid out one after another (no triangular operands
// with a full output).
template <class T, int BM, int BN>
bool xcd_ranges_balanced(const GemmGroup<T>& g) {
  const int per = g.total / 8;
  long long wx[8] = {}, sum = 0;
  int pi = 0;
  for (int b = 0; b < g.total; ++b) {
    while (pi + 1 < g.count && b >= g.p[pi + 1].tile_begin) ++pi;
    const GemmProblemT<T>& P = g.p[pi];
    const int tz = (b - P.tile_begin) % P.tiles_per_batch;
    const int ks = tz / P.tiles, t = tz - ks * P.tiles;
    int I, J, kb;
    tile_coords<BM, BN>(P, t, I, J);
    const long long n = (long long)tile_band<BM, BN>(P, I, J, kb) * (P.kseg > 0 ? P.nseg : 1);
    const long long w = n * (ks + 1) / P.ksplit - n * ks / P.ksplit;
    wx[b / per] += w;
    sum += w;
  }
  for (int x = 0; x < 8; ++x)
    if (80 * wx[x] > 11 * sum) return false;
  return true;
}

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
  // XCD placement.  Tiles of equal K take one contiguous range of tiles per XCD, so each
  // XCD's L2 serves a compact part of the operands.  Triangular operands make the K
  // extents differ and enumerate the tiles longest first, so such ranges can differ in
  // work several-fold (an N = W W^T product at m = 8192 ran twice as long); they keep the
  // ranges only while those are balanced, else groups of 4 tiles go round-robin.  With a
  // full output they interleave batch entries and take the plain round-robin dispatch.
  bool tri_full = false, tri_any = false;
  for (int q = 0; q < g.count; ++q) {
    const int f = g.p[q].flags;
    const bool tri = f & (kAUpper | kALower | kBUpper | kBLower);
    tri_any = tri_any || tri;
    tri_full = tri_full || (tri && !(f & (kOutUpper | kOutLower)));
  }
  g.group = (total % 8 == 0 && total >= 64) ? total / 8 : 0;
  if (tri_full)
    g.group = 0;
  else if (tri_any && g.group > 0 && !xcd_ranges_balanced<T, BM, BN>(g))
    g.group = 4;
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

// Large tiles on a stream-K schedule (see gemm_streamk_kernel), one launch pair per
// problem, for groups of single problems with a symmetric output (too few tiles for the
// machine) and a long K, when a problem's workspace can hold the partial tiles: each
// workgroup then gets a long K range, and the schedule replaces a uniform split-K whose
// partial tiles cost more traffic.  With short ranges (a few dozen K steps per
// workgroup) the staggered K positions of the workgroups share the caches worse than
// the full tiles in lockstep do, and triangular operands (K differing per tile) measure
// faster on the small tiles, so those stay on the regular schedule.  Returns false
// (nothing launched) when the schedule does not apply.
template <class T, int TA, int TB>
void streamk_one(hipStream_t s, const GemmProblemT<T>& p, long long units, T* slots, int nwg) {
  constexpr int BM = 128, BN = 128;
  if (p.beta != 0.0)
    hipLaunchKernelGGL((gemm_streamk_kernel<T, BM, BN, 4, 4, TA, TB, true>), dim3(nwg), dim3(1024), 0,
                       s, p, units, slots);
  else
    hipLaunchKernelGGL((gemm_streamk_kernel<T, BM, BN, 4, 4, TA, TB, false>), dim3(nwg), dim3(1024),
                       0, s, p, units, slots);
  PS_HIP(hipGetLastError());
  hipLaunchKernelGGL((gemm_streamk_reduce_kernel<T, BM, BN, 1024>), dim3(p.tiles), dim3(1024), 0, s,
                     p, units, slots, nwg);
  PS_HIP(hipGetLastError());
}

template <class T>
bool launch_streamk(hipStream_t s, const GemmProblemT<T>* probs, int count) {
  constexpr int BM = 128, BN = 128, NWG = 256;   // one 16-wave workgroup per compute unit
  GemmProblemT<T> ps[kMaxGroup];
  long long units[kMaxGroup];
  int n = 0, total = 0;
  bool skew = false;
  T* ws = nullptr;
  long long ws_elems = 0;
  for (int q = 0; q < count; ++q) {
    GemmProblemT<T> p = probs[q];
    if (p.M <= 0 || p.N <= 0) continue;
    if (p.nb1 * p.nb2 != 1 || p.alpha_b || p.beta_b) return false;
    if (!ws && p.ws && p.ws_slots > 0) {
      ws = p.ws;
      ws_elems = (long long)p.ws_slots * p.M * p.N;
    }
    if (p.flags & (kAUpper | kALower | kBUpper | kBLower)) return false;
    if (p.flags & (kOutUpper | kOutLower)) skew = true;
    p.ksplit = 1;
    p.tm = p.M / BM;
    p.tn = p.N / BN;
    p.tiles = (p.flags & (kOutUpper | kOutLower)) ? p.tm * (p.tm + 1) / 2 : p.tm * p.tn;
    p.tiles_per_batch = p.tiles;
    p.tile_begin = 0;
    total += p.tiles;
    const int nseg = p.kseg > 0 ? p.nseg : 1;
    long long u = 0;
    for (int t = 0; t < p.tiles; ++t) {
      int I, J, kb;
      tile_coords<BM, BN>(p, t, I, J);
      u += (long long)tile_band<BM, BN>(p, I, J, kb) * nseg;
    }
    if (u < 128LL * NWG) return false;   // K steps per workgroup
    units[n] = u;
    ps[n++] = p;
  }
  if (n == 0 || !(skew || total < NWG)) return false;
  if (!ws || ws_elems < 2LL * NWG * BM * BN) return false;
  const int slot = krec_begin(s);
  for (int q = 0; q < n; ++q) {
    const int v = ps[q].tA * 2 + ps[q].tB;
    if (v == 0)
      streamk_one<T, 0, 0>(s, ps[q], units[q], ws, NWG);
    else if (v == 1)
      streamk_one<T, 0, 1>(s, ps[q], units[q], ws, NWG);
    else if (v == 2)
      streamk_one<T, 1, 0>(s, ps[q], units[q], ws, NWG);
    else
      streamk_one<T, 1, 1>(s, ps[q], units[q], ws, NWG);
  }
  if (slot >= 0) {
    double f = 0.0;
    for (int q = 0; q < n; ++q) f += gemm_algorithmic_flops(ps[q]);
    krec_end(s, slot, std::is_same<T, float>::value ? kKcGemm32 : kKcGemm128, f);
  }
  return true;
}

}  // namespace

void kernel_set_recorder(KernelRecorder* r) { g_rec = r; }
void gemm_set_tuning(const GemmTuneTable* t) { g_tune = t; }
const GemmTuneTable* gemm_get_tuning() { return g_tune; }
void gemm_set_force(const GemmChoice* c) { g_force = c; }
void gemm_set_log(GemmLog* log) { g_log = log; }
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
  const unsigned long long key = launch_key(probs, count);
  if (g_log) log_launch(probs, count, key);
  const GemmChoice* c = g_force;
  if (!c && g_tune)
    for (size_t i = 0; i < g_tune->keys.size(); ++i)
      if (g_tune->keys[i] == key) c = &g_tune->choices[i];
  if (c) {   // a tuned (or, while tuning, a trial) choice, made legal per problem
    GemmProblemT<T> ps[kMaxGroup];
    for (int q = 0; q < count; ++q) {
      ps[q] = probs[q];
      const GemmProblemT<T>& p = probs[q];
      const bool can_split = p.nb1 * p.nb2 == 1 && p.ws && p.ws_slots >= c->ksplit &&
                             !p.alpha_b && !p.beta_b && p.K / BK >= 4 * c->ksplit;
      ps[q].ksplit = (c->ksplit > 1 && can_split) ? c->ksplit : (c->ksplit > 1 ? p.ksplit : 1);
    }
    if (c->streamk && big && launch_streamk<T>(s, ps, count)) return;
    if (c->tile == 128 && big)
      launch_group<T, 128, 128, 4, 4>(s, ps, count);
    else
      launch_group<T, 64, 64, 2, 2>(s, ps, count);
    return;
  }
  if (big && launch_streamk<T>(s, probs, count)) return;
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
