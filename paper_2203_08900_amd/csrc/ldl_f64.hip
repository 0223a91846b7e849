// Alg. 7 (robust Sigma-orthonormal bases): truncated LDL^T of Z = Sigma P_+ (or of
// -Sigma P_-) with 1x1 pivots and diagonal pivoting.  Z is positive semidefinite with a
// known rank k (Thm. DefDivConq, Thm. EVREalSigmaOrth), so D is diagonal and the basis is
// Q = Sigma C with C = L D^{1/2} restricted to the first k pivots (C C^T = Z).
//
// The factorization goes by panels of 64 pivots.  Choosing each pivot over all rows
// would make every pivot a dependency across the whole matrix; instead one workgroup
// picks the panel's candidates, the 128 largest diagonal entries of the current Schur
// complement (ties: lower index), gathers their 128 x 128 block into LDS and takes the 64
// pivots greedily inside it (largest remaining Schur diagonal, ties: lower index), which
// gives the panel's 64 x 64 pivot factor L_pp.  Every other row then solves
// C(i, panel) L_pp^T = Z(i, pivots) by forward substitution (one thread per row, L_pp
// broadcast from LDS), and the Schur complement takes a rank-64 update on the matrix
// cores.  C keeps the original row order; Z is stored as its upper triangle only.
#include "ps_internal.h"

namespace ps {
namespace {

constexpr int NT = 256;
inline unsigned blocks_for(size_t n) {
  return (unsigned)std::min<size_t>((n + NT - 1) / NT, 8192);
}

constexpr int kPanel = kLdlPanel;         // pivots per panel
constexpr int kCand = kLdlCand;           // candidates per panel
constexpr int kThr = 1024;                // threads of the panel kernel
constexpr int kKeysPerThread = kLdlMaxN / kThr;
constexpr int kTri = kCand * (kCand + 1) / 2;
static_assert(kPanel * (kPanel + 1) <= kTri, "the inverse reuses the candidate block's area");
static_assert(kCand == 2 * 64 && kPanel <= kCand, "two candidate slots per lane of one wave");

// Order-preserving 64-bit key of a double (a larger value has a larger key, -0 and +0 the
// same); key 0 is reserved for rows that are not candidates.
__device__ inline unsigned long long ord_key(double d) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(d + 0.0);
  const unsigned long long k = (u >> 63) ? ~u : (u | 0x8000000000000000ull);
  return k == 0ull ? 1ull : k;
}

// Symmetric access to the upper triangle of Z (column-major, leading dimension np)
__device__ inline double zsym(const double* Z, int np, int i, int j) {
  return i <= j ? Z[i + (size_t)j * np] : Z[j + (size_t)i * np];
}

__device__ inline int tri_at(int a, int b) {   // packed lower triangle, a, b < kCand
  return a >= b ? a * (a + 1) / 2 + b : b * (b + 1) / 2 + a;
}

// Exclusive prefix sum of one int per thread over the workgroup; *total gets the sum.
__device__ inline int block_excl_scan(int v, int* wsum, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int w = 0; w < kThr / 64; ++w) {
      const int t = wsum[w];
      wsum[w] = run;
      run += t;
    }
    wsum[kThr / 64] = run;
  }
  __syncthreads();
  const int r = wsum[wave] + x - v;
  *total = wsum[kThr / 64];
  __syncthreads();
  return r;
}

// One panel's pivots.  Inputs: Z (upper triangle of the Schur complement), mask (1 for
// rows already pivoted and for padding rows), nb <= 64 pivots wanted.  Outputs:
// piv[0:64] (global row of pivot q, -1 where none), L (64 x 64, column-major: L_pp,
// identity rows beyond the pivots taken), and on a non-positive pivot or too few rows
// info[0] = 1.
__global__ void __launch_bounds__(kThr) ldl_panel_kernel(const double* Z, int np, int n,
                                                         const int* mask, int nb, int* piv,
                                                         double* Lout, int* info) {
  __shared__ double tri[kTri];                  // the candidate block, packed lower triangle
  __shared__ double cbT[kPanel][kCand];         // panel columns of the candidate rows
  __shared__ int cand[kCand];                   // global row of each candidate slot
  __shared__ int pslot[kPanel];                 // candidate slot of pivot q, -1: none
  __shared__ int hist[256];
  __shared__ int wsum[kThr / 64 + 1];
  __shared__ int sel[4];                        // digit, remaining want, count, #candidates
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  // ---- keys of the free rows' Schur diagonals
  unsigned long long key[kKeysPerThread];
  int nfree = 0;
#pragma unroll
  for (int u = 0; u < kKeysPerThread; ++u) {
    const int i = tid + kThr * u;
    key[u] = 0ull;
    if (i < n && !mask[i]) {
      key[u] = ord_key(Z[i + (size_t)i * np]);
      ++nfree;
    }
  }
  int total;
  block_excl_scan(nfree, wsum, &total);
  const int T = min(kCand, total);
  if (T < nb) {   // fewer free rows than pivots wanted (uniform)
    if (tid < kPanel) piv[tid] = -1;
    if (tid == 0) info[0] = 1;
    for (int e = tid; e < kPanel * kPanel; e += kThr) {
      const int i = e % kPanel, j = e / kPanel;
      Lout[e] = (i == j) ? 1.0 : 0.0;
    }
    return;
  }

  // ---- the T-th largest key, eight bits at a time from the top
  unsigned long long prefix = 0ull, pmask = 0ull;
  int want = T, eqcount = 0;
  for (int pass = 0; pass < 8; ++pass) {
    const int shift = 56 - 8 * pass;
    if (tid < 256) hist[tid] = 0;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kKeysPerThread; ++u)
      if (key[u] != 0ull && (key[u] & pmask) == prefix)
        atomicAdd(&hist[(int)((key[u] >> shift) & 255ull)], 1);
    __syncthreads();
    if (wave == 0) {
      int c[4], s = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        c[q] = hist[4 * lane + q];
        s += c[q];
      }
      // entries in the bins above this lane's four
      int above = s;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_down(above, o, 64);
        if (lane + o < 64) above += y;
      }
      above -= s;
      if (above < want && want <= above + s) {
        int cum = above;
        for (int q = 3; q >= 0; --q) {
          if (cum + c[q] >= want) {
            sel[0] = 4 * lane + q;
            sel[1] = want - cum;
            sel[2] = c[q];
            break;
          }
          cum += c[q];
        }
      }
    }
    __syncthreads();
    prefix |= (unsigned long long)sel[0] << shift;
    pmask |= 255ull << shift;
    want = sel[1];
    eqcount = sel[2];
    __syncthreads();
  }
  // ---- candidates: every key above the threshold, and the `want` lowest-index rows
  // whose key equals it (T of them; the count is capped and re-read, so a slot is only
  // used once written).  The ranks among equal keys need a scan only when some of them
  // are left out (uniform branch).
  if (tid == 0) sel[3] = 0;
  if (tid < kCand) cand[tid] = -1;
  const bool all_eq = want == eqcount;
  const int kpt = (np + kThr - 1) / kThr;
  int eqbase = 0;
#pragma unroll
  for (int u = 0; u < kKeysPerThread; ++u) {
    if (u < kpt) {
      const int eq = key[u] == prefix ? 1 : 0;
      int rank = 0;
      if (!all_eq) {
        int tot;
        rank = eqbase + block_excl_scan(eq, wsum, &tot);
        eqbase += tot;
      }
      const bool take = key[u] > prefix || (eq && rank < want);
      if (take) {
        const int slot = atomicAdd(&sel[3], 1);
        if (slot < kCand) cand[slot] = tid + kThr * u;
      }
    }
  }
  __syncthreads();
  const int nc = min(T, sel[3]);   // equal to T

  // ---- the candidate block (lower triangle) into LDS
  for (int e = tid; e < kTri; e += kThr) {
    int a = (int)((sqrtf(8.0f * e + 1.0f) - 1.0f) * 0.5f);
    while (a * (a + 1) / 2 > e) --a;
    while ((a + 1) * (a + 2) / 2 <= e) ++a;
    const int b = e - a * (a + 1) / 2;
    tri[e] = (a < nc && cand[a] >= 0 && cand[b] >= 0) ? zsym(Z, np, cand[a], cand[b]) : 0.0;
  }
  __syncthreads();

  // ---- greedy pivots inside the block (one wave; lane l owns slots l and l + 64)
  if (wave == 0) {
    const int a0 = lane, a1 = lane + 64;
    bool f0 = a0 < nc && cand[a0] >= 0, f1 = a1 < nc && cand[a1] >= 0;
    double d0 = f0 ? tri[tri_at(a0, a0)] : 0.0;
    double d1 = f1 ? tri[tri_at(a1, a1)] : 0.0;
    const int g0 = f0 ? cand[a0] : 0x7fffffff, g1 = f1 ? cand[a1] : 0x7fffffff;
    int taken = 0;
    for (int jj = 0; jj < nb; ++jj) {
      // argmax of the free slots' Schur diagonals, ties to the lower row
      // (a NaN diagonal never wins, so every lane reaches the same winner)
      double bd = -INFINITY;
      int bg = 0x7fffffff, bs = -1;
      if (f0 && d0 == d0) { bd = d0; bg = g0; bs = a0; }
      if (f1 && d1 == d1 && (d1 > bd || (d1 == bd && g1 < bg))) { bd = d1; bg = g1; bs = a1; }
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        const double od = __shfl_xor(bd, o, 64);
        const int og = __shfl_xor(bg, o, 64), os = __shfl_xor(bs, o, 64);
        if (od > bd || (od == bd && og < bg)) { bd = od; bg = og; bs = os; }
      }
      if (!(bd > 0.0) || bs < 0) break;   // uniform: every lane has the same winner
      const int p = bs;
      const double sq = sqrt(bd), inv = 1.0 / sq;
      double c0 = 0.0, c1 = 0.0;
      // both slots' dot products with the pivot row in one pass over the earlier
      // columns (consecutive lanes read consecutive candidates: no bank conflicts), two
      // partial sums per slot
      double s0 = 0.0, s1 = 0.0, t0 = 0.0, t1 = 0.0;
      int j = 0;
#pragma unroll 2
      for (; j + 1 < jj; j += 2) {
        const double pj = cbT[j][p], pk = cbT[j + 1][p];
        s0 += cbT[j][a0] * pj;
        s1 += cbT[j][a1] * pj;
        t0 += cbT[j + 1][a0] * pk;
        t1 += cbT[j + 1][a1] * pk;
      }
      if (j < jj) {
        const double pj = cbT[j][p];
        s0 += cbT[j][a0] * pj;
        s1 += cbT[j][a1] * pj;
      }
      if (a0 == p) c0 = sq;
      else if (f0) c0 = (tri[tri_at(a0, p)] - (s0 + t0)) * inv;
      if (a1 == p) c1 = sq;
      else if (f1) c1 = (tri[tri_at(a1, p)] - (s1 + t1)) * inv;
      cbT[jj][a0] = c0;
      cbT[jj][a1] = c1;
      if (a0 == p) f0 = false;
      else if (f0) d0 -= c0 * c0;
      if (a1 == p) f1 = false;
      else if (f1) d1 -= c1 * c1;
      if (lane == 0) pslot[jj] = p;
      taken = jj + 1;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (lane == 0 && taken < nb) info[0] = 1;
    for (int q = taken + lane; q < kPanel; q += 64) pslot[q] = -1;
  }
  __syncthreads();

  // ---- outputs: pivots, L_pp (identity rows beyond the pivots taken)
  if (tid < kPanel) piv[tid] = pslot[tid] >= 0 ? cand[pslot[tid]] : -1;
  for (int e = tid; e < kPanel * kPanel; e += kThr) {
    const int i = e % kPanel, j = e / kPanel;
    const int ps = pslot[i];
    Lout[e] = ps >= 0 ? (j <= i ? cbT[j][ps] : 0.0) : (i == j ? 1.0 : 0.0);
  }
}

// The panel's columns of every row: rows pivoted in earlier panels get zeros, the
// panel's pivot rows get L_pp, and every other row i solves c L_pp^T = Z(i, pivots) by
// forward substitution (one thread per row, c in registers, L_pp and the reciprocals of
// its diagonal broadcast from LDS); the pivot rows are marked pivoted.
__global__ void __launch_bounds__(64) ldl_rows_kernel(const double* Z, int np, double* Cp,
                                                      int* mask, const int* piv,
                                                      const double* L) {
  __shared__ double Ls[kPanel][kPanel + 1];
  __shared__ double rd[kPanel];
  __shared__ int pv[kPanel];
  for (int e = threadIdx.x; e < kPanel * kPanel; e += blockDim.x)
    Ls[e % kPanel][e / kPanel] = L[e];
  pv[threadIdx.x] = piv[threadIdx.x];
  __syncthreads();
  rd[threadIdx.x] = 1.0 / Ls[threadIdx.x][threadIdx.x];
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  int q = -1;
  for (int t = 0; t < kPanel; ++t)
    if (pv[t] == i) q = t;
  double* out = Cp + i;
  if (q >= 0) {
    for (int j = 0; j < kPanel; ++j) out[(size_t)j * np] = j <= q ? Ls[q][j] : 0.0;
    mask[i] = 1;
    return;
  }
  if (mask[i] != 0) {
    for (int j = 0; j < kPanel; ++j) out[(size_t)j * np] = 0.0;
    return;
  }
  double c[kPanel];
#pragma unroll
  for (int j = 0; j < kPanel; ++j) c[j] = pv[j] >= 0 ? zsym(Z, np, i, pv[j]) : 0.0;
#pragma unroll
  for (int j = 0; j < kPanel; ++j) {
    double sacc = c[j];
#pragma unroll
    for (int k = 0; k < j; ++k) sacc -= c[k] * Ls[j][k];
    c[j] = pv[j] >= 0 ? sacc * rd[j] : 0.0;
  }
#pragma unroll
  for (int j = 0; j < kPanel; ++j) out[(size_t)j * np] = c[j];
}

__global__ void ldl_mask_kernel(int* mask, int n, int np) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += gridDim.x * blockDim.x)
    mask[i] = i < n ? 0 : 1;
}

// Upper triangle of Z = (Sigma S + a Sigma)/2 for the Casida form: Sigma = diag(I, -I),
// Sigma S = [[A_s, B_s], [B_s, A_s]] (symmetrized), n = 2m, padding zero.
__global__ void ldl_form_casida_kernel(const double* as, const double* bs, int m, int mp, int np,
                                       double a, double* Z) {
  const size_t tot = (size_t)np * np;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % np), j = (int)(e / np);
    double v = 0.0;
    if (i <= j && j < 2 * m) {
      const int ii = i < m ? i : i - m, jj = j < m ? j : j - m;
      const double* X = ((i < m) == (j < m)) ? as : bs;
      v = 0.25 * (X[ii + (size_t)jj * mp] + X[jj + (size_t)ii * mp]);
      if (i == j) v += 0.5 * a * (i < m ? 1.0 : -1.0);
    }
    Z[e] = v;
  }
}

// Upper triangle of Z = (Sigma S + a Sigma)/2 for a general signature (S: n x n, ld np)
__global__ void ldl_form_general_kernel(const double* S, const double* sg, int n, int np, double a,
                                        double* Z) {
  const size_t tot = (size_t)np * np;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % np), j = (int)(e / np);
    double v = 0.0;
    if (i <= j && j < n) {
      v = 0.25 * (sg[i] * S[i + (size_t)j * np] + sg[j] * S[j + (size_t)i * np]);
      if (i == j) v += 0.5 * a * sg[i];
    }
    Z[e] = v;
  }
}

// Casida basis from the factor (ld np): Q_+ = Sigma C, top = C(0:m, :), bottom
// = -C(m:2m, :), and the mix [(top + bottom), (top - bottom)] / sqrt(2) of the
// decoupling; padding zero
__global__ void ldl_casida_out_kernel(const double* C, int np, int m, int mp, double* top,
                                      double* qbot, double* ab) {
  const size_t n = (size_t)mp * mp;
  const double h = 0.70710678118654752440;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % mp), j = (int)(e / mp);
    double tv = 0.0, bv = 0.0;
    if (i < m && j < m) {
      tv = C[i + (size_t)j * np];
      bv = -C[m + i + (size_t)j * np];
    }
    top[e] = tv;
    qbot[e] = bv;
    ab[e] = h * (tv + bv);
    ab[n + e] = h * (tv - bv);
  }
}

// Q = Sigma C for a general signature (rows beyond n zero), np x kp
__global__ void ldl_scale_rows_kernel(const double* C, int np, int kp, const double* sg, int n,
                                      double* Q) {
  const size_t tot = (size_t)np * kp;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % np);
    Q[e] = i < n ? sg[i] * C[e] : 0.0;
  }
}

}  // namespace

void ldl_factor(hipStream_t s, double* Z, int n, int np, int k, double* C, const LdlScratch& w,
                int* info) {
  if (k <= 0) return;
  if (np > kLdlMaxN || np % 64 != 0 || n > np)
    throw HipError{hipErrorInvalidValue, "ldl_factor: size"};
  hipLaunchKernelGGL(ldl_mask_kernel, dim3(blocks_for(np)), dim3(NT), 0, s, w.mask, n, np);
  PS_HIP(hipGetLastError());
  for (int t0 = 0; t0 < k; t0 += kPanel) {
    const int nb = std::min(kPanel, k - t0);
    int* pv = w.piv + t0;
    hipLaunchKernelGGL(ldl_panel_kernel, dim3(1), dim3(kThr), 0, s, Z, np, n, w.mask, nb, pv, w.L,
                       info);
    PS_HIP(hipGetLastError());
    double* Cp = C + (size_t)t0 * np;
    hipLaunchKernelGGL(ldl_rows_kernel, dim3((np + 63) / 64), dim3(64), 0, s, Z, np, Cp, w.mask,
                       pv, w.L);
    PS_HIP(hipGetLastError());
    if (t0 + kPanel < k) {   // Schur complement, upper triangle, in place
      GemmProblem pu = gemm_problem(np, np, kPanel, Cp, np, 0, Cp, np, 1, Z, np, -1.0, 1.0, Z, np,
                                    kOutUpper);
      gemm_f64(s, pu);
    }
  }
}

void ldl_form_casida(hipStream_t s, const double* as, const double* bs, int m, int mp, int np,
                     double a, double* Z) {
  hipLaunchKernelGGL(ldl_form_casida_kernel, dim3(blocks_for((size_t)np * np)), dim3(NT), 0, s, as,
                     bs, m, mp, np, a, Z);
  PS_HIP(hipGetLastError());
}

void ldl_form_general(hipStream_t s, const double* S, const double* sg, int n, int np, double a,
                      double* Z) {
  hipLaunchKernelGGL(ldl_form_general_kernel, dim3(blocks_for((size_t)np * np)), dim3(NT), 0, s, S,
                     sg, n, np, a, Z);
  PS_HIP(hipGetLastError());
}

void ldl_casida_out(hipStream_t s, const double* C, int np, int m, int mp, double* top,
                    double* qbot, double* ab) {
  hipLaunchKernelGGL(ldl_casida_out_kernel, dim3(blocks_for((size_t)mp * mp)), dim3(NT), 0, s, C,
                     np, m, mp, top, qbot, ab);
  PS_HIP(hipGetLastError());
}

void ldl_scale_rows(hipStream_t s, const double* C, int np, int kp, const double* sg, int n,
                    double* Q) {
  hipLaunchKernelGGL(ldl_scale_rows_kernel, dim3(blocks_for((size_t)np * kp)), dim3(NT), 0, s, C,
                     np, kp, sg, n, Q);
  PS_HIP(hipGetLastError());
}

}  // namespace ps
