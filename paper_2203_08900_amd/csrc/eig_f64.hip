// Kernels of the full eigen-decomposition: the symmetric divide-and-conquer (Alg. 2)
// on H_+ with the Cholesky bases of Alg. 4, its small leaves, and the assembly of
// the eigenpairs of H from those of H_+ (Thm. DefDivConq, Thm. EVREalSigmaOrth).
//
// Subproblem sizes are arbitrary (they follow the ranks of the projectors), so the
// copy kernels here move between the padded layout of the matrix-core kernels
// (multiples of 64, zero or identity padding) and arbitrary column offsets and
// row index lists.
#include "ps_internal.h"

namespace ps {

namespace {
constexpr int NT = 256;
inline unsigned grid_for(size_t n) {
  size_t b = (n + NT - 1) / NT;
  return (unsigned)(b > 65535u * 64u ? 65535u * 64u : (b ? b : 1));
}
#define PS_GRID_LOOP(e, n) \
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < (n); e += (size_t)gridDim.x * blockDim.x)
}  // namespace

__global__ void shift_diag_kernel(double* y, int ld, int n, double b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i + (size_t)i * ld] += b;
}

void shift_diag(hipStream_t s, double* y, int ld, int n, double b) {
  if (n <= 0) return;
  hipLaunchKernelGGL(shift_diag_kernel, dim3((n + NT - 1) / NT), dim3(NT), 0, s, y, ld, n, b);
  PS_HIP(hipGetLastError());
}

__global__ void spd_pad_kernel(const double* g, double* z, int n, int np, double c) {
  PS_GRID_LOOP(e, (size_t)np * np) {
    const int i = (int)(e % np), j = (int)(e / np);
    double v = 0.0;
    if (i < j) v = g[e];
    else if (i == j) v = (i < n) ? g[e] + c : 1.0;
    z[e] = v;
  }
}

void spd_pad(hipStream_t s, const double* g, double* z, int n, int np, double c) {
  hipLaunchKernelGGL(spd_pad_kernel, dim3(grid_for((size_t)np * np)), dim3(NT), 0, s, g, z, n,
                     np, c);
  PS_HIP(hipGetLastError());
}

__global__ void get_diag_kernel(const double* x, int ld, int n, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = x[i + (size_t)i * ld];
}

void get_diag(hipStream_t s, const double* x, int ld, int n, double* out) {
  if (n <= 0) return;
  hipLaunchKernelGGL(get_diag_kernel, dim3((n + NT - 1) / NT), dim3(NT), 0, s, x, ld, n, out);
  PS_HIP(hipGetLastError());
}

// Sum of squares of the off-diagonal entries of the leading n x n block (two passes:
// per-workgroup partials, then one workgroup adds them in a fixed order).
constexpr int kOffParts = 256;

__device__ inline double wg_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
  __syncthreads();
  return r;
}

__global__ void offdiag_part_kernel(const double* x, int ld, int n, double* part) {
  __shared__ double sh[NT / 64];
  double q = 0.0;
  PS_GRID_LOOP(e, (size_t)n * n) {
    const int i = (int)(e % n), j = (int)(e / n);
    if (i != j) {
      const double v = x[i + (size_t)j * ld];
      q += v * v;
    }
  }
  const double t = wg_sum(q, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void offdiag_sum_kernel(const double* part, double* out) {
  __shared__ double sh[NT / 64];
  double q = 0.0;
  for (int e = threadIdx.x; e < kOffParts; e += blockDim.x) q += part[e];
  const double t = wg_sum(q, sh);
  if (threadIdx.x == 0) out[0] = t;
}

void offdiag_norm2(hipStream_t s, const double* x, int ld, int n, double* out) {
  // out[0] receives the result; out[1 .. kOffParts] hold the partials
  hipLaunchKernelGGL(offdiag_part_kernel, dim3(kOffParts), dim3(NT), 0, s, x, ld, n, out + 1);
  hipLaunchKernelGGL(offdiag_sum_kernel, dim3(1), dim3(NT), 0, s, out + 1, out);
  PS_HIP(hipGetLastError());
}

__global__ void copy_pad_kernel(const double* src, int lds, int rows, int cols, double* dst,
                                int ldd, int rows_pad, int cols_pad) {
  PS_GRID_LOOP(e, (size_t)rows_pad * cols_pad) {
    const int i = (int)(e % rows_pad), j = (int)(e / rows_pad);
    dst[i + (size_t)j * ldd] = (i < rows && j < cols) ? src[i + (size_t)j * lds] : 0.0;
  }
}

void copy_pad(hipStream_t s, const double* src, int lds, int rows, int cols, double* dst,
              int ldd, int rows_pad, int cols_pad) {
  if (rows_pad <= 0 || cols_pad <= 0) return;
  hipLaunchKernelGGL(copy_pad_kernel, dim3(grid_for((size_t)rows_pad * cols_pad)), dim3(NT), 0,
                     s, src, lds, rows, cols, dst, ldd, rows_pad, cols_pad);
  PS_HIP(hipGetLastError());
}

__global__ void put_cols_kernel(const double* src, int lds, double* dst, int ldd, int o, int n,
                                int rows) {
  PS_GRID_LOOP(e, (size_t)rows * n) {
    const int i = (int)(e % rows), j = (int)(e / rows);
    dst[i + (size_t)(o + j) * ldd] = src[i + (size_t)j * lds];
  }
}

void put_cols(hipStream_t s, const double* src, int lds, double* dst, int ldd, int o, int n,
              int rows) {
  if (n <= 0 || rows <= 0) return;
  hipLaunchKernelGGL(put_cols_kernel, dim3(grid_for((size_t)rows * n)), dim3(NT), 0, s, src, lds,
                     dst, ldd, o, n, rows);
  PS_HIP(hipGetLastError());
}

__global__ void gather_sym_kernel(const double* src, int lds, const int* ri, const int* ci,
                                  int rows, int cols, double sc, double dg, double* dst, int ldd,
                                  int rows_pad, int cols_pad, double padval, int upper_only) {
  PS_GRID_LOOP(e, (size_t)rows_pad * cols_pad) {
    const int i = (int)(e % rows_pad), j = (int)(e / rows_pad);
    double v;
    if (upper_only && i > j) {
      v = 0.0;
    } else if (i < rows && j < cols) {
      const int r = ri[i], c = ci[j];
      v = sc * src[r + (size_t)c * lds] + (r == c ? dg : 0.0);
    } else {
      v = (i == j) ? padval : 0.0;
    }
    dst[i + (size_t)j * ldd] = v;
  }
}

void gather_sym(hipStream_t s, const double* src, int lds, const int* ri, const int* ci, int rows,
                int cols, double sc, double dg, double* dst, int ldd, int rows_pad, int cols_pad,
                double padval, int upper_only) {
  if (rows_pad <= 0 || cols_pad <= 0) return;
  hipLaunchKernelGGL(gather_sym_kernel, dim3(grid_for((size_t)rows_pad * cols_pad)), dim3(NT), 0,
                     s, src, lds, ri, ci, rows, cols, sc, dg, dst, ldd, rows_pad, cols_pad, padval,
                     upper_only);
  PS_HIP(hipGetLastError());
}

__global__ void scatter_rows_kernel(const double* src, int lds, int trans, const int* ri, int rows,
                                    int cols, double* dst, int ldd, int c0) {
  PS_GRID_LOOP(e, (size_t)rows * cols) {
    const int i = (int)(e % rows), j = (int)(e / rows);
    const double v = trans ? src[j + (size_t)i * lds] : src[i + (size_t)j * lds];
    dst[ri[i] + (size_t)(c0 + j) * ldd] = v;
  }
}

void scatter_rows(hipStream_t s, const double* src, int lds, int trans, const int* ri, int rows,
                  int cols, double* dst, int ldd, int c0) {
  if (rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL(scatter_rows_kernel, dim3(grid_for((size_t)rows * cols)), dim3(NT), 0, s,
                     src, lds, trans, ri, rows, cols, dst, ldd, c0);
  PS_HIP(hipGetLastError());
}

__global__ void permute_cols_kernel(const double* src, int lds, const int* perm, int rows,
                                    int cols, double* dst, int ldd) {
  PS_GRID_LOOP(e, (size_t)rows * cols) {
    const int i = (int)(e % rows), j = (int)(e / rows);
    dst[i + (size_t)j * ldd] = src[i + (size_t)perm[j] * lds];
  }
}

void permute_cols(hipStream_t s, const double* src, int lds, const int* perm, int rows, int cols,
                  double* dst, int ldd) {
  if (rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL(permute_cols_kernel, dim3(grid_for((size_t)rows * cols)), dim3(NT), 0, s,
                     src, lds, perm, rows, cols, dst, ldd);
  PS_HIP(hipGetLastError());
}

__global__ void permute_vec_kernel(const double* src, const int* perm, int n, double* dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[perm[i]];
}

void permute_vec(hipStream_t s, const double* src, const int* perm, int n, double* dst) {
  if (n <= 0) return;
  hipLaunchKernelGGL(permute_vec_kernel, dim3((n + NT - 1) / NT), dim3(NT), 0, s, src, perm, n,
                     dst);
  PS_HIP(hipGetLastError());
}

// lam[i] = w[i] and lam[m + i] = -w[i]: the eigenvalues of H come in pairs +-lambda
// (Thm. EVREalSigmaOrth); the positive ones are those of H_+ (Thm. DefDivConq).
__global__ void eig_lambda_kernel(const double* w, int m, double* lam) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) {
    lam[i] = w[i];
    lam[m + i] = -w[i];
  }
}

void eig_lambda(hipStream_t s, const double* w, int m, double* lam) {
  hipLaunchKernelGGL(eig_lambda_kernel, dim3((m + NT - 1) / NT), dim3(NT), 0, s, w, m, lam);
  PS_HIP(hipGetLastError());
}

// V(:, m + j) = Pi V(:, j), Pi = [[0, I], [I, 0]]: the eigenvector of -lambda_j.
__global__ void pi_columns_kernel(double* v, int ldv, int m) {
  PS_GRID_LOOP(e, (size_t)m * m) {
    const int i = (int)(e % m), j = (int)(e / m);
    const double top = v[i + (size_t)j * ldv];
    const double bot = v[m + i + (size_t)j * ldv];
    v[i + (size_t)(m + j) * ldv] = bot;
    v[m + i + (size_t)(m + j) * ldv] = top;
  }
}

void pi_columns(hipStream_t s, double* v, int ldv, int m) {
  hipLaunchKernelGGL(pi_columns_kernel, dim3(grid_for((size_t)m * m)), dim3(NT), 0, s, v, ldv, m);
  PS_HIP(hipGetLastError());
}

// Per column: flip the sign so that the entry of largest modulus (lowest row index on
// ties) is positive.  One workgroup per column.
__global__ __launch_bounds__(NT) void canon_sign_kernel(double* v, int ldv, int rows) {
  __shared__ double bv[NT];
  __shared__ int bi[NT];
  double* col = v + (size_t)blockIdx.x * ldv;
  double best = -1.0;
  int idx = rows;
  for (int i = threadIdx.x; i < rows; i += NT) {
    const double a = fabs(col[i]);
    if (a > best) {   // increasing i within a thread: strict > keeps the lowest index
      best = a;
      idx = i;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = idx;
  __syncthreads();
  for (int off = NT / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      const double b2 = bv[threadIdx.x + off];
      const int i2 = bi[threadIdx.x + off];
      if (b2 > bv[threadIdx.x] || (b2 == bv[threadIdx.x] && i2 < bi[threadIdx.x])) {
        bv[threadIdx.x] = b2;
        bi[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  const int k = bi[0];
  const bool flip = k < rows && col[k] < 0.0;
  __syncthreads();
  if (flip)
    for (int i = threadIdx.x; i < rows; i += NT) col[i] = -col[i];
}

void canon_sign(hipStream_t s, double* v, int ldv, int rows, int cols) {
  if (cols <= 0) return;
  hipLaunchKernelGGL(canon_sign_kernel, dim3(cols), dim3(NT), 0, s, v, ldv, rows);
  PS_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ Jacobi leaves
// Eigen-decomposition of the small symmetric diagonal blocks B(o:o+n, o:o+n), n <= 64,
// one workgroup each: cyclic two-sided Jacobi with the round-robin ordering, so the
// n/2 rotations of a round act on disjoint index pairs and are applied together
// (columns of B and V, then rows of B).  Rotation of the pair (p, q), p < q:
// t = sign(tau) / (|tau| + sqrt(1 + tau^2)), tau = (b_qq - b_pp) / (2 b_pq),
// c = 1/sqrt(1 + t^2), s = t c; afterwards b_pq = 0, b_pp -= t b_pq, b_qq += t b_pq
// exactly.  A pair is rotated when |b_pq| > u sqrt(|b_pp b_qq|) (u = 2^-53); sweeps
// stop when none is.  Output: ascending eigenvalues lam[o..o+n) and the eigenvectors
// in the diagonal block of Z (ld ldz), columns in the same order.
__global__ __launch_bounds__(NT) void jacobi_kernel(const double* B, int ld, const int* lo,
                                                    const int* ln, double* Z, int ldz,
                                                    double* lam, int* sweeps_out, int max_sweeps) {
  __shared__ double a[64][65];
  __shared__ double v[64][65];
  __shared__ double rc[32], rs[32], rt[32], rpq[32], rpp[32], rqq[32];
  __shared__ int rp[32], rq[32];
  __shared__ int rotated;
  __shared__ int order[64];
  const int o = lo[blockIdx.x], n = ln[blockIdx.x];
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * 64; e += NT) {
    const int i = e & 63, j = e >> 6;
    // the upper triangle defines the symmetric block
    a[i][j] = (i < n && j < n) ? B[(o + (i < j ? i : j)) + (size_t)(o + (i < j ? j : i)) * ld]
                               : 0.0;
    v[i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int N = n + (n & 1);
  const int half = N / 2;
  const double u = 1.1102230246251565e-16;
  int sweep = 0;
  if (n > 1) {
    for (sweep = 0; sweep < max_sweeps; ++sweep) {
      if (tid == 0) rotated = 0;
      __syncthreads();
      for (int round = 0; round < N - 1; ++round) {
        if (tid < half) {
          const int k = tid;
          int p = (k == 0) ? 0 : ((k - 1 + round) % (N - 1)) + 1;
          int q = ((N - 2 - k + round) % (N - 1)) + 1;
          if (p > q) {
            const int t0 = p;
            p = q;
            q = t0;
          }
          double c = 1.0, sn = 0.0, t = 0.0, apq = 0.0, app = 0.0, aqq = 0.0;
          if (q < n) {
            apq = a[p][q];
            app = a[p][p];
            aqq = a[q][q];
            if (apq != 0.0 && fabs(apq) > u * sqrt(fabs(app * aqq))) {
              const double tau = (aqq - app) / (2.0 * apq);
              t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
              c = 1.0 / sqrt(1.0 + t * t);
              sn = t * c;
              rotated = 1;
            }
          }
          rp[k] = p;
          rq[k] = q;
          rc[k] = c;
          rs[k] = sn;
          rt[k] = t;
          rpq[k] = apq;
          rpp[k] = app;
          rqq[k] = aqq;
        }
        __syncthreads();
        // columns of a and v
        for (int e = tid; e < half * n; e += NT) {
          const int k = e / n, i = e - k * n;
          const double sn = rs[k];
          if (sn == 0.0) continue;
          const double c = rc[k];
          const int p = rp[k], q = rq[k];
          const double x = a[i][p], y = a[i][q];
          a[i][p] = c * x - sn * y;
          a[i][q] = sn * x + c * y;
          const double xv = v[i][p], yv = v[i][q];
          v[i][p] = c * xv - sn * yv;
          v[i][q] = sn * xv + c * yv;
        }
        __syncthreads();
        // rows of a
        for (int e = tid; e < half * n; e += NT) {
          const int k = e / n, j = e - k * n;
          const double sn = rs[k];
          if (sn == 0.0) continue;
          const double c = rc[k];
          const int p = rp[k], q = rq[k];
          const double x = a[p][j], y = a[q][j];
          a[p][j] = c * x - sn * y;
          a[q][j] = sn * x + c * y;
        }
        __syncthreads();
        if (tid < half && rs[tid] != 0.0) {
          const int p = rp[tid], q = rq[tid];
          const double t = rt[tid], apq = rpq[tid];
          // the 2 x 2 block exactly, from the values before the rotation
          a[p][p] = rpp[tid] - t * apq;
          a[q][q] = rqq[tid] + t * apq;
          a[p][q] = 0.0;
          a[q][p] = 0.0;
        }
        __syncthreads();
      }
      const int any = rotated;
      __syncthreads();
      if (!any) break;
    }
  }
  if (tid == 0) {
    for (int i = 0; i < n; ++i) order[i] = i;
    for (int i = 1; i < n; ++i) {   // insertion sort by eigenvalue (stable)
      const int key = order[i];
      const double kv = a[key][key];
      int j = i - 1;
      while (j >= 0 && a[order[j]][order[j]] > kv) {
        order[j + 1] = order[j];
        --j;
      }
      order[j + 1] = key;
    }
    atomicMax(sweeps_out, sweep);
  }
  __syncthreads();
  for (int e = tid; e < n * n; e += NT) {
    const int i = e % n, r = e / n;
    Z[(o + i) + (size_t)(o + r) * ldz] = v[i][order[r]];
  }
  if (tid < n) lam[o + tid] = a[order[tid]][order[tid]];
}

void jacobi_leaves(hipStream_t s, const double* b, int ld, const int* leaf_o, const int* leaf_n,
                   int nleaves, double* z, int ldz, double* lam, int* sweeps_out) {
  if (nleaves <= 0) return;
  hipLaunchKernelGGL(jacobi_kernel, dim3(nleaves), dim3(NT), 0, s, b, ld, leaf_o, leaf_n, z, ldz,
                     lam, sweeps_out, 40);
  PS_HIP(hipGetLastError());
}

}  // namespace ps

namespace ps {

// ------------------------------------------------------------------ adjoint helpers
// G (np x np, zero padded) = [[gA, -gB], [0, 0]]: the loss gradient with respect to
// sign(H) = [[S_A, S_B], [-S_B, -S_A]], placed in the first block row, times Sigma.
__global__ void build_gbar_kernel(const double* ga, const double* gb, int ldg, int m, double* g,
                                  int np) {
  PS_GRID_LOOP(e, (size_t)np * np) {
    const int i = (int)(e % np), j = (int)(e / np);
    double v = 0.0;
    if (i < m) {
      if (j < m) v = ga[i + (size_t)j * ldg];
      else if (j < 2 * m) v = -gb[i + (size_t)(j - m) * ldg];
    }
    g[e] = v;
  }
}

void build_gbar(hipStream_t s, const double* ga, const double* gb, int ldg, int m, double* g,
                int np) {
  hipLaunchKernelGGL(build_gbar_kernel, dim3(grid_for((size_t)np * np)), dim3(NT), 0, s, ga, gb,
                     ldg, m, g, np);
  PS_HIP(hipGetLastError());
}

// T(i, j) <- -F_ij T(i, j), F_ij = (s_i - s_j) / (lambda_i - lambda_j) (0 when s_i = s_j),
// s = +1 on the first m indices, -1 on the next m; padding (>= 2m) cleared.
__global__ void dk_hadamard_kernel(double* t, int np, const double* lam, int m) {
  PS_GRID_LOOP(e, (size_t)np * np) {
    const int i = (int)(e % np), j = (int)(e / np);
    double v = 0.0;
    if (i < 2 * m && j < 2 * m && ((i < m) != (j < m))) {
      const double si = i < m ? 1.0 : -1.0;
      v = -t[e] * (si - (-si)) / (lam[i] - lam[j]);
    }
    t[e] = v;
  }
}

void dk_hadamard(hipStream_t s, double* t, int np, const double* lam, int m) {
  hipLaunchKernelGGL(dk_hadamard_kernel, dim3(grid_for((size_t)np * np)), dim3(NT), 0, s, t, np,
                     lam, m);
  PS_HIP(hipGetLastError());
}

// gA = sym(K11 + K22), gB = sym(K12 + K21) for K (np x np), blocks of size m
__global__ void grad_assemble_kernel(const double* k, int np, int m, double* ga, double* gb,
                                     int ldo) {
  PS_GRID_LOOP(e, (size_t)m * m) {
    const int i = (int)(e % m), j = (int)(e / m);
    auto K = [&](int r, int c) { return k[r + (size_t)c * np]; };
    ga[i + (size_t)j * ldo] =
        0.5 * ((K(i, j) + K(m + i, m + j)) + (K(j, i) + K(m + j, m + i)));
    gb[i + (size_t)j * ldo] =
        0.5 * ((K(i, m + j) + K(m + i, j)) + (K(j, m + i) + K(m + j, i)));
  }
}

void grad_assemble(hipStream_t s, const double* k, int np, int m, double* ga, double* gb,
                   int ldo) {
  hipLaunchKernelGGL(grad_assemble_kernel, dim3(grid_for((size_t)m * m)), dim3(NT), 0, s, k, np, m,
                     ga, gb, ldo);
  PS_HIP(hipGetLastError());
}

}  // namespace ps
