// Element-wise kernels of the batched division (one launch over a class of problems
// of equal padded size mp): each takes its per-matrix scalars from device arrays, so a
// class needs no per-problem launches for them.
#include "ps_internal.h"

namespace ps {

namespace {
constexpr int NT = 256;
inline unsigned blocks_for(size_t n) {
  const size_t b = (n + NT - 1) / NT;
  return (unsigned)(b < 4096 ? b : 4096);
}

__device__ inline double warp_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}
}  // namespace

// y_b = f[b] x_b  (x_b = x + b sx, y_b = y + b sy, n elements each)
__global__ void scale_b_kernel(const double* x, long long sx, double* y, long long sy,
                               const double* f, size_t n) {
  const int b = blockIdx.y;
  const double a = f[b];
  const double* X = x + b * sx;
  double* Y = y + b * sy;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    Y[e] = a * X[e];
}

void scale_b(hipStream_t s, const double* x, long long sx, double* y, long long sy,
             const double* f, size_t n, int nb) {
  hipLaunchKernelGGL(scale_b_kernel, dim3(blocks_for(n), nb), dim3(NT), 0, s, x, sx, y, sy, f, n);
  PS_HIP(hipGetLastError());
}

// z_{b r + j} = upper(g_b) + c[b r + j] I (strictly lower part 0): the shifted Gram
// matrices of a Zolotarev step for every problem of the class
__global__ void form_shifts_b_kernel(const double* g, double* z, int mp, const double* c, int r) {
  const size_t n = (size_t)mp * mp;
  const int q = blockIdx.y, b = q / r;
  const double sh = c[q];
  const double* G = g + b * n;
  double* Z = z + q * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % mp), j = (int)(e / mp);
    Z[e] = (i < j) ? G[e] : ((i == j) ? G[e] + sh : 0.0);
  }
}

void form_shifts_b(hipStream_t s, const double* g, double* z, int mp, const double* c, int r,
                   int nb) {
  hipLaunchKernelGGL(form_shifts_b_kernel, dim3(blocks_for((size_t)mp * mp), nb * r), dim3(NT), 0,
                     s, g, z, mp, c, r);
  PS_HIP(hipGetLastError());
}

// y_b = a[b] x_b + c[b] I  (x, y may alias; stride mp^2)
__global__ void axpb_identity_b_kernel(const double* x, double* y, const double* a,
                                       const double* c, int mp) {
  const size_t n = (size_t)mp * mp;
  const int b = blockIdx.y;
  const double aa = a[b], cc = c[b];
  const double* X = x + b * n;
  double* Y = y + b * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % mp), j = (int)(e / mp);
    Y[e] = aa * X[e] + (i == j ? cc : 0.0);
  }
}

void axpb_identity_b(hipStream_t s, const double* x, double* y, const double* a,
                     const double* c, int mp, int nb) {
  hipLaunchKernelGGL(axpb_identity_b_kernel, dim3(blocks_for((size_t)mp * mp), nb), dim3(NT), 0,
                     s, x, y, a, c, mp);
  PS_HIP(hipGetLastError());
}

// out[2b] = ||x2_b - x1_b||_F^2, out[2b+1] = ||x2_b||_F^2, one workgroup per matrix (a
// fixed summation order)
__global__ void diff_norms_b_kernel(const double* x1, const double* x2, size_t n, double* out) {
  __shared__ double sh[2][NT / 64];
  const int b = blockIdx.x;
  const double* A = x1 + b * n;
  const double* B = x2 + b * n;
  double d = 0.0, q = 0.0;
  for (size_t e = threadIdx.x; e < n; e += NT) {
    const double u = A[e], v = B[e];
    d += (v - u) * (v - u);
    q += v * v;
  }
  d = warp_sum(d);
  q = warp_sum(q);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    sh[0][w] = d;
    sh[1][w] = q;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sd = 0.0, sq = 0.0;
    for (int i = 0; i < NT / 64; ++i) {
      sd += sh[0][i];
      sq += sh[1][i];
    }
    out[2 * b] = sd;
    out[2 * b + 1] = sq;
  }
}

void diff_norms_b(hipStream_t s, const double* x1, const double* x2, size_t n, double* out,
                  int nb) {
  hipLaunchKernelGGL(diff_norms_b_kernel, dim3(nb), dim3(NT), 0, s, x1, x2, n, out);
  PS_HIP(hipGetLastError());
}

// Golub-Kahan start vectors for a batch of matrices with their own sizes m[q] (the same
// values as gk_init: positive, hashed from the index, zero beyond m[q], unit norm).
__global__ void gk_init_b_kernel(double* v, const int* m, int mp, int per) {
  __shared__ double sh[NT / 64];
  __shared__ double tot;
  const int q = blockIdx.x;
  const int mq = m[q / per];
  double* V = v + (size_t)q * mp;
  double acc = 0.0;
  for (int i = threadIdx.x; i < mp; i += blockDim.x) {
    double x = 0.0;
    if (i < mq) {
      unsigned h = (unsigned)i * 2654435761u + 0x9e3779b9u * ((q % per) + 1);
      h ^= h >> 16;
      h *= 0x85ebca6bu;
      h ^= h >> 13;
      x = 1.0 + (double)(h & 0xffff) / 65536.0;
    }
    V[i] = x;
    acc += x * x;
  }
  acc = warp_sum(acc);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int i = 0; i < NT / 64; ++i) r += sh[i];
    tot = r;
  }
  __syncthreads();
  const double inv = 1.0 / sqrt(tot);
  for (int i = threadIdx.x; i < mp; i += blockDim.x) V[i] *= inv;
}

void gk_init_b(hipStream_t s, double* v, const int* m_dev, int mp, int count, int per) {
  hipLaunchKernelGGL(gk_init_b_kernel, dim3(count), dim3(NT), 0, s, v, m_dev, mp, per);
  PS_HIP(hipGetLastError());
}

// Alg. 6 tail of a class, one launch per kernel over all its problems (stride mp^2; the
// same element-wise arithmetic as the single-problem kernels).
// A_s = sym(S21 + S12) / 2, B_s = sym(S21 - S12) / 2
__global__ void sign_blocks_b_kernel(const double* s12, const double* s21, double* as, double* bs,
                                     int mp) {
  const size_t n = (size_t)mp * mp, off = blockIdx.y * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % mp), j = (int)(e / mp);
    const size_t et = j + (size_t)i * mp;
    const double p = 0.5 * (s12[off + e] + s12[off + et]);
    const double q = 0.5 * (s21[off + e] + s21[off + et]);
    as[off + e] = 0.5 * (q + p);
    bs[off + e] = 0.5 * (q - p);
  }
}

void sign_blocks_b(hipStream_t s, const double* s12, const double* s21, double* as, double* bs,
                   int mp, int nb) {
  hipLaunchKernelGGL(sign_blocks_b_kernel, dim3(blocks_for((size_t)mp * mp), nb), dim3(NT), 0, s,
                     s12, s21, as, bs, mp);
  PS_HIP(hipGetLastError());
}

// p11 = upper((I + A_s) / 2), strictly lower part zero
__global__ void half_shift_upper_b_kernel(const double* as, double* p11, int mp) {
  const size_t n = (size_t)mp * mp, off = blockIdx.y * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % mp), j = (int)(e / mp);
    p11[off + e] = (i < j) ? 0.5 * as[off + e] : ((i == j) ? 0.5 * (1.0 + as[off + e]) : 0.0);
  }
}

void half_shift_upper_b(hipStream_t s, const double* as, double* p11, int mp, int nb) {
  hipLaunchKernelGGL(half_shift_upper_b_kernel, dim3(blocks_for((size_t)mp * mp), nb), dim3(NT), 0,
                     s, as, p11, mp);
  PS_HIP(hipGetLastError());
}

// top = C^T;  ab_b = [(top + qbot), (top - qbot)] / sqrt 2  (ab stride 2 mp^2)
__global__ void basis_mix_b_kernel(const double* c, const double* qbot, double* top_out,
                                   double* ab, int mp) {
  const size_t n = (size_t)mp * mp, off = blockIdx.y * n;
  double* AB = ab + 2 * off;
  const double h = 0.70710678118654752440;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % mp), j = (int)(e / mp);
    const double tv = (i >= j) ? c[off + j + (size_t)i * mp] : 0.0;
    const double bv = qbot[off + e];
    top_out[off + e] = tv;
    AB[e] = h * (tv + bv);
    AB[n + e] = h * (tv - bv);
  }
}

void basis_mix_b(hipStream_t s, const double* c, const double* qbot, double* top_out, double* ab,
                 int mp, int nb) {
  hipLaunchKernelGGL(basis_mix_b_kernel, dim3(blocks_for((size_t)mp * mp), nb), dim3(NT), 0, s, c,
                     qbot, top_out, ab, mp);
  PS_HIP(hipGetLastError());
}

// zero rows and columns >= m of matrix q (stride mp^2), m = m_dev[q / per]
__global__ void mask_pad_b_kernel(double* x, const int* m_dev, int mp, int per) {
  const size_t n = (size_t)mp * mp;
  const int q = blockIdx.y, m = m_dev[q / per];
  double* X = x + q * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % mp), j = (int)(e / mp);
    if (i >= m || j >= m) X[e] = 0.0;
  }
}

void mask_pad_b(hipStream_t s, double* x, const int* m_dev, int mp, int per, int count) {
  hipLaunchKernelGGL(mask_pad_b_kernel, dim3(blocks_for((size_t)mp * mp), count), dim3(NT), 0, s,
                     x, m_dev, mp, per);
  PS_HIP(hipGetLastError());
}

}  // namespace ps
