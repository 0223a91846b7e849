// Element-wise, copy and reduction kernels of the pseudosym pipeline (FP64).
#include "ps_internal.h"

namespace ps {

namespace {
constexpr int NT = 256;
inline unsigned blocks_for(size_t n, int per = NT) {
  size_t b = (n + per - 1) / per;
  return (unsigned)(b > 65535u * 64u ? 65535u * 64u : b);
}

__device__ inline double warp_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// block-wide sum (NT threads); result valid in thread 0
__device__ inline double block_sum(double v, double* sh) {
  v = warp_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
  __syncthreads();
  return r;
}
}  // namespace

// mk[0] = upper(A + B), mk[1] = upper(A - B); padded diagonal 1, strictly lower 0.
__global__ void pack_casida_kernel(int m, int mp, const double* A, int lda, const double* B,
                                   int ldb, double* mk) {
  const size_t n = (size_t)mp * mp;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % mp), j = (int)(e / mp);
    double sp = 0.0, sm = 0.0;
    if (i <= j) {
      if (j < m) {
        const double a = A[i + (size_t)j * lda], b = B[i + (size_t)j * ldb];
        sp = a + b;
        sm = a - b;
      } else if (i == j) {
        sp = 1.0;
        sm = 1.0;
      }
    }
    mk[e] = sp;
    mk[n + e] = sm;
  }
}

void pack_casida(hipStream_t s, int m, int mp, const double* A, int lda, const double* B,
                 int ldb, double* mk) {
  hipLaunchKernelGGL(pack_casida_kernel, dim3(blocks_for((size_t)mp * mp)), dim3(NT), 0, s, m,
                     mp, A, lda, B, ldb, mk);
  PS_HIP(hipGetLastError());
}

__global__ void mask_pad_kernel(double* x, int m, int mp, long long stride) {
  double* X = x + blockIdx.y * stride;
  const size_t n = (size_t)mp * mp;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % mp), j = (int)(e / mp);
    if (i >= m || j >= m) X[e] = 0.0;
  }
}

void mask_pad(hipStream_t s, double* x, int m, int mp, long long stride, int batch) {
  if (m == mp) return;
  hipLaunchKernelGGL(mask_pad_kernel, dim3(blocks_for((size_t)mp * mp), batch), dim3(NT), 0, s,
                     x, m, mp, stride);
  PS_HIP(hipGetLastError());
}

__global__ void fill_kernel(double* x, size_t n, double v) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    x[e] = v;
}

void fill_zero(hipStream_t s, double* x, size_t n) {
  if (!n) return;
  hipLaunchKernelGGL(fill_kernel, dim3(blocks_for(n)), dim3(NT), 0, s, x, n, 0.0);
  PS_HIP(hipGetLastError());
}

template <class T>
__global__ void zero_lower_kernel(T* x, int mp, long long stride) {
  T* X = x + blockIdx.y * stride;
  const size_t n = (size_t)mp * mp;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % mp), j = (int)(e / mp);
    if (i > j) X[e] = T(0);
  }
}

template <class T>
void zero_lower_t(hipStream_t s, T* x, int mp, long long stride, int batch) {
  hipLaunchKernelGGL(zero_lower_kernel<T>, dim3(blocks_for((size_t)mp * mp), batch), dim3(NT), 0,
                     s, x, mp, stride);
  PS_HIP(hipGetLastError());
}
void zero_lower(hipStream_t s, double* x, int mp, long long stride, int batch) {
  zero_lower_t(s, x, mp, stride, batch);
}
void zero_lower(hipStream_t s, float* x, int mp, long long stride, int batch) {
  zero_lower_t(s, x, mp, stride, batch);
}

template <class T>
__global__ void zero_block_kernel(T* x, int rows, int cols, int ld, int nb1, long long s1,
                                  long long s2) {
  const int b = blockIdx.y;
  T* X = x + (b % nb1) * s1 + (b / nb1) * s2;
  const size_t n = (size_t)rows * cols;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % rows), j = (int)(e / rows);
    X[i + (size_t)j * ld] = T(0);
  }
}

template <class T>
void zero_block_t(hipStream_t s, T* x, int rows, int cols, int ld, int nb1, long long s1, int nb2,
                  long long s2) {
  if (rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL(zero_block_kernel<T>, dim3(blocks_for((size_t)rows * cols), nb1 * nb2),
                     dim3(NT), 0, s, x, rows, cols, ld, nb1, s1, s2);
  PS_HIP(hipGetLastError());
}
void zero_block(hipStream_t s, double* x, int rows, int cols, int ld, int nb1, long long s1,
                int nb2, long long s2) {
  zero_block_t(s, x, rows, cols, ld, nb1, s1, nb2, s2);
}
void zero_block(hipStream_t s, float* x, int rows, int cols, int ld, int nb1, long long s1,
                int nb2, long long s2) {
  zero_block_t(s, x, rows, cols, ld, nb1, s1, nb2, s2);
}

// 64 x 64 tiles through LDS
__global__ void transpose_kernel(const double* x, double* y, int mp, long long stride) {
  __shared__ double t[64][65];
  const double* X = x + blockIdx.z * stride;
  double* Y = y + blockIdx.z * stride;
  const int bi = blockIdx.x * 64, bj = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int j = ty; j < 64; j += 4) t[j][tx] = X[(bi + tx) + (size_t)(bj + j) * mp];
  __syncthreads();
  for (int i = ty; i < 64; i += 4) Y[(bj + tx) + (size_t)(bi + i) * mp] = t[tx][i];
}

void transpose(hipStream_t s, const double* x, double* y, int mp, long long stride, int batch) {
  hipLaunchKernelGGL(transpose_kernel, dim3(mp / 64, mp / 64, batch), dim3(NT), 0, s, x, y, mp,
                     stride);
  PS_HIP(hipGetLastError());
}

// z[j] = upper(G) + shifts[j] I with strictly lower part zero (G holds its upper triangle)
__global__ void form_shifts_kernel(const double* g, double* z, int mp, const double* shifts) {
  const size_t n = (size_t)mp * mp;
  const double c = shifts[blockIdx.y];
  double* Z = z + blockIdx.y * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % mp), j = (int)(e / mp);
    Z[e] = (i < j) ? g[e] : ((i == j) ? g[e] + c : 0.0);
  }
}

void form_shifts(hipStream_t s, const double* g, double* z, int mp, const double* shifts,
                 int r) {
  hipLaunchKernelGGL(form_shifts_kernel, dim3(blocks_for((size_t)mp * mp), r), dim3(NT), 0, s,
                     g, z, mp, shifts);
  PS_HIP(hipGetLastError());
}

struct ShiftList {
  double c[kMaxSeg];
};

// same as form_shifts_kernel with the shifts passed by value (no host-device copy); the
// padded diagonal (indices >= m, where G is zero) is 1, so that a zero shift (the Newton
// step) still leaves the padding positive definite
__global__ void form_shifts_v_kernel(const double* g, double* z, int m, int mp, ShiftList sl) {
  const size_t n = (size_t)mp * mp;
  const double c = sl.c[blockIdx.y];
  double* Z = z + blockIdx.y * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % mp), j = (int)(e / mp);
    Z[e] = (i < j) ? g[e] : ((i == j) ? (i < m ? g[e] + c : 1.0) : 0.0);
  }
}

void form_shifts_v(hipStream_t s, const double* g, double* z, int m, int mp,
                   const double* shifts_host, int r) {
  ShiftList sl{};
  for (int j = 0; j < r && j < kMaxSeg; ++j) sl.c[j] = shifts_host[j];
  hipLaunchKernelGGL(form_shifts_v_kernel, dim3(blocks_for((size_t)mp * mp), r), dim3(NT), 0, s,
                     g, z, m, mp, sl);
  PS_HIP(hipGetLastError());
}

__global__ void fill_int_kernel(int* x, int n) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) x[e] = 0;
}

void fill_int_zero(hipStream_t s, int* x, int n) {
  hipLaunchKernelGGL(fill_int_kernel, dim3((n + NT - 1) / NT), dim3(NT), 0, s, x, n);
  PS_HIP(hipGetLastError());
}

// y = a x + b I (x, y may alias)
__global__ void axpb_identity_kernel(const double* x, double* y, double a, double b, int mp) {
  const size_t n = (size_t)mp * mp;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % mp), j = (int)(e / mp);
    y[e] = a * x[e] + (i == j ? b : 0.0);
  }
}

void axpb_identity(hipStream_t s, const double* x, double* y, double a, double b, int mp) {
  hipLaunchKernelGGL(axpb_identity_kernel, dim3(blocks_for((size_t)mp * mp)), dim3(NT), 0, s, x,
                     y, a, b, mp);
  PS_HIP(hipGetLastError());
}

__global__ void scale_copy_kernel(const double* x, double* y, double a, size_t n) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    y[e] = a * x[e];
}

void scale_copy(hipStream_t s, const double* x, double* y, double a, size_t n) {
  hipLaunchKernelGGL(scale_copy_kernel, dim3(blocks_for(n)), dim3(NT), 0, s, x, y, a, n);
  PS_HIP(hipGetLastError());
}

// A_s = sym(S21 + S12)/2, B_s = sym(S21 - S12)/2 (the blocks of sign(H))
__global__ void sign_blocks_kernel(const double* s12, const double* s21, double* as,
                                   double* bs, int mp) {
  const size_t n = (size_t)mp * mp;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % mp), j = (int)(e / mp);
    const size_t et = j + (size_t)i * mp;
    const double p = 0.5 * (s12[e] + s12[et]);
    const double q = 0.5 * (s21[e] + s21[et]);
    as[e] = 0.5 * (q + p);
    bs[e] = 0.5 * (q - p);
  }
}

void sign_blocks(hipStream_t s, const double* s12, const double* s21, double* as, double* bs,
                 int mp) {
  hipLaunchKernelGGL(sign_blocks_kernel, dim3(blocks_for((size_t)mp * mp)), dim3(NT), 0, s,
                     s12, s21, as, bs, mp);
  PS_HIP(hipGetLastError());
}

// p11 = upper((I + A_s)/2), strictly lower zero (padded A_s is zero: padded diagonal 1/2)
__global__ void half_shift_upper_kernel(const double* as, double* p11, int mp) {
  const size_t n = (size_t)mp * mp;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % mp), j = (int)(e / mp);
    p11[e] = (i < j) ? 0.5 * as[e] : ((i == j) ? 0.5 * (1.0 + as[e]) : 0.0);
  }
}

void half_shift_upper(hipStream_t s, const double* as, double* p11, int mp) {
  hipLaunchKernelGGL(half_shift_upper_kernel, dim3(blocks_for((size_t)mp * mp)), dim3(NT), 0, s,
                     as, p11, mp);
  PS_HIP(hipGetLastError());
}

// top = C^T;  ab[0] = (top + qbot)/sqrt2, ab[1] = (top - qbot)/sqrt2
__global__ void basis_mix_kernel(const double* c, const double* qbot, double* top_out,
                                 double* ab, int mp) {
  const size_t n = (size_t)mp * mp;
  const double h = 0.70710678118654752440;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % mp), j = (int)(e / mp);
    const double tv = (i >= j) ? c[j + (size_t)i * mp] : 0.0;
    const double bv = qbot[e];
    top_out[e] = tv;
    ab[e] = h * (tv + bv);
    ab[n + e] = h * (tv - bv);
  }
}

void basis_mix(hipStream_t s, const double* c, const double* qbot, double* top_out, double* ab,
               int mp) {
  hipLaunchKernelGGL(basis_mix_kernel, dim3(blocks_for((size_t)mp * mp)), dim3(NT), 0, s, c,
                     qbot, top_out, ab, mp);
  PS_HIP(hipGetLastError());
}

__global__ void copy_out_kernel(const double* x, int ldx, double* y, int ldy, int rows,
                                int cols) {
  const size_t n = (size_t)rows * cols;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % rows), j = (int)(e / rows);
    y[i + (size_t)j * ldy] = x[i + (size_t)j * ldx];
  }
}

void copy_out(hipStream_t s, const double* x, int ldx, double* y, int ldy, int rows, int cols) {
  if (rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL(copy_out_kernel, dim3(blocks_for((size_t)rows * cols)), dim3(NT), 0, s, x,
                     ldx, y, ldy, rows, cols);
  PS_HIP(hipGetLastError());
}

// out2[0] += ||x2 - x1||^2 partials, out2[1] += ||x2||^2 partials: two-pass (per-block
// partials then a single-block sum) for a deterministic result.
__global__ void diff_norm_partial_kernel(const double* x1, const double* x2, size_t n,
                                         double* part) {
  __shared__ double sh[NT / 64];
  double d = 0.0, q = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const double a = x1[e], b = x2[e];
    d += (b - a) * (b - a);
    q += b * b;
  }
  const double sd = block_sum(d, sh);
  const double sq = block_sum(q, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sd;
    part[2 * blockIdx.x + 1] = sq;
  }
}

__global__ void sum_pairs_kernel(const double* part, int nb, double* out2) {
  __shared__ double sh[NT / 64];
  double d = 0.0, q = 0.0;
  for (int e = threadIdx.x; e < nb; e += blockDim.x) {
    d += part[2 * e];
    q += part[2 * e + 1];
  }
  const double sd = block_sum(d, sh);
  const double sq = block_sum(q, sh);
  if (threadIdx.x == 0) {
    out2[0] = sd;
    out2[1] = sq;
  }
}

void diff_norms(hipStream_t s, const double* x1, const double* x2, size_t n, double* out2) {
  // out2 must have room for 2 + 2*1024 doubles (partials after the two results)
  const int nb = 1024;
  hipLaunchKernelGGL(diff_norm_partial_kernel, dim3(nb), dim3(NT), 0, s, x1, x2, n, out2 + 2);
  hipLaunchKernelGGL(sum_pairs_kernel, dim3(1), dim3(NT), 0, s, out2 + 2, nb, out2);
  PS_HIP(hipGetLastError());
}

// ------------------------------------------------------------ Golub-Kahan bidiagonalization
// deterministic unit start vector per batch item (entries of the padding are zero)
__global__ void gk_init_kernel(double* v, int m, int mp) {
  __shared__ double sh[NT / 64];
  double* V = v + blockIdx.x * (size_t)mp;
  double q = 0.0;
  for (int i = threadIdx.x; i < mp; i += blockDim.x) {
    double x = 0.0;
    if (i < m) {
      unsigned h = (unsigned)i * 2654435761u + 0x9e3779b9u * (blockIdx.x + 1);
      h ^= h >> 16;
      h *= 0x85ebca6bu;
      h ^= h >> 13;
      x = 1.0 + (double)(h & 0xffff) / 65536.0;   // positive, well spread
    }
    V[i] = x;
    q += x * x;
  }
  __shared__ double tot;
  const double s = block_sum(q, sh);
  if (threadIdx.x == 0) tot = s;
  __syncthreads();
  const double inv = 1.0 / sqrt(tot);
  for (int i = threadIdx.x; i < mp; i += blockDim.x) V[i] *= inv;
}

void gk_init(hipStream_t s, double* v, int m, int mp, int batch, unsigned) {
  hipLaunchKernelGGL(gk_init_kernel, dim3(batch), dim3(NT), 0, s, v, m, mp);
  PS_HIP(hipGetLastError());
}

// One half-step of the bidiagonalization per launch, with the vectors kept unnormalized
// (w~ = ||w~|| w): w~ = M x / ||x~|| - ||x~|| wprev~ / ||wprev~||, where x~ is the previous
// half-step's vector and wprev~ the one before (the coefficient of the recurrence is the
// norm of x~).  Each workgroup owns four entries of w~ (one column dot per wave) and
// writes the sum of their squares to its slot of wpart; norms are the sums of such
// partials, taken in a fixed order by every workgroup of the next launch, so there is
// no cross-workgroup traffic within a launch and the result is deterministic.  Workgroup
// 0 also stores ||x~|| at hist[hist_x] (hist_x < 0: none).  Partials: npart = gridDim.x
// per batch item.
__device__ inline double gk_norm2(const double* part, int npart, double* sh) {
  double q = 0.0;
  for (int i = threadIdx.x; i < npart; i += blockDim.x) q += part[i];
  __shared__ double tot;
  const double r = block_sum(q, sh);
  if (threadIdx.x == 0) tot = r;
  __syncthreads();
  return tot;
}

__global__ void gk_step_kernel(const double* mat, long long mstride, const double* x,
                               long long xstride, const double* xpart, double* w,
                               long long wstride, const double* wprev, long long wpstride,
                               const double* wppart, double* wpart, double* hist, int hist_x,
                               int hist_ld, int mp) {
  constexpr int U = 8;
  __shared__ double sh[NT / 64];
  __shared__ double wv[NT / 64];
  const int b = blockIdx.y, npart = gridDim.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col = blockIdx.x * (NT / 64) + wave;
  double dot = 0.0;
  if (col < mp) {
    const double2* Mc = reinterpret_cast<const double2*>(mat + b * mstride + (size_t)col * mp);
    const double2* X = reinterpret_cast<const double2*>(x + b * xstride);
    const int n2 = mp / 2;
    double acc0 = 0.0, acc1 = 0.0;
    for (int base = 0; base < n2; base += 64 * U) {
      double2 a[U], v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = base + lane + 64 * u;
        a[u] = i < n2 ? Mc[i] : double2{0.0, 0.0};
        v[u] = i < n2 ? X[i] : double2{0.0, 0.0};
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        acc0 += a[u].x * v[u].x;
        acc1 += a[u].y * v[u].y;
      }
    }
    dot = warp_sum(acc0 + acc1);
  }
  const double nx = sqrt(gk_norm2(xpart + (size_t)b * npart, npart, sh));
  const double nwp = wprev ? sqrt(gk_norm2(wppart + (size_t)b * npart, npart, sh)) : 1.0;
  const double inx = nx > 0.0 ? 1.0 / nx : 0.0;
  const double cw = (wprev && nwp > 0.0) ? nx / nwp : 0.0;
  double val = 0.0;
  if (col < mp && lane == 0) {
    val = dot * inx;
    if (wprev) val -= cw * wprev[b * wpstride + col];
    w[b * wstride + col] = val;
    wv[wave] = val * val;
  } else if (lane == 0) {
    wv[wave] = 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double q = 0.0;
    for (int i = 0; i < NT / 64; ++i) q += wv[i];
    wpart[(size_t)b * npart + blockIdx.x] = q;
    if (blockIdx.x == 0 && hist_x >= 0) hist[(size_t)b * hist_ld + hist_x] = nx;
  }
}

// partials of a unit vector's squared norm: 1 in slot 0 of every batch item
__global__ void gk_seed_kernel(double* part, int npart) {
  for (int i = threadIdx.x; i < npart; i += blockDim.x) part[(size_t)blockIdx.x * npart + i] = i == 0 ? 1.0 : 0.0;
}
// hist[hist_out] = the norm given by the partials (the last half-step's vector)
__global__ void gk_finish_kernel(const double* part, int npart, double* hist, int hist_out,
                                 int hist_ld) {
  __shared__ double sh[NT / 64];
  const double n2 = gk_norm2(part + (size_t)blockIdx.x * npart, npart, sh);
  if (threadIdx.x == 0) hist[(size_t)blockIdx.x * hist_ld + hist_out] = sqrt(n2);
}

int gk_parts(int mp) { return (mp + NT / 64 - 1) / (NT / 64); }

void gk_seed(hipStream_t s, double* part, int mp, int batch) {
  hipLaunchKernelGGL(gk_seed_kernel, dim3(batch), dim3(NT), 0, s, part, gk_parts(mp));
  PS_HIP(hipGetLastError());
}

void gk_step(hipStream_t s, const double* mat, long long mstride, const double* x,
             long long xstride, const double* xpart, double* w, long long wstride,
             const double* wprev, long long wpstride, const double* wppart, double* wpart,
             double* hist, int hist_x, int hist_ld, int mp, int batch) {
  hipLaunchKernelGGL(gk_step_kernel, dim3(gk_parts(mp), batch), dim3(NT), 0, s, mat, mstride, x,
                     xstride, xpart, w, wstride, wprev, wpstride, wppart, wpart, hist, hist_x,
                     hist_ld, mp);
  PS_HIP(hipGetLastError());
}

void gk_finish(hipStream_t s, const double* part, int mp, double* hist, int hist_out, int hist_ld,
               int batch) {
  hipLaunchKernelGGL(gk_finish_kernel, dim3(batch), dim3(NT), 0, s, part, gk_parts(mp), hist,
                     hist_out, hist_ld);
  PS_HIP(hipGetLastError());
}

__global__ void sym_scale_upper_kernel(const double* x, double* z, int m, int mp, double scale) {
  const size_t n = (size_t)mp * mp;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % mp), j = (int)(e / mp);
    double v = 0.0;
    if (i < m && j < m && i <= j) v = scale * (x[e] + x[j + (size_t)i * mp]);
    else if (i == j) v = 1.0;
    z[e] = v;
  }
}

void sym_scale_upper(hipStream_t s, const double* x, double* z, int m, int mp, double scale) {
  hipLaunchKernelGGL(sym_scale_upper_kernel, dim3(blocks_for((size_t)mp * mp)), dim3(NT), 0, s, x,
                     z, m, mp, scale);
  PS_HIP(hipGetLastError());
}

__global__ void sum_diff_scaled_kernel(const double* e1, const double* e2, double* top,
                                       double* bot, double c, size_t n) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const double a = e1[e], b = e2[e];
    top[e] = c * (a + b);
    bot[e] = c * (a - b);
  }
}

void sum_diff_scaled(hipStream_t s, const double* e1, const double* e2, double* top, double* bot,
                     double c, int mp) {
  const size_t n = (size_t)mp * mp;
  hipLaunchKernelGGL(sum_diff_scaled_kernel, dim3(blocks_for(n)), dim3(NT), 0, s, e1, e2, top, bot,
                     c, n);
  PS_HIP(hipGetLastError());
}

// ------------------------------------------------------- power steps on a symmetric matrix
// Start vector of the power steps: fixed, of both signs, zero past the live size m.
__global__ void power_start_kernel(double* v, int m, int mp) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < mp; i += gridDim.x * blockDim.x) {
    double x = 0.0;
    if (i < m) {
      unsigned h = (unsigned)i * 2654435761u + 0x7f4a7c15u;
      h ^= h >> 15;
      h *= 0x2c1b3c6du;
      h ^= h >> 12;
      x = (double)(int)(h & 0xffffu) / 32768.0 - 1.0;
    }
    v[i] = x;
  }
}

// y = (M - shift I) x on the live block (rows and columns below m); y is zero past m.
// M is symmetric in full storage, so row i is column i, which one wave reads
// contiguously as 16-byte vectors, eight in flight per lane (NT / 64 columns per
// workgroup).  x is zero past m, so whole columns are read (padded entries of M are
// finite).
__global__ void sym_apply_kernel(const double* M, int m, int mp, double shift, const double* x,
                                 double* y) {
  constexpr int U = 8;
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
  if (i >= mp) return;
  double acc0 = 0.0, acc1 = 0.0;
  if (i < m) {
    const double2* Mc = reinterpret_cast<const double2*>(M + (size_t)i * mp);
    const double2* X = reinterpret_cast<const double2*>(x);
    const int n2 = mp / 2;
    for (int base = 0; base < n2; base += 64 * U) {
      double2 a[U], v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = base + lane + 64 * u;
        a[u] = j < n2 ? Mc[j] : double2{0.0, 0.0};
        v[u] = j < n2 ? X[j] : double2{0.0, 0.0};
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        acc0 += a[u].x * v[u].x;
        acc1 += a[u].y * v[u].y;
      }
    }
  }
  const double acc = warp_sum(acc0 + acc1);
  if (lane == 0) y[i] = i < m ? acc - shift * x[i] : 0.0;
}

__global__ void two_norms2_kernel(const double* a, const double* b, int n, double* out2) {
  __shared__ double sh[NT / 64];
  double qa = 0.0, qb = 0.0;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    qa += a[e] * a[e];
    qb += b[e] * b[e];
  }
  const double sa = block_sum(qa, sh);
  const double sb = block_sum(qb, sh);
  if (threadIdx.x == 0) {
    out2[0] = sa;
    out2[1] = sb;
  }
}

void sym_power_norm(hipStream_t s, const double* M, int m, int mp, double shift, int steps,
                    double* v0, double* v1, double* out2) {
  hipLaunchKernelGGL(power_start_kernel, dim3(blocks_for(mp)), dim3(NT), 0, s, v0, m, mp);
  double* v[2] = {v0, v1};
  const unsigned nb = (unsigned)((mp + NT / 64 - 1) / (NT / 64));
  for (int k = 0; k < steps; ++k)
    hipLaunchKernelGGL(sym_apply_kernel, dim3(nb), dim3(NT), 0, s, M, m, mp, shift, v[k & 1],
                       v[(k + 1) & 1]);
  hipLaunchKernelGGL(two_norms2_kernel, dim3(1), dim3(NT), 0, s, v[steps & 1],
                     v[(steps + 1) & 1], mp, out2);
  PS_HIP(hipGetLastError());
}

// ------------------------------------------------------- full sign matrix from its blocks
// S = [[S_A, S_B], [-S_B, -S_A]] (2m x 2m, ld lds2) from the m x m blocks (ld lds)
__global__ void sign_full_kernel(const double* sa, const double* sb, int lds, int m, double* S,
                                 int lds2) {
  const int n = 2 * m;
  const size_t total = (size_t)n * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    const int bi = i >= m, bj = j >= m;
    const size_t src = (i - bi * m) + (size_t)(j - bj * m) * lds;
    // row block 0: (S_A, S_B); row block 1: (-S_B, -S_A)
    const double v = (bi == bj) ? sa[src] : sb[src];
    S[i + (size_t)j * lds2] = bi ? -v : v;
  }
}

void sign_full(hipStream_t s, const double* sa, const double* sb, int lds, int m, double* S,
               int lds2) {
  hipLaunchKernelGGL(sign_full_kernel, dim3(blocks_for((size_t)4 * m * m)), dim3(NT), 0, s, sa, sb,
                     lds, m, S, lds2);
  PS_HIP(hipGetLastError());
}

}  // namespace ps
