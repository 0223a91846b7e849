// Conversion and element-wise kernels of the mixed-precision Zolotarev steps: the
// well-conditioned shifted Gram matrices are factorized in FP32 and the second step's
// correction polynomial runs in FP32, while the iterate, X^T X and every quantity whose
// rounding is not damped by a small factor stay in FP64.
#include "ps_internal.h"

namespace ps {

namespace {
constexpr int NT = 256;
inline unsigned grid_for(size_t n) {
  size_t b = (n + NT - 1) / NT;
  return (unsigned)(b > 65535u * 64u ? 65535u * 64u : (b ? b : 1));
}
}  // namespace

struct ShiftList32 {
  double c[kMaxSeg];
};

// z[j] = fp32(upper(G) + c_j I), zero below the diagonal
__global__ void form_shifts_f32_kernel(const double* g, float* z, int mp, ShiftList32 sl) {
  const size_t n = (size_t)mp * mp;
  const double c = sl.c[blockIdx.y];
  float* Z = z + blockIdx.y * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % mp), j = (int)(e / mp);
    Z[e] = (i < j) ? (float)g[e] : ((i == j) ? (float)(g[e] + c) : 0.0f);
  }
}

void form_shifts_f32(hipStream_t s, const double* g, float* z, int mp, const double* shifts,
                     int r) {
  if (r <= 0) return;
  ShiftList32 sl{};
  for (int j = 0; j < r && j < kMaxSeg; ++j) sl.c[j] = shifts[j];
  hipLaunchKernelGGL(form_shifts_f32_kernel, dim3(grid_for((size_t)mp * mp), r), dim3(NT), 0, s, g,
                     z, mp, sl);
  PS_HIP(hipGetLastError());
}

// y = fp32(x)
__global__ void cvt_f64_f32_kernel(const double* x, float* y, size_t n) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    y[e] = (float)x[e];
}

void cvt_f64_f32(hipStream_t s, const double* x, float* y, size_t n) {
  hipLaunchKernelGGL(cvt_f64_f32_kernel, dim3(grid_for(n)), dim3(NT), 0, s, x, y, n);
  PS_HIP(hipGetLastError());
}

__global__ void cvt_f32_f64_kernel(const float* x, double* y, size_t n) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    y[e] = (double)x[e];
}

void cvt_f32_f64(hipStream_t s, const float* x, double* y, size_t n) {
  hipLaunchKernelGGL(cvt_f32_f64_kernel, dim3(grid_for(n)), dim3(NT), 0, s, x, y, n);
  PS_HIP(hipGetLastError());
}

// y = a y + b fp64(x)
__global__ void axpy_f32_kernel(double* y, double a, double b, const float* x, size_t n) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    y[e] = a * y[e] + b * (double)x[e];
}

void axpy_f32(hipStream_t s, double* y, double a, double b, const float* x, size_t n) {
  hipLaunchKernelGGL(axpy_f32_kernel, dim3(grid_for(n)), dim3(NT), 0, s, y, a, b, x, n);
  PS_HIP(hipGetLastError());
}

// y = a x + b I on an mp x mp FP32 matrix
__global__ void axpb_identity_f32_kernel(const float* x, float* y, float a, float b, int mp) {
  const size_t n = (size_t)mp * mp;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % mp), j = (int)(e / mp);
    y[e] = a * x[e] + (i == j ? b : 0.0f);
  }
}

void axpb_identity_f32(hipStream_t s, const float* x, float* y, float a, float b, int mp) {
  hipLaunchKernelGGL(axpb_identity_f32_kernel, dim3(grid_for((size_t)mp * mp)), dim3(NT), 0, s, x,
                     y, a, b, mp);
  PS_HIP(hipGetLastError());
}

}  // namespace ps
