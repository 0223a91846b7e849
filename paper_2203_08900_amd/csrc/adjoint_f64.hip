// Element-wise kernels of the stored-factor adjoint of the sign blocks (reverse mode
// through the division's own composition: the Cholesky factorizations of A + B and A - B,
// Y0 = R_M R_K^T, the Zolotarev steps of Alg. 8 on the core and the sign-block products).
// The products themselves run on the GEMM kernel.
#include "ps_internal.h"

namespace ps {
namespace {

constexpr int NT = 256;
inline unsigned blocks_for(size_t n) {
  return (unsigned)std::min<size_t>((n + NT - 1) / NT, 8192);
}

// The sign blocks are S_A = (q + p)/2 and S_B = (q - p)/2 with p = sym(S12),
// q = sym(S21), so the seeds are g12 = sym(gA - gB)/2 and g21 = sym(gA + gB)/2 (mp x mp,
// zero past m).
__global__ void adj_seed_kernel(const double* ga, const double* gb, int ldg, int m, int mp,
                                double* g12, double* g21) {
  const size_t n = (size_t)mp * mp;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % mp), j = (int)(e / mp);
    double p = 0.0, q = 0.0;
    if (i < m && j < m) {
      const size_t a = i + (size_t)j * ldg, t = j + (size_t)i * ldg;
      const double sa = 0.5 * (ga[a] + ga[t]), sb = 0.5 * (gb[a] + gb[t]);
      p = 0.5 * (sa - sb);
      q = 0.5 * (sa + sb);
    }
    g12[e] = p;
    g21[e] = q;
  }
}

// y = x + x^T
__global__ void sym2_kernel(const double* x, double* y, int mp) {
  const size_t n = (size_t)mp * mp;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % mp), j = (int)(e / mp);
    y[e] = x[e] + x[j + (size_t)i * mp];
  }
}

// x <- the lower triangle of x with its diagonal halved (the Cholesky adjoint's map)
__global__ void phi_lower_kernel(double* x, int mp) {
  const size_t n = (size_t)mp * mp;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % mp), j = (int)(e / mp);
    if (i < j)
      x[e] = 0.0;
    else if (i == j)
      x[e] *= 0.5;
  }
}

// gA = sym(gm + gk), gB = sym(gm - gk) on the live m x m block
__global__ void adj_out_kernel(const double* gm, const double* gk, int mp, int m, double* ga,
                               double* gb, int ldo) {
  const size_t n = (size_t)m * m;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % m), j = (int)(e / m);
    const size_t a = i + (size_t)j * mp, t = j + (size_t)i * mp;
    const double sm = 0.5 * (gm[a] + gm[t]), sk = 0.5 * (gk[a] + gk[t]);
    ga[i + (size_t)j * ldo] = sm + sk;
    gb[i + (size_t)j * ldo] = sm - sk;
  }
}

}  // namespace

void adj_seed(hipStream_t s, const double* ga, const double* gb, int ldg, int m, int mp,
              double* g12, double* g21) {
  hipLaunchKernelGGL(adj_seed_kernel, dim3(blocks_for((size_t)mp * mp)), dim3(NT), 0, s, ga, gb,
                     ldg, m, mp, g12, g21);
  PS_HIP(hipGetLastError());
}

void sym2(hipStream_t s, const double* x, double* y, int mp) {
  hipLaunchKernelGGL(sym2_kernel, dim3(blocks_for((size_t)mp * mp)), dim3(NT), 0, s, x, y, mp);
  PS_HIP(hipGetLastError());
}

void phi_lower(hipStream_t s, double* x, int mp) {
  hipLaunchKernelGGL(phi_lower_kernel, dim3(blocks_for((size_t)mp * mp)), dim3(NT), 0, s, x, mp);
  PS_HIP(hipGetLastError());
}

void adj_out(hipStream_t s, const double* gm, const double* gk, int mp, int m, double* ga,
             double* gb, int ldo) {
  hipLaunchKernelGGL(adj_out_kernel, dim3(blocks_for((size_t)m * m)), dim3(NT), 0, s, gm, gk, mp,
                     m, ga, gb, ldo);
  PS_HIP(hipGetLastError());
}

}  // namespace ps
