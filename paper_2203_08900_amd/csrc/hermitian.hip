// The complex Bethe-Salpeter forms (Sec. 5) on the real pipeline.
//
// A complex number z = x + iy acts on R^2 as the 2 x 2 block [[x, -y], [y, x]];
// writing every entry of a complex matrix so (the interleaved realification R) maps
// products to products, the conjugate transpose to the transpose, inverses to inverses
// and Hermitian positive definite matrices to symmetric positive definite ones.  For
// Eq:BSE2 (A, B Hermitian) the realified H is the real Casida form of twice the size
// with blocks R(A), R(B), so its sign blocks are R(A_s), R(B_s); and since every 2 x 2
// diagonal block of a realified Hermitian matrix is a multiple of I, a real Cholesky
// factor of it is R of the complex one, so the Alg. 6 basis and the core basis come
// out realified as well.  For Eq:BSE1 (B complex symmetric, the lower blocks
// conjugated) the bottom half is realified with the imaginary parts flipped, which
// makes the off-diagonal blocks R(B) D with D = diag(1, -1) per entry: symmetric, and
// the real Casida form again, whose sign blocks are R(A_s) and R(B_s) D.  In both forms
// the first column of each 2 x 2 block holds (re, im) of the complex entry.
#include "ps_internal.h"

namespace ps {
namespace {

constexpr int NT = 256;
inline unsigned blocks_for(size_t n) {
  return (unsigned)std::min<size_t>((n + NT - 1) / NT, 8192);
}

// Y (2m x 2m, ld ldy) from complex X (m x m, ld ldx in complex entries):
// flip = 0: [[re, -im], [im, re]]; flip = 1: [[re, im], [im, -re]]
__global__ void realify_kernel(const double2* X, int ldx, int m, double* Y, int ldy, int flip) {
  const int m2 = 2 * m;
  const size_t n = (size_t)m2 * m2;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % m2), c = (int)(e / m2);
    const int a = r & 1, b = c & 1;
    const double2 x = X[(r >> 1) + (size_t)(c >> 1) * ldx];
    double v;
    if (!flip) v = (a == b) ? x.x : (a ? x.y : -x.y);
    else v = a ? (b ? -x.x : x.y) : (b ? x.y : x.x);
    Y[r + (size_t)c * ldy] = v;
  }
}

// complex X (rows x cols, ld ldx) from the first columns of the 2 x 2 blocks of Y
__global__ void complexify_kernel(const double* Y, int ldy, int rows, int cols, double2* X,
                                  int ldx) {
  const size_t n = (size_t)rows * cols;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % rows), j = (int)(e / rows);
    const double* y = Y + 2 * i + (size_t)(2 * j) * ldy;
    X[i + (size_t)j * ldx] = double2{y[0], y[1]};
  }
}

// Nearest matrix of the realified form ([[re, -im], [im, re]] blocks) to X (m2 x m2,
// m2 even, column-major, ld ldx): each block's two copies of re and of im are averaged.
__global__ void pair_project_kernel(double* X, int half, int ldx) {
  const size_t n = (size_t)half * half;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % half), j = (int)(e / half);
    double* c0 = X + 2 * i + (size_t)(2 * j) * ldx;   // column 2j
    double* c1 = c0 + ldx;                             // column 2j + 1
    const double re = 0.5 * (c0[0] + c1[1]);
    const double im = 0.5 * (c0[1] - c1[0]);
    c0[0] = re;
    c0[1] = im;
    c1[0] = -im;
    c1[1] = re;
  }
}

}  // namespace

void pair_project(hipStream_t s, double* X, int m2, int ldx) {
  const int half = m2 / 2;
  hipLaunchKernelGGL(pair_project_kernel, dim3(blocks_for((size_t)half * half)), dim3(NT), 0, s, X,
                     half, ldx);
  PS_HIP(hipGetLastError());
}

void realify(hipStream_t s, const double* X, int ldx, int m, double* Y, int ldy, int flip) {
  hipLaunchKernelGGL(realify_kernel, dim3(blocks_for((size_t)4 * m * m)), dim3(NT), 0, s,
                     reinterpret_cast<const double2*>(X), ldx, m, Y, ldy, flip);
  PS_HIP(hipGetLastError());
}

void complexify(hipStream_t s, const double* Y, int ldy, int rows, int cols, double* X, int ldx) {
  hipLaunchKernelGGL(complexify_kernel, dim3(blocks_for((size_t)rows * cols)), dim3(NT), 0, s, Y,
                     ldy, rows, cols, reinterpret_cast<double2*>(X), ldx);
  PS_HIP(hipGetLastError());
}

}  // namespace ps
