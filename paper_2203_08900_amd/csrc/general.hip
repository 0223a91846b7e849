// Element-wise kernels of the division of a definite pseudosymmetric H of any signature
// Sigma = diag(sigma), Sigma H symmetric positive definite (the matrices of Sec. 6.1).
// The division runs on the congruent symmetric T = R Sigma R^T with M = Sigma H = R^T R
// (H = R^{-1} T R), so these kernels only move signs, blocks and padding; the
// arithmetic is in the GEMM, Cholesky and Zolotarev code shared with the Casida form.
// Padded layout as elsewhere: n x n operands in np x np buffers (np a multiple of 64).
#include "ps_internal.h"

namespace ps {

namespace {
constexpr int NT = 256;
inline unsigned grid_for(size_t n) {
  size_t b = (n + NT - 1) / NT;
  return (unsigned)(b > 65535u * 64u ? 65535u * 64u : (b ? b : 1));
}
#define PS_GEN_LOOP(e, n) \
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < (n); e += (size_t)gridDim.x * blockDim.x)
}  // namespace

// m(i, j) = (sigma_i H(i, j) + sigma_j H(j, i)) / 2 for i <= j < n (the symmetric part of
// Sigma H), zero below the diagonal, 1 on the padded diagonal
__global__ void pack_general_kernel(int n, int np, const double* H, int ldh, const double* sg,
                                    double* m) {
  PS_GEN_LOOP(e, (size_t)np * np) {
    const int i = (int)(e % np), j = (int)(e / np);
    double v = 0.0;
    if (i < n && j < n) {
      if (i <= j) v = 0.5 * (sg[i] * H[i + (size_t)j * ldh] + sg[j] * H[j + (size_t)i * ldh]);
    } else if (i == j) {
      v = 1.0;
    }
    m[e] = v;
  }
}

void pack_general(hipStream_t s, int n, int np, const double* H, int ldh, const double* sg,
                  double* m) {
  hipLaunchKernelGGL(pack_general_kernel, dim3(grid_for((size_t)np * np)), dim3(NT), 0, s, n, np,
                     H, ldh, sg, m);
  PS_HIP(hipGetLastError());
}

// y = diag(sigma) x (rows) or x diag(sigma) (columns); sigma_i = 0 beyond n, so the
// padding of y is zero
__global__ void scale_signs_kernel(const double* x, double* y, int n, int np, const double* sg,
                                   int cols) {
  PS_GEN_LOOP(e, (size_t)np * np) {
    const int i = (int)(e % np), j = (int)(e / np);
    const int k = cols ? j : i;
    y[e] = (i < n && j < n) ? sg[k] * x[e] : 0.0;
  }
}

void scale_signs(hipStream_t s, const double* x, double* y, int n, int np, const double* sg,
                 bool cols) {
  hipLaunchKernelGGL(scale_signs_kernel, dim3(grid_for((size_t)np * np)), dim3(NT), 0, s, x, y,
                     n, np, sg, cols ? 1 : 0);
  PS_HIP(hipGetLastError());
}

// Leading k x k block of +-Sigma P_+- for P_+- = (I +- S)/2 in the form
//   out(i, j) = sigma_i (a delta_ij + S(i, j)) / 2   (a = +1: Sigma P_+; a = -1: -Sigma P_-),
// symmetrized, upper triangle stored (zero below), 1 on the padded diagonal (kp x kp)
__global__ void lead_block_kernel(const double* S, int lds, const double* sg, int k, int kp,
                                  double a, double* out) {
  PS_GEN_LOOP(e, (size_t)kp * kp) {
    const int i = (int)(e % kp), j = (int)(e / kp);
    double v = 0.0;
    if (i < k && j < k) {
      if (i <= j) {
        const double d = (i == j) ? a : 0.0;
        v = 0.25 * (sg[i] * (d + S[i + (size_t)j * lds]) + sg[j] * (d + S[j + (size_t)i * lds]));
      }
    } else if (i == j) {
      v = 1.0;
    }
    out[e] = v;
  }
}

void lead_block(hipStream_t s, const double* S, int lds, const double* sg, int k, int kp, double a,
                double* out) {
  hipLaunchKernelGGL(lead_block_kernel, dim3(grid_for((size_t)kp * kp)), dim3(NT), 0, s, S, lds,
                     sg, k, kp, a, out);
  PS_HIP(hipGetLastError());
}

// The top block of an Alg. 6 basis: top(i, j) = t sigma_i C(j, i), i, j < k (t = +-1),
// zero in the padding (kp x kp)
__global__ void chol_top_kernel(const double* c, int kp, const double* sg, int k, double t,
                                double* top) {
  PS_GEN_LOOP(e, (size_t)kp * kp) {
    const int i = (int)(e % kp), j = (int)(e / kp);
    top[e] = (i < k && j < k) ? t * sg[i] * c[j + (size_t)i * kp] : 0.0;
  }
}

void chol_top(hipStream_t s, const double* c, int kp, const double* sg, int k, double t,
              double* top) {
  hipLaunchKernelGGL(chol_top_kernel, dim3(grid_for((size_t)kp * kp)), dim3(NT), 0, s, c, kp, sg,
                     k, t, top);
  PS_HIP(hipGetLastError());
}

// Upper triangle of the projector Z = (I + a sym(U))/2 of the symmetric T, U = sign(T)
// (n x n in np x np, a = +-1): positive semidefinite of rank r_+ (a = +1) or r_- (a = -1);
// zero below the diagonal and in the padding
__global__ void proj_form_kernel(const double* U, int n, int np, double a, double* Z) {
  PS_GEN_LOOP(e, (size_t)np * np) {
    const int i = (int)(e % np), j = (int)(e / np);
    double v = 0.0;
    if (i <= j && j < n) {
      v = 0.25 * a * (U[e] + U[j + (size_t)i * np]);
      if (i == j) v += 0.5;
    }
    Z[e] = v;
  }
}

void proj_form(hipStream_t s, const double* U, int n, int np, double a, double* Z) {
  hipLaunchKernelGGL(proj_form_kernel, dim3(grid_for((size_t)np * np)), dim3(NT), 0, s, U, n, np,
                     a, Z);
  PS_HIP(hipGetLastError());
}

// x(i, j) = 1 if i == j else 0 wherever i >= k or j >= k (kp x kp, ld kp): the padding
// of a k x k Gram matrix made the identity, so that its Cholesky factor and inverse are
// the identity there
__global__ void unit_pad_kernel(double* x, int k, int kp) {
  PS_GEN_LOOP(e, (size_t)kp * kp) {
    const int i = (int)(e % kp), j = (int)(e / kp);
    if (i >= k || j >= k) x[e] = i == j ? 1.0 : 0.0;
  }
}

void unit_pad(hipStream_t s, double* x, int k, int kp) {
  if (k == kp) return;
  hipLaunchKernelGGL(unit_pad_kernel, dim3(grid_for((size_t)kp * kp)), dim3(NT), 0, s, x, k, kp);
  PS_HIP(hipGetLastError());
}

}  // namespace ps
