// Internal declarations of the pseudosym HIP library (not part of the C-ABI).
//
// Storage convention inside the library: every m x m operand is held in a padded
// column-major buffer of size mp x mp (mp = m rounded up to a multiple of 64,
// leading dimension mp).  Padding rows/columns are kept block-diagonal with the
// real part (zeros off the diagonal block, and a positive constant on the padded
// diagonal of matrices that get factorized), so that no kernel needs bounds checks
// and the padded block never mixes into the real block.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "zolo_host.h"

namespace ps {

constexpr int kTile = 64;   // padding granule and GEMM tile edge
constexpr int kNb = 64;     // Cholesky diagonal block size
constexpr int kMaxSeg = 16; // K segments with separate scale (shift terms of one step)
constexpr int kMaxGroup = 4;

inline int pad_to(int m, int g = kTile) { return (m + g - 1) / g * g; }

struct HipError {
  hipError_t code;
  const char* where;
};

#define PS_HIP(call)                                                  \
  do {                                                                \
    hipError_t e_ = (call);                                           \
    if (e_ != hipSuccess) throw ::ps::HipError{e_, #call};            \
  } while (0)

// ----------------------------------------------------------------- static scratch
// Size of the file-scope device array behind pseudosym_divide_static (static_scratch.hip)
// and the address of the current device's copy (null if its lookup failed).
constexpr size_t kStaticScratchBytes = (size_t)128 << 20;
void* static_scratch_ptr();

// ----------------------------------------------------------------- FP64 GEMM
// D = alpha * op(A) op(B) + beta * C  for a grouped, two-level batched set of
// problems.  op(X) = X (t = 0) or X^T (t = 1); all matrices column-major.
enum GemmFlags : int {
  kOutUpper = 1,   // compute tiles I <= J only, store entries i <= j only
  kOutLower = 2,   // compute tiles I >= J only, store entries i >= j only
  kMirror = 4,     // also store D(j,i) = D(i,j) for the stored off-diagonal entries
  kAUpper = 8,     // op(A)(i,k) = 0 for k < i  (within each K segment)
  kALower = 16,    // op(A)(i,k) = 0 for k > i
  kBUpper = 32,    // op(B)(k,j) = 0 for k > j
  kBLower = 64,    // op(B)(k,j) = 0 for k < j
};

template <class T>
struct GemmProblemT {
  const T* A;
  const T* B;
  const T* C;
  T* D;
  long long sA[2], sB[2], sC[2], sD[2];  // strides of the two batch indices
  int M, N, K;
  int lda, ldb, ldc, ldd;
  int tA, tB, flags;
  int nb1, nb2;     // batch extents (batch index z = z1 + nb1 * z2)
  int kseg, nseg;   // K = nseg * kseg; segment s scales op(A) by kscale[s]
  int ksplit;       // > 1: split the K loop; partial products go to ws, then a reduction
  double alpha, beta;
  double kscale[kMaxSeg];
  T* ws;            // ksplit * M * N elements per batch entry (only when ksplit > 1)
  int ws_slots;     // ws holds ws_slots * M * N elements (0: unknown); the launcher may
                    // then use it for the partial tiles of a stream-K schedule
  // optional per-batch-entry scalars in device memory (entry z = z1 + nb1 * z2); when
  // set they replace alpha, beta and kscale (kscale_b[z * nseg + s])
  const double* alpha_b;
  const double* beta_b;
  const double* kscale_b;
  // filled by the launcher
  int tm, tn, tiles, tiles_per_batch, tile_begin;
};
using GemmProblem = GemmProblemT<double>;
using GemmProblemF = GemmProblemT<float>;

GemmProblem gemm_problem(int M, int N, int K, const double* A, int lda, int tA,
                         const double* B, int ldb, int tB, double* D, int ldd,
                         double alpha = 1.0, double beta = 0.0, const double* C = nullptr,
                         int ldc = 0, int flags = 0);
GemmProblemF gemm_problem(int M, int N, int K, const float* A, int lda, int tA, const float* B,
                          int ldb, int tB, float* D, int ldd, double alpha = 1.0,
                          double beta = 0.0, const float* C = nullptr, int ldc = 0,
                          int flags = 0);

// Autotuning of the GEMM launches.  A launch is identified by a key hashed from the
// sizes, transposes, flags, batch layout and split of its problems (not their pointers).
// A choice names the tile (64 or 128), a split-K factor (1: none) and whether to take the
// stream-K schedule; a choice that a launch cannot take (large tiles on a shape that is
// not a multiple of 128 of at least 512, a split without room for the partial tiles or on
// a batch) falls back to the legal one nearest to it.  All three hooks are per host
// thread: a table consulted by every launch, a choice forced on every launch (the
// tuner's trials), and a log of the launches issued (the tuner's inventory).
struct GemmChoice {
  int tile;
  int ksplit;
  int streamk;
};
struct GemmTuneTable {
  std::vector<unsigned long long> keys;
  std::vector<GemmChoice> choices;
};
struct GemmLog {
  std::vector<unsigned long long> keys;
  std::vector<std::vector<GemmProblem>> p64;   // per logged launch (empty for FP32)
  std::vector<std::vector<GemmProblemF>> p32;
};
void gemm_set_tuning(const GemmTuneTable* t);
const GemmTuneTable* gemm_get_tuning();
void gemm_set_force(const GemmChoice* c);
void gemm_set_log(GemmLog* log);

// Optional per-launch timing of the matrix-core kernels: when a recorder is set (for the
// calling host thread), every launch of a recorded class is bracketed by a pair of
// events on its own stream (a GEMM's window also covers its split-K reduction) and its
// algorithmic flops are noted.  Classes (ps_info.kclass_*):
enum KernelClass : int {
  kKcCholWide = 0,     // chol_step_kernel<double, wide>   (one or two matrices)
  kKcCholNarrow = 1,   // chol_step_kernel<double, narrow> (more matrices)
  kKcChol32 = 2,       // chol_step_kernel<float, *>
  kKcGemm128 = 3,      // FP64 GEMM, 128 x 128 tiles
  kKcGemm64 = 4,       // FP64 GEMM, 64 x 64 tiles
  kKcGemm32 = 5,       // FP32 GEMM, either tile
  kKcCount = 8
};
struct KernelRecorder {
  hipEvent_t* ev = nullptr;   // pairs (start, stop)
  double* flops = nullptr;    // per recorded window
  int* cls = nullptr;         // class per recorded window
  int* nl = nullptr;          // launches per recorded window
  int cap = 0;                // number of pairs available
  int n = 0;                  // pairs used
};
void kernel_set_recorder(KernelRecorder* r);
KernelRecorder* kernel_recorder();
// start / stop of one recorded window on stream s (no-ops without a recorder or room):
// one launch, or a run of back-to-back launches of one class (a Cholesky chain), so that
// no event separates them
int krec_begin(hipStream_t s);
void krec_end(hipStream_t s, int slot, int cls, double flops, int launches = 1);
template <class T>
double gemm_algorithmic_flops(const GemmProblemT<T>& p);

// Launch up to kMaxGroup independent problems in one kernel.  Problems with
// ksplit > 1 are followed by a reduction launch (sum of partials, beta C, triangle
// and mirror handling); their batch extent must be 1.
void gemm_f64(hipStream_t s, const GemmProblem* probs, int count);
inline void gemm_f64(hipStream_t s, const GemmProblem& p) { gemm_f64(s, &p, 1); }
// the same on FP32 operands (v_mfma_f32_16x16x4_f32, FP32 accumulation)
void gemm_f32(hipStream_t s, const GemmProblemF* probs, int count);
inline void gemm_f32(hipStream_t s, const GemmProblemF& p) { gemm_f32(s, &p, 1); }

// ----------------------------------------------------------------- Cholesky
// Kernel launches recorded for later issue (each closure enqueues on its own stream).
using LaunchList = std::vector<std::function<void()>>;
// Issue two recorded launch sequences alternately, one launch of each in turn, so that
// two independent chains on different streams both start at once whatever the host's
// launch rate.
void issue_interleaved(LaunchList& a, LaunchList& b);

// In-place upper Cholesky Z = R^T R of `batch` SPD matrices (mp x mp, ld = mp,
// matrix stride sz) with the strictly lower part zero on entry, producing the
// inverse factor W = R^{-1} (upper) in `w` (stride sw).  `tmp` is unused.  A
// non-positive pivot in matrix b sets bit min(b, 30) of the device int *info.  With
// `defer`, the launches are appended there instead of issued.  With `v` (mp x mp per
// matrix, stride sv, contents irrelevant, clobbered) and one or two matrices below the
// outer-block size, W is formed alongside the factorization instead of afterwards.
void potrf_inv_f64(hipStream_t s, double* z, long long sz, double* w, long long sw,
                   double* tmp, int mp, int batch, int* info, bool inverse = true,
                   LaunchList* defer = nullptr, double* v = nullptr, long long sv = 0);
// the same in FP32 (pivots taken and inverted through FP64 square roots)
void potrf_inv_f32(hipStream_t s, float* z, long long sz, float* w, long long sw, int mp,
                   int batch, int* info, LaunchList* defer = nullptr);

// ----------------------------------------------------------------- elementwise
void pack_casida(hipStream_t s, int m, int mp, const double* A, int lda, const double* B,
                 int ldb, double* mk);  // mk[0] = upper(A+B), mk[1] = upper(A-B), pad diag 1
void mask_pad(hipStream_t s, double* x, int m, int mp, long long stride, int batch);
void fill_zero(hipStream_t s, double* x, size_t n);
void zero_lower(hipStream_t s, double* x, int mp, long long stride, int batch);
void zero_lower(hipStream_t s, float* x, int mp, long long stride, int batch);
// zero `rows x cols` blocks (leading dimension ld) at x + b1*s1 + b2*s2
void zero_block(hipStream_t s, double* x, int rows, int cols, int ld, int nb1, long long s1,
                int nb2, long long s2);
void zero_block(hipStream_t s, float* x, int rows, int cols, int ld, int nb1, long long s1,
                int nb2, long long s2);
void transpose(hipStream_t s, const double* x, double* y, int mp, long long stride, int batch);
void form_shifts(hipStream_t s, const double* g, double* z, int mp, const double* shifts,
                 int r);   // z[j] = upper(G) + shifts[j] I, strictly lower zero
void scale_copy(hipStream_t s, const double* x, double* y, double a, size_t n);
void axpb_identity(hipStream_t s, const double* x, double* y, double a, double b, int mp);
void sign_blocks(hipStream_t s, const double* s12, const double* s21, double* as,
                 double* bs, int mp);   // A_s = sym(S21+S12)/2, B_s = sym(S21-S12)/2
void half_shift_upper(hipStream_t s, const double* as, double* p11, int mp);  // (I+A_s)/2
void basis_mix(hipStream_t s, const double* c, const double* qbot, double* top_out,
               double* ab, int mp);     // Q_top = C^T, a=(Q_top+Q_bot)/sqrt2, b=(..-..)/sqrt2
void copy_out(hipStream_t s, const double* x, int ldx, double* y, int ldy, int rows,
              int cols);
void diff_norms(hipStream_t s, const double* x1, const double* x2, size_t n, double* out2);
// Power steps on M - shift I (M symmetric, full storage, padded size mp, live size m) from
// a fixed start vector: out2 = (||v_k||^2, ||v_{k-1}||^2) after k = steps >= 1 products, so
// sqrt(out2[0] / out2[1]) estimates ||M - shift I||_2 from below.  v0, v1: mp doubles each.
void sym_power_norm(hipStream_t s, const double* M, int m, int mp, double shift, int steps,
                    double* v0, double* v1, double* out2);

// z = upper(scale (x + x^T)) on the first m rows/columns, 1 on the padded diagonal
void sym_scale_upper(hipStream_t s, const double* x, double* z, int m, int mp, double scale);
// top = c (e1 + e2), bot = c (e1 - e2)
void sum_diff_scaled(hipStream_t s, const double* e1, const double* e2, double* top, double* bot,
                     double c, int mp);

// mixed-precision helpers (mixed.hip)
void form_shifts_f32(hipStream_t s, const double* g, float* z, int mp, const double* shifts,
                     int r);   // z[j] = fp32(upper(G) + shifts[j] I)
void cvt_f64_f32(hipStream_t s, const double* x, float* y, size_t n);
void cvt_f32_f64(hipStream_t s, const float* x, double* y, size_t n);
void axpy_f32(hipStream_t s, double* y, double a, double b, const float* x, size_t n);
void axpb_identity_f32(hipStream_t s, const float* x, float* y, float a, float b, int mp);

// eigen-decomposition helpers (eig_f64.hip)
void shift_diag(hipStream_t s, double* y, int ld, int n, double b);   // y(i,i) += b, i < n
// z = upper(g) + c I on the first n diagonal entries, 1 on the padded diagonal
void spd_pad(hipStream_t s, const double* g, double* z, int n, int np, double c);
void get_diag(hipStream_t s, const double* x, int ld, int n, double* out);
// out[0] = sum of squares of the off-diagonal entries of the leading n x n block of x;
// out must hold 1 + 256 doubles
void offdiag_norm2(hipStream_t s, const double* x, int ld, int n, double* out);
// dst(i,j) = src(i,j) for i < rows, j < cols, 0 elsewhere in rows_pad x cols_pad
void copy_pad(hipStream_t s, const double* src, int lds, int rows, int cols, double* dst,
              int ldd, int rows_pad, int cols_pad);
void put_cols(hipStream_t s, const double* src, int lds, double* dst, int ldd, int o, int n,
              int rows);   // dst(:, o + j) = src(:, j), j < n
// dst(i,j) = sc src(ri[i], ci[j]) + dg [ri[i] == ci[j]] on rows x cols; padval on the
// padded diagonal, 0 elsewhere; upper_only: 0 below the diagonal
void gather_sym(hipStream_t s, const double* src, int lds, const int* ri, const int* ci, int rows,
                int cols, double sc, double dg, double* dst, int ldd, int rows_pad, int cols_pad,
                double padval, int upper_only);
// dst(ri[i], c0 + j) = trans ? src(j, i) : src(i, j)
void scatter_rows(hipStream_t s, const double* src, int lds, int trans, const int* ri, int rows,
                  int cols, double* dst, int ldd, int c0);
void permute_cols(hipStream_t s, const double* src, int lds, const int* perm, int rows, int cols,
                  double* dst, int ldd);
void permute_vec(hipStream_t s, const double* src, const int* perm, int n, double* dst);
void eig_lambda(hipStream_t s, const double* w, int m, double* lam);
void pi_columns(hipStream_t s, double* v, int ldv, int m);
void canon_sign(hipStream_t s, double* v, int ldv, int rows, int cols);
void jacobi_leaves(hipStream_t s, const double* b, int ld, const int* leaf_o, const int* leaf_n,
                   int nleaves, double* z, int ldz, double* lam, int* sweeps_out);
void fill_int_zero(hipStream_t s, int* x, int n);
// stored-factor adjoint of the sign blocks (adjoint_f64.hip): seeds g12 = sym(gA - gB)/2,
// g21 = sym(gA + gB)/2 padded to mp; y = x + x^T; x <- tril(x) with the diagonal halved;
// gA = sym(gm + gk), gB = sym(gm - gk) on the live block
void adj_seed(hipStream_t s, const double* ga, const double* gb, int ldg, int m, int mp,
              double* g12, double* g21);
void sym2(hipStream_t s, const double* x, double* y, int mp);
// S = [[S_A, S_B], [-S_B, -S_A]] (2m x 2m, ld lds2) from the blocks (m x m, ld lds)
void sign_full(hipStream_t s, const double* sa, const double* sb, int lds, int m, double* S,
               int lds2);
void phi_lower(hipStream_t s, double* x, int mp);
void adj_out(hipStream_t s, const double* gm, const double* gk, int mp, int m, double* ga,
             double* gb, int ldo);
// adjoint of the sign function (divided-difference form in the eigenbasis)
void build_gbar(hipStream_t s, const double* ga, const double* gb, int ldg, int m, double* g,
                int np);
void dk_hadamard(hipStream_t s, double* t, int np, const double* lam, int m);
void grad_assemble(hipStream_t s, const double* k, int np, int m, double* ga, double* gb,
                   int ldo);

// division for any signature (general.hip); sg holds sigma (0 beyond n)
void pack_general(hipStream_t s, int n, int np, const double* H, int ldh, const double* sg,
                  double* m);   // upper(sym(Sigma H)), pad diag 1
void scale_signs(hipStream_t s, const double* x, double* y, int n, int np, const double* sg,
                 bool cols);    // y = Sigma x (rows) or x Sigma (cols), zero padding
void lead_block(hipStream_t s, const double* S, int lds, const double* sg, int k, int kp, double a,
                double* out);   // upper(sym(Sigma (a I + S)/2)) on the leading k x k, pad diag 1
void chol_top(hipStream_t s, const double* c, int kp, const double* sg, int k, double t,
              double* top);     // top(i, j) = t sigma_i C(j, i)
void proj_form(hipStream_t s, const double* U, int n, int np, double a,
               double* Z);      // upper((I + a sym(U))/2), zero padding
void unit_pad(hipStream_t s, double* x, int k, int kp);   // identity outside the leading k x k

// Golub-Kahan bidiagonalization (batch of two matrices M_b with transposes Mt_b).
void gk_init(hipStream_t s, double* v, int m, int mp, int batch, unsigned seed);
// batched division (batch.hip): per-matrix scalars from device arrays
void scale_b(hipStream_t s, const double* x, long long sx, double* y, long long sy,
             const double* f, size_t n, int nb);
void form_shifts_b(hipStream_t s, const double* g, double* z, int mp, const double* c, int r,
                   int nb);
void axpb_identity_b(hipStream_t s, const double* x, double* y, const double* a,
                     const double* c, int mp, int nb);
void diff_norms_b(hipStream_t s, const double* x1, const double* x2, size_t n, double* out,
                  int nb);
void gk_init_b(hipStream_t s, double* v, const int* m_dev, int mp, int count, int per);
// the Alg. 6 tail of a class: the single-problem kernels over nb problems (stride mp^2;
// ab and its halves stride 2 mp^2); mask_pad_b zeroes rows and columns >= m_dev[q / per]
// of matrix q for q < count
void sign_blocks_b(hipStream_t s, const double* s12, const double* s21, double* as, double* bs,
                   int mp, int nb);
void half_shift_upper_b(hipStream_t s, const double* as, double* p11, int mp, int nb);
void basis_mix_b(hipStream_t s, const double* c, const double* qbot, double* top_out, double* ab,
                 int mp, int nb);
void mask_pad_b(hipStream_t s, double* x, const int* m_dev, int mp, int per, int count);
// Bidiagonalization half-steps with unnormalized vectors and per-workgroup partial
// sums of squares (gk_parts(mp) per batch item): gk_seed writes the partials of a unit
// vector, gk_step forms w~ = M x / ||x~|| - ||x~|| wprev~ / ||wprev~|| (wprev null: none)
// and stores ||x~|| at hist[hist_x], gk_finish stores the norm of the last vector.
int gk_parts(int mp);
void gk_seed(hipStream_t s, double* part, int mp, int batch);
void gk_step(hipStream_t s, const double* mat, long long mstride, const double* x,
             long long xstride, const double* xpart, double* w, long long wstride,
             const double* wprev, long long wpstride, const double* wppart, double* wpart,
             double* hist, int hist_x, int hist_ld, int mp, int batch);
void gk_finish(hipStream_t s, const double* part, int mp, double* hist, int hist_out, int hist_ld,
               int batch);

// ----------------------------------------------------------------- Alg. 7 (ldl_f64.hip)
// Truncated LDL^T with 1x1 pivots and diagonal pivoting of a positive semidefinite Z of
// rank k (upper triangle, n x n in np x np, np a multiple of 64 up to kLdlMaxN), by
// panels of kLdlPanel pivots chosen greedily among the kLdlCand largest Schur diagonals.
// C (np x pad(k), ld np) gets L D^{1/2} in the original row order; Z is overwritten by
// Schur complements.  info[0] = 1 on a non-positive pivot.
constexpr int kLdlPanel = 64;
constexpr int kLdlCand = 128;
constexpr int kLdlMaxN = 16384;
struct LdlScratch {
  double* L;   // 64 x 64: the panel's pivot factor L_pp
  int* piv;    // pad(k): pivots in the order taken
  int* mask;   // np: rows pivoted so far
};
void ldl_factor(hipStream_t s, double* Z, int n, int np, int k, double* C, const LdlScratch& w,
                int* info);
// Z = (Sigma S + a Sigma)/2 (upper triangle): a = +1 gives Sigma P_+, a = -1 gives
// -Sigma P_-.  Casida form from the sign blocks (n = 2m), or any signature from S.
void ldl_form_casida(hipStream_t s, const double* as, const double* bs, int m, int mp, int np,
                     double a, double* Z);
void ldl_form_general(hipStream_t s, const double* S, const double* sg, int n, int np, double a,
                      double* Z);
void ldl_casida_out(hipStream_t s, const double* C, int np, int m, int mp, double* top,
                    double* qbot, double* ab);
void ldl_scale_rows(hipStream_t s, const double* C, int np, int kp, const double* sg, int n,
                    double* Q);

// ----------------------------------------------------------------- complex forms (hermitian.hip)
// Interleaved realification of a complex m x m matrix (double pairs, ld in complex
// entries) into a real 2m x 2m one: each entry becomes [[re, -im], [im, re]] (flip = 0)
// or [[re, im], [im, -re]] (flip = 1); complexify reads (re, im) back from the first
// column of each 2 x 2 block (rows x cols complex).
void realify(hipStream_t s, const double* X, int ldx, int m, double* Y, int ldy, int flip);
void complexify(hipStream_t s, const double* Y, int ldy, int rows, int cols, double* X, int ldx);
// the nearest realified matrix: each 2 x 2 block becomes [[re, -im], [im, re]] with re and
// im the averages of their two copies (m2 even)
void pair_project(hipStream_t s, double* X, int m2, int ldx);

}  // namespace ps
