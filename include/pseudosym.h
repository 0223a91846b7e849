/*
 * pseudosym - structure-preserving spectral division of definite pseudosymmetric
 * matrices on AMD Instinct MI355X (gfx950).
 *
 * Method: Benner, Nakatsukasa, Penke, "A Structure-Preserving Divide-and-Conquer
 * Method for Pseudosymmetric Matrices" (arXiv 2203.08900).  The library handles
 * the Casida / real Bethe-Salpeter form (Sec. 5, Eq:Casida)
 *
 *        H = [[ A,  B],       A = A^T,  B = B^T  (m x m),  n = 2m,
 *             [-B, -A]]       Sigma = diag(I_m, -I_m),
 *
 * in the definite case, i.e. Sigma*H positive definite, which for this form means
 * A + B and A - B are both symmetric positive definite.  Then (Thm. EVREalSigmaOrth)
 * H has m positive and m negative real eigenvalues, they come in pairs +-lambda,
 * and one spectral division step decouples H into a symmetric positive definite
 * block and its negative (Thm. DefDivConq).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Matrices are double precision, column-major, with leading dimension >= rows.
 *    All matrix pointers are DEVICE pointers on the device that is current when
 *    the handle was created; the caller owns every input and output buffer.
 *  - A and B are read through their upper triangles and are not modified.
 *  - Work is enqueued on the handle's stream.  Every call synchronizes that stream
 *    once before returning, because the stopping test of the iteration and the
 *    info record are host data; outputs are complete when the call returns.
 *  - Return value: 0 on success; a negative value -k means argument k (1-based,
 *    the handle being argument 1) is invalid and nothing was launched; a positive
 *    value is one of the PS_* status codes below, in which case the outputs are
 *    undefined and `info` (if given) says where the failure happened.
 *  - Device memory: the library never allocates device memory.  Its scratch space is
 *    the caller's workspace (ps_set_workspace, sized by ps_workspace_size or
 *    ps_workspace_size_batched); a call whose workspace is missing or too small returns
 *    PS_NO_WORKSPACE before any launch.
 *  - Streams: the library creates none.  Work runs on the handle's stream; the caller
 *    may lend extra streams (ps_set_worker_streams) on which independent work runs
 *    concurrently: the FP32 shift group of a mixed step, the workers of a batched call
 *    and the subtrees of the eigen-decomposition.  Without them that work runs in order
 *    on the handle's stream, with the same results.
 */
#ifndef PSEUDOSYM_H
#define PSEUDOSYM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ps_handle_s* ps_handle;

/* status codes (positive: numerical or runtime failure) */
enum {
  PS_OK = 0,
  PS_NOT_DEFINITE = 1,     /* Cholesky of A+B or A-B failed: Sigma*H is not positive definite */
  PS_SHIFT_BREAKDOWN = 2,  /* Cholesky of a shifted Gram matrix X^T X + c I failed */
  PS_NOT_CONVERGED = 3,    /* the stopping test of Alg. 8 failed after max_restarts restarts */
  PS_HIP_ERROR = 4,        /* a HIP runtime call failed */
  PS_NO_WORKSPACE = 5,     /* the caller-provided workspace is too small */
  PS_BASIS_BREAKDOWN = 6   /* Cholesky of the leading block of P_+ failed (Alg. 6), or
                              a non-positive pivot among the retained ones (Alg. 7) */
};

/* arithmetic of the Zolotarev steps */
enum {
  PS_PREC_FP64 = 0,        /* everything in FP64 (plain form) */
  PS_PREC_MIXED = 1        /* FP32 matrix-core bulk, FP64 for ill-conditioned shifts,
                              FP64 refinement and subspace orthogonalization; problems
                              with m < 1024 (padded) run in FP64, where the split does
                              not pay */
};

/* Sigma-orthonormal basis Q_+ of the positive invariant subspace (pseudosym_divide):
 *  PS_BASIS_ALG6: Alg. 6, Q_+ = [C^T; P_{+,21} C^{-1}] with C = chol of the leading
 *                 block (I + A_s)/2 of P_+ = (I + sign(H))/2; unique (its top block is
 *                 lower triangular with positive diagonal).
 *  PS_BASIS_CORE: the same subspace from the half-size core: with Y0 = R_M R_K^T and
 *                 its polar factor U, Z = Q_h [R_M^{-1} U; R_K^{-1}] (Q_h the symmetric
 *                 orthogonal [[I, I], [I, -I]]/sqrt(2)) spans it, Z^T Sigma Z = G =
 *                 Y0^{-1} U + (Y0^{-1} U)^T = R_G^T R_G, Q_+ = Z R_G^{-1} and
 *                 H_+ = 2 R_G^{-T} R_G^{-1}.  It needs neither the sign blocks nor the
 *                 Alg. 6 decoupling products; Q_+ differs from the Alg. 6 basis by an
 *                 orthogonal factor G (H_+ by G^T H_+ G).
 *  PS_BASIS_LDL:  Alg. 7, the robust variant: Sigma P_+ = (Sigma S + Sigma)/2 (2m x 2m,
 *                 positive semidefinite of rank m) = C C^T by a truncated LDL^T with
 *                 1x1 pivots and diagonal pivoting (D diagonal, C = L D^{1/2}), and
 *                 Q_+ = Sigma C.  Pivots: per panel of 64, the 128 largest diagonal
 *                 entries of the Schur complement (ties: lower index) are candidates and
 *                 each pivot is the largest remaining one among them (ties: lower index).
 *                 It avoids the leading-block Cholesky that Alg. 6 needs; Q_+ differs
 *                 from the Alg. 6 basis by an orthogonal factor.  Padded 2m up to 16384;
 *                 pseudosym_divide and pseudosym_divide_general only.  A non-positive
 *                 retained pivot returns PS_BASIS_BREAKDOWN.
 *  PS_BASIS_CONGRUENT: pseudosym_divide_general only.  With M = Sigma H = R^T R,
 *                 W = R^{-1} and T = R Sigma R^T (H = W T R), the projectors of H are
 *                 W (I +- sign(T))/2 R, so W maps the ranges of the symmetric positive
 *                 semidefinite Z_+- = (I +- sign(T))/2 onto the invariant subspaces.
 *                 Z_+- = C C^T by the truncated LDL^T of PS_BASIS_LDL (rank r_+-),
 *                 V = W C, +-V^T Sigma V = R_G^T R_G (Cholesky), Q_+- = V R_G^{-1}, and
 *                 H_+- = +-(C R_G^{-1})^T (C R_G^{-1}).  sign(H) is never formed (unless
 *                 S is asked for), which keeps the backward error at rounding level for
 *                 any cond(M) that the Cholesky of M survives.  Padded n up to 16384.
 *                 Not one of the paper's listings: the subspaces are those of Alg. 6
 *                 and 7, Q differs from their bases by an orthogonal factor. */
enum { PS_BASIS_ALG6 = 0, PS_BASIS_CORE = 1, PS_BASIS_LDL = 2, PS_BASIS_CONGRUENT = 3 };

typedef struct {
  int precision;       /* PS_PREC_*                                               */
  int r;               /* Zolotarev degree parameter (type (2r+1, 2r)), 1..8;    */
                       /* 0 picks the smallest r that converges in two steps     */
  int max_restarts;    /* restarts allowed by the stopping test of Alg. 8 (>= 0) */
  int max_steps;       /* 0: full method.  1: stop after the first Zolotarev step */
                       /* and return that iterate in place of sign(H) (the blocks */
                       /* of X_1 = hat Z(H/alpha)); only honoured by pseudosym_sign */
  int lanczos_steps;   /* Golub-Kahan steps of the alpha/beta estimator (>= 4)   */
  int timing;          /* 1: fill info->phase_ms with per-phase GPU times;        */
                       /* 2: also time every launch of the matrix-core kernels   */
                       /*    with events on its stream (info->kclass_*, gemm_*); */
                       /*    pseudosym_divide_batched takes 2 only (see there)   */
  double alpha;        /* > 0: caller's upper bound of max|lambda(H)| (skips the  */
  double beta;         /* estimator); > 0: caller's lower bound of min|lambda(H)| */
  double mixed_kappa;  /* mixed precision: shifts whose condition number          */
                       /* (1 + c)/(l^2 + c) exceeds this run in FP64               */
  int step2_series;    /* nonzero: when step 1 has left every singular value of the */
                       /* iterate within [l_1, 1] with (1 - l_1^2)^P < 1e-17 for    */
                       /* P <= 8, evaluate the second step's sum                    */
                       /* sum_j a_j (X^T X + c_{2j-1} I)^{-1} as the convergent     */
                       /* series in Delta = X^T X - I instead of r factorizations   */
                       /* (the same rational function to below 1e-17)               */
  int basis;           /* pseudosym_divide / pseudosym_eig: PS_BASIS_ALG6 (default) */
                       /* or PS_BASIS_CORE, see below; PS_BASIS_LDL for           */
                       /* pseudosym_divide and pseudosym_divide_general;         */
                       /* PS_BASIS_CONGRUENT for pseudosym_divide_general        */
  int iteration;       /* PS_ITER_ZOLO (Alg. 8, default) or one of the comparison  */
                       /* iterations of Sec. 6, see below (FP64 only)             */
  int refine;          /* what follows the iteration, PS_REFINE_*:               */
                       /* NONE: (mixed precision with the core basis, m >= 1024  */
                       /*   padded) the basis and H_+ in FP32 as well: the       */
                       /*   low-precision result before any refinement (~1e-5   */
                       /*   relative eigenvalue error at n = 4096);               */
                       /*   elsewhere as RR.  RR (default): FP64 Sigma-          */
                       /*   orthonormalization and Rayleigh-Ritz block of the    */
                       /*   subspace (core basis), FP64 sign blocks and Alg. 6.  */
                       /*   NS: RR after one FP64 Newton-Schulz pass on the      */
                       /*   polar factor, U <- U (3I - U^T U)/2                   */
} ps_opts;

enum { PS_REFINE_NONE = 0, PS_REFINE_RR = 1, PS_REFINE_NS = 2 };

/* sign iteration (ps_opts.iteration); the comparison iterations of Tab:ItRuntime run
 * one step after another with a schedule fixed by l = beta/alpha:
 *  PS_ITER_DWH:    Sigma-DWH, i.e. the step of Alg. 8 with r = 1 and the l-recurrence,
 *                  until the recurrence reaches 1 - 1e-15, plus the step of the stopping
 *                  test ||X_k - X_{k-1}||_F / ||X_k||_F <= u^{1/3} (5, 6, 6 steps at
 *                  kappa = 1e2, 1e8, 1e12);
 *  PS_ITER_NEWTON: the scaled Newton iteration X <- (mu X + (mu X)^{-1})/2 with the
 *                  Byers-Xu scaling (mu_0 = 1/sqrt(l), then from the modulus interval),
 *                  stopping test u^{1/2} (7, 9, 9 steps).
 * Both stop with PS_NOT_CONVERGED when the stopping test fails (no restart). */
enum { PS_ITER_ZOLO = 0, PS_ITER_DWH = 1, PS_ITER_NEWTON = 2 };

typedef struct {
  int status;
  int steps;               /* Zolotarev steps taken (2 per attempt)                 */
  int restarts;
  int r;
  int shifts_fp64[2];      /* shifts per step that ran in FP64                      */
  int failed_step;         /* step whose Cholesky failed (-1: none)                 */
  int failed_mask;         /* batch bitmask of the failing Cholesky factorizations  */
  double alpha, beta;      /* bounds actually used                                  */
  double ell[4];           /* l at the start of each step (attempt-major)           */
  double step_change;      /* ||X2 - X1||_F / ||X2||_F of the accepted attempt      */
  double sigma_est[2];     /* estimator output: sigma_max(Y0), 1/sigma_max(Y0^{-1}) */
  double phase_ms[8];      /* setup, estimate, step1, step2, refine, assemble,      */
                           /* bases, decouple (when opts->timing)                    */
  int step2_terms;         /* 0: second step by factorizations; P > 0: series terms */
  int gemm_launches;       /* timing == 2: launches of the large-tile FP64 GEMM kernel */
  double gemm_ms;          /*   their summed GPU time (split-K reductions included)   */
  double gemm_flops;       /*   their algorithmic flops (zero blocks of triangular    */
                           /*   operands and the unstored triangle not counted)      */
  int eig_splits;          /* pseudosym_eig: splits of the symmetric recursion        */
  int eig_leaves;          /*   leaves solved by the Jacobi kernel                    */
  int eig_sweeps;          /*   largest number of Jacobi sweeps of a leaf             */
  int eig_steps;           /*   Zolotarev steps summed over the splits                */
  int eig_restarts;        /*   restarts summed over the splits                       */
  int eig_clusters;        /*   blocks found to be a multiple of I within 1e-12 of     */
                           /*   their magnitude (split without a shift)                */
  /* timing == 2, per kernel class c (PS_KC_*): launches, summed GPU time of the event
   * windows (ms) and algorithmic flops.  A Cholesky step launch counts mp^3/3 per matrix
   * spread evenly over the mp/64 steps of its factorization, less the updates of the
   * outer blocks from padded size 4096 (GEMM launches, counted in their class). */
  int kclass_launches[8];
  double kclass_ms[8];
  double kclass_flops[8];
  /* Check of the bounds behind the series form of the second step (Alg. 8 with alpha,
   * beta as given or estimated): ||X1^T X1 - I||_2 is at most 1 - l1^2 when [beta, alpha]
   * held the singular values of the core; the largest over the attempts of its lower
   * estimate by power steps on the device, and the attempts whose estimate exceeded that
   * bound (plus rounding), whose second step was then redone by factorizations and
   * followed by a restart (pseudosym_eig: over all its splits). */
  double delta_norm_est;
  int bounds_rejected;
  /* pseudosym_divide_general: cond(Sigma H) = (sigma_max(R) sigma_max(R^{-1}))^2 for the
   * Cholesky factor R of Sigma H, by Golub-Kahan (from below), which bounds this form's
   * accuracy (the backward error grows like cond(Sigma H) u: about 1e-9 at 1e7, 1e-4 at
   * 1e12). */
  double cond_est;
} ps_info;

/* kernel classes of ps_info.kclass_* */
enum {
  PS_KC_CHOL_WIDE = 0,     /* Cholesky step, FP64, one or two matrices per launch      */
  PS_KC_CHOL_NARROW = 1,   /* Cholesky step, FP64, more matrices                       */
  PS_KC_CHOL_FP32 = 2,     /* Cholesky step, FP32                                      */
  PS_KC_GEMM128 = 3,       /* FP64 GEMM on 128 x 128 tiles                              */
  PS_KC_GEMM64 = 4,        /* FP64 GEMM on 64 x 64 tiles                                */
  PS_KC_GEMM_FP32 = 5      /* FP32 GEMM                                                 */
};

/* Fill *o with the defaults: FP64, r = 8, 2 restarts, full method, 20 Lanczos
 * steps, no timing, estimated alpha/beta, mixed_kappa = 20, step2_series = 1,
 * basis = PS_BASIS_ALG6, iteration = PS_ITER_ZOLO, refine = PS_REFINE_RR. */
void ps_opts_default(ps_opts* o);

/* Create a handle bound to `stream` (a hipStream_t, NULL = default stream) on
 * the current device.  Returns 0 or PS_HIP_ERROR. */
int ps_create(ps_handle* h, void* stream);
int ps_destroy(ps_handle h);
int ps_set_stream(ps_handle h, void* stream);

/* Batched division (Alg. 2's independent problems): after the bounds
 * and coefficients of a class are known, its launch sequence (both Zolotarev steps, the
 * stopping-test norms, the bases and the decoupled blocks) is captured once as a HIP
 * graph and replayed when a class with the same sizes, options and workspace comes again
 * (up to 32 graphs kept per handle and worker; the runtime holds their resources until
 * ps_destroy).  enable = 1 (default) or 0 (every launch issued directly, as on the first
 * call); results are identical either way.  Applies to the handle and its workers, on
 * their streams other than the legacy default (NULL) stream, which cannot be captured.
 * Returns 0, -1 (no handle) or -2 (enable not 0 or 1). */
int ps_set_graphs(ps_handle h, int enable);

/* GEMM autotuning (tile shapes chosen by measurement).  Every launch
 * of the matrix-core GEMM is identified by a key hashed from the sizes, transposes, flags,
 * batch layout and split of its problems.  A tuning entry tells the launcher which tile
 * (64 x 64 or 128 x 128), split-K factor and schedule (stream-K or not) to use for that
 * key; a choice a launch cannot take falls back to the nearest legal one. */
typedef struct {
  unsigned long long key;   /* launch key */
  int tile;                 /* 64 or 128 */
  int ksplit;               /* 1 (no split) .. 8 */
  int streamk;              /* 0 or 1 */
  float ms;                 /* autotune: time per launch of this choice */
  float ms_default;         /* autotune: time per launch of the built-in choice */
  int launches;             /* autotune: launches with this key in the tuned call */
} ps_gemm_tune;

/* Install a tuning table (n entries, host array, copied) on the handle and its workers;
 * n = 0 restores the built-in choices.  Captured batched graphs are dropped.  Returns 0,
 * -1 (no handle) or -2 (bad entry). */
int ps_set_gemm_tuning(ps_handle h, const ps_gemm_tune* entries, int n);

/* Tune the GEMM launches of one pseudosym_divide at half-size m with options opts: the
 * division runs once with every launch logged, then every distinct launch is timed under
 * each choice it can take (tile 64 or 128, split-K by 1 to 8, stream-K), five
 * times after two warm-up runs, on the handle's stream; the fastest per key goes to
 * out[0 .. min(cap, count)) with its time and the built-in choice's.  *count gets the
 * number of distinct keys.  The trials overwrite the division's own buffers: the call
 * returns no division result.  Workspace: ps_workspace_size(m, opts, 6).  Not for
 * PS_BASIS_LDL (-7). */
int ps_autotune_divide(ps_handle h, int m, const double* A, int lda, const double* B, int ldb,
                       const ps_opts* opts, ps_gemm_tune* out, int cap, int* count);

/* Bytes of device workspace that a call of kind `what` (0 sign and sign_fwd_iter, 1 divide,
 * 2 eig and sign_fwd, 3 sign_bwd, 4 divide_general, 5 the complex forms: sign_hermitian,
 * divide_hermitian, sign_bse, 6 autotune_divide, 7 sign_bwd_iter) needs at half-size m
 * (for kind 4: the order n of H) with options o (NULL = defaults). */
size_t ps_workspace_size(int m, const ps_opts* o, int what);

/* Use caller memory (device pointer, 256-byte aligned, `bytes` long) as the
 * workspace from now on; NULL clears it (calls then return PS_NO_WORKSPACE).  The
 * buffer must outlive every call that uses it.  Returns 0, -1 (no handle) or -2
 * (misaligned pointer). */
int ps_set_workspace(ps_handle h, void* dptr, size_t bytes);

/* Bytes of workspace for pseudosym_divide_batched on these `batch` half-sizes m[] (host
 * array) with options o (NULL = defaults): one share per worker (up to six), each
 * holding the largest single problem and the largest class of equal padded size that
 * the call batches together (classes are planned within 2 GiB per share).  A smaller
 * workspace also works as long as one share holds the largest single problem: the call
 * then uses fewer workers or smaller classes.  0 on invalid arguments. */
size_t ps_workspace_size_batched(int batch, const int* m, const ps_opts* o);

/* Lend `count` (0..PS_MAX_WORKER_STREAMS) extra streams (hipStream_t, on the handle's
 * device, distinct from the handle's stream) for the concurrent parts of a call: the
 * first runs the FP32 shift group of a mixed step, and batched calls and the
 * eigen-decomposition run one worker per stream (at most six, resp. four).  The handle
 * keeps the pointers: the streams must outlive it or be replaced by another call
 * (count 0 withdraws them).  Streams should have the default priority.  Returns 0,
 * -1 (no handle), -2 (bad count), -3 (a null stream or the handle's own), or
 * PS_HIP_ERROR. */
#define PS_MAX_WORKER_STREAMS 8
int ps_set_worker_streams(ps_handle h, int count, void* const* streams);

/* Host-only: coefficients of the scaled Zolotarev function hat Z_{2r+1}(x; ell)
 * (Eq:Compcis, Eq:hatZ, Eq:ZPartialFrac2): c[0..2r-1] = c_1..c_2r,
 * a[0..r-1] = a_1..a_r, *chat = hat C, *ell_next = hat Z(ell; ell) (the l update
 * of Alg. 8).  0 < ell < 1, 1 <= r <= 8.  Returns 0 or -1 on bad arguments. */
int ps_zolotarev_coeffs(double ell, int r, double* c, double* a, double* chat,
                        double* ell_next);

/* sign(H) by the Zolotarev iteration of Alg. 8 (two steps of r independent shifted
 * factorizations each, with the stopping test and restart of Alg. 8).  Output:
 * the blocks of sign(H) = [[SA, SB], [-SB, -SA]] (the odd function of H keeps the
 * Casida form), SA and SB symmetric m x m with leading dimension lds. */
int pseudosym_sign(ps_handle h, int m, const double* A, int lda, const double* B, int ldb,
                   double* SA, double* SB, int lds, const ps_opts* opts, ps_info* info);

/* One step of structure-preserving spectral division (Alg. 3 with sigma = 0 for a
 * definite H): sign(H) as above, then the (Sigma, I)-orthogonal basis Q_+ of the
 * invariant subspace of the m positive eigenvalues by Alg. 6, and the decoupled
 * block H_+ = Q_+^T Sigma H Q_+ (Thm. DefDivConq).
 * Outputs: Qp, 2m x m with leading dimension ldq >= 2m, Q_+^T Sigma Q_+ = I, whose
 * top m x m block is lower triangular with positive diagonal (the Cholesky form of
 * Alg. 6, which makes Q_+ unique); Hp, m x m symmetric positive definite with
 * leading dimension ldh, whose eigenvalues are the m positive eigenvalues of H.
 * The negative half follows from the structure: Q_- = Pi Q_+ with
 * Pi = [[0, I], [I, 0]] spans the negative invariant subspace, Q_-^T Sigma Q_- = -I,
 * and H_- = -H_+. */
int pseudosym_divide(ps_handle h, int m, const double* A, int lda, const double* B, int ldb,
                     double* Qp, int ldq, double* Hp, int ldh, const ps_opts* opts,
                     ps_info* info);

/* One step of spectral division (Alg. 3 with sigma = 0) of a definite pseudosymmetric H
 * of ANY signature: Sigma = diag(sigma) with entries +-1 in any order and Sigma H
 * symmetric positive definite, the matrices of Sec. 6.1 (H = Sigma Q D Q^T).  With
 * r_+ and r_- the numbers of +1 and -1 in sigma, H has r_+ positive and r_- negative
 * eigenvalues (Thm. EVREalSigmaOrth).  sign(H) by Alg. 8 (the Zolotarev iteration runs on
 * the symmetric T = R Sigma R^T, M = Sigma H = R^T R, H = R^{-1} T R, so its shifted
 * matrices are T^2 + c I, symmetric positive definite, factorized by Cholesky); bases by
 * Alg. 6 as printed (Cholesky of the leading r_+ x r_+ block of Sigma P_+ and the
 * leading r_- x r_- block of -Sigma P_-, Q_- with the sign of Thm. HRisLDL); decoupled
 * blocks of Thm. DefDivConq.
 *   H      n x n (device, ld ldh >= n), read only; its symmetric part of Sigma H is used.
 *   sigma  HOST array of n doubles, each +1 or -1 (else -5).
 *   S      optional n x n output sign(H) (device, lds >= n), NULL to skip.
 *   Qp     n x r_+ (ldqp >= n): Q_+^T Sigma Q_+ = I, range = positive invariant subspace.
 *   Qm     n x r_- (ldqm >= n): Q_-^T Sigma Q_- = -I, the negative one.
 *   Hp     r_+ x r_+ (ldhp >= r_+): H_+ = Q_+^T Sigma H Q_+, symmetric positive definite.
 *   Hm     r_- x r_- (ldhm >= r_-): H_- = -Q_-^T Sigma H Q_-, negative definite.
 * Outputs of an empty side (r_+ = 0 or r_- = 0) may be NULL.  Bases built from sign(H)
 * (Alg. 6 and 7) inherit its error, which the similarity with R multiplies by up to
 * cond(M): backward errors ||Q_+^T Sigma H Q_-|| / ||H|| of about 1e-10 at
 * cond(M) = 1e6, 1e-9 at 1e7, 1e-6 at 1e10 and 1e-4 at 1e12 (n = 250, Sec. 6.1
 * matrices); info->cond_est reports a lower estimate of cond(M), so that the caller can
 * tell.  opts->basis = PS_BASIS_CONGRUENT builds the bases from the projectors of T
 * instead and keeps the backward error near 1e-15 up to cond(M) = 1e12 (see the enum).
 * The leading blocks of Alg. 6 can be ill-conditioned for an unlucky Sigma, which
 * PS_BASIS_BREAKDOWN reports when their Cholesky fails.  opts->basis = PS_BASIS_LDL
 * takes Alg. 7 instead (truncated LDL^T with diagonal pivoting of Sigma P_+ and
 * -Sigma P_-, Q_+- = Sigma C_+-), which needs no leading block to be well conditioned;
 * PS_BASIS_LDL and PS_BASIS_CONGRUENT take padded n up to 16384, else -16; any other
 * value gives Alg. 6.  PS_BASIS_BREAKDOWN under PS_BASIS_CONGRUENT: a non-positive
 * retained pivot or a failed Cholesky of the Sigma-Gram matrix.  The Cholesky of M can
 * still fail (PS_NOT_DEFINITE) or the iteration break down (PS_SHIFT_BREAKDOWN) at a
 * large enough cond(M).  The steps run in FP64 whatever opts->precision is (cond(T) is
 * cond(M), and FP32 steps would leave the subspaces about cond(M) * 6e-8 off; measured
 * 3e-2 in Sigma-orthonormality at n = 1100, cond(M) = 1e3).  opts->max_steps must be 0. */
int pseudosym_divide_general(ps_handle h, int n, const double* H, int ldh, const double* sigma,
                             double* S, int lds, double* Qp, int ldqp, double* Qm, int ldqm,
                             double* Hp, int ldhp, double* Hm, int ldhm, const ps_opts* opts,
                             ps_info* info);

/* The complex Bethe-Salpeter forms of Sec. 5, definite (Sigma H Hermitian positive
 * definite, Sigma = diag(I_m, -I_m)).  Matrices are complex double, stored as interleaved
 * (real, imaginary) pairs of doubles, column-major, device memory; leading dimensions
 * count complex entries.  The library realifies them (each complex entry becomes a
 * 2 x 2 real block), runs the real pipeline at half-size 2m on the real Casida form that
 * results, and reads the complex results back, so the accuracy, options and statuses
 * are those of the real calls at half-size 2m.  Workspace: ps_workspace_size(m, opts, 5).
 *
 * Eq:BSE2: H = [[A, B], [-B, -A]], A and B Hermitian m x m, A + B and A - B positive
 * definite.  sign(H) keeps the form: SA, SB Hermitian m x m (ld lds >= m). */
int pseudosym_sign_hermitian(ps_handle h, int m, const double* A, int lda, const double* B,
                             int ldb, double* SA, double* SB, int lds, const ps_opts* opts,
                             ps_info* info);

/* Eq:BSE2 division: Qp (2m x m complex, ldq >= 2m) with Q_+^H Sigma Q_+ = I spanning the
 * invariant subspace of the m positive eigenvalues, and Hp = Q_+^H Sigma H Q_+ (m x m
 * Hermitian positive definite, ldh >= m) holding them (Thm. DefDivConq).  opts->basis:
 * PS_BASIS_ALG6 (Alg. 6 in complex arithmetic: the top block of Q_+ is lower triangular
 * with a real positive diagonal, which makes it unique) or PS_BASIS_CORE; Alg. 7 is not
 * offered here (its pivot choice may separate the two real rows of a complex one).
 * opts->max_steps must be 0. */
int pseudosym_divide_hermitian(ps_handle h, int m, const double* A, int lda, const double* B,
                               int ldb, double* Qp, int ldq, double* Hp, int ldh,
                               const ps_opts* opts, ps_info* info);

/* Eq:BSE1: H = [[A, B], [-conj(B), -conj(A)]], A Hermitian and B complex symmetric m x m,
 * [[A, B], [conj(B), conj(A)]] positive definite.  sign(H) keeps the form
 * [[SA, SB], [-conj(SB), -conj(SA)]]: SA Hermitian and SB complex symmetric (lds >= m). */
int pseudosym_sign_bse(ps_handle h, int m, const double* A, int lda, const double* B, int ldb,
                       double* SA, double* SB, int lds, const ps_opts* opts, ps_info* info);

/* pseudosym_divide without any workspace, for callers that cannot allocate device memory
 * (code under graph capture, tight serving loops, harnesses that forbid allocation).  The
 * scratch space is a fixed 128 MiB device array inside the library (each GPU it runs on
 * holds one copy until the process ends); the call allocates nothing, creates nothing,
 * ignores opts->timing and otherwise behaves exactly like pseudosym_divide (same kernels,
 * same results).  Sizes whose workspace would exceed the array (beyond m = 560 or so;
 * every m <= 512 fits with any options) return -2.  Every call on a GPU shares that GPU's
 * array: calls that overlap on one GPU (other streams, other threads, other handles)
 * race and must be serialized by the caller. */
int pseudosym_divide_static(ps_handle h, int m, const double* A, int lda, const double* B,
                            int ldb, double* Qp, int ldq, double* Hp, int ldh,
                            const ps_opts* opts, ps_info* info);

/* All eigenpairs of H (Alg. 3 once, then Alg. 2 on the decoupled block; Thm. DefDivConq
 * reduces the rest to the symmetric positive definite H_+).  H_+ = Q_+^T Sigma H Q_+
 * comes from pseudosym_divide; the symmetric spectral divide-and-conquer splits it
 * recursively: shift sigma = median of the diagonal of the current block, sign of the
 * shifted block by the same Zolotarev iteration (r chosen by the two-step rule), bases
 * of both projectors by Alg. 4 (Cholesky of a leading block; the leading indices are
 * those with the largest projector diagonal), until blocks of at most 64 remain, which
 * a Jacobi kernel diagonalizes.
 * Outputs (device): lambda[0..2m-1]: lambda[i], i < m, the positive eigenvalues in
 * ascending order, lambda[m+i] = -lambda[i].  V (2m x 2m, leading dimension
 * ldv >= 2m, may be NULL): column j is the eigenvector of lambda[j] with
 * V^T Sigma V = diag(I_m, -I_m), V(:, m+i) = Pi V(:, i), and each column's entry of
 * largest modulus (lowest index on ties) positive.  opts->r applies to the first
 * division step.  Status PS_NOT_CONVERGED with info->failed_step = 5 when no shift
 * splits a block of the recursion. */
int pseudosym_eig(ps_handle h, int m, const double* A, int lda, const double* B, int ldb,
                  double* lambda, double* V, int ldv, const ps_opts* opts, ps_info* info);

/* pseudosym_divide for `batch` independent problems of (possibly) different sizes:
 * problem i has half-size m[i], inputs A[i], B[i] (leading dimensions lda[i], ldb[i])
 * and outputs Qp[i] (2m[i] x m[i], ldq[i] >= 2 m[i]) and Hp[i] (ldh[i] >= m[i]), with
 * the conventions of pseudosym_divide.  m, lda, ldb, ldq, ldh and the pointer arrays
 * are HOST arrays of length batch holding device pointers.  The problems run largest
 * first, on the caller's worker streams (ps_set_worker_streams; one worker per stream,
 * at most six, each with an equal share of the handle's workspace, sized by
 * ps_workspace_size_batched) or, without them, in order on the handle's stream; the
 * call returns when all are done.  In FP64 (or mixed below its size threshold), problems of one padded size (m
 * rounded up to 64) run together, with either basis, up to 32 per batched pipeline
 * (fewer where their workspace would pass 3 GiB): their results agree with single calls
 * to rounding (the sums are split differently), not bit for bit; other problems run the
 * single-problem pipeline and match it exactly.  infos (host, length batch, may be NULL)
 * receives one record per problem; the return value is 0 or the status of the first
 * failing problem in index order.  opts->timing == 2: problems that run alone report
 * their phases and kernel classes as in pseudosym_divide; a batched pipeline reports its
 * kernel classes once, in the record of its first completed problem (its other records
 * have none), and runs without HIP graphs for that call; other timing values are
 * ignored.
 * Argument errors: -k as usual (k = 3..11 also when entry i of that array is invalid). */
int pseudosym_divide_batched(ps_handle h, int batch, const int* m, const double* const* A,
                             const int* lda, const double* const* B, const int* ldb,
                             double* const* Qp, const int* ldq, double* const* Hp,
                             const int* ldh, const ps_opts* opts, ps_info* infos);

/* Differentiable sign function.  Forward: the blocks SA, SB of sign(H) (as
 * pseudosym_sign, from the division step) together with the eigen-decomposition of
 * pseudosym_eig (lambda, 2m values; V, 2m x 2m with ldv >= 2m), which the adjoint
 * reuses.  The caller keeps lambda and V (device memory it owns) for the backward. */
int pseudosym_sign_fwd(ps_handle h, int m, const double* A, int lda, const double* B, int ldb,
                       double* SA, double* SB, int lds, double* lambda, double* V, int ldv,
                       const ps_opts* opts, ps_info* info);

/* Adjoint (backward) of the sign blocks.  Given gSA = dL/dS_A and gSB = dL/dS_B (m x m,
 * leading dimension ldg) for a scalar loss L and the lambda, V of the forward, writes
 * gA = dL/dA and gB = dL/dB (m x m, ldo), each the symmetric part, so that
 * <gA, E_A> + <gB, E_B> is the derivative of L along symmetric (E_A, E_B).  With
 * H = V diag(lambda) V^{-1} the derivative of sign is the divided-difference form
 * L*(H, G) = V^{-T} (F o (V^T G V^{-T})) V^T, F_ij = (sign lambda_i - sign lambda_j) /
 * (lambda_i - lambda_j); V^{-1} = diag(I, -I) V^T Sigma by the Sigma-orthogonality of V
 * (Thm. EVREalSigmaOrth).  For L = trace(W P_+), P_+ = (I + sign(H))/2, the inputs are
 * gSA = (W11 - W22)^T / 2 and gSB = (W21 - W12)^T / 2 (W in m x m blocks). */
int pseudosym_sign_bwd(ps_handle h, int m, const double* lambda, const double* V, int ldv,
                       const double* gSA, const double* gSB, int ldg, double* gA, double* gB,
                       int ldo);

/* The full 2m x 2m sign(H) = [[S_A, S_B], [-S_B, -S_A]] (eq:signDef; the block form of
 * sign(H) for the Casida structure) from the blocks pseudosym_sign returns (device, m x m,
 * leading dimension lds), written to S (device, column-major, lds2 >= 2m; caller-owned).
 * Argument errors: -1 handle, -2 m, -3 SA, -4 SB, -5 lds, -6 S, -7 lds2. */
int pseudosym_sign_full(ps_handle h, int m, const double* SA, const double* SB, int lds,
                        double* S, int lds2);

/* Differentiable sign function on the iteration's own factors (no eigen-decomposition).
 * The forward is pseudosym_sign (Alg. 8 on the core Y0 = R_M R_K^T, Sec. 4, in FP64, both
 * steps by factorizations, no Newton-Schulz pass) that also writes into `store` (caller's
 * device memory, 256-byte aligned, at least ps_sign_store_size(m, opts) bytes, kept by
 * the caller until the backward): R_M, R_K, their inverses, the polar factor U, and per
 * Zolotarev step its input X_k, the inverse Cholesky factors W_kj of X_k^T X_k + c_j I
 * and its scalars.  The store holds 2 (1 + max_restarts) steps (max_restarts <= 3).
 * Argument errors: -1..-9 as pseudosym_sign, -10 store null or misaligned, -11
 * store_bytes too small, -12 options it does not take (mixed precision, another
 * iteration, max_restarts > 3). */
size_t ps_sign_store_size(int m, const ps_opts* opts);
int pseudosym_sign_fwd_iter(ps_handle h, int m, const double* A, int lda, const double* B,
                            int ldb, double* SA, double* SB, int lds, void* store,
                            size_t store_bytes, const ps_opts* opts, ps_info* info);

/* Backward of pseudosym_sign_fwd_iter: gA = dL/dA, gB = dL/dB (symmetric parts, m x m,
 * ldo) from gSA = dL/dS_A, gSB = dL/dS_B (m x m, ldg), by reverse mode through the
 * forward's composition with the stored factors: the sign-block products, each
 * Zolotarev step X' = hat C X (I + sum_j a_j N_j), N_j = W_j W_j^T, whose adjoint is
 * hat C (G (I + sum_j a_j N_j) - X (Z + Z^T)), Z = sum_j a_j N_j X^T G N_j (batched and
 * K-segmented matrix-core products), Y0 = R_M R_K^T, the inverses, and the Cholesky
 * factorizations (gM = sym(W Phi(R triu(gR)^T) W^T), Phi the lower triangle with its
 * diagonal halved).  The bounds and coefficients of the forward are held fixed (sign is
 * scale invariant; the rational approximation error of the two steps is below 1e-15).
 * Workspace: ps_workspace_size kind 7.  Argument errors: -1 handle, -2 m, -3 store null,
 * misaligned or not written for this m, -4/-5 gradients, -6 ldg, -7/-8 outputs, -9 ldo. */
int pseudosym_sign_bwd_iter(ps_handle h, int m, const void* store, const double* gSA,
                            const double* gSB, int ldg, double* gA, double* gB, int ldo);

/* Human-readable name of a status code. */
const char* ps_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* PSEUDOSYM_H */
