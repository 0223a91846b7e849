// Host driver of the pseudosym pipeline and the C-ABI entry points.
//
// The Zolotarev iteration runs on the half-size core of H.  With
//   M = A + B = R^T R,   K = A - B = L L^T  (L = R_K^T),   Y0 = R L,
// Q_h = [[I, I], [I, -I]]/sqrt(2) gives Q_h H Q_h = [[0, K], [M, 0]], so the
// eigenvalues of H are +-sigma(Y0), and every odd function f(x) = x h(x^2) of H is
//   f(H) = Q_h [[0, R^{-1} f(Y0) L^T], [R^T f(Y0) L^{-1}, 0]] Q_h,  f(Y0) = Y0 h(Y0^T Y0).
// Alg. 8 applied to H therefore equals the Zolotarev polar iteration applied to Y0,
//   Y <- hat C (Y + sum_j a_j Y (Y^T Y + c_{2j-1} I)^{-1}),
// whose shifted matrices are symmetric positive definite (SYRK, Cholesky and the
// triangular inverse, all on matrix cores).  The blocks of sign(H) are assembled
// from the polar factor U of Y0 as A_s = (S21 + S12)/2, B_s = (S21 - S12)/2 with
// S12 = R^{-1} U L^T and S21 = R^T U L^{-1}; the bases follow Alg. 6 and the
// decoupled block is H_+ = Q_+^T Sigma H Q_+ = (Q_h Q_+)^T diag(M, K) (Q_h Q_+).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/pseudosym.h"
#include "ps_internal.h"

namespace ps {
void fill_int_zero(hipStream_t s, int* x, int n);
void form_shifts_v(hipStream_t s, const double* g, double* z, int m, int mp,
                   const double* shifts_host, int r);
}  // namespace ps

struct ps_handle_s {
  hipStream_t stream = nullptr;
  int device = 0;
  void* user_ws = nullptr;      // the caller's workspace (the library allocates none)
  size_t user_bytes = 0;
  double* pinned = nullptr;  // host staging for scalars
  hipEvent_t ev[10] = {};
  bool events = false;
  std::vector<hipEvent_t> kev;  // per-launch kernel timing (opts.timing == 2)
  std::vector<double> kflops;
  std::vector<int> kcls;
  std::vector<int> knl;
  // the caller's extra streams (ps_set_worker_streams): the first is also the second
  // stream of a mixed step (FP32 shift group); without any, that work is serialized on
  // `stream`
  std::vector<hipStream_t> wstreams;
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  std::vector<ps_handle_s*> workers;   // one per worker stream (batched calls, recursion)
  // captured launch sequences of the batched pipeline, replayed when a class with the
  // same key comes again (ps_set_graphs; oldest dropped beyond kGraphCache)
  struct GraphEntry {
    std::vector<long long> key;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  bool use_graphs = true;
  ps::GemmTuneTable tuning;   // ps_set_gemm_tuning (empty: the built-in heuristic)
};

namespace ps {
namespace {

constexpr size_t kAlign = 256;
constexpr int kPinned = 1 << 16;  // doubles (host staging: up to m = 32768 values)
// below this padded size the FP32 group of a mixed step costs more in extra launches and
// stream hand-offs than its arithmetic saves (measured on 256 problems of 32..512): such
// problems run in FP64
constexpr int kMixedMin = 1024;
constexpr int kGraphCache = 32;   // captured class pipelines kept per handle

// whether a problem of half-size m runs the mixed-precision steps (and needs their FP32
// buffers)
inline bool mixed_arith(const ps_opts& o, int m) {
  return o.precision == PS_PREC_MIXED && pad_to(m) >= kMixedMin;
}

struct Arena {
  char* base = nullptr;
  size_t off = 0;
  bool dry = true;
  template <class T>
  T* take(size_t n) {
    const size_t bytes = (n * sizeof(T) + kAlign - 1) / kAlign * kAlign;
    T* p = dry ? nullptr : reinterpret_cast<T*>(base + off);
    off += bytes;
    return p;
  }
};

struct Buffers {
  int m = 0, mp = 0, r = 0;
  size_t S = 0;
  double *mk, *wmk, *tmp, *y, *yt, *x0, *x1, *x2, *g, *z, *w, *nmat;
  double *t1, *t2, *s12, *s21, *as, *bs, *p11, *wc, *qbot, *top, *ab, *F, *hp;
  double *vv, *uu, *pp, *hist, *norms;
  double* gkpart;    // partial norms of the bidiagonalization vectors (3 generations)
  double* splitws;   // kMaxSplit partial products of split-K GEMMs
  int* dinfo;
  // mixed precision (null in FP64 mode)
  float *z32, *w32, *n32, *x32, *d32, *t32, *u32, *y32;
};

constexpr int kMaxSplit = 8;

// Choose a split-K factor for a launch of few tiles: the pieces run in rounds of
// `slots` resident workgroups (one 16-wave large tile per compute unit, or two small
// ones), so the factor that fills the last round best wins, less 2 % per extra split
// for the partial sums' traffic and the shorter K loops (at least 8 steps of 16).
void auto_split(GemmProblem& p, double* ws, int maxsplit = kMaxSplit) {
  // the workspace also serves a stream-K schedule, which the launcher may choose
  p.ws = ws;
  p.ws_slots = kMaxSplit;
  const bool big = p.M % 128 == 0 && p.N % 128 == 0 && std::min(p.M, p.N) >= 512;
  const int T = big ? 128 : 64;
  const long long slots = big ? 256 : 512;
  long long tiles = (p.flags & (kOutUpper | kOutLower)) ? (long long)(p.M / T) * (p.M / T + 1) / 2
                                                        : (long long)(p.M / T) * (p.N / T);
  tiles *= (long long)p.nb1 * p.nb2;
  if (p.nb1 * p.nb2 != 1 || tiles >= 512) return;
  int best = 1;
  double best_score = -1.0;
  for (int ks = 1; ks <= maxsplit; ++ks) {
    if (ks > 1 && p.K / 16 / ks < 8) break;
    const long long pieces = tiles * ks;
    const long long rounds = (pieces + slots - 1) / slots;
    const double score = (double)pieces / (double)(rounds * slots) - 0.02 * (ks - 1);
    if (score > best_score + 1e-12) {
      best_score = score;
      best = ks;
    }
  }
  if (best > 1) {
    p.ksplit = best;
    p.ws = ws;
  }
}

// Hand the split workspace (kMaxSplit * M * N elements) to a problem that is launched
// without auto_split, so that the launcher may give it a stream-K schedule.
void with_ws(GemmProblem& p, double* ws) {
  p.ws = ws;
  p.ws_slots = kMaxSplit;
}

void carve(Arena& a, Buffers& b, int m, int r, int what, bool mixed = false) {
  b.m = m;
  b.mp = pad_to(m);
  b.r = r;
  const size_t S = (size_t)b.mp * b.mp;
  b.S = S;
  // the eig subproblems use 8 slots; a division at least 4 (the 2m x 2m matrix of the
  // Alg. 7 factorization goes there)
  const int rr = std::max(r, what >= 2 ? 8 : (what == 1 ? 4 : 2));
  b.mk = a.take<double>(2 * S);
  b.wmk = a.take<double>(2 * S);
  b.tmp = a.take<double>((size_t)rr * b.mp * kNb);
  b.y = a.take<double>(2 * S);
  b.yt = a.take<double>(2 * S);
  b.x0 = a.take<double>(S);
  b.x1 = a.take<double>(S);
  b.x2 = a.take<double>(S);
  b.g = a.take<double>(S);
  b.z = a.take<double>((size_t)rr * S);
  b.w = a.take<double>((size_t)rr * S);
  b.nmat = a.take<double>(S);
  b.t1 = a.take<double>(S);
  b.t2 = a.take<double>(S);
  b.s12 = a.take<double>(S);
  b.s21 = a.take<double>(S);
  b.as = a.take<double>(S);
  b.bs = a.take<double>(S);
  if (what >= 1) {
    b.p11 = a.take<double>(S);
    b.wc = a.take<double>(S);
    b.qbot = a.take<double>(S);
    b.top = a.take<double>(S);
    b.ab = a.take<double>(2 * S);
    b.F = a.take<double>(2 * S);
    b.hp = a.take<double>(S);
  } else {
    b.p11 = b.wc = b.qbot = b.top = b.ab = b.F = b.hp = nullptr;
  }
  b.vv = a.take<double>(2 * (size_t)b.mp);
  b.uu = a.take<double>(2 * (size_t)b.mp);
  b.pp = a.take<double>(2 * (size_t)b.mp);
  b.hist = a.take<double>(2 * 256);
  b.gkpart = a.take<double>(3 * 2 * (size_t)gk_parts(b.mp));
  b.norms = a.take<double>(2 + 2 * 1024 + 16);
  b.splitws = a.take<double>((size_t)kMaxSplit * S);
  b.dinfo = a.take<int>(16);
  if (mixed) {
    b.z32 = a.take<float>((size_t)rr * S);
    b.w32 = a.take<float>((size_t)rr * S);
    b.n32 = a.take<float>(S);
    b.x32 = a.take<float>(S);
    b.d32 = a.take<float>(S);
    b.t32 = a.take<float>(S);
    b.u32 = a.take<float>(S);
    b.y32 = a.take<float>(S);
  } else {
    b.z32 = b.w32 = b.n32 = b.x32 = b.d32 = b.t32 = b.u32 = b.y32 = nullptr;
  }
}

// r = 0: the smallest r for which the two steps map [l, 1] into [1 - 1e-15, 1] (the
// criterion the paper takes from a table of its reference [NakF16]); workspace sizing
// assumes the largest r.
int auto_r(double ell) {
  for (int r = 1; r < 8; ++r) {
    ZoloHost c1, c2;
    if (zolotarev_host(ell, r, &c1)) continue;
    const double e1 = std::min(c1.ell_next, 1.0 - 1e-16);
    if (zolotarev_host(e1, r, &c2)) continue;
    if (1.0 - c2.ell_next <= 1e-15) return r;
  }
  return 8;
}

int resolve_r(const ps_opts& o) { return o.r <= 0 ? 8 : std::min(o.r, 8); }

// Zolotarev degree of the recursion's splits.  The shifted blocks have eigenvalues
// spread over [l, 1] with l small; with the smallest r that reaches 1 - 1e-15 in two
// steps, 1 - l_1 after the first step is about u^{1/(2r+1)}, the stopping test's own
// tolerance, so most splits restarted (26 of 31 at n = 4096); the factorization chains
// are latency-bound, so r = 8 costs about the same per step and takes 1 - l_1 well
// below it.
constexpr int kEigR = 8;

// Device buffers of the eigen-decomposition, placed after the largest divide or
// subproblem layout (the recursion reuses that region for every subproblem).
struct EigBuffers {
  double *qf, *hraw, *hs, *qt, *qb, *vacc, *t, *vs, *zbd, *w, *wsorted, *dscratch;
  int *perm, *leaf_o, *leaf_n, *sweeps;
};

size_t eig_region_offset(int m, const ps_opts& o) {
  Arena a1, a2;
  Buffers b1, b2;
  carve(a1, b1, m, resolve_r(o), 1, mixed_arith(o, m));
  carve(a2, b2, m, 8, 2);
  return std::max(a1.off, a2.off);
}

void carve_eig(Arena& a, EigBuffers& e, int m) {
  const int mp = pad_to(m);
  const size_t S = (size_t)mp * mp;
  e.qf = a.take<double>((size_t)2 * m * m);
  e.hraw = a.take<double>((size_t)m * m);
  e.hs = a.take<double>(S);
  e.qt = a.take<double>(S);
  e.qb = a.take<double>(S);
  e.vacc = a.take<double>(S);
  e.t = a.take<double>(S);
  e.vs = a.take<double>(S);
  e.zbd = a.take<double>(S);
  e.w = a.take<double>(mp);
  e.wsorted = a.take<double>(mp);
  e.dscratch = a.take<double>(mp);
  e.perm = a.take<int>(mp);
  e.leaf_o = a.take<int>(mp);
  e.leaf_n = a.take<int>(mp);
  e.sweeps = a.take<int>(16);
}

// Subtrees of at most this many columns run on the recursion workers, each with a
// scratch region sized for it.
inline int eig_worker_cap(int m) { return std::max(64, pad_to((m + 1) / 2)); }
constexpr int kEigWorkers = 4;

void carve_eig_worker(Arena& a, int m, char** base, double** vs, double** t, double** zbd,
                      double** dscr, int** perm) {
  const int mp = pad_to(m), cap = eig_worker_cap(m);
  Arena d;
  Buffers b;
  carve(d, b, cap, 8, 2);
  *base = a.take<char>(d.off);
  *vs = a.take<double>((size_t)mp * cap);
  *t = a.take<double>((size_t)mp * cap);
  *zbd = a.take<double>((size_t)cap * cap);
  *dscr = a.take<double>(mp);
  *perm = a.take<int>(mp);
}

size_t workspace_bytes(int m, const ps_opts& o, int what) {
  Arena a;
  Buffers b;
  if (what >= 2) {
    a.off = eig_region_offset(m, o);
    EigBuffers e;
    carve_eig(a, e, m);
    for (int k = 0; k < kEigWorkers; ++k) {
      char* base;
      double *vs, *t, *zbd, *dscr;
      int* perm;
      carve_eig_worker(a, m, &base, &vs, &t, &zbd, &dscr, &perm);
    }
    return a.off + kAlign;
  }
  carve(a, b, m, resolve_r(o), what, mixed_arith(o, m));
  return a.off + kAlign;
}

struct Timer {
  ps_handle h;
  bool on;
  int n = 0;
  int phase_of[10];
  void mark(int phase) {
    if (!on || n >= 10) return;
    PS_HIP(hipEventRecord(h->ev[n], h->stream));
    phase_of[n] = phase;
    ++n;
  }
  void finish(double* ms) {
    if (!on) return;
    for (int i = 0; i < 8; ++i) ms[i] = 0.0;
    for (int i = 1; i < n; ++i) {
      float t = 0.f;
      PS_HIP(hipEventElapsedTime(&t, h->ev[i - 1], h->ev[i]));
      if (phase_of[i] >= 0 && phase_of[i] < 8) ms[phase_of[i]] += t;
    }
  }
};

// Golub-Kahan bidiagonalization of two matrices at once: M_0 = mats[0], M_1 = mats[S],
// transposes in mats_t.  Returns sigma_max of each bidiagonal projection.
// dinfo_dev: flags to bring back with the same synchronization (to pinned + 512)
void gk_estimate(hipStream_t s, Buffers& b, const double* mats, const double* mats_t, int steps,
                 double* pinned, double smax[2], const int* dinfo_dev = nullptr) {
  const int mp = b.mp;
  const long long S = (long long)b.S;
  gk_init(s, b.vv, b.m, mp, 2, 0);
  // half-step h writes the partial norms of its vector to generation h % 3; the unit
  // start vector's are generation 2
  const size_t np2 = 2 * (size_t)gk_parts(mp);
  auto part = [&](int h) { return b.gkpart + (size_t)((h + 3) % 3) * np2; };
  gk_seed(s, part(-1), mp, 2);
  for (int k = 0; k < steps; ++k) {
    // u_k = M v_k - beta_{k-1} u_{k-1}   (M x = column dots of M^T; beta_{k-1} = ||v~_k||)
    gk_step(s, mats_t, S, b.vv, mp, part(2 * k - 1), b.uu, mp, k > 0 ? b.uu : nullptr, mp,
            part(2 * k - 2), part(2 * k), b.hist, 2 * k - 1, 256, mp, 2);
    // v_{k+1} = M^T u_k - alpha_k v_k   (alpha_k = ||u~_k||)
    gk_step(s, mats, S, b.uu, mp, part(2 * k), b.vv, mp, b.vv, mp, part(2 * k - 1),
            part(2 * k + 1), b.hist, 2 * k, 256, mp, 2);
  }
  gk_finish(s, part(2 * steps - 1), mp, b.hist, 2 * steps - 1, 256, 2);
  PS_HIP(hipMemcpyAsync(pinned, b.hist, 2 * 256 * sizeof(double), hipMemcpyDeviceToHost, s));
  if (dinfo_dev)
    PS_HIP(hipMemcpyAsync(pinned + 512, dinfo_dev, 16 * sizeof(int), hipMemcpyDeviceToHost, s));
  PS_HIP(hipStreamSynchronize(s));
  for (int q = 0; q < 2; ++q) {
    double d[128], e[128];
    for (int k = 0; k < steps; ++k) {
      d[k] = pinned[q * 256 + 2 * k];
      e[k] = pinned[q * 256 + 2 * k + 1];
    }
    double smn;
    bidiag_extreme_sv(d, e, steps, &smax[q], &smn);
  }
}

// One Zolotarev step on the core: xn = hat C x (I + sum_j a_j (x^T x + c_{2j-1} I)^{-1})
void zolo_step_f64(hipStream_t s, Buffers& b, const double* x, double* xn, const ZoloHost& co,
                   int* dinfo_slot) {
  const int mp = b.mp, r = co.r;
  const long long S = (long long)b.S;
  {
    GemmProblem pg = gemm_problem(mp, mp, mp, x, mp, 1, x, mp, 0, b.g, mp, 1.0, 0.0, nullptr, 0,
                                  kOutUpper);
    auto_split(pg, b.splitws);
    gemm_f64(s, pg);
  }
  double shifts[8];
  for (int j = 0; j < r; ++j) shifts[j] = co.c[2 * j];
  form_shifts_v(s, b.g, b.z, b.m, mp, shifts, r);
  potrf_inv_f64(s, b.z, S, b.w, S, b.tmp, mp, r, dinfo_slot);
  GemmProblem pn = gemm_problem(mp, mp, r * mp, b.w, mp, 0, b.w, mp, 1, b.nmat, mp, 1.0, 0.0,
                                nullptr, 0, kAUpper | kBLower | kOutUpper | kMirror);
  pn.kseg = mp;
  pn.nseg = r;
  for (int j = 0; j < r; ++j) pn.kscale[j] = co.a[j];
  if (r > 1 && r <= kMaxSplit) {   // one partial per shift term (measured faster here
    pn.ksplit = r;                  // than the round-filling choice of auto_split)
    pn.ws = b.splitws;
  }
  gemm_f64(s, pn);
  GemmProblem px = gemm_problem(mp, mp, mp, x, mp, 0, b.nmat, mp, 0, xn, mp, co.chat, co.chat, x,
                                mp, 0);
  auto_split(px, b.splitws);
  gemm_f64(s, px);
}

// Number of series terms for the second step, or 0 when the factorization form is
// needed.  After the first step the singular values of X lie in [l1, 1], so
// Delta = X^T X - I has ||Delta|| <= 1 - l1^2 and, with (G + c I)^{-1} =
// (1 + c)^{-1} sum_p (-Delta / (1 + c))^p, the p-th term of sum_j a_j (G + c_j I)^{-1} is
// bounded by gamma_p ||Delta||^p, gamma_p = sum_j a_j / (1 + c_j)^{p+1}.  P terms are
// used when the first omitted one is below 1e-17 relative to gamma_0.
constexpr int kMaxSeries = 8;

int series_terms(const ZoloHost& co, double ell_in, double gam[kMaxSeries]) {
  const long double d = 1.0L - (long double)ell_in * ell_in;
  long double g[kMaxSeries + 2] = {};
  for (int j = 0; j < co.r; ++j) {
    long double f = 1.0L / (1.0L + co.c[2 * j]);
    long double t = co.a[j] * f;
    for (int p = 0; p < kMaxSeries + 2; ++p) {
      g[p] += t;
      t *= f;
    }
  }
  for (int P = 1; P <= kMaxSeries; ++P) {
    long double bound = g[P];
    for (int q = 0; q < P; ++q) bound *= d;
    if (bound <= 1e-17L * g[0]) {
      for (int p = 0; p < kMaxSeries; ++p) gam[p] = (double)((p & 1) ? -g[p] : g[p]);
      return P;
    }
  }
  return 0;
}

// Check of the bounds behind the series: power steps on Delta = X^T X - I (or on X^T X
// with the identity subtracted on the fly) on the side stream, launched from the point
// where the step has formed that matrix in b.g, which the rest of the step only reads.
// The caller waits for `join` before b.g is written again.
constexpr int kPowerSteps = 6;

struct SeriesCheck {
  hipStream_t side;   // null: run in order on the step's stream
  hipEvent_t fork, join;
  double* v;          // 2 mp doubles
  double* out2;       // ||v_k||^2, ||v_{k-1}||^2
};

void launch_series_check(hipStream_t s, const Buffers& b, const SeriesCheck* chk, double shift) {
  if (!chk) return;
  hipStream_t t = chk->side ? chk->side : s;
  if (t != s) {
    PS_HIP(hipEventRecord(chk->fork, s));
    PS_HIP(hipStreamWaitEvent(t, chk->fork, 0));
  }
  sym_power_norm(t, b.g, b.m, b.mp, shift, kPowerSteps, chk->v, chk->v + b.mp, chk->out2);
  if (t != s) PS_HIP(hipEventRecord(chk->join, t));
}

// Second Zolotarev step by the series: xn = hat C x (I + sum_{p<P} gam_p Delta^p),
// Delta = x^T x - I, evaluated by Horner's rule on the right.
void zolo_step_series(hipStream_t s, Buffers& b, const double* x, double* xn, const ZoloHost& co,
                      int P, const double gam[kMaxSeries], const SeriesCheck* chk = nullptr) {
  const int mp = b.mp;
  GemmProblem pg = gemm_problem(mp, mp, mp, x, mp, 1, x, mp, 0, b.g, mp, 1.0, 0.0, nullptr, 0,
                                kOutUpper | kMirror);
  auto_split(pg, b.splitws);
  gemm_f64(s, pg);
  axpb_identity(s, b.g, b.g, 1.0, -1.0, mp);                 // Delta
  launch_series_check(s, b, chk, 0.0);
  // T = (1 + gam_0) I + gam_1 Delta + ... + gam_{P-1} Delta^{P-1}
  double* T = b.nmat;
  double* T2 = b.t1;
  if (P == 1) {
    axpb_identity(s, b.g, T, 0.0, 1.0 + gam[0], mp);
  } else {
    axpb_identity(s, b.g, T, gam[P - 1], (P - 2 == 0 ? 1.0 + gam[0] : gam[P - 2]), mp);
    for (int q = P - 3; q >= 0; --q) {
      // Delta and T are symmetric and commute, so Delta T is symmetric: upper tiles only
      GemmProblem ph = gemm_problem(mp, mp, mp, b.g, mp, 0, T, mp, 0, T2, mp, 1.0, 0.0, nullptr,
                                    0, kOutUpper | kMirror);
      auto_split(ph, b.splitws);
      gemm_f64(s, ph);
      axpb_identity(s, T2, T, 1.0, q == 0 ? 1.0 + gam[0] : gam[q], mp);
    }
  }
  GemmProblem px = gemm_problem(mp, mp, mp, x, mp, 0, T, mp, 0, xn, mp, co.chat, 0.0, nullptr, 0,
                                0);
  auto_split(px, b.splitws);
  gemm_f64(s, px);
}

// Mixed precision.  The iterate X and X^T X stay in FP64.  In a factorization step,
// shift c_{2j-1} goes to FP32 when the condition number of its shifted Gram matrix,
// at most (1 + c)/(l^2 + c) on [l, 1], is at most kappa; FP32 rounding then perturbs
// X (I + N) by about kappa u_32 relative, which moves the polar factor's subspace by
// the same order and the Rayleigh-Ritz eigenvalues of H_+ by its square.  The FP32
// group is factorized on a second stream while the FP64 group runs on the first.
struct MixedCtx {
  hipStream_t side;
  hipEvent_t fork, join;
  double kappa;
};

void zolo_step_mixed(hipStream_t s, const MixedCtx& mx, Buffers& b, const double* x, double* xn,
                     const ZoloHost& co, double ell, int* dinfo64, int* dinfo32, int* n64_out) {
  const int mp = b.mp, r = co.r;
  const long long S = (long long)b.S;
  {
    GemmProblem pg = gemm_problem(mp, mp, mp, x, mp, 1, x, mp, 0, b.g, mp, 1.0, 0.0, nullptr, 0,
                                  kOutUpper);
    auto_split(pg, b.splitws);
    gemm_f64(s, pg);
  }
  double c64[8], a64[8], c32[8], a32[8];
  int n64 = 0, n32 = 0;
  for (int j = 0; j < r; ++j) {
    const double c = co.c[2 * j];
    const double kap = (1.0 + c) / (ell * ell + c);
    if (kap > mx.kappa) {
      c64[n64] = c;
      a64[n64++] = co.a[j];
    } else {
      c32[n32] = c;
      a32[n32++] = co.a[j];
    }
  }
  *n64_out = n64;
  // the two groups' factorizations are latency-bound chains of launches: record both and
  // issue them alternately, so that neither waits for the host to enqueue the other
  LaunchList chain32, chain64;
  hipStream_t s2 = mx.side ? mx.side : s;   // no second stream: both groups in order on s
  if (n32 > 0) {
    if (s2 != s) {
      PS_HIP(hipEventRecord(mx.fork, s));
      PS_HIP(hipStreamWaitEvent(s2, mx.fork, 0));
    }
    form_shifts_f32(s2, b.g, b.z32, mp, c32, n32);
    potrf_inv_f32(s2, b.z32, S, b.w32, S, mp, n32, dinfo32, &chain32);
  }
  if (n64 > 0) {
    form_shifts_v(s, b.g, b.z, b.m, mp, c64, n64);
    potrf_inv_f64(s, b.z, S, b.w, S, b.tmp, mp, n64, dinfo64, true, &chain64);
  }
  issue_interleaved(chain32, chain64);
  if (n32 > 0) {
    GemmProblemF pn = gemm_problem(mp, mp, n32 * mp, b.w32, mp, 0, b.w32, mp, 1, b.n32, mp, 1.0,
                                   0.0, nullptr, 0, kAUpper | kBLower | kOutUpper | kMirror);
    pn.kseg = mp;
    pn.nseg = n32;
    for (int j = 0; j < n32; ++j) pn.kscale[j] = a32[j];
    // the FP32 shifted matrices are no longer needed (the factors are in w32): split-K or
    // stream-K partials there (rr slices of S)
    pn.ws = b.z32;
    pn.ws_slots = b.r > 2 ? b.r : 2;
    if (n32 > 1 && n32 <= kMaxSplit) pn.ksplit = n32;
    gemm_f32(s2, pn);
    if (s2 != s) PS_HIP(hipEventRecord(mx.join, s2));
  }
  if (n64 > 0) {
    GemmProblem pn = gemm_problem(mp, mp, n64 * mp, b.w, mp, 0, b.w, mp, 1, b.nmat, mp, 1.0, 0.0,
                                  nullptr, 0, kAUpper | kBLower | kOutUpper | kMirror);
    pn.kseg = mp;
    pn.nseg = n64;
    for (int j = 0; j < n64; ++j) pn.kscale[j] = a64[j];
    auto_split(pn, b.splitws);
    gemm_f64(s, pn);
  } else {
    fill_zero(s, b.nmat, b.S);
  }
  if (n32 > 0) {
    if (s2 != s) PS_HIP(hipStreamWaitEvent(s, mx.join, 0));
    axpy_f32(s, b.nmat, 1.0, 1.0, b.n32, b.S);
  }
  GemmProblem px = gemm_problem(mp, mp, mp, x, mp, 0, b.nmat, mp, 0, xn, mp, co.chat, co.chat, x,
                                mp, 0);
  auto_split(px, b.splitws);
  gemm_f64(s, px);
}

// Second step by the series with Delta = X^T X - I in FP64 and the correction
// T' = sum_{p >= 1} gam_p Delta^p and X T' in FP32: ||Delta|| <= 1 - l_1^2 is small, so
// FP32 rounding of the correction is damped by that factor, and
// X2 = hat C (1 + gam_0) X + hat C X T' is formed in FP64.
void zolo_step_series_mixed(hipStream_t s, Buffers& b, const double* x, double* xn,
                            const ZoloHost& co, int P, const double gam[kMaxSeries],
                            const SeriesCheck* chk = nullptr) {
  const int mp = b.mp;
  GemmProblem pg = gemm_problem(mp, mp, mp, x, mp, 1, x, mp, 0, b.g, mp, 1.0, 0.0, nullptr, 0,
                                kOutUpper | kMirror);
  auto_split(pg, b.splitws);
  gemm_f64(s, pg);
  scale_copy(s, x, xn, co.chat * (1.0 + gam[0]), b.S);
  if (P < 2) {
    launch_series_check(s, b, chk, 1.0);   // b.g holds X^T X
    return;
  }
  axpb_identity(s, b.g, b.g, 1.0, -1.0, mp);   // Delta
  launch_series_check(s, b, chk, 0.0);
  cvt_f64_f32(s, b.g, b.d32, b.S);
  cvt_f64_f32(s, x, b.x32, b.S);
  // inner = gam_1 I + gam_2 Delta + ... + gam_{P-1} Delta^{P-2}, then T' = Delta inner
  float* inner = b.t32;
  float* tmp = b.u32;
  axpb_identity_f32(s, b.d32, inner, P >= 3 ? (float)gam[P - 1] : 0.0f,
                    (float)(P >= 3 ? gam[P - 2] : gam[1]), mp);
  for (int q = P - 3; q >= 1; --q) {
    GemmProblemF ph = gemm_problem(mp, mp, mp, b.d32, mp, 0, inner, mp, 0, tmp, mp, 1.0, 0.0,
                                   nullptr, 0, kOutUpper | kMirror);   // symmetric, as above
    gemm_f32(s, ph);
    axpb_identity_f32(s, tmp, inner, 1.0f, (float)gam[q], mp);
  }
  GemmProblemF pt = gemm_problem(mp, mp, mp, b.d32, mp, 0, inner, mp, 0, tmp, mp, 1.0, 0.0,
                                 nullptr, 0, kOutUpper | kMirror);
  gemm_f32(s, pt);
  GemmProblemF py = gemm_problem(mp, mp, mp, b.x32, mp, 0, tmp, mp, 0, b.y32, mp);
  gemm_f32(s, py);
  axpy_f32(s, xn, 1.0, co.chat, b.y32, b.S);
}

// alpha, beta for the core matrix: sigma_max(Y) and 1/sigma_max(Y^{-1}) by Golub-Kahan.
void estimate_bounds(hipStream_t s, Buffers& b, const double* ymats, int steps, double* pinned,
                     double* alpha, double* beta, double est[2],
                     const int* dinfo_dev = nullptr) {
  transpose(s, ymats, b.yt, b.mp, (long long)b.S, 2);
  double smax[2];
  gk_estimate(s, b, ymats, b.yt, steps, pinned, smax, dinfo_dev);
  est[0] = smax[0];
  est[1] = smax[1] > 0 ? 1.0 / smax[1] : 0.0;
  *alpha = 1.01 * smax[0];
  *beta = 0.99 / smax[1];
}

// The caller's workspace (ps_set_workspace, 256-byte aligned), or null when there is
// none or it is smaller than `need`: the library never allocates device memory.
char* workspace_base(ps_handle h, size_t need) {
  if (!h->user_ws || h->user_bytes < need) return nullptr;
  return (char*)h->user_ws;
}

// Worker handles bound to the caller's worker streams (created on first use; they hold
// host staging and events only, and borrow their streams).
int ensure_workers(ps_handle h, int n) {
  n = std::min(n, (int)h->wstreams.size());
  while ((int)h->workers.size() < n) {
    ps_handle w = nullptr;
    if (ps_create(&w, h->wstreams[h->workers.size()]) != PS_OK) return -1;
    w->use_graphs = h->use_graphs;
    w->tuning = h->tuning;
    h->workers.push_back(w);
  }
  return n;
}

// The comparison iterations of Sec. 6 (Tab:ItRuntime) on the core matrix y, one step per
// launch sequence with a schedule fixed on the host from l = beta / alpha:
//  Sigma-DWH: Zolotarev steps with r = 1 (the l-recurrence updated per step) until
//    1 - l <= 1e-15, plus one step for the stopping test with u^{1/3};
//  scaled Newton, X <- (mu X + (mu X)^{-T}) / 2 (the odd rational map of the sign
//    iteration, on the core): the step X (mu/2) (I + mu^{-2} (X^T X)^{-1}) is the r = 1
//    step with c = 0, a = mu^{-2}, hat C = mu/2; Byers-Xu scaling mu_0 = 1/sqrt(l),
//    mu_k = 1/sqrt(u_k), u_{k+1} = (mu_k + 1/mu_k)/2, until u_k - 1 <= 1e-15, plus one
//    step for the stopping test with u^{1/2}.
// Steps whose shifted Gram matrices are within the series' reach (the singular values of
// the iterate in [l_k, 1]) use the series form of the second Zolotarev step.  The final
// iterate is in b.x2.
int single_step_iterate(hipStream_t s, Buffers& b, const double* y, double alpha, double beta,
                        const ps_opts& o, double* pin, ps_info& inf, Timer& tm) {
  scale_copy(s, y, b.x0, 1.0 / alpha, b.S);
  const double ell0 = std::min(beta / alpha, 1.0 - 1e-15);
  std::vector<ZoloHost> sched;
  std::vector<double> ells;   // lower bound of the singular values before each step
  const bool newton = o.iteration == PS_ITER_NEWTON;
  double tol;
  if (!newton) {
    tol = std::pow(std::ldexp(1.0, -53), 1.0 / 3.0);
    double ell = ell0;
    for (int k = 0; k < 30; ++k) {
      ZoloHost c;
      if (zolotarev_host(std::min(ell, 1.0 - 1e-16), 1, &c)) return PS_NOT_CONVERGED;
      sched.push_back(c);
      ells.push_back(ell);
      const bool done = 1.0 - ell <= 1e-15;
      ell = std::min(c.ell_next, 1.0 - 1e-16);
      if (done) break;
      if (1.0 - ell <= 1e-15) {
        if (zolotarev_host(ell, 1, &c)) return PS_NOT_CONVERGED;
        sched.push_back(c);
        ells.push_back(ell);
        break;
      }
    }
  } else {
    tol = std::pow(std::ldexp(1.0, -53), 0.5);
    double mu = 1.0 / std::sqrt(ell0), u = 0.5 * (mu + 1.0 / mu), lo = ell0;
    for (int k = 0; k < 60; ++k) {
      ZoloHost c{};
      c.r = 1;
      c.c[0] = 0.0;
      c.a[0] = 1.0 / (mu * mu);
      c.chat = 0.5 * mu;
      sched.push_back(c);
      ells.push_back(lo);
      if (k > 0 && u - 1.0 <= 1e-15) break;
      if (k > 0) u = 0.5 * (mu + 1.0 / mu);
      mu = 1.0 / std::sqrt(u);
      lo = 1.0;   // after the first step the moduli lie in [1, u]
    }
  }
  inf.r = 1;
  const double* xin = b.x0;
  double* bufs[2] = {b.x1, b.x2};
  int k = 0;
  for (const ZoloHost& c : sched) {
    double* xout = bufs[k & 1];
    // Sigma-DWH steps after the first: the series form when it reaches 1e-17 (Newton
    // steps always factorize: their iterates' singular values lie above 1)
    double gam[kMaxSeries];
    const int P = (o.step2_series && k > 0 && !newton) ? series_terms(c, ells[k], gam) : 0;
    if (P > 0)
      zolo_step_series(s, b, xin, xout, c, P, gam);
    else
      zolo_step_f64(s, b, xin, xout, c, b.dinfo + 1);
    xin = xout;
    ++k;
  }
  tm.mark(2);
  inf.steps = k;
  inf.shifts_fp64[0] = 1;
  // stopping test on the last two iterates
  const double* last = bufs[(k - 1) & 1];
  const double* prev = k >= 2 ? bufs[(k - 2) & 1] : b.x0;
  diff_norms(s, prev, last, b.S, b.norms);
  PS_HIP(hipMemcpyAsync(pin, b.norms, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  PS_HIP(hipMemcpyAsync(pin + 8, b.dinfo, 16 * sizeof(int), hipMemcpyDeviceToHost, s));
  PS_HIP(hipStreamSynchronize(s));
  const int* di = (const int*)(pin + 8);
  if (di[1]) {
    inf.failed_step = 1;
    inf.failed_mask = di[1];
    return PS_SHIFT_BREAKDOWN;
  }
  inf.step_change = std::sqrt(pin[0]) / std::sqrt(pin[1]);
  if (last != b.x2) PS_HIP(hipMemcpyAsync(b.x2, last, b.S * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (!(inf.step_change <= tol)) return PS_NOT_CONVERGED;
  return PS_OK;
}

// Factor store of the stored-factor adjoint (pseudosym_sign_fwd_iter): the forward keeps,
// per Zolotarev step k, the step's input X_k and its inverse Cholesky factors
// W_kj = R_kj^{-1} (X_k^T X_k + c_j I = R_kj^T R_kj), with the step's scalars, and run()
// adds R_M, R_K, W_M, W_K and the polar factor U.  Layout in doubles: a header of
// kStoreHeader values, then R_M, R_K, W_M, W_K, U (S each), then per step X_k (S) and
// its r factors (r S).  Header: [0] layout version, [1] m, [2] mp, [3] r, [4] steps;
// step k at 16 + 16 k: the scale from the previous step's output (or Y0) to X_k, hat C,
// a_1..a_r.
constexpr int kStoreHeader = 256;
constexpr int kStoreMaxSteps = 8;
constexpr double kStoreVersion = 1.0;

size_t store_doubles(int mp, int r, int steps) {
  return kStoreHeader + (size_t)(5 + steps * (1 + r)) * mp * mp;
}

struct StepStore {
  double* base = nullptr;   // device, 256-byte aligned
  int mp = 0, r = 0, max_steps = 0, n = 0;
  double hdr[kStoreHeader] = {};
  double* mats() const { return base + kStoreHeader; }   // R_M, R_K, W_M, W_K, U
  double* x(int k) const { return mats() + (size_t)(5 + k * (1 + r)) * mp * mp; }
  double* w(int k) const { return x(k) + (size_t)mp * mp; }
  // before step k: its input and scalars (the factors follow with after_step)
  void before_step(hipStream_t s, const double* xin, double scale, const ZoloHost& co) {
    if (n >= max_steps) throw HipError{hipErrorInvalidValue, "factor store: too many steps"};
    const size_t S = (size_t)mp * mp;
    PS_HIP(hipMemcpyAsync(x(n), xin, S * sizeof(double), hipMemcpyDeviceToDevice, s));
    double* h = hdr + 16 + 16 * n;
    h[0] = scale;
    h[1] = co.chat;
    for (int j = 0; j < co.r; ++j) h[2 + j] = co.a[j];
  }
  void after_step(hipStream_t s, const double* wfac) {
    const size_t S = (size_t)mp * mp;
    PS_HIP(hipMemcpyAsync(w(n), wfac, (size_t)r * S * sizeof(double), hipMemcpyDeviceToDevice, s));
    ++n;
  }
};

// The Zolotarev iteration of Alg. 8 on the core matrix y (padded b.mp x b.mp, zero
// padding): X0 = y / alpha, l = beta / alpha, two steps per attempt, the stopping
// test ||X2 - X1||_F / ||X2||_F <= u^{1/(2r+1)} and restarts from X2 with bounds
// re-estimated on X2.  r_opt <= 0 picks r by the two-step rule.  Fills the iteration
// fields of inf; on PS_OK the polar factor of y is in b.x2.  Uses b.dinfo[1..3].
int polar_iterate(hipStream_t s, Buffers& b, const double* y, double alpha, double beta,
                  int r_opt, const ps_opts& o, double* pin, ps_info& inf, Timer& tm,
                  const MixedCtx* mx = nullptr, const MixedCtx* aux = nullptr,
                  StepStore* keep = nullptr) {
  if (o.iteration != PS_ITER_ZOLO) return single_step_iterate(s, b, y, alpha, beta, o, pin, inf, tm);
  const int mp = b.mp;
  const long long S = (long long)b.S;
  const int r = r_opt <= 0 ? 8 : std::min(r_opt, 8);
  scale_copy(s, y, b.x0, 1.0 / alpha, b.S);

  double ell = std::min(beta / alpha, 1.0 - 1e-15);
  const int r_run = (r_opt <= 0) ? auto_r(ell) : r;
  inf.r = r_run;
  const double tol = std::pow(std::ldexp(1.0, -53), 1.0 / (2 * r_run + 1));
  int status = PS_OK;
  const double* xin = b.x0;
  int attempt = 0;
  int ell_slot = 0;
  double in_scale = 1.0 / alpha;   // X0 from y (then from X2 on a restart)
  for (;; ++attempt) {
    ZoloHost c1, c2;
    if (zolotarev_host(ell, r_run, &c1)) return PS_NOT_CONVERGED;
    double ell1 = std::min(c1.ell_next, 1.0 - 1e-15);
    if (ell_slot < 4) inf.ell[ell_slot++] = ell;
    if (ell_slot < 4) inf.ell[ell_slot++] = ell1;
    if (mx) {
      int n64 = 0;
      zolo_step_mixed(s, *mx, b, xin, b.x1, c1, ell, b.dinfo + 1, b.dinfo + 7, &n64);
      inf.shifts_fp64[0] = n64;
    } else {
      if (keep) keep->before_step(s, xin, in_scale, c1);
      zolo_step_f64(s, b, xin, b.x1, c1, b.dinfo + 1);
      if (keep) keep->after_step(s, b.w);
      inf.shifts_fp64[0] = r_run;
    }
    tm.mark(2);
    if (o.max_steps == 1) {
      inf.steps += 1;
      std::swap(b.x1, b.x2);  // the sign assembly reads x2
      break;
    }
    // the second step's coefficients, on the host while the first step runs
    if (zolotarev_host(ell1, r_run, &c2)) return PS_NOT_CONVERGED;
    double gam[kMaxSeries];
    const int P = o.step2_series ? series_terms(c2, ell1, gam) : 0;
    inf.step2_terms = P;
    // the FP32 correction is damped by ||Delta|| <= 1 - l1^2; use it only while that
    // keeps its rounding below 1e-13 (else the FP64 series)
    const bool series32 = mx && (1.0 - ell1 * ell1) * 6.0e-8 <= 1e-13;
    // The series length rests on ||Delta|| <= 1 - l1^2, i.e. on [beta, alpha] holding the
    // singular values of the core; beta is an estimate from below of 1/sigma_max(Y0^{-1}) or
    // the caller's.  A few singular values outside it barely move the Frobenius stopping
    // test, so ||Delta|| is estimated on the device while the step runs.
    const MixedCtx* sc = aux ? aux : mx;
    SeriesCheck chk{sc ? sc->side : nullptr, sc ? sc->fork : nullptr, sc ? sc->join : nullptr,
                    b.pp, b.norms + 2 + 2 * 1024};
    const SeriesCheck* pc = P > 0 ? &chk : nullptr;
    if (P > 0 && series32) {
      zolo_step_series_mixed(s, b, b.x1, b.x2, c2, P, gam, pc);
    } else if (P > 0) {
      zolo_step_series(s, b, b.x1, b.x2, c2, P, gam, pc);
    } else {
      if (keep) keep->before_step(s, b.x1, 1.0, c2);
      zolo_step_f64(s, b, b.x1, b.x2, c2, b.dinfo + 2);
      if (keep) keep->after_step(s, b.w);
    }
    inf.shifts_fp64[1] = (P > 0) ? 0 : r_run;
    if (pc && chk.side) PS_HIP(hipStreamWaitEvent(s, chk.join, 0));
    tm.mark(3);
    inf.steps += 2;
    diff_norms(s, b.x1, b.x2, b.S, b.norms);
    PS_HIP(hipMemcpyAsync(pin, b.norms, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    if (pc) PS_HIP(hipMemcpyAsync(pin + 4, chk.out2, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    PS_HIP(hipMemcpyAsync(pin + 8, b.dinfo, 16 * sizeof(int), hipMemcpyDeviceToHost, s));
    PS_HIP(hipStreamSynchronize(s));
    const int* di = (const int*)(pin + 8);
    if (di[1] || di[2] || di[7]) {
      status = PS_SHIFT_BREAKDOWN;
      inf.failed_step = (di[1] || di[7]) ? 1 : 2;
      inf.failed_mask = di[1] ? di[1] : (di[7] ? di[7] : di[2]);
      break;
    }
    // Bound violated (beyond half the bound again, rounding of X^T X, and in mixed mode
    // the FP32 group's perturbation of X1): the series may have been cut too short, and
    // the stopping test cannot be trusted with it.  Redo the step by factorizations (its
    // multipliers stay positive for any singular value) and restart from X2, whose
    // bounds are then estimated afresh.
    bool bounds_hold = true;
    if (pc) {
      const double rho = pin[5] > 0.0 ? std::sqrt(pin[4] / pin[5]) : 0.0;
      inf.delta_norm_est = std::max(inf.delta_norm_est, rho);
      const double allowed = 1.5 * (1.0 - ell1 * ell1) + 64.0 * b.m * 0x1p-53 +
                             (mx ? 64.0 * mx->kappa * 0x1p-24 : 0.0);
      if (!(rho <= allowed)) {
        bounds_hold = false;
        inf.bounds_rejected += 1;
        zolo_step_f64(s, b, b.x1, b.x2, c2, b.dinfo + 2);
        inf.step2_terms = 0;
        inf.shifts_fp64[1] = r_run;
        diff_norms(s, b.x1, b.x2, b.S, b.norms);
        PS_HIP(hipMemcpyAsync(pin, b.norms, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        PS_HIP(hipMemcpyAsync(pin + 8, b.dinfo, 16 * sizeof(int), hipMemcpyDeviceToHost, s));
        PS_HIP(hipStreamSynchronize(s));
        if (di[2]) {
          status = PS_SHIFT_BREAKDOWN;
          inf.failed_step = 2;
          inf.failed_mask = di[2];
          break;
        }
      }
    }
    const double change = std::sqrt(pin[0]) / std::sqrt(pin[1]);
    inf.step_change = change;
    if (bounds_hold && change <= tol) break;
    if (attempt >= o.max_restarts) {
      status = PS_NOT_CONVERGED;
      break;
    }
    // restart from X2: new bounds from Golub-Kahan on X2 and on chol(X2^T X2)^{-1}
    inf.restarts += 1;
    {
      GemmProblem pg = gemm_problem(mp, mp, mp, b.x2, mp, 1, b.x2, mp, 0, b.g, mp, 1.0, 0.0,
                                    nullptr, 0, kOutUpper);
      auto_split(pg, b.splitws);
      gemm_f64(s, pg);
      spd_pad(s, b.g, b.z, b.m, mp, 0.0);
      potrf_inv_f64(s, b.z, S, b.w, S, b.tmp, mp, 1, b.dinfo + 3, true, nullptr, b.z + S, S);
      // estimator pair: y = [X2, W_G]
      PS_HIP(hipMemcpyAsync(b.y, b.x2, b.S * sizeof(double), hipMemcpyDeviceToDevice, s));
      PS_HIP(hipMemcpyAsync(b.y + S, b.w, b.S * sizeof(double), hipMemcpyDeviceToDevice, s));
      double est[2], a2, b2;
      estimate_bounds(s, b, b.y, std::max(4, std::min(o.lanczos_steps, 120)), pin, &a2, &b2,
                      est);
      // sigma_max(W_G) = 1 / sigma_min(X2)
      scale_copy(s, b.x2, b.x0, 1.0 / a2, b.S);
      in_scale = 1.0 / a2;
      xin = b.x0;
      ell = std::min(b2 / a2, 1.0 - 1e-15);
    }
  }
  return status;
}

// Per-class kernel timing (opts.timing == 2): a recorder on the calling thread that uses
// the handle's event pairs; collect() adds the recorded windows to inf once the handle's
// stream has been synchronized.
struct ClassTiming {
  ps_handle h;
  KernelRecorder rec;
  bool on;
  ClassTiming(ps_handle h_, bool on_) : h(h_), on(on_) {
    if (!on) return;
    const int cap = 1024;
    while ((int)h->kev.size() < 2 * cap) {
      hipEvent_t e;
      PS_HIP(hipEventCreate(&e));
      h->kev.push_back(e);
    }
    h->kflops.assign(cap, 0.0);
    h->kcls.assign(cap, -1);
    h->knl.assign(cap, 1);
    rec.ev = h->kev.data();
    rec.flops = h->kflops.data();
    rec.cls = h->kcls.data();
    rec.nl = h->knl.data();
    rec.cap = cap;
    kernel_set_recorder(&rec);
  }
  ~ClassTiming() {
    if (on) kernel_set_recorder(nullptr);
  }
  void collect(ps_info& inf) const {
    for (int q = 0; q < rec.n; ++q) {
      const int c = rec.cls[q];
      if (c < 0 || c >= kKcCount) continue;
      float t = 0.f;
      PS_HIP(hipEventElapsedTime(&t, rec.ev[2 * q], rec.ev[2 * q + 1]));
      inf.kclass_launches[c] += rec.nl[q];
      inf.kclass_ms[c] += t;
      inf.kclass_flops[c] += rec.flops[q];
    }
    inf.gemm_launches = inf.kclass_launches[kKcGemm128];
    inf.gemm_ms = inf.kclass_ms[kKcGemm128];
    inf.gemm_flops = inf.kclass_flops[kKcGemm128];
  }
};

// pairs: A and B are realified complex matrices (Eq:BSE2): the polar factor is projected
// back onto the realified form, which the mixed steps' FP32 factorizations perturb
int run(ps_handle h, int m, const double* A, int lda, const double* B, int ldb, double* out1,
        int ld1, double* out2, int ld2, const ps_opts& o, ps_info* info, int what,
        char* ws = nullptr, bool pairs = false, StepStore* keep = nullptr) {
  hipStream_t s = h->stream;
  const int r = resolve_r(o);
  // workspace: the caller's (or `ws`, which the caller has checked for size)
  char* base = ws ? ws : workspace_base(h, workspace_bytes(m, o, what));
  if (!base) return PS_NO_WORKSPACE;
  Arena ar;
  ar.base = base;
  ar.dry = false;
  Buffers b;
  carve(ar, b, m, r, what, mixed_arith(o, m));
  const int mp = b.mp;
  const long long S = (long long)b.S;
  double* pin = h->pinned;

  ps_info inf{};
  inf.failed_step = -1;
  inf.r = r;
  Timer tm{h, o.timing != 0};
  tm.mark(-1);
  const ClassTiming ktime(h, o.timing >= 2);

  fill_int_zero(s, b.dinfo, 16);
  // ---- setup: M = A + B = R_M^T R_M, K = A - B = R_K^T R_K, Y0 = R_M R_K^T, Y0^{-1} = W_K^T W_M
  pack_casida(s, m, mp, A, lda, B, ldb, b.mk);
  potrf_inv_f64(s, b.mk, S, b.wmk, S, b.tmp, mp, 2, b.dinfo + 0, true, nullptr, b.y, S);
  {
    GemmProblem pg[2];
    pg[0] = gemm_problem(mp, mp, mp, b.mk, mp, 0, b.mk + S, mp, 1, b.y, mp, 1.0, 0.0, nullptr, 0,
                         kAUpper | kBLower);
    pg[1] = gemm_problem(mp, mp, mp, b.wmk + S, mp, 1, b.wmk, mp, 0, b.y + S, mp, 1.0, 0.0,
                         nullptr, 0, kALower | kBUpper);
    with_ws(pg[0], b.splitws);
    gemm_f64(s, pg, 2);
  }
  mask_pad(s, b.y, m, mp, S, 2);
  tm.mark(0);

  // ---- parameter estimation (Alg. 8 step 1)
  double alpha = o.alpha, beta = o.beta;
  inf.sigma_est[0] = inf.sigma_est[1] = 0.0;
  // a failed setup Cholesky shows up as non-finite estimates; its flag comes back with
  // the estimator's results (or on its own when the caller gave both bounds)
  int setup_flag;
  if (!(alpha > 0.0) || !(beta > 0.0)) {
    double a_est, b_est;
    estimate_bounds(s, b, b.y, std::max(4, std::min(o.lanczos_steps, 120)), pin, &a_est, &b_est,
                    inf.sigma_est, b.dinfo);
    setup_flag = ((const int*)(pin + 512))[0];
    if (!(alpha > 0.0)) alpha = a_est;
    if (!(beta > 0.0)) beta = b_est;
  } else {
    PS_HIP(hipMemcpyAsync(pin, b.dinfo, 16 * sizeof(int), hipMemcpyDeviceToHost, s));
    PS_HIP(hipStreamSynchronize(s));
    setup_flag = ((const int*)pin)[0];
  }
  if (setup_flag != 0) {
    inf.status = PS_NOT_DEFINITE;
    inf.failed_step = 0;
    inf.failed_mask = setup_flag;
    if (info) *info = inf;
    return PS_NOT_DEFINITE;
  }
  inf.alpha = alpha;
  inf.beta = beta;
  tm.mark(1);

  // ---- Zolotarev steps with the stopping test of Alg. 8
  MixedCtx mxc{h->side, h->fork, h->join, o.mixed_kappa > 1.0 ? o.mixed_kappa : 20.0};
  const bool mixed = mixed_arith(o, m);
  const int status = polar_iterate(s, b, b.y, alpha, beta, o.r, o, pin, inf, tm,
                                   mixed ? &mxc : nullptr, &mxc, keep);
  if (status != PS_OK) {
    inf.status = status;
    tm.finish(inf.phase_ms);
    if (info) *info = inf;
    return status;
  }

  if (pairs) pair_project(s, b.x2, m, mp);
  const double* U = b.x2;
  // ---- FP64 Newton-Schulz pass on the polar factor: U <- U (3I - U^T U)/2 (refine 2)
  if (o.refine >= PS_REFINE_NS) {
    GemmProblem pg = gemm_problem(mp, mp, mp, U, mp, 1, U, mp, 0, b.g, mp, 1.0, 0.0, nullptr, 0,
                                  kOutUpper | kMirror);
    auto_split(pg, b.splitws);
    gemm_f64(s, pg);
    axpb_identity(s, b.g, b.g, -0.5, 1.5, mp);
    GemmProblem pu = gemm_problem(mp, mp, mp, U, mp, 0, b.g, mp, 0, b.x1, mp);
    auto_split(pu, b.splitws);
    gemm_f64(s, pu);
    mask_pad(s, b.x1, m, mp, S, 1);
    U = b.x1;
  }
  tm.mark(4);
  if (what == 1 && o.basis == PS_BASIS_CORE && o.refine == PS_REFINE_NONE && mixed) {
    // ---- the core basis in the bulk precision (no FP64 refinement): the same products
    // and Cholesky factorization as below on FP32 matrix cores, the element-wise steps
    // in FP64; the result of the low-precision path before any refinement
    float* u32 = b.x32;    // U
    float* wm32 = b.d32;   // R_M^{-1}
    float* wk32 = b.t32;   // R_K^{-1}
    float* t132 = b.u32;   // R_M^{-1} U
    float* g32 = b.z32;    // G, then its factor
    float* wg32 = b.w32;   // R_G^{-1}
    cvt_f64_f32(s, U, u32, b.S);
    cvt_f64_f32(s, b.wmk, wm32, b.S);
    cvt_f64_f32(s, b.wmk + S, wk32, b.S);
    tm.mark(5);
    gemm_f32(s, gemm_problem(mp, mp, mp, wm32, mp, 0, u32, mp, 0, t132, mp, 1.0, 0.0, nullptr,
                             0, kAUpper));
    gemm_f32(s, gemm_problem(mp, mp, mp, wk32, mp, 1, t132, mp, 0, b.y32, mp, 1.0, 0.0, nullptr,
                             0, kALower));
    cvt_f32_f64(s, b.y32, b.t2, b.S);
    sym_scale_upper(s, b.t2, b.p11, m, mp, 1.0);
    cvt_f64_f32(s, b.p11, g32, b.S);
    potrf_inv_f32(s, g32, S, wg32, S, mp, 1, b.dinfo + 4);
    gemm_f32(s, gemm_problem(mp, mp, mp, t132, mp, 0, wg32, mp, 0, b.y32, mp, 1.0, 0.0, nullptr,
                             0, kBUpper));
    gemm_f32(s, gemm_problem(mp, mp, mp, wk32, mp, 0, wg32, mp, 0, b.n32, mp, 1.0, 0.0, nullptr,
                             0, kAUpper | kBUpper));
    cvt_f32_f64(s, b.y32, b.t2, b.S);
    cvt_f32_f64(s, b.n32, b.s12, b.S);
    sum_diff_scaled(s, b.t2, b.s12, b.top, b.qbot, M_SQRT1_2, mp);
    tm.mark(6);
    gemm_f32(s, gemm_problem(mp, mp, mp, wg32, mp, 1, wg32, mp, 0, t132, mp, 2.0, 0.0, nullptr,
                             0, kALower | kBUpper | kOutUpper | kMirror));
    cvt_f32_f64(s, t132, b.hp, b.S);
    tm.mark(7);
    copy_out(s, b.top, mp, out1, ld1, m, m);
    copy_out(s, b.qbot, mp, out1 + m, ld1, m, m);
    copy_out(s, b.hp, mp, out2, ld2, m, m);
  } else if (what == 1 && o.basis == PS_BASIS_CORE) {
    // ---- basis from the half-size core (no sign blocks needed).  With Q_h the
    // orthogonal symmetric [[I, I], [I, -I]]/sqrt(2), Q_h H Q_h = [[0, K], [M, 0]] maps
    // Z = Q_h [R_M^{-1} U; R_K^{-1}] onto Z P, P = U^T Y0, when U is the polar factor of
    // Y0, so range(Z) is the invariant subspace of the positive eigenvalues.  For any U,
    // Z^T Sigma Z = G = Y0^{-1} U + (Y0^{-1} U)^T (Y0^{-1} = R_K^{-T} R_M^{-1}) and
    // Z^T Sigma H Z = I + U^T U; with G = R_G^T R_G the basis Q_+ = Z R_G^{-1} is
    // Sigma-orthonormal whatever the accuracy of U, and H_+ = R_G^{-T} (I + U^T U) R_G^{-1}
    // = 2 R_G^{-T} R_G^{-1} (U orthogonal), the Rayleigh-Ritz block of that subspace.
    tm.mark(5);
    GemmProblem pt = gemm_problem(mp, mp, mp, b.wmk, mp, 0, U, mp, 0, b.t1, mp, 1.0, 0.0, nullptr,
                                  0, kAUpper);                    // T1 = R_M^{-1} U
    auto_split(pt, b.splitws);
    gemm_f64(s, pt);
    GemmProblem pv = gemm_problem(mp, mp, mp, b.wmk + S, mp, 1, b.t1, mp, 0, b.t2, mp, 1.0, 0.0,
                                  nullptr, 0, kALower);           // R_K^{-T} T1 = Y0^{-1} U
    auto_split(pv, b.splitws);
    gemm_f64(s, pv);
    sym_scale_upper(s, b.t2, b.p11, m, mp, 1.0);              // upper(G), padding I
    potrf_inv_f64(s, b.p11, S, b.wc, S, b.tmp, mp, 1, b.dinfo + 4, true, nullptr, b.t2, S);
    {
      GemmProblem pe[2];
      pe[0] = gemm_problem(mp, mp, mp, b.t1, mp, 0, b.wc, mp, 0, b.t2, mp, 1.0, 0.0, nullptr, 0,
                           kBUpper);                              // R_M^{-1} U R_G^{-1}
      pe[1] = gemm_problem(mp, mp, mp, b.wmk + S, mp, 0, b.wc, mp, 0, b.s12, mp, 1.0, 0.0,
                           nullptr, 0, kAUpper | kBUpper);        // R_K^{-1} R_G^{-1}
      with_ws(pe[0], b.splitws);
      gemm_f64(s, pe, 2);
      sum_diff_scaled(s, b.t2, b.s12, b.top, b.qbot, M_SQRT1_2, mp);
    }
    tm.mark(6);
    {
      GemmProblem ph = gemm_problem(mp, mp, mp, b.wc, mp, 1, b.wc, mp, 0, b.hp, mp, 2.0, 0.0,
                                    nullptr, 0, kALower | kBUpper | kOutUpper | kMirror);
      auto_split(ph, b.splitws);
      gemm_f64(s, ph);
    }
    tm.mark(7);
    copy_out(s, b.top, mp, out1, ld1, m, m);
    copy_out(s, b.qbot, mp, out1 + m, ld1, m, m);
    copy_out(s, b.hp, mp, out2, ld2, m, m);
  } else {
  // ---- blocks of sign(H):  S12 = W_M U R_K,  S21 = R_M^T U W_K^T
  {
    GemmProblem pg[2];
    pg[0] = gemm_problem(mp, mp, mp, U, mp, 0, b.mk + S, mp, 0, b.t1, mp, 1.0, 0.0, nullptr, 0,
                         kBUpper);
    pg[1] = gemm_problem(mp, mp, mp, U, mp, 0, b.wmk + S, mp, 1, b.t2, mp, 1.0, 0.0, nullptr, 0,
                         kBLower);
    with_ws(pg[0], b.splitws);
    gemm_f64(s, pg, 2);
    pg[0] = gemm_problem(mp, mp, mp, b.wmk, mp, 0, b.t1, mp, 0, b.s12, mp, 1.0, 0.0, nullptr, 0,
                         kAUpper);
    pg[1] = gemm_problem(mp, mp, mp, b.mk, mp, 1, b.t2, mp, 0, b.s21, mp, 1.0, 0.0, nullptr, 0,
                         kALower);
    with_ws(pg[0], b.splitws);
    gemm_f64(s, pg, 2);
    sign_blocks(s, b.s12, b.s21, b.as, b.bs, mp);
  }
  tm.mark(5);
  if (keep) {   // R_M, R_K, W_M, W_K and U for the adjoint, then the header
    double* st = keep->mats();
    PS_HIP(hipMemcpyAsync(st, b.mk, 2 * S * sizeof(double), hipMemcpyDeviceToDevice, s));
    PS_HIP(hipMemcpyAsync(st + 2 * S, b.wmk, 2 * S * sizeof(double), hipMemcpyDeviceToDevice, s));
    PS_HIP(hipMemcpyAsync(st + 4 * S, U, S * sizeof(double), hipMemcpyDeviceToDevice, s));
    keep->hdr[0] = kStoreVersion;
    keep->hdr[1] = m;
    keep->hdr[2] = mp;
    keep->hdr[3] = keep->r;
    keep->hdr[4] = keep->n;
    std::memcpy(pin, keep->hdr, kStoreHeader * sizeof(double));
    PS_HIP(hipMemcpyAsync(keep->base, pin, kStoreHeader * sizeof(double), hipMemcpyHostToDevice, s));
    PS_HIP(hipStreamSynchronize(s));   // the staging area is reused below
  }

  if (what == 0) {
    copy_out(s, b.as, mp, out1, ld1, m, m);
    copy_out(s, b.bs, mp, out2, ld2, m, m);
  } else {
    if (o.basis == PS_BASIS_LDL) {
    // ---- Alg. 7: Sigma P_+ = (Sigma S + Sigma)/2 (2m x 2m, rank m) = C C^T by the
    // truncated LDL^T with diagonal pivoting, Q_+ = Sigma C
    const int np = pad_to(2 * m);
    int* iw = reinterpret_cast<int*>(b.t2);
    const LdlScratch lw{b.wc, iw, iw + mp};
    ldl_form_casida(s, b.as, b.bs, m, mp, np, 1.0, b.z);
    ldl_factor(s, b.z, 2 * m, np, m, b.w, lw, b.dinfo + 4);
    ldl_casida_out(s, b.w, np, m, mp, b.top, b.qbot, b.ab);
    } else {
    // ---- Alg. 6: C = chol((I + A_s)/2), Q_+ = [C^T; P_{+,21} C^{-1}], P_{+,21} = -B_s/2
    half_shift_upper(s, b.as, b.p11, mp);
    potrf_inv_f64(s, b.p11, S, b.wc, S, b.tmp, mp, 1, b.dinfo + 4, true, nullptr, b.t1, S);
    {
      GemmProblem pq = gemm_problem(mp, mp, mp, b.bs, mp, 0, b.wc, mp, 0, b.qbot, mp, -0.5, 0.0,
                                    nullptr, 0, kBUpper);
      auto_split(pq, b.splitws);
      gemm_f64(s, pq);
    }
    mask_pad(s, b.qbot, m, mp, S, 1);
    basis_mix(s, b.p11, b.qbot, b.top, b.ab, mp);
    }
    mask_pad(s, b.ab, m, mp, S, 2);
    tm.mark(6);
    // ---- decoupling: H_+ = (R_M a)^T (R_M a) + (R_K b)^T (R_K b)
    {
      GemmProblem pf = gemm_problem(mp, mp, mp, b.mk, mp, 0, b.ab, mp, 0, b.F, 2 * mp, 1.0, 0.0,
                                    nullptr, 0, kAUpper);
      pf.nb1 = 2;
      pf.sA[0] = S;
      pf.sB[0] = S;
      pf.sC[0] = mp;
      pf.sD[0] = mp;
      gemm_f64(s, pf);
      GemmProblem ph = gemm_problem(mp, mp, 2 * mp, b.F, 2 * mp, 1, b.F, 2 * mp, 0, b.hp, mp, 1.0,
                                    0.0, nullptr, 0, kOutUpper | kMirror);
      auto_split(ph, b.splitws);
      gemm_f64(s, ph);
    }
    tm.mark(7);
    copy_out(s, b.top, mp, out1, ld1, m, m);
    copy_out(s, b.qbot, mp, out1 + m, ld1, m, m);
    copy_out(s, b.hp, mp, out2, ld2, m, m);
  }
  }
  PS_HIP(hipMemcpyAsync(pin + 8, b.dinfo, 16 * sizeof(int), hipMemcpyDeviceToHost, s));
  PS_HIP(hipStreamSynchronize(s));
  const int* di = (const int*)(pin + 8);
  if (what >= 1 && di[4]) {
    inf.status = PS_BASIS_BREAKDOWN;
    inf.failed_step = 4;
    inf.failed_mask = di[4];
    if (info) *info = inf;
    return PS_BASIS_BREAKDOWN;
  }
  tm.finish(inf.phase_ms);
  ktime.collect(inf);
  inf.status = PS_OK;
  if (info) *info = inf;
  return PS_OK;
}


// ---------------------------------------------------------------- any signature
// Division of a definite pseudosymmetric H of any signature Sigma = diag(sigma) (Sigma H
// symmetric positive definite; the random matrices of Sec. 6.1).  With
// M = Sigma H = R^T R and T = R Sigma R^T, H = R^{-1} T R, so sign(H) = R^{-1} sign(T) R,
// and sign(T) of the symmetric T is its polar factor: the Zolotarev iteration of Alg. 8
// on T (same alpha, beta, coefficients and stopping test, T^2 + c I SPD) runs on the
// kernels of the Casida form at size n.  The bases follow Alg. 6 as printed (Cholesky of
// the leading r_+ x r_+ block of Sigma P_+ and the leading r_- x r_- block of
// -Sigma P_-, r_+- the numbers of +-1 in Sigma, Thm. EVREalSigmaOrth), Q_- with the sign
// of Thm. HRisLDL, and the decoupled blocks H_+ = Q_+^T M Q_+ = (R Q_+)^T (R Q_+),
// H_- = -(R Q_-)^T (R Q_-) (Thm. DefDivConq).
size_t general_bytes(int n, const ps_opts& o) {
  Arena a;
  Buffers b;
  carve(a, b, n, resolve_r(o), 1, false);   // FP64 only, see run_general
  a.take<double>(pad_to(n));   // the signs
  return a.off + kAlign;
}

int run_general(ps_handle h, int n, const double* H, int ldh, const double* sigma, double* S_out,
                int ldso, double* Qp, int ldqp, double* Qm, int ldqm, double* Hp, int ldhp,
                double* Hm, int ldhm, const ps_opts& o, ps_info* info) {
  hipStream_t s = h->stream;
  const int r = resolve_r(o);
  char* base = workspace_base(h, general_bytes(n, o));
  if (!base) return PS_NO_WORKSPACE;
  Arena ar;
  ar.base = base;
  ar.dry = false;
  Buffers b;
  carve(ar, b, n, r, 1, false);
  double* sg = ar.take<double>(pad_to(n));
  const int np = b.mp;
  const long long S = (long long)b.S;
  double* pin = h->pinned;
  int p = 0;
  for (int i = 0; i < n; ++i) p += sigma[i] > 0 ? 1 : 0;
  const int q = n - p;
  for (int i = 0; i < np; ++i) pin[i] = i < n ? sigma[i] : 0.0;
  PS_HIP(hipMemcpyAsync(sg, pin, np * sizeof(double), hipMemcpyHostToDevice, s));
  PS_HIP(hipStreamSynchronize(s));   // the staging area is reused below

  ps_info inf{};
  inf.failed_step = -1;
  inf.r = r;
  Timer tm{h, o.timing != 0};
  const ClassTiming ktime(h, o.timing >= 2);
  tm.mark(-1);
  fill_int_zero(s, b.dinfo, 16);
  // ---- M = Sigma H = R^T R (in mk), W = R^{-1} (in wmk)
  double* R = b.mk;
  double* W = b.wmk;
  pack_general(s, n, np, H, ldh, sg, R);
  potrf_inv_f64(s, R, S, W, S, b.tmp, np, 1, b.dinfo + 0, true, nullptr, b.y, S);
  // ---- T = R Sigma R^T (y) and T^{-1} = W^T Sigma W (y + S): symmetric, zero padding
  scale_signs(s, R, b.t1, n, np, sg, true);    // R Sigma
  scale_signs(s, W, b.t2, n, np, sg, false);   // Sigma W
  {
    GemmProblem pg[2];
    pg[0] = gemm_problem(np, np, np, b.t1, np, 0, R, np, 1, b.y, np, 1.0, 0.0, nullptr, 0,
                         kAUpper | kBLower | kOutUpper | kMirror);
    pg[1] = gemm_problem(np, np, np, W, np, 1, b.t2, np, 0, b.y + S, np, 1.0, 0.0, nullptr, 0,
                         kALower | kBUpper | kOutUpper | kMirror);
    with_ws(pg[0], b.splitws);
    gemm_f64(s, pg, 2);
  }
  tm.mark(0);
  // ---- alpha >= sigma_max(T) = max |lambda(H)|, beta <= 1 / sigma_max(T^{-1}) (Alg. 8)
  double alpha = o.alpha, beta = o.beta;
  if (!(alpha > 0.0) || !(beta > 0.0)) {
    double a_est, b_est;
    estimate_bounds(s, b, b.y, std::max(4, std::min(o.lanczos_steps, 120)), pin, &a_est, &b_est,
                    inf.sigma_est);
    if (!(alpha > 0.0)) alpha = a_est;
    if (!(beta > 0.0)) beta = b_est;
  }
  // cond(M) = (sigma_max(R) sigma_max(R^{-1}))^2, which bounds this form's accuracy:
  // Golub-Kahan on the pair [R, W] (W copied next to R), estimates from below
  {
    PS_HIP(hipMemcpyAsync(R + S, W, S * sizeof(double), hipMemcpyDeviceToDevice, s));
    double est[2], a_r, b_r;
    estimate_bounds(s, b, R, std::max(4, std::min(o.lanczos_steps, 120)), pin, &a_r, &b_r, est);
    inf.cond_est = est[1] > 0.0 ? (est[0] / est[1]) * (est[0] / est[1]) : HUGE_VAL;
  }
  PS_HIP(hipMemcpyAsync(pin, b.dinfo, 16 * sizeof(int), hipMemcpyDeviceToHost, s));
  PS_HIP(hipStreamSynchronize(s));
  if (((int*)pin)[0] != 0) {
    inf.status = PS_NOT_DEFINITE;
    inf.failed_step = 0;
    inf.failed_mask = ((int*)pin)[0];
    if (info) *info = inf;
    return PS_NOT_DEFINITE;
  }
  inf.alpha = alpha;
  inf.beta = beta;
  tm.mark(1);
  // ---- sign(T) by the Zolotarev iteration with the stopping test of Alg. 8
  // FP64 steps whatever opts.precision says: cond(T) = cond(M), far above the shifted
  // conditions the FP32 bulk is chosen for, and the invariant subspaces an FP32 step
  // leaves about cond(T) u_32 off are not rotated back by an FP64 polish of U
  MixedCtx mxc{h->side, h->fork, h->join, o.mixed_kappa > 1.0 ? o.mixed_kappa : 20.0};
  const int status = polar_iterate(s, b, b.y, alpha, beta, o.r, o, pin, inf, tm, nullptr, &mxc);
  if (status != PS_OK) {
    inf.status = status;
    tm.finish(inf.phase_ms);
    if (info) *info = inf;
    return status;
  }
  const bool congruent = o.basis == PS_BASIS_CONGRUENT;
  // ---- sign(H) = W U R (s12), zero padding; the congruent bases do not need it
  if (S_out || !congruent) {
    GemmProblem p1 = gemm_problem(np, np, np, W, np, 0, b.x2, np, 0, b.t1, np, 1.0, 0.0, nullptr,
                                  0, kAUpper);
    auto_split(p1, b.splitws);
    gemm_f64(s, p1);
    GemmProblem p2 = gemm_problem(np, np, np, b.t1, np, 0, R, np, 0, b.s12, np, 1.0, 0.0, nullptr,
                                  0, kBUpper);
    auto_split(p2, b.splitws);
    gemm_f64(s, p2);
  }
  const double* Sg = b.s12;
  if (S_out) copy_out(s, Sg, np, S_out, ldso, n, n);
  tm.mark(5);
  // ---- Alg. 6 for one sign: k leading indices, a = +1 (Sigma P_+) or -1 (-Sigma P_-),
  // top block t Sigma C^T (t = +1, resp. -1), bottom (a/2) S(k:n, 0:k) C^{-1}; then the
  // decoupled block hs (R Q)^T (R Q)
  auto basis = [&](int k, double a, double t, double hs, double* Qout, int ldqo, double* Hout,
                   int ldho, int slot) {
    if (k == 0) return;
    const int kp = pad_to(k), rp = pad_to(std::max(n - k, 1));
    double* Q = b.ab;   // np x kp, ld np
    lead_block(s, Sg, np, sg, k, kp, a, b.p11);
    potrf_inv_f64(s, b.p11, 0, b.wc, 0, b.tmp, kp, 1, b.dinfo + slot, true, nullptr, b.t2, 0);
    chol_top(s, b.p11, kp, sg, k, t, b.top);
    copy_pad(s, b.top, kp, k, k, Q, np, k, kp);
    if (n > k) {
      copy_pad(s, Sg + k, np, n - k, k, b.qbot, rp, rp, kp);
      GemmProblem pb = gemm_problem(rp, kp, kp, b.qbot, rp, 0, b.wc, kp, 0, b.t1, rp, 0.5 * a, 0.0,
                                    nullptr, 0, kBUpper);
      gemm_f64(s, pb);
      copy_pad(s, b.t1, rp, n - k, k, Q + k, np, np - k, kp);
    } else if (np > k) {
      copy_pad(s, b.t1, rp, 0, 0, Q + k, np, np - k, kp);   // zero padding rows
    }
    GemmProblem pf = gemm_problem(np, kp, np, R, np, 0, Q, np, 0, b.F, np, 1.0, 0.0, nullptr, 0,
                                  kAUpper);
    gemm_f64(s, pf);
    GemmProblem ph = gemm_problem(kp, kp, np, b.F, np, 1, b.F, np, 0, b.hp, kp, hs, 0.0, nullptr,
                                  0, kOutUpper | kMirror);
    auto_split(ph, b.splitws);
    gemm_f64(s, ph);
    copy_out(s, Q, np, Qout, ldqo, n, k);
    copy_out(s, b.hp, kp, Hout, ldho, k, k);
  };
  // ---- bases from the projectors of T: (I + a U)/2 (rank k) = C C^T by the truncated
  // LDL^T with diagonal pivoting, V = W C spans the invariant subspace of H, its
  // Sigma-Gram matrix a V^T Sigma V = R_G^T R_G, Q = V R_G^{-1}, and the decoupled block
  // a (R Q)^T (R Q) = a F^T F with F = C R_G^{-1} (R V = C).  No product with sign(H),
  // whose projectors carry cond(M) u of error.
  // The two sides are independent chains of latency-bound LDL^T panels: with a side
  // stream the negative one runs there, on its own buffers, while the positive one runs
  // on the caller's stream (split-K only on the latter, whose workspace is not shared).
  struct CBuf {
    hipStream_t st;
    double *Z, *C, *V, *Q, *G, *D, *F, *Hb, *tmp, *pv, *ws, *L;
    int* iw;
  };
  auto cbasis = [&](const CBuf& u, int k, double a, double* Qout, int ldqo, double* Hout,
                    int ldho, int slot) {
    if (k == 0) return;
    const hipStream_t st = u.st;
    const int kp = pad_to(k);
    const LdlScratch lw{u.L, u.iw, u.iw + kp};
    proj_form(st, b.x2, n, np, a, u.Z);
    ldl_factor(st, u.Z, n, np, k, u.C, lw, b.dinfo + slot);
    GemmProblem pv = gemm_problem(np, kp, np, W, np, 0, u.C, np, 0, u.V, np, 1.0, 0.0, nullptr,
                                  0, kAUpper);
    gemm_f64(st, pv);
    ldl_scale_rows(st, u.V, np, kp, sg, n, u.Q);   // Sigma V
    GemmProblem pg = gemm_problem(kp, kp, np, u.V, np, 1, u.Q, np, 0, u.G, kp, a, 0.0, nullptr,
                                  0, kOutUpper | kMirror);
    if (u.ws) auto_split(pg, u.ws);
    gemm_f64(st, pg);
    unit_pad(st, u.G, k, kp);
    potrf_inv_f64(st, u.G, 0, u.D, 0, u.tmp, kp, 1, b.dinfo + slot, true, nullptr, u.pv, 0);
    GemmProblem pq[2];
    pq[0] = gemm_problem(np, kp, kp, u.V, np, 0, u.D, kp, 0, u.Q, np, 1.0, 0.0, nullptr, 0,
                         kBUpper);
    pq[1] = gemm_problem(np, kp, kp, u.C, np, 0, u.D, kp, 0, u.F, np, 1.0, 0.0, nullptr, 0,
                         kBUpper);
    gemm_f64(st, pq, 2);
    GemmProblem ph = gemm_problem(kp, kp, np, u.F, np, 1, u.F, np, 0, u.Hb, kp, a, 0.0, nullptr,
                                  0, kOutUpper | kMirror);
    if (u.ws) auto_split(ph, u.ws);
    gemm_f64(st, ph);
    copy_out(st, u.Q, np, Qout, ldqo, n, k);
    copy_out(st, u.Hb, kp, Hout, ldho, k, k);
  };
  // Alg. 7 on the same per-side buffers: a Sigma P_a = (Sigma S + a Sigma)/2 = C C^T,
  // Q = Sigma C, and the decoupled block hs (R Q)^T (R Q)
  auto lbasis = [&](const CBuf& u, int k, double a, double hs, double* Qout, int ldqo,
                    double* Hout, int ldho, int slot) {
    if (k == 0) return;
    const hipStream_t st = u.st;
    const int kp = pad_to(k);
    const LdlScratch lw{u.L, u.iw, u.iw + kp};
    ldl_form_general(st, Sg, sg, n, np, a, u.Z);
    ldl_factor(st, u.Z, n, np, k, u.C, lw, b.dinfo + slot);
    ldl_scale_rows(st, u.C, np, kp, sg, n, u.Q);
    GemmProblem pf = gemm_problem(np, kp, np, R, np, 0, u.Q, np, 0, u.F, np, 1.0, 0.0, nullptr,
                                  0, kAUpper);
    gemm_f64(st, pf);
    GemmProblem ph = gemm_problem(kp, kp, np, u.F, np, 1, u.F, np, 0, u.Hb, kp, hs, 0.0, nullptr,
                                  0, kOutUpper | kMirror);
    if (u.ws) auto_split(ph, u.ws);
    gemm_f64(st, ph);
    copy_out(st, u.Q, np, Qout, ldqo, n, k);
    copy_out(st, u.Hb, kp, Hout, ldho, k, k);
  };
  if (congruent || o.basis == PS_BASIS_LDL) {
    const hipStream_t t = (h->side && p > 0 && q > 0) ? h->side : s;
    const CBuf pos{s,     b.z,   b.w,    b.t1,   b.ab,  b.p11, b.wc, b.F, b.hp,
                   b.tmp, b.t2,  b.splitws, b.wc, reinterpret_cast<int*>(b.t2)};
    const CBuf neg{t,         b.z + S,  b.w + S, b.z + 2 * S, b.ab + S, b.s21, b.top, b.F + S,
                   b.as,      b.tmp + (size_t)np * kNb, b.bs, t == s ? b.splitws : nullptr,
                   b.top,     reinterpret_cast<int*>(b.qbot)};
    if (t != s) {
      PS_HIP(hipEventRecord(h->fork, s));
      PS_HIP(hipStreamWaitEvent(t, h->fork, 0));
    }
    if (congruent) {
      cbasis(neg, q, -1.0, Qm, ldqm, Hm, ldhm, 5);
      if (t != s) PS_HIP(hipEventRecord(h->join, t));
      cbasis(pos, p, 1.0, Qp, ldqp, Hp, ldhp, 4);
    } else {
      lbasis(neg, q, -1.0, -1.0, Qm, ldqm, Hm, ldhm, 5);
      if (t != s) PS_HIP(hipEventRecord(h->join, t));
      lbasis(pos, p, 1.0, 1.0, Qp, ldqp, Hp, ldhp, 4);
    }
    if (t != s) PS_HIP(hipStreamWaitEvent(s, h->join, 0));
    tm.mark(6);
  } else {
    basis(p, 1.0, 1.0, 1.0, Qp, ldqp, Hp, ldhp, 4);
    tm.mark(6);
    basis(q, -1.0, -1.0, -1.0, Qm, ldqm, Hm, ldhm, 5);
  }
  tm.mark(7);
  PS_HIP(hipMemcpyAsync(pin + 8, b.dinfo, 16 * sizeof(int), hipMemcpyDeviceToHost, s));
  PS_HIP(hipStreamSynchronize(s));
  const int* di = (const int*)(pin + 8);
  if (di[4] || di[5]) {
    inf.status = PS_BASIS_BREAKDOWN;
    inf.failed_step = 4;
    inf.failed_mask = di[4] ? 1 : 2;
    if (info) *info = inf;
    return PS_BASIS_BREAKDOWN;
  }
  tm.finish(inf.phase_ms);
  ktime.collect(inf);
  inf.status = PS_OK;
  if (info) *info = inf;
  return PS_OK;
}

// ---------------------------------------------------------------- complex forms
// The Bethe-Salpeter forms of Sec. 5 through the interleaved realification (see
// hermitian.hip): A and B realified into the real Casida blocks of half-size 2m, the
// real pipeline on those, and the complex results read back from the realified ones.
// Workspace: the realified blocks and outputs (5 (2m)^2 doubles), then the real
// pipeline's own.
size_t hermitian_bytes(int m, const ps_opts& o) {
  const size_t n2 = (size_t)(2 * m) * (2 * m);
  return (5 * n2 * sizeof(double) + kAlign - 1) / kAlign * kAlign + workspace_bytes(2 * m, o, 1);
}

// what: 0 sign blocks, 1 division (Q_+ 2m x m, H_+ m x m); flip_b: Eq:BSE1 (B complex
// symmetric, lower blocks conjugated) instead of Eq:BSE2 (B Hermitian)
int run_hermitian(ps_handle h, int m, const double* A, int lda, const double* B, int ldb,
                  double* O1, int ld1, double* O2, int ld2, const ps_opts& o, ps_info* info,
                  int what, bool flip_b) {
  hipStream_t s = h->stream;
  char* base = workspace_base(h, hermitian_bytes(m, o));
  if (!base) return PS_NO_WORKSPACE;
  const int m2 = 2 * m;
  const size_t n2 = (size_t)m2 * m2;
  double* Ar = reinterpret_cast<double*>(base);
  double* Br = Ar + n2;
  double* R1 = Br + n2;        // sign block A_s or Q_+ (4m x 2m)
  double* R2 = R1 + 2 * n2;    // sign block B_s or H_+
  char* ws = base + (5 * n2 * sizeof(double) + kAlign - 1) / kAlign * kAlign;
  realify(s, A, lda, m, Ar, m2, 0);
  realify(s, B, ldb, m, Br, m2, flip_b ? 1 : 0);
  int rc;
  if (what == 0) {
    rc = run(h, m2, Ar, m2, Br, m2, R1, m2, R2, m2, o, info, 0, ws, !flip_b);
    if (rc == PS_OK) {
      complexify(s, R1, m2, m, m, O1, ld1);
      complexify(s, R2, m2, m, m, O2, ld2);
    }
  } else {
    rc = run(h, m2, Ar, m2, Br, m2, R1, 2 * m2, R2, m2, o, info, 1, ws, !flip_b);
    if (rc == PS_OK) {
      complexify(s, R1, 2 * m2, 2 * m, m, O1, ld1);
      complexify(s, R2, m2, m, m, O2, ld2);
    }
  }
  if (rc == PS_OK) PS_HIP(hipStreamSynchronize(s));
  return rc;
}

// ---------------------------------------------------------------- GEMM autotuning
// One division with every GEMM launch logged (the built-in choices), then each distinct
// launch timed again under every choice it can take: 64 or 128 tiles, split-K by 1 to 8,
// and the stream-K schedule.  The trials rerun the logged launches
// on the division's own buffers (their contents are then garbage, which the timing does
// not depend on).  Workspace: the division's outputs, then its own.
size_t tune_bytes(int m, const ps_opts& o) {
  const size_t outs = (size_t)3 * m * m * sizeof(double);
  return (outs + kAlign - 1) / kAlign * kAlign + workspace_bytes(m, o, 1);
}

int run_autotune(ps_handle h, int m, const double* A, int lda, const double* B, int ldb,
                 const ps_opts& o, ps_gemm_tune* out, int cap, int* count) {
  hipStream_t s = h->stream;
  char* base = workspace_base(h, tune_bytes(m, o));
  if (!base) return PS_NO_WORKSPACE;
  double* Qp = reinterpret_cast<double*>(base);
  double* Hp = Qp + (size_t)2 * m * m;
  char* ws = base + ((size_t)3 * m * m * sizeof(double) + kAlign - 1) / kAlign * kAlign;
  GemmLog log;
  const GemmTuneTable* prev = gemm_get_tuning();
  gemm_set_tuning(nullptr);
  gemm_set_log(&log);
  ps_info inf{};
  int rc;
  try {
    rc = run(h, m, A, lda, B, ldb, Qp, 2 * m, Hp, m, o, &inf, 1, ws);
  } catch (...) {
    gemm_set_log(nullptr);
    gemm_set_tuning(prev);
    throw;
  }
  gemm_set_log(nullptr);
  if (rc != PS_OK) {
    gemm_set_tuning(prev);
    return rc;
  }
  if (h->side) PS_HIP(hipStreamSynchronize(h->side));
  PS_HIP(hipStreamSynchronize(s));
  // distinct launches: first occurrence and count
  std::vector<int> first;
  std::vector<int> times;
  for (size_t i = 0; i < log.keys.size(); ++i) {
    int f = -1;
    for (size_t j = 0; j < first.size(); ++j)
      if (log.keys[first[j]] == log.keys[i]) f = (int)j;
    if (f < 0) {
      first.push_back((int)i);
      times.push_back(1);
    } else {
      ++times[f];
    }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  PS_HIP(hipEventCreate(&e0));
  PS_HIP(hipEventCreate(&e1));
  auto trial = [&](int li, const GemmChoice* c) -> float {
    gemm_set_force(c);
    auto launch = [&] {
      if (!log.p64[li].empty())
        gemm_f64(s, log.p64[li].data(), (int)log.p64[li].size());
      else
        gemm_f32(s, log.p32[li].data(), (int)log.p32[li].size());
    };
    constexpr int kReps = 5;
    launch();
    launch();
    PS_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < kReps; ++r) launch();
    PS_HIP(hipEventRecord(e1, s));
    PS_HIP(hipEventSynchronize(e1));
    gemm_set_force(nullptr);
    float ms = 0.f;
    PS_HIP(hipEventElapsedTime(&ms, e0, e1));
    return ms / kReps;
  };
  int n = 0;
  try {
    for (size_t u = 0; u < first.size(); ++u) {
      const int li = first[u];
      // what the launch can take
      bool big = true, single = true, split_ok = true, ws_any = false;
      int kmin = 1 << 30;
      auto scan = [&](const auto& v) {
        single = v.size() == 1;
        for (const auto& p : v) {
          if (p.M % 128 || p.N % 128 || std::min(p.M, p.N) < 512) big = false;
          if (p.nb1 * p.nb2 != 1 || !p.ws || p.alpha_b || p.beta_b) split_ok = false;
          if (p.ws && p.ws_slots > 0) ws_any = true;
          kmin = std::min(kmin, p.K / 32);
        }
      };
      if (!log.p64[li].empty()) scan(log.p64[li]);
      else scan(log.p32[li]);
      const float t_default = trial(li, nullptr);
      GemmChoice best{0, 0, 0};
      float t_best = 0.f;
      bool have = false;
      for (int tile : {64, 128}) {
        if (tile == 128 && !big) continue;
        for (int k = 1; k <= kMaxSplit; ++k) {
          if (k > 1 && (!single || !split_ok || kmin < 4 * k)) continue;
          for (int sk : {0, 1}) {
            if (sk && (tile != 128 || !ws_any || k != 1)) continue;
            const GemmChoice c{tile, k, sk};
            const float t = trial(li, &c);
            if (!have || t < t_best) {
              best = c;
              t_best = t;
              have = true;
            }
          }
        }
      }
      if (n < cap && out) {
        ps_gemm_tune& e = out[n];
        e.key = log.keys[li];
        e.tile = best.tile;
        e.ksplit = best.ksplit;
        e.streamk = best.streamk;
        e.ms = t_best;
        e.ms_default = t_default;
        e.launches = times[u];
      }
      ++n;
    }
  } catch (...) {
    gemm_set_force(nullptr);
    gemm_set_tuning(prev);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  gemm_set_tuning(prev);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (count) *count = n;
  return PS_OK;
}

// ---------------------------------------------------------------- eigen-decomposition
// Leaves of the recursion: subproblems of at most this size go to the Jacobi kernel.
constexpr int kLeaf = 64;

// One split of Alg. 2 on the subproblem spanned by columns o..o+n of the accumulated
// basis V (H_+ restricted to it is A_sub = V_sub^T H_+ V_sub): shift sigma = median of
// the diagonal of A_sub, U = sign(A_sub - sigma I) by the Zolotarev iteration (the
// polar factor of a symmetric matrix is its sign), r_+ = trace((I + U)/2), bases of
// range(P_+) and range(P_-) by Alg. 4 (Cholesky of a leading block of each projector,
// the leading indices chosen as those with the largest diagonal of the projector), a
// Cholesky-QR pass over [Q_- Q_+], and V_sub <- V_sub [Q_- Q_+].  On success *rminus is
// the size of the lower part (eigenvalues below sigma), which occupies the first
// columns.
// Scratch of one recursion worker: the subproblem layout at `base` and the column
// block buffers (vs, t: mp x pad(n); zbd: pad(n)^2), host staging and stream.
struct SplitCtx {
  hipStream_t s;
  char* base;
  double *vs, *t, *zbd, *dscratch;
  int* perm;
  double* pin;
};

int eig_split(const SplitCtx& c, const EigBuffers& gl, int m, int o, int n, const ps_opts& o_,
              ps_info& inf, int* rminus) {
  hipStream_t s = c.s;
  double* pin = c.pin;
  struct {
    double *vacc, *hs, *vs, *t, *zbd, *dscratch;
    int* perm;
  } e{gl.vacc, gl.hs, c.vs, c.t, c.zbd, c.dscratch, c.perm};
  const int mp = pad_to(m);
  Arena sa;
  sa.base = c.base;
  sa.dry = false;
  Buffers b;
  carve(sa, b, n, 8, 2);
  const int np = b.mp;
  const long long Sn = (long long)b.S;
  // A_sub = V_sub^T (H_+ V_sub)
  copy_pad(s, e.vacc + (size_t)o * mp, mp, mp, n, e.vs, mp, mp, np);
  {
    GemmProblem pt = gemm_problem(mp, np, mp, e.hs, mp, 0, e.vs, mp, 0, e.t, mp);
    gemm_f64(s, pt);
    GemmProblem pa = gemm_problem(np, np, mp, e.vs, mp, 1, e.t, mp, 0, e.zbd, np, 1.0, 0.0,
                                  nullptr, 0, kOutUpper | kMirror);
    gemm_f64(s, pa);
  }
  get_diag(s, e.zbd, np, n, e.dscratch);
  offdiag_norm2(s, e.zbd, np, n, b.norms);
  PS_HIP(hipMemcpyAsync(pin, e.dscratch, n * sizeof(double), hipMemcpyDeviceToHost, s));
  PS_HIP(hipMemcpyAsync(pin + n, b.norms, sizeof(double), hipMemcpyDeviceToHost, s));
  PS_HIP(hipStreamSynchronize(s));
  const double off = std::sqrt(std::max(0.0, pin[n]));
  std::vector<double> dg(pin, pin + n);
  std::sort(dg.begin(), dg.end());
  const double lo = dg.front(), hi = dg.back();
  // A block whose eigenvalues all lie within (hi - lo) + 2 ||offdiag||_F of each other,
  // at most kClusterTol of its magnitude, is lambda I to that accuracy: every basis is an
  // eigenbasis, no shift can split it, and any split loses at most that much.  Its
  // columns are halved as they are (the halves end as leaves of this same kind or as
  // Jacobi leaves, which diagonalize what coupling is left).
  constexpr double kClusterTol = 1e-12;
  if ((hi - lo) + 2.0 * off <= kClusterTol * std::max(std::fabs(lo), std::fabs(hi))) {
    *rminus = n / 2;
    inf.eig_clusters += 1;
    return PS_OK;
  }
  double sigma = (n & 1) ? dg[n / 2] : 0.5 * (dg[n / 2 - 1] + dg[n / 2]);
  int rp = 0;
  bool ok = false;
  for (int attempt = 0; attempt < 8 && !ok; ++attempt) {
    if (attempt > 0) {
      // nudge the shift away from the side that received everything (or, after a
      // breakdown, just move it); the spread of the diagonal sets the step
      const double step = (hi - lo > 0 ? hi - lo : std::fabs(hi) + 1.0) * 0.25 / attempt;
      sigma += (rp == n) ? step : -step;
      if (rp != 0 && rp != n) sigma += 1e-3 * step;
    }
    fill_int_zero(s, b.dinfo, 16);
    scale_copy(s, e.zbd, b.y, 1.0, b.S);
    shift_diag(s, b.y, np, n, -sigma);
    // alpha >= sigma_max(Y), beta <= sigma_min(Y) = 1 / sigma_max(chol(Y^T Y)^{-1})
    {
      GemmProblem pg = gemm_problem(np, np, np, b.y, np, 1, b.y, np, 0, b.g, np, 1.0, 0.0,
                                    nullptr, 0, kOutUpper);
      auto_split(pg, b.splitws);
      gemm_f64(s, pg);
      spd_pad(s, b.g, b.z, n, np, 0.0);
      potrf_inv_f64(s, b.z, Sn, b.w, Sn, b.tmp, np, 1, b.dinfo + 3, true, nullptr, b.z + Sn,
                    Sn);
      PS_HIP(hipMemcpyAsync(b.y + Sn, b.w, b.S * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    // the estimator pair overwrites b.y: keep Y in x1 meanwhile
    scale_copy(s, b.y, b.x1, 1.0, b.S);
    double est[2], alpha, beta;
    estimate_bounds(s, b, b.y, std::max(4, std::min(o_.lanczos_steps, 120)), pin, &alpha, &beta,
                    est);
    PS_HIP(hipMemcpyAsync(pin, b.dinfo, 16 * sizeof(int), hipMemcpyDeviceToHost, s));
    PS_HIP(hipStreamSynchronize(s));
    if (((int*)pin)[3] != 0 || !(beta > 0.0) || !(alpha > beta)) {
      rp = -1;   // (nearly) singular shift: move it
      continue;
    }
    scale_copy(s, b.x1, b.y, 1.0, b.S);
    ps_info pinf{};
    Timer tm0{nullptr, false};
    const int st = polar_iterate(s, b, b.y, alpha, beta, kEigR, o_, pin, pinf, tm0);
    inf.eig_steps += pinf.steps;
    inf.eig_restarts += pinf.restarts;
    inf.bounds_rejected += pinf.bounds_rejected;
    inf.delta_norm_est = std::max(inf.delta_norm_est, pinf.delta_norm_est);
    if (st != PS_OK) {
      rp = -1;
      continue;
    }
    get_diag(s, b.x2, np, n, e.dscratch);
    PS_HIP(hipMemcpyAsync(pin, e.dscratch, n * sizeof(double), hipMemcpyDeviceToHost, s));
    PS_HIP(hipStreamSynchronize(s));
    double tr = 0.0;
    for (int i = 0; i < n; ++i) tr += pin[i];
    rp = (int)std::lround(0.5 * (n + tr));
    ok = rp > 0 && rp < n;
  }
  if (!ok) return PS_NOT_CONVERGED;
  const int rm = n - rp;
  // pivot order: indices by decreasing diagonal of P_+ = (I + U)/2 (ties by index)
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::vector<double> du(pin, pin + n);
  std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return du[x] > du[y]; });
  int* ipin = (int*)pin;
  for (int i = 0; i < n; ++i) ipin[i] = idx[i];
  PS_HIP(hipMemcpyAsync(e.perm, ipin, n * sizeof(int), hipMemcpyHostToDevice, s));
  const int* pp = e.perm;        // r_+ pivots of P_+
  const int* pm = e.perm + rp;   // the other r_- indices: pivots of P_-
  const int npp = pad_to(rp), npm = pad_to(rm);
  const double* U = b.x2;
  double* z[8];
  double* w[8];
  for (int k = 0; k < 8; ++k) {
    z[k] = b.z + k * Sn;
    w[k] = b.w + k * Sn;
  }
  fill_int_zero(s, b.dinfo, 16);
  // Alg. 4: P_+(pp, pp) = C_+ C_+^T (C_+ = R_+^T), Q_+ rows pp = C_+, rows pm = P_+(pm, pp) C_+^{-T}
  gather_sym(s, U, np, pp, pp, rp, rp, 0.5, 0.5, z[0], npp, npp, npp, 1.0, 1);
  gather_sym(s, U, np, pm, pp, rm, rp, 0.5, 0.5, z[1], npm, npm, npp, 0.0, 0);
  gather_sym(s, U, np, pm, pm, rm, rm, -0.5, 0.5, z[3], npm, npm, npm, 1.0, 1);
  gather_sym(s, U, np, pp, pm, rp, rm, -0.5, 0.5, z[4], npp, npp, npm, 0.0, 0);
  potrf_inv_f64(s, z[0], 0, w[0], 0, b.tmp, npp, 1, b.dinfo + 4, true, nullptr, w[3], 0);
  potrf_inv_f64(s, z[3], 0, w[1], 0, b.tmp, npm, 1, b.dinfo + 5, true, nullptr, w[4], 0);
  {
    GemmProblem q1 = gemm_problem(npm, npp, npp, z[1], npm, 0, w[0], npp, 0, z[2], npm, 1.0, 0.0,
                                  nullptr, 0, kBUpper);
    GemmProblem q2 = gemm_problem(npp, npm, npm, z[4], npp, 0, w[1], npm, 0, z[5], npp, 1.0, 0.0,
                                  nullptr, 0, kBUpper);
    gemm_f64(s, q1);
    gemm_f64(s, q2);
  }
  // Q0 = [Q_- Q_+]
  fill_zero(s, z[6], b.S);
  scatter_rows(s, z[3], npm, 1, pm, rm, rm, z[6], np, 0);
  scatter_rows(s, z[5], npp, 0, pp, rp, rm, z[6], np, 0);
  scatter_rows(s, z[0], npp, 1, pp, rp, rp, z[6], np, rm);
  scatter_rows(s, z[2], npm, 0, pm, rm, rp, z[6], np, rm);
  // one Cholesky-QR pass: Q0 <- Q0 chol(Q0^T Q0)^{-1}
  {
    GemmProblem pg = gemm_problem(np, np, np, z[6], np, 1, z[6], np, 0, b.g, np, 1.0, 0.0,
                                  nullptr, 0, kOutUpper);
    auto_split(pg, b.splitws);
    gemm_f64(s, pg);
    spd_pad(s, b.g, z[7], n, np, 0.0);
    potrf_inv_f64(s, z[7], 0, w[2], 0, b.tmp, np, 1, b.dinfo + 6, true, nullptr, w[3], 0);
    GemmProblem pq = gemm_problem(np, np, np, z[6], np, 0, w[2], np, 0, b.x0, np, 1.0, 0.0,
                                  nullptr, 0, kBUpper);
    gemm_f64(s, pq);
    mask_pad(s, b.x0, n, np, Sn, 1);
  }
  // V_sub <- V_sub Q0
  {
    GemmProblem pv = gemm_problem(mp, np, np, e.vs, mp, 0, b.x0, np, 0, e.t, mp);
    gemm_f64(s, pv);
    put_cols(s, e.t, mp, e.vacc, mp, o, n, mp);
  }
  PS_HIP(hipMemcpyAsync(pin, b.dinfo, 16 * sizeof(int), hipMemcpyDeviceToHost, s));
  PS_HIP(hipStreamSynchronize(s));
  const int* di = (const int*)pin;
  if (di[4] || di[5] || di[6]) return PS_BASIS_BREAKDOWN;
  *rminus = rm;
  return PS_OK;
}

int run_eig(ps_handle h, int m, const double* A, int lda, const double* B, int ldb, double* lam,
            double* V, int ldv, const ps_opts& o, ps_info* info, double* SA = nullptr,
            double* SB = nullptr, int lds = 0) {
  hipStream_t s = h->stream;
  char* base = workspace_base(h, workspace_bytes(m, o, 2));
  if (!base) return PS_NO_WORKSPACE;
  const int mp = pad_to(m);
  const size_t S = (size_t)mp * mp;
  Arena ea;
  ea.base = base;
  ea.off = eig_region_offset(m, o);
  ea.dry = false;
  EigBuffers e;
  carve_eig(ea, e, m);
  double* pin = h->pinned;
  // ---- one spectral division step (Alg. 3 with Alg. 6 bases)
  ps_info inf{};
  int st = run(h, m, A, lda, B, ldb, e.qf, 2 * m, e.hraw, m, o, &inf, 1);
  if (st != PS_OK) {
    if (info) *info = inf;
    return st;
  }
  if (SA && SB) {
    // the blocks of sign(H) from the division step, before the recursion reuses its buffers
    Arena ra;
    ra.base = base;
    ra.dry = false;
    Buffers db;
    carve(ra, db, m, resolve_r(o), 1, mixed_arith(o, m));
    copy_out(s, db.as, mp, SA, lds, m, m);
    copy_out(s, db.bs, mp, SB, lds, m, m);
  }
  copy_pad(s, e.qf, 2 * m, m, m, e.qt, mp, mp, mp);
  copy_pad(s, e.qf + m, 2 * m, m, m, e.qb, mp, mp, mp);
  copy_pad(s, e.hraw, m, m, m, e.hs, mp, mp, mp);
  // ---- Alg. 2 on H_+: splits down to leaves of at most kLeaf.  Blocks wider than the
  // worker cap are split here; the subtrees below it are independent and go, largest
  // first, to kEigWorkers host threads with their own streams and scratch.
  fill_zero(s, e.vacc, S);
  shift_diag(s, e.vacc, mp, m, 1.0);
  SplitCtx main_ctx{s, base, e.vs, e.t, e.zbd, e.dscratch, e.perm, pin};
  const int cap = eig_worker_cap(m);
  std::vector<std::pair<int, int>> stack{{0, m}}, leaves, subtrees;
  while (!stack.empty()) {
    const auto [o0, n0] = stack.back();
    stack.pop_back();
    if (n0 <= kLeaf) {
      leaves.push_back({o0, n0});
      continue;
    }
    if (n0 <= cap) {
      subtrees.push_back({o0, n0});
      continue;
    }
    int rm = 0;
    st = eig_split(main_ctx, e, m, o0, n0, o, inf, &rm);
    if (st != PS_OK) {
      inf.status = st;
      inf.failed_step = 5;
      if (info) *info = inf;
      return st;
    }
    inf.eig_splits += 1;
    stack.push_back({o0 + rm, n0 - rm});
    stack.push_back({o0, rm});
  }
  if (!subtrees.empty()) {
    PS_HIP(hipStreamSynchronize(s));   // the workers' streams start from the current V
    // the caller's worker streams (up to kEigWorkers); without any, the subtrees run on
    // the handle's own stream and scratch, one after the other
    const int nwk = ensure_workers(h, kEigWorkers);
    if (nwk < 0) return PS_HIP_ERROR;
    const int nw = std::max(1, nwk);
    std::vector<SplitCtx> ctx(nw);
    for (int k = 0; k < nw; ++k) {
      if (nwk == 0) {
        ctx[k] = main_ctx;
        continue;
      }
      ctx[k].s = h->workers[k]->stream;
      ctx[k].pin = h->workers[k]->pinned;
      carve_eig_worker(ea, m, &ctx[k].base, &ctx[k].vs, &ctx[k].t, &ctx[k].zbd,
                       &ctx[k].dscratch, &ctx[k].perm);
    }
    // shared pool: a worker takes the widest pending block and returns its two halves
    std::mutex mu;
    std::condition_variable cv;
    int busy = 0;
    bool failed = false;
    std::vector<std::vector<std::pair<int, int>>> wleaves(nw);
    std::vector<ps_info> winf(nw);
    std::vector<int> wst(nw, PS_OK);
    auto work = [&](int k) {
      if (hipSetDevice(h->device) != hipSuccess) {
        std::lock_guard<std::mutex> g(mu);
        wst[k] = PS_HIP_ERROR;
        failed = true;
        cv.notify_all();
        return;
      }
      for (;;) {
        std::pair<int, int> node;
        {
          std::unique_lock<std::mutex> g(mu);
          cv.wait(g, [&] { return failed || !subtrees.empty() || busy == 0; });
          if (failed || subtrees.empty()) return;
          auto it = std::max_element(subtrees.begin(), subtrees.end(),
                                     [](const std::pair<int, int>& x,
                                        const std::pair<int, int>& y) {
                                       return x.second < y.second;
                                     });
          node = *it;
          subtrees.erase(it);
          ++busy;
        }
        int rm = 0, r1 = PS_HIP_ERROR;
        if (node.second <= kLeaf) {
          r1 = PS_OK;
        } else {
          try {
            r1 = eig_split(ctx[k], e, m, node.first, node.second, o, winf[k], &rm);
          } catch (...) {
            r1 = PS_HIP_ERROR;
          }
        }
        std::lock_guard<std::mutex> g(mu);
        --busy;
        if (r1 != PS_OK) {
          wst[k] = r1;
          failed = true;
        } else if (node.second <= kLeaf) {
          wleaves[k].push_back(node);
        } else {
          winf[k].eig_splits += 1;
          for (const auto& c : {std::make_pair(node.first, rm),
                                std::make_pair(node.first + rm, node.second - rm)}) {
            if (c.second <= kLeaf)
              wleaves[k].push_back(c);
            else
              subtrees.push_back(c);
          }
        }
        cv.notify_all();
      }
    };
    std::vector<std::thread> threads;
    for (int k = 1; k < nw; ++k) threads.emplace_back(work, k);
    work(0);
    for (auto& t : threads) t.join();
    for (int k = 0; k < nw; ++k) {
      inf.eig_splits += winf[k].eig_splits;
      inf.eig_clusters += winf[k].eig_clusters;
      inf.eig_steps += winf[k].eig_steps;
      inf.eig_restarts += winf[k].eig_restarts;
      leaves.insert(leaves.end(), wleaves[k].begin(), wleaves[k].end());
      if (wst[k] != PS_OK) {
        inf.status = wst[k];
        inf.failed_step = 5;
        if (info) *info = inf;
        return wst[k];
      }
    }
  }
  // ---- leaves: B = V^T H_+ V is block diagonal up to rounding; Jacobi on its blocks
  {
    GemmProblem pt = gemm_problem(mp, mp, mp, e.hs, mp, 0, e.vacc, mp, 0, e.t, mp);
    gemm_f64(s, pt);
    GemmProblem pb = gemm_problem(mp, mp, mp, e.vacc, mp, 1, e.t, mp, 0, e.vs, mp, 1.0, 0.0,
                                  nullptr, 0, kOutUpper | kMirror);
    gemm_f64(s, pb);
  }
  const int nl = (int)leaves.size();
  int* ipin = (int*)pin;
  for (int l = 0; l < nl; ++l) {
    ipin[l] = leaves[l].first;
    ipin[nl + l] = leaves[l].second;
  }
  PS_HIP(hipMemcpyAsync(e.leaf_o, ipin, nl * sizeof(int), hipMemcpyHostToDevice, s));
  PS_HIP(hipMemcpyAsync(e.leaf_n, ipin + nl, nl * sizeof(int), hipMemcpyHostToDevice, s));
  fill_int_zero(s, e.sweeps, 16);
  fill_zero(s, e.zbd, S);
  jacobi_leaves(s, e.vs, mp, e.leaf_o, e.leaf_n, nl, e.zbd, mp, e.w, e.sweeps);
  {
    GemmProblem pz = gemm_problem(mp, mp, mp, e.vacc, mp, 0, e.zbd, mp, 0, e.t, mp);
    gemm_f64(s, pz);
  }
  // ---- ascending order (the splits already order the blocks; this is a check)
  PS_HIP(hipMemcpyAsync(pin, e.w, m * sizeof(double), hipMemcpyDeviceToHost, s));
  PS_HIP(hipMemcpyAsync(pin + m, e.sweeps, sizeof(int), hipMemcpyDeviceToHost, s));
  PS_HIP(hipStreamSynchronize(s));
  inf.eig_leaves = nl;
  inf.eig_sweeps = *(int*)(pin + m);
  std::vector<int> ord(m);
  for (int i = 0; i < m; ++i) ord[i] = i;
  {
    std::vector<double> wv(pin, pin + m);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return wv[x] < wv[y]; });
  }
  bool sorted = true;
  for (int i = 0; i < m; ++i) sorted = sorted && ord[i] == i;
  const double* wfin = e.w;
  const double* vfin = e.t;
  if (!sorted) {
    for (int i = 0; i < m; ++i) ipin[i] = ord[i];
    PS_HIP(hipMemcpyAsync(e.perm, ipin, m * sizeof(int), hipMemcpyHostToDevice, s));
    permute_vec(s, e.w, e.perm, m, e.wsorted);
    permute_cols(s, e.t, mp, e.perm, mp, m, e.vs, mp);
    wfin = e.wsorted;
    vfin = e.vs;
  }
  eig_lambda(s, wfin, m, lam);
  if (V) {
    // V = [Q_+ Z, Pi Q_+ Z], Q_+ = [Qt; Qb]
    double* vt = (vfin == e.t) ? e.vs : e.t;
    GemmProblem p1 = gemm_problem(mp, mp, mp, e.qt, mp, 0, vfin, mp, 0, vt, mp);
    gemm_f64(s, p1);
    copy_out(s, vt, mp, V, ldv, m, m);
    GemmProblem p2 = gemm_problem(mp, mp, mp, e.qb, mp, 0, vfin, mp, 0, vt, mp);
    gemm_f64(s, p2);
    copy_out(s, vt, mp, V + m, ldv, m, m);
    pi_columns(s, V, ldv, m);
    canon_sign(s, V, ldv, 2 * m, 2 * m);
  }
  PS_HIP(hipStreamSynchronize(s));
  inf.status = PS_OK;
  if (info) *info = inf;
  return PS_OK;
}



// Adjoint of the sign function: with H = V diag(lambda) V^{-1} from the eigen-
// decomposition (V^{-1} = Sigma_hat V^T Sigma, Thm. EVREalSigmaOrth), the gradient of a
// loss with respect to H is V^{-T} (F o (V^T G V^{-T})) V^T, F the divided differences
// of sign on the eigenvalues; the blocks of dH = [[dA, dB], [-dB, -dA]] then give the
// gradients of A and B.  Four 2m x 2m matrix-core GEMMs and element-wise kernels.
size_t adjoint_bytes(int m) {
  const size_t np = (size_t)pad_to(2 * m);
  return 4 * np * np * sizeof(double) + 5 * kAlign;
}

int run_sign_bwd(ps_handle h, int m, const double* lam, const double* V, int ldv,
                 const double* gSA, const double* gSB, int ldg, double* gA, double* gB,
                 int ldo) {
  hipStream_t s = h->stream;
  char* base = workspace_base(h, adjoint_bytes(m));
  if (!base) return PS_NO_WORKSPACE;
  const int np = pad_to(2 * m);
  const size_t S = (size_t)np * np;
  Arena a;
  a.base = base;
  a.dry = false;
  double* vp = a.take<double>(S);
  double* g = a.take<double>(S);
  double* u = a.take<double>(S);
  double* t = a.take<double>(S);
  copy_pad(s, V, ldv, 2 * m, 2 * m, vp, np, np, np);
  build_gbar(s, gSA, gSB, ldg, m, g, np);
  GemmProblem p1 = gemm_problem(np, np, np, g, np, 0, vp, np, 0, u, np);     // (G Sigma) V
  gemm_f64(s, p1);
  GemmProblem p2 = gemm_problem(np, np, np, vp, np, 1, u, np, 0, t, np);     // V^T (G Sigma) V
  gemm_f64(s, p2);
  dk_hadamard(s, t, np, lam, m);
  GemmProblem p3 = gemm_problem(np, np, np, vp, np, 0, t, np, 0, u, np);     // V M
  gemm_f64(s, p3);
  GemmProblem p4 = gemm_problem(np, np, np, u, np, 0, vp, np, 1, g, np);     // V M V^T
  gemm_f64(s, p4);
  grad_assemble(s, g, np, m, gA, gB, ldo);
  PS_HIP(hipStreamSynchronize(s));
  return PS_OK;
}

// Workspace of the stored-factor backward: 13 matrices, two stacks of r and the split-K
// partials.
size_t sign_bwd_iter_bytes(int m, int r) {
  const size_t S = (size_t)pad_to(m) * pad_to(m);
  return (13 + 2 * (size_t)r + kMaxSplit) * S * sizeof(double) + 16 * kAlign;
}

// Reverse mode through the forward that filled `store` (see StepStore):
//   S12 = W_M U R_K, S21 = R_M^T U W_K^T, S_A = (sym S21 + sym S12)/2,
//   S_B = (sym S21 - sym S12)/2;
//   Zolotarev step X' = hat C X (I + sum_j a_j N_j), N_j = (X^T X + c_j I)^{-1} = W_j W_j^T:
//   gX = hat C (G (I + sum_j a_j N_j) - X (Z + Z^T)), Z = sum_j a_j N_j X^T G N_j
//   (Z + Z^T = sum_j a_j N_j (X^T G + G^T X) N_j);
//   X_k = scale_k (previous output or Y0), Y0 = R_M R_K^T, W = R^{-1}: gR -= W^T gW W^T;
//   M = R^T R: gM = sym(W Phi(R triu(gR)^T) W^T), Phi = lower triangle, diagonal halved;
//   gA = gM + gK, gB = gM - gK.
int run_sign_bwd_iter(ps_handle h, int m, const double* store, const double* gSA,
                      const double* gSB, int ldg, double* gA, double* gB, int ldo) {
  hipStream_t s = h->stream;
  double* pin = h->pinned;
  PS_HIP(hipMemcpyAsync(pin, store, kStoreHeader * sizeof(double), hipMemcpyDeviceToHost, s));
  PS_HIP(hipStreamSynchronize(s));
  double hdr[kStoreHeader];
  std::memcpy(hdr, pin, sizeof(hdr));
  const int mp = pad_to(m);
  const int r = (int)hdr[3], nsteps = (int)hdr[4];
  if (hdr[0] != kStoreVersion || (int)hdr[1] != m || (int)hdr[2] != mp || r < 1 || r > 8 ||
      nsteps < 1 || nsteps > kStoreMaxSteps)
    return -3;
  char* base = workspace_base(h, sign_bwd_iter_bytes(m, r));
  if (!base) return PS_NO_WORKSPACE;
  const size_t S = (size_t)mp * mp;
  Arena a;
  a.base = base;
  a.dry = false;
  double* g12 = a.take<double>(S);
  double* g21 = a.take<double>(S);
  double* gu1 = a.take<double>(S);
  double* gu2 = a.take<double>(S);
  double* G = a.take<double>(S);
  double* t1 = a.take<double>(S);
  double* t2 = a.take<double>(S);
  double* Z = a.take<double>(S);
  double* P = a.take<double>(S);
  double* grm = a.take<double>(S);
  double* grk = a.take<double>(S);
  double* gmm = a.take<double>(S);
  double* gkk = a.take<double>(S);
  double* sa = a.take<double>((size_t)r * S);
  double* sb = a.take<double>((size_t)r * S);
  double* sws = a.take<double>((size_t)kMaxSplit * S);   // split-K / stream-K partials
  StepStore st;
  st.base = const_cast<double*>(store);
  st.mp = mp;
  st.r = r;
  const double* RM = st.mats();
  const double* RK = RM + S;
  const double* WM = RM + 2 * S;
  const double* WK = RM + 3 * S;
  const double* U = RM + 4 * S;
  auto gemm = [&](const double* A_, int tA, const double* B_, int tB, double* D, double al,
                  double be, const double* C, int flags) {
    GemmProblem p = gemm_problem(mp, mp, mp, A_, mp, tA, B_, mp, tB, D, mp, al, be, C, mp, flags);
    auto_split(p, sws);
    gemm_f64(s, p);
  };
  // batch of r products, operand A (or B) stepping through the stack
  auto gemm_r = [&](const double* A_, long long sA, int tA, const double* B_, long long sB, int tB,
                    double* D, int flags) {
    GemmProblem p = gemm_problem(mp, mp, mp, A_, mp, tA, B_, mp, tB, D, mp, 1.0, 0.0, nullptr, 0,
                                 flags);
    p.nb1 = r;
    p.sA[0] = sA;
    p.sB[0] = sB;
    p.sD[0] = (long long)S;
    gemm_f64(s, p);
  };
  // sum_j a_j L_j W_j^T over the stacks (K segments of mp), plus beta C
  auto gemm_seg = [&](const double* L, const double* W, const double* aj, double* D, double be,
                      const double* C, int flags) {
    GemmProblem p = gemm_problem(mp, mp, r * mp, L, mp, 0, W, mp, 1, D, mp, 1.0, be, C, mp,
                                 kBLower | flags);
    p.kseg = mp;
    p.nseg = r;
    for (int j = 0; j < r; ++j) p.kscale[j] = aj[j];
    if (r > 1 && r <= kMaxSplit) {   // one partial per segment, as the forward's N product
      p.ksplit = r;
      p.ws = sws;
      p.ws_slots = kMaxSplit;
    }
    gemm_f64(s, p);
  };
  // ---- sign blocks: g12 = dL/dS12, g21 = dL/dS21; gU = W_M^T g12 R_K^T + R_M g21 W_K
  adj_seed(s, gSA, gSB, ldg, m, mp, g12, g21);
  gemm(WM, 1, g12, 0, t1, 1.0, 0.0, nullptr, kALower);
  gemm(t1, 0, RK, 1, gu1, 1.0, 0.0, nullptr, kBLower);
  gemm(RM, 0, g21, 0, t2, 1.0, 0.0, nullptr, kAUpper);
  gemm(t2, 0, WK, 0, gu2, 1.0, 0.0, nullptr, kBUpper);
  sum_diff_scaled(s, gu1, gu2, G, t1, 1.0, mp);                      // G = gU
  // ---- the Zolotarev steps in reverse order
  for (int k = nsteps - 1; k >= 0; --k) {
    const double* X = st.x(k);
    const double* W = st.w(k);
    const double* hk = hdr + 16 + 16 * k;
    const double scale = hk[0], chat = hk[1];
    // Z + Z^T = sum_j a_j N_j (X^T G + G^T X) N_j: symmetric, so two of its products
    // form only their upper triangles
    gemm(X, 1, G, 0, t1, 1.0, 0.0, nullptr, 0);                       // X^T G
    sym2(s, t1, Z, mp);                                               // X^T G + G^T X
    gemm_r(W, (long long)S, 1, Z, 0, 0, sa, kALower);                 // W_j^T (.)
    gemm_r(sa, (long long)S, 0, W, (long long)S, 0, sb,
           kBUpper | kOutUpper | kMirror);                            // (.) W_j
    gemm_r(W, (long long)S, 0, sb, (long long)S, 0, sa, kAUpper);     // W_j (.)
    gemm_seg(sa, W, hk + 2, t2, 0.0, nullptr, kOutUpper | kMirror);   // Z + Z^T
    gemm_r(G, 0, 0, W, (long long)S, 0, sb, kBUpper);                 // G W_j
    gemm_seg(sb, W, hk + 2, P, 1.0, G, 0);                            // G (I + sum a_j N_j)
    gemm(X, 0, t2, 0, G, -scale * chat, scale * chat, P, 0);         // gradient of the input
  }
  // ---- Y0 = R_M R_K^T (G = dL/dY0), W = R^{-1}:
  //   gR_M = U W_K^T g21 - gU1 U^T W_M^T + gY0 R_K,  gR_K = U^T W_M^T g12 - gU2^T U W_K^T + gY0^T R_M
  gemm(U, 0, WK, 1, t1, 1.0, 0.0, nullptr, kBLower);
  gemm(t1, 0, g21, 0, grm, 1.0, 0.0, nullptr, 0);
  gemm(gu1, 0, U, 1, t1, 1.0, 0.0, nullptr, 0);
  gemm(t1, 0, WM, 1, grm, -1.0, 1.0, grm, kBLower);
  gemm(G, 0, RK, 0, grm, 1.0, 1.0, grm, kBUpper);
  gemm(U, 1, WM, 1, t1, 1.0, 0.0, nullptr, kBLower);
  gemm(t1, 0, g12, 0, grk, 1.0, 0.0, nullptr, 0);
  gemm(gu2, 1, U, 0, t1, 1.0, 0.0, nullptr, 0);
  gemm(t1, 0, WK, 1, grk, -1.0, 1.0, grk, kBLower);
  gemm(G, 1, RM, 0, grk, 1.0, 1.0, grk, kBUpper);
  // ---- Cholesky adjoints: gM = W Phi(R triu(gR)^T) W^T (symmetrized at the output)
  auto chol_adj = [&](const double* R, const double* Wf, double* gR, double* out) {
    zero_lower(s, gR, mp, 0, 1);
    gemm(R, 0, gR, 1, t1, 1.0, 0.0, nullptr, kAUpper | kBLower);
    phi_lower(s, t1, mp);
    gemm(Wf, 0, t1, 0, t2, 1.0, 0.0, nullptr, kAUpper | kBLower);
    gemm(t2, 0, Wf, 1, out, 1.0, 0.0, nullptr, kBLower);
  };
  chol_adj(RM, WM, grm, gmm);
  chol_adj(RK, WK, grk, gkk);
  adj_out(s, gmm, gkk, mp, m, gA, gB, ldo);
  PS_HIP(hipStreamSynchronize(s));
  return PS_OK;
}

int check_common(ps_handle h, int m, const double* A, int lda, const double* B, int ldb,
                 const ps_opts* o) {
  if (!h) return -1;
  if (m < 1) return -2;
  if (!A) return -3;
  if (lda < m) return -4;
  if (!B) return -5;
  if (ldb < m) return -6;
  if (o && (o->r < 0 || o->r > 8 || o->max_restarts < 0 || o->max_steps < 0 ||
            o->max_steps > 1 || (o->precision != PS_PREC_FP64 && o->precision != PS_PREC_MIXED) ||
            (o->basis != PS_BASIS_ALG6 && o->basis != PS_BASIS_CORE &&
             o->basis != PS_BASIS_LDL) ||
            (o->basis == PS_BASIS_LDL && pad_to(2 * m) > kLdlMaxN) ||
            o->iteration < PS_ITER_ZOLO || o->iteration > PS_ITER_NEWTON ||
            o->refine < PS_REFINE_NONE || o->refine > PS_REFINE_NS ||
            (o->iteration != PS_ITER_ZOLO &&
             (o->precision != PS_PREC_FP64 || o->max_steps != 0))))
    return -11;
  return 0;
}

template <class F>
int guarded(ps_handle h, F&& f) {
  // the handle's GEMM tuning table for the launches of this call on this host thread
  struct TuneScope {
    const GemmTuneTable* prev;
    explicit TuneScope(const GemmTuneTable* t) : prev(gemm_get_tuning()) { gemm_set_tuning(t); }
    ~TuneScope() { gemm_set_tuning(prev); }
  } scope(h->tuning.keys.empty() ? nullptr : &h->tuning);
  try {
    int dev = 0;
    PS_HIP(hipGetDevice(&dev));
    if (dev != h->device) PS_HIP(hipSetDevice(h->device));
    return f();
  } catch (const HipError&) {
    return PS_HIP_ERROR;
  } catch (...) {
    return PS_HIP_ERROR;
  }
}

// Batched division of independent problems of uneven sizes.  The problems are dealt,
// largest first, to kWorkers host threads; each drives its own handle (stream,
// workspace, pinned staging) through the single-problem pipeline, so that the
// latency-bound small factorizations of different problems overlap on the device.
// Measured on 256 problems of m = 32..512: 3 workers 146 ms, 4: 143, 6: 136, 8: 136
// (the process has 4 hardware queues; more streams than queues still fill gaps).
constexpr int kWorkers = 6;

// ---- One batched pipeline for a class of problems with the same padded size (core
// basis, FP64 arithmetic, no restarts): every launch of the single-problem path covers
// the whole class, with the per-problem scalars (bounds, Zolotarev coefficients, shifts,
// series coefficients) in small device arrays.  Problems the class cannot finish (a
// failed factorization, a step needing a restart or the Cholesky form of step 2) are
// returned in `redo` for the single-problem path.  The arithmetic per problem is that
// of the single path; sums split differently (no split-K), so results agree with it to
// rounding, not bit for bit.
struct ClassBufs {
  int nb = 0, mp = 0, r = 0;
  long long S = 0;
  double *mk, *wmk, *y, *yt, *x0, *x1, *x2, *g, *z, *w, *nmat, *t1, *t2, *s12, *p11, *wc, *top,
      *qbot, *hp, *vv, *uu, *pp, *hist, *norms, *scal;
  int *dinfo, *mdev;
  double* gkpart;    // partial norms of the bidiagonalization vectors (3 generations)
};

constexpr int kClassScal = 64;   // per-problem scalar slots (see run_class)

void carve_class(Arena& a, ClassBufs& c, int nb, int mp, int r) {
  c.nb = nb;
  c.mp = mp;
  c.r = r;
  c.S = (long long)mp * mp;
  const size_t S = (size_t)c.S, n = (size_t)nb;
  c.mk = a.take<double>(2 * n * S);
  c.wmk = a.take<double>(2 * n * S);
  c.y = a.take<double>(2 * n * S);
  c.yt = a.take<double>(2 * n * S);
  c.x0 = a.take<double>(n * S);
  c.x1 = a.take<double>(n * S);
  c.x2 = a.take<double>(n * S);
  c.g = a.take<double>(n * S);
  c.z = a.take<double>((size_t)r * n * S);
  c.w = a.take<double>((size_t)r * n * S);
  c.nmat = a.take<double>(n * S);
  c.t1 = a.take<double>(n * S);
  c.t2 = a.take<double>(n * S);
  c.s12 = a.take<double>(n * S);
  c.p11 = a.take<double>(n * S);
  c.wc = a.take<double>(n * S);
  c.top = a.take<double>(n * S);
  c.qbot = a.take<double>(n * S);
  c.hp = a.take<double>(n * S);
  c.vv = a.take<double>(2 * n * mp);
  c.uu = a.take<double>(2 * n * mp);
  c.pp = a.take<double>(2 * n * mp);
  c.hist = a.take<double>(2 * n * 256);
  c.gkpart = a.take<double>(3 * 2 * (size_t)n * gk_parts(mp));
  c.norms = a.take<double>(2 * n);
  c.scal = a.take<double>(n * kClassScal);
  c.dinfo = a.take<int>(16);
  c.mdev = a.take<int>(n);
}

size_t class_bytes(int nb, int mp, int r) {
  Arena a;
  ClassBufs c;
  carve_class(a, c, nb, mp, r);
  return a.off + kAlign;
}

// At most this many problems per class, and at most the worker's share of the
// workspace for one (about (37 + 2r) mp^2 doubles per problem).  Measured on 256
// problems of m = 32..512 (about 32 per padded size): classes of 8, 16, 32, 64: 41, 36,
// 33, 32 ms.  kClassBytes is the share per worker that ps_workspace_size_batched asks
// for (classes of 19 at padded size 512, 32 from 384 down).
constexpr int kClassMax = 32;
constexpr size_t kClassBytes = (size_t)2 << 30;

int class_limit(int mp, int r, size_t region) {
  int nb = 1;
  while (nb < kClassMax && class_bytes(nb + 1, mp, r) <= region) ++nb;
  return class_bytes(nb, mp, r) <= region ? nb : 0;
}

// Jobs of a batched call, largest problems first: in FP64 arithmetic (mixed requests
// below the mixed threshold run in FP64 anyway) problems of one padded size form
// classes of up to kClassMax that fit `region` bytes and run as one batched pipeline;
// everything else, and what a class hands back, runs one problem at a time.
std::vector<std::vector<int>> plan_batch(int batch, const int* m, const ps_opts& o,
                                         size_t region) {
  // (timing: a class reports its kernel classes, not phases; see run_class)
  const bool classes = o.max_steps != 1 &&
                       (o.precision == PS_PREC_FP64 || o.precision == PS_PREC_MIXED);
  std::vector<std::vector<int>> jobs;
  std::vector<int> order(batch);
  for (int i = 0; i < batch; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return m[x] > m[y]; });
  size_t i = 0;
  while (i < order.size()) {
    const int mp = pad_to(m[order[i]]);
    size_t j = i;
    while (j < order.size() && pad_to(m[order[j]]) == mp) ++j;
    const int lim = classes ? class_limit(mp, resolve_r(o), region) : 0;
    const bool cls = classes && j - i >= 2 && lim >= 2 &&
                     (o.precision == PS_PREC_FP64 || mp < kMixedMin);
    if (cls) {
      for (size_t a = i; a < j; a += lim)
        jobs.emplace_back(order.begin() + a, order.begin() + std::min(j, a + (size_t)lim));
    } else {
      for (size_t a = i; a < j; ++a) jobs.push_back({order[a]});
    }
    i = j;
  }
  return jobs;
}

size_t max_single_bytes(int batch, const int* m, const ps_opts& o) {
  size_t need = 0;
  for (int i = 0; i < batch; ++i) need = std::max(need, workspace_bytes(m[i], o, 1));
  return need;
}

// Workspace of a batched call with `nw` workers: nw regions, each holding the largest
// single problem and the largest class planned within kClassBytes.
size_t batched_bytes(int batch, const int* m, const ps_opts& o, int nw) {
  size_t region = max_single_bytes(batch, m, o);
  for (const auto& job : plan_batch(batch, m, o, std::max(region, kClassBytes)))
    if (job.size() > 1)
      region = std::max(region, class_bytes((int)job.size(), pad_to(m[job[0]]), resolve_r(o)));
  region = (region + kAlign - 1) / kAlign * kAlign;
  return (size_t)nw * region;
}

int run_class(ps_handle h, const std::vector<int>& idx, const int* m, const double* const* A,
              const int* lda, const double* const* B, const int* ldb, double* const* Qp,
              const int* ldq, double* const* Hp, const int* ldh, const ps_opts& o,
              ps_info* infos, std::vector<int>& redo) {
  hipStream_t s = h->stream;
  const int nb = (int)idx.size();
  const int mp = pad_to(m[idx[0]]);
  const int rmax = resolve_r(o);
  char* base = workspace_base(h, class_bytes(nb, mp, rmax));
  if (!base) return PS_NO_WORKSPACE;
  Arena ar;
  ar.base = base;
  ar.dry = false;
  ClassBufs c;
  carve_class(ar, c, nb, mp, rmax);
  const long long S = c.S;
  double* pin = h->pinned;
  // timing == 2: this class's launches, reported in the record of its first problem
  // that completes (the class then runs without graphs, whose replays record nothing)
  const ClassTiming ktime(h, o.timing >= 2);
  auto fail_all = [&] {
    for (int p : idx) redo.push_back(p);
    return PS_OK;
  };
  // ---- setup (a0): M_b, K_b packed as matrices 2b, 2b + 1; one batched factorization
  fill_int_zero(s, c.dinfo, 16);
  int* ipin = (int*)pin;
  for (int b = 0; b < nb; ++b) {
    const int p = idx[b];
    pack_casida(s, m[p], mp, A[p], lda[p], B[p], ldb[p], c.mk + 2 * b * S);
    ipin[b] = m[p];
  }
  PS_HIP(hipMemcpyAsync(c.mdev, ipin, nb * sizeof(int), hipMemcpyHostToDevice, s));
  potrf_inv_f64(s, c.mk, S, c.wmk, S, nullptr, mp, 2 * nb, c.dinfo + 0);
  {
    GemmProblem pg[2];
    pg[0] = gemm_problem(mp, mp, mp, c.mk, mp, 0, c.mk + S, mp, 1, c.y, mp, 1.0, 0.0, nullptr, 0,
                         kAUpper | kBLower);
    pg[1] = gemm_problem(mp, mp, mp, c.wmk + S, mp, 1, c.wmk, mp, 0, c.y + S, mp, 1.0, 0.0, nullptr,
                         0, kALower | kBUpper);
    for (auto& q : pg) {
      q.nb1 = nb;
      q.sA[0] = q.sB[0] = q.sC[0] = q.sD[0] = 2 * S;
    }
    gemm_f64(s, pg, 2);
  }
  for (int b = 0; b < nb; ++b) mask_pad(s, c.y + 2 * b * S, m[idx[b]], mp, S, 2);
  // ---- bounds (a1): Golub-Kahan on all 2 nb matrices at once
  const int steps = std::max(4, std::min(o.lanczos_steps, 120));
  transpose(s, c.y, c.yt, mp, S, 2 * nb);
  gk_init_b(s, c.vv, c.mdev, mp, 2 * nb, 2);
  const size_t np2 = 2 * (size_t)nb * gk_parts(mp);
  auto part = [&](int h) { return c.gkpart + (size_t)((h + 3) % 3) * np2; };
  gk_seed(s, part(-1), mp, 2 * nb);
  for (int k = 0; k < steps; ++k) {
    gk_step(s, c.yt, S, c.vv, mp, part(2 * k - 1), c.uu, mp, k > 0 ? c.uu : nullptr, mp,
            part(2 * k - 2), part(2 * k), c.hist, 2 * k - 1, 256, mp, 2 * nb);
    gk_step(s, c.y, S, c.uu, mp, part(2 * k), c.vv, mp, c.vv, mp, part(2 * k - 1),
            part(2 * k + 1), c.hist, 2 * k, 256, mp, 2 * nb);
  }
  gk_finish(s, part(2 * steps - 1), mp, c.hist, 2 * steps - 1, 256, 2 * nb);
  const size_t hist_n = (size_t)2 * nb * 256;
  if (hist_n + 16 > (size_t)kPinned) return fail_all();
  PS_HIP(hipMemcpyAsync(pin, c.hist, hist_n * sizeof(double), hipMemcpyDeviceToHost, s));
  PS_HIP(hipMemcpyAsync(pin + hist_n, c.dinfo, 16 * sizeof(int), hipMemcpyDeviceToHost, s));
  PS_HIP(hipStreamSynchronize(s));
  if (((int*)(pin + hist_n))[0] != 0) return fail_all();   // not definite somewhere
  std::vector<double> alpha(nb), beta(nb), ell(nb);
  int r = (o.r <= 0) ? 1 : rmax;
  for (int b = 0; b < nb; ++b) {
    double smax[2];
    for (int q = 0; q < 2; ++q) {
      double d[128], e[128], smn;
      for (int k = 0; k < steps; ++k) {
        d[k] = pin[(2 * b + q) * 256 + 2 * k];
        e[k] = pin[(2 * b + q) * 256 + 2 * k + 1];
      }
      bidiag_extreme_sv(d, e, steps, &smax[q], &smn);
    }
    alpha[b] = o.alpha > 0.0 ? o.alpha : 1.01 * smax[0];
    beta[b] = o.beta > 0.0 ? o.beta : 0.99 / smax[1];
    if (!(alpha[b] > 0.0) || !(beta[b] > 0.0) || !std::isfinite(alpha[b]) ||
        !std::isfinite(beta[b]))
      return fail_all();
    ell[b] = std::min(beta[b] / alpha[b], 1.0 - 1e-15);
    if (o.r <= 0) r = std::max(r, auto_r(ell[b]));
  }
  // ---- coefficients per problem (a2) and their device arrays
  //   scal[0 .. nb)          1/alpha_b               scal[nb .. 2nb)   hat C of step 1
  //   scal[2nb .. 2nb+nb r)  a_j of step 1 (b-major)  then c_{2j-1} of step 1 (b-major)
  //   then hat C of step 2 (nb), then the Horner coefficients of step 2 (p-major, nb each)
  std::vector<ZoloHost> c1(nb), c2(nb);
  std::vector<double> gam((size_t)nb * kMaxSeries);
  int P = 0;
  for (int b = 0; b < nb; ++b) {
    if (zolotarev_host(ell[b], r, &c1[b])) return fail_all();
    const double ell1 = std::min(c1[b].ell_next, 1.0 - 1e-15);
    if (zolotarev_host(ell1, r, &c2[b])) return fail_all();
    const int Pb = o.step2_series ? series_terms(c2[b], ell1, &gam[(size_t)b * kMaxSeries]) : 0;
    if (Pb == 0) return fail_all();
    P = std::max(P, Pb);
  }
  double* hs = pin;   // staging for the upload (the downloads above are complete)
  const int o_inva = 0, o_chat1 = nb, o_a1 = 2 * nb, o_c1 = 2 * nb + nb * r,
            o_chat2 = 2 * nb + 2 * nb * r, o_h = o_chat2 + nb;
  const int n_scal = o_h + nb * (kMaxSeries + 3);
  if (n_scal > nb * kClassScal) return fail_all();
  for (int b = 0; b < nb; ++b) {
    hs[o_inva + b] = 1.0 / alpha[b];
    hs[o_chat1 + b] = c1[b].chat;
    for (int j = 0; j < r; ++j) {
      hs[o_a1 + b * r + j] = c1[b].a[j];
      hs[o_c1 + b * r + j] = c1[b].c[2 * j];
    }
    hs[o_chat2 + b] = c2[b].chat;
    const double* gb = &gam[(size_t)b * kMaxSeries];
    // Horner stages: T = gam_{P-1} Delta + gam'_{P-2} I, then T <- Delta T + gam'_q I,
    // gam'_0 = 1 + gam_0 (slot p holds gam'_p; slots kMaxSeries.. hold 1, -1 and 0)
    for (int p = 0; p < kMaxSeries; ++p) hs[o_h + p * nb + b] = p == 0 ? 1.0 + gb[0] : gb[p];
    hs[o_h + kMaxSeries * nb + b] = 1.0;
    hs[o_h + (kMaxSeries + 1) * nb + b] = -1.0;
    hs[o_h + (kMaxSeries + 2) * nb + b] = 0.0;
  }
  PS_HIP(hipMemcpyAsync(c.scal, hs, n_scal * sizeof(double), hipMemcpyHostToDevice, s));
  const double* d_inva = c.scal + o_inva;
  const double* d_chat1 = c.scal + o_chat1;
  const double* d_a1 = c.scal + o_a1;
  const double* d_c1 = c.scal + o_c1;
  const double* d_chat2 = c.scal + o_chat2;
  auto d_h = [&](int p) { return c.scal + o_h + (size_t)p * nb; };
  const double* d_one = d_h(kMaxSeries);
  const double* d_mone = d_h(kMaxSeries + 1);
  const double* d_zero = d_h(kMaxSeries + 2);
  auto batched = [&](GemmProblem q, long long sa, long long sb, long long sd) {
    q.nb1 = nb;
    q.sA[0] = sa;
    q.sB[0] = sb;
    q.sC[0] = sd;
    q.sD[0] = sd;
    return q;
  };
  // ---- steps 1 and 2, the stopping-test norms, bases and decoupling: launches only (the
  // coefficients are device arrays), captured once per class key as a graph and replayed
  auto body = [&]() {
    // ---- step 1 (a3): X1 = hat C X0 (I + sum_j a_j (X0^T X0 + c_j I)^{-1})
    scale_b(s, c.y, 2 * S, c.x0, S, d_inva, (size_t)S, nb);
    {
      GemmProblem pg = batched(gemm_problem(mp, mp, mp, c.x0, mp, 1, c.x0, mp, 0, c.g, mp, 1.0, 0.0,
                                            nullptr, 0, kOutUpper), S, S, S);
      gemm_f64(s, pg);
      form_shifts_b(s, c.g, c.z, mp, d_c1, r, nb);
      potrf_inv_f64(s, c.z, S, c.w, S, nullptr, mp, r * nb, c.dinfo + 1);
      GemmProblem pn = batched(gemm_problem(mp, mp, r * mp, c.w, mp, 0, c.w, mp, 1, c.nmat, mp, 1.0,
                                            0.0, nullptr, 0,
                                            kAUpper | kBLower | kOutUpper | kMirror),
                               r * S, r * S, S);
      pn.kseg = mp;
      pn.nseg = r;
      pn.kscale_b = d_a1;
      gemm_f64(s, pn);
      GemmProblem px = batched(gemm_problem(mp, mp, mp, c.x0, mp, 0, c.nmat, mp, 0, c.x1, mp, 1.0,
                                            1.0, c.x0, mp, 0),
                               S, S, S);
      px.alpha_b = d_chat1;
      px.beta_b = d_chat1;
      gemm_f64(s, px);
    }
    // ---- step 2 (a3) by the series: X2 = hat C X1 T(Delta), Delta = X1^T X1 - I
    {
      GemmProblem pg = batched(gemm_problem(mp, mp, mp, c.x1, mp, 1, c.x1, mp, 0, c.g, mp, 1.0, 0.0,
                                            nullptr, 0, kOutUpper | kMirror), S, S, S);
      gemm_f64(s, pg);
      axpb_identity_b(s, c.g, c.g, d_one, d_mone, mp, nb);   // Delta
      double* T = c.nmat;
      double* T2 = c.t1;
      if (P == 1) {
        axpb_identity_b(s, c.g, T, d_zero, d_h(0), mp, nb);   // T = (1 + gam_0) I
      } else {
        axpb_identity_b(s, c.g, T, d_h(P - 1), d_h(P - 2), mp, nb);
        for (int q = P - 3; q >= 0; --q) {
          GemmProblem ph = batched(gemm_problem(mp, mp, mp, c.g, mp, 0, T, mp, 0, T2, mp, 1.0, 0.0,
                                                nullptr, 0, kOutUpper | kMirror),
                                   S, S, S);   // symmetric (Delta and T commute)
          gemm_f64(s, ph);
          axpb_identity_b(s, T2, T, d_one, d_h(q), mp, nb);
        }
      }
      GemmProblem px = batched(gemm_problem(mp, mp, mp, c.x1, mp, 0, T, mp, 0, c.x2, mp), S, S, S);
      px.alpha_b = d_chat2;
      gemm_f64(s, px);
    }
    // ---- stopping test (a4) per problem: the norms now, the decision after the bases
    diff_norms_b(s, c.x1, c.x2, (size_t)S, c.norms, nb);
    const double* U = c.x2;
    if (o.basis == PS_BASIS_CORE) {
      // ---- core basis (a7, a8): Q_+ = Z R_G^{-1}, H_+ = 2 R_G^{-T} R_G^{-1}
      GemmProblem pt = batched(gemm_problem(mp, mp, mp, c.wmk, mp, 0, U, mp, 0, c.t1, mp, 1.0, 0.0,
                                            nullptr, 0, kAUpper), 2 * S, S, S);
      gemm_f64(s, pt);
      GemmProblem pv = batched(gemm_problem(mp, mp, mp, c.wmk + S, mp, 1, c.t1, mp, 0, c.t2, mp, 1.0,
                                            0.0, nullptr, 0, kALower), 2 * S, S, S);
      gemm_f64(s, pv);
      for (int b = 0; b < nb; ++b)
        sym_scale_upper(s, c.t2 + b * S, c.p11 + b * S, m[idx[b]], mp, 1.0);
      potrf_inv_f64(s, c.p11, S, c.wc, S, nullptr, mp, nb, c.dinfo + 4);
      GemmProblem pe[2];
      pe[0] = batched(gemm_problem(mp, mp, mp, c.t1, mp, 0, c.wc, mp, 0, c.t2, mp, 1.0, 0.0, nullptr,
                                   0, kBUpper), S, S, S);
      pe[1] = batched(gemm_problem(mp, mp, mp, c.wmk + S, mp, 0, c.wc, mp, 0, c.s12, mp, 1.0, 0.0,
                                   nullptr, 0, kAUpper | kBUpper), 2 * S, S, S);
      gemm_f64(s, pe, 2);
      for (int b = 0; b < nb; ++b)   // (sum_diff_scaled takes the matrix edge, not a length)
        sum_diff_scaled(s, c.t2 + b * S, c.s12 + b * S, c.top + b * S, c.qbot + b * S, M_SQRT1_2,
                        mp);
      GemmProblem ph = batched(gemm_problem(mp, mp, mp, c.wc, mp, 1, c.wc, mp, 0, c.hp, mp, 2.0, 0.0,
                                            nullptr, 0, kALower | kBUpper | kOutUpper | kMirror),
                               S, S, S);
      gemm_f64(s, ph);
    } else {
      // ---- blocks of sign(H) (a6): S12 = W_M U R_K, S21 = R_M^T U W_K^T (S21 in p11 until
      // the sign blocks are formed; A_s, B_s in the first matrices of z and w, free since
      // step 1)
      double* as = c.z;
      double* bs = c.w;
      GemmProblem pg[2];
      pg[0] = batched(gemm_problem(mp, mp, mp, U, mp, 0, c.mk + S, mp, 0, c.t1, mp, 1.0, 0.0,
                                   nullptr, 0, kBUpper), S, 2 * S, S);
      pg[1] = batched(gemm_problem(mp, mp, mp, U, mp, 0, c.wmk + S, mp, 1, c.t2, mp, 1.0, 0.0,
                                   nullptr, 0, kBLower), S, 2 * S, S);
      gemm_f64(s, pg, 2);
      pg[0] = batched(gemm_problem(mp, mp, mp, c.wmk, mp, 0, c.t1, mp, 0, c.s12, mp, 1.0, 0.0,
                                   nullptr, 0, kAUpper), 2 * S, S, S);
      pg[1] = batched(gemm_problem(mp, mp, mp, c.mk, mp, 1, c.t2, mp, 0, c.p11, mp, 1.0, 0.0,
                                   nullptr, 0, kALower), 2 * S, S, S);
      gemm_f64(s, pg, 2);
      sign_blocks_b(s, c.s12, c.p11, as, bs, mp, nb);
      // ---- Alg. 6 (a7): C = chol((I + A_s)/2), Q_+ = [C^T; P_{+,21} C^{-1}], P_{+,21} = -B_s/2
      half_shift_upper_b(s, as, c.p11, mp, nb);
      potrf_inv_f64(s, c.p11, S, c.wc, S, nullptr, mp, nb, c.dinfo + 4);
      GemmProblem pq = batched(gemm_problem(mp, mp, mp, bs, mp, 0, c.wc, mp, 0, c.qbot, mp, -0.5, 0.0,
                                            nullptr, 0, kBUpper), S, S, S);
      gemm_f64(s, pq);
      mask_pad_b(s, c.qbot, c.mdev, mp, 1, nb);
      double* ab = c.yt;   // [a_b, b_b] per problem (stride 2 S), free since the estimator
      basis_mix_b(s, c.p11, c.qbot, c.top, ab, mp, nb);
      mask_pad_b(s, ab, c.mdev, mp, 2, 2 * nb);
      // ---- decoupling (a8): H_+ = F^T F, F = [R_M a; R_K b] (2 mp x mp, ld 2 mp; in y)
      double* F = c.y;
      GemmProblem pf = gemm_problem(mp, mp, mp, c.mk, mp, 0, ab, mp, 0, F, 2 * mp, 1.0, 0.0, nullptr,
                                    0, kAUpper);
      pf.nb1 = 2;
      pf.sA[0] = pf.sB[0] = S;
      pf.sC[0] = pf.sD[0] = mp;
      pf.nb2 = nb;
      pf.sA[1] = pf.sB[1] = pf.sC[1] = pf.sD[1] = 2 * S;
      gemm_f64(s, pf);
      GemmProblem ph = batched(gemm_problem(mp, mp, 2 * mp, F, 2 * mp, 1, F, 2 * mp, 0, c.hp, mp,
                                            1.0, 0.0, nullptr, 0, kOutUpper | kMirror),
                               2 * S, 2 * S, S);
      gemm_f64(s, ph);
    }
  };
  if (h->use_graphs && s != nullptr && !ktime.on) {   // the legacy default stream cannot be captured
    std::vector<long long> key = {(long long)(uintptr_t)base, nb, mp, r, P, o.basis};
    for (int b = 0; b < nb; ++b) key.push_back(m[idx[b]]);
    hipGraphExec_t exec = nullptr;
    for (auto& g : h->graphs)
      if (g.key == key) exec = g.exec;
    if (!exec) {
      hipGraph_t graph = nullptr;
      PS_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      try {
        body();
      } catch (...) {
        (void)hipStreamEndCapture(s, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        throw;
      }
      PS_HIP(hipStreamEndCapture(s, &graph));
      const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      PS_HIP(e);
      if ((int)h->graphs.size() >= kGraphCache) {
        (void)hipGraphExecDestroy(h->graphs.front().exec);
        h->graphs.erase(h->graphs.begin());
      }
      h->graphs.push_back({key, exec});
    }
    PS_HIP(hipGraphLaunch(exec, s));
  } else {
    body();
  }
  PS_HIP(hipMemcpyAsync(pin, c.norms, 2 * nb * sizeof(double), hipMemcpyDeviceToHost, s));
  PS_HIP(hipMemcpyAsync(pin + 2 * nb, c.dinfo, 16 * sizeof(int), hipMemcpyDeviceToHost, s));
  PS_HIP(hipStreamSynchronize(s));
  if (((int*)(pin + 2 * nb))[1] != 0 || ((int*)(pin + 2 * nb))[4] != 0) return fail_all();
  const double tol = std::pow(std::ldexp(1.0, -53), 1.0 / (2 * r + 1));
  std::vector<char> ok(nb, 1);
  std::vector<double> change(nb);
  for (int b = 0; b < nb; ++b) {
    change[b] = std::sqrt(pin[2 * b]) / std::sqrt(pin[2 * b + 1]);
    if (!(change[b] <= tol)) ok[b] = 0;
  }
  for (int b = 0; b < nb; ++b) {
    const int p = idx[b];
    if (!ok[b]) {
      redo.push_back(p);
      continue;
    }
    const int mm = m[p];
    copy_out(s, c.top + b * S, mp, Qp[p], ldq[p], mm, mm);
    copy_out(s, c.qbot + b * S, mp, Qp[p] + mm, ldq[p], mm, mm);
    copy_out(s, c.hp + b * S, mp, Hp[p], ldh[p], mm, mm);
    if (infos) {
      ps_info& inf = infos[p];
      inf = ps_info{};
      inf.status = PS_OK;
      inf.failed_step = -1;
      inf.steps = 2;
      inf.r = r;
      inf.alpha = alpha[b];
      inf.beta = beta[b];
      inf.ell[0] = ell[b];
      inf.ell[1] = std::min(c1[b].ell_next, 1.0 - 1e-15);
      inf.step_change = change[b];
      inf.step2_terms = P;
      inf.shifts_fp64[0] = r;    // classes run every shift of step 1 in FP64
      inf.shifts_fp64[1] = 0;    // step 2 by the series
    }
  }
  PS_HIP(hipStreamSynchronize(s));
  if (ktime.on && infos)
    for (int b = 0; b < nb; ++b)
      if (ok[b]) {
        ktime.collect(infos[idx[b]]);
        break;
      }
  return PS_OK;
}

int run_batched(ps_handle h, int batch, const int* m, const double* const* A, const int* lda,
                const double* const* B, const int* ldb, double* const* Qp, const int* ldq,
                double* const* Hp, const int* ldh, const ps_opts& o, ps_info* infos) {
  // Workers: one per caller worker stream (up to kWorkers), each with an equal share of
  // the caller's workspace that holds the largest single problem (fewer workers if the
  // shares would not); without worker streams the handle itself is the one worker.
  if (!h->user_ws) return PS_NO_WORKSPACE;
  const int nwk = ensure_workers(h, std::min(kWorkers, batch));
  if (nwk < 0) return PS_HIP_ERROR;
  int nw = std::max(1, nwk);
  const size_t single = max_single_bytes(batch, m, o);
  auto share = [&](int n) { return h->user_bytes / (size_t)n / kAlign * kAlign; };
  while (nw > 1 && share(nw) < single) --nw;
  const size_t region = share(nw);
  if (region < single) return PS_NO_WORKSPACE;
  std::vector<ps_handle> wk;
  if (nwk == 0) {
    wk.push_back(h);
  } else {
    for (int k = 0; k < nw; ++k) {
      ps_handle w = h->workers[k];
      w->user_ws = (char*)h->user_ws + (size_t)k * region;
      w->user_bytes = region;
      wk.push_back(w);
    }
    // the inputs may still be in flight on the caller's stream
    PS_HIP(hipEventRecord(h->fork, h->stream));
    for (int k = 0; k < nw; ++k) PS_HIP(hipStreamWaitEvent(wk[k]->stream, h->fork, 0));
  }
  const std::vector<std::vector<int>> jobs = plan_batch(batch, m, o, region);
  std::vector<int> status(batch, PS_OK);
  std::atomic<int> next{0};
  const int njobs = (int)jobs.size();
  auto work = [&](int k) {
    ps_handle w = wk[k];
    if (hipSetDevice(h->device) != hipSuccess) {
      for (int i; (i = next.fetch_add(1)) < njobs;)
        for (int p : jobs[i]) status[p] = PS_HIP_ERROR;
      return;
    }
    auto single = [&](int p) {
      ps_info local{};
      ps_info* inf = infos ? &infos[p] : &local;
      status[p] = guarded(w, [&] {
        return run(w, m[p], A[p], lda[p], B[p], ldb[p], Qp[p], ldq[p], Hp[p], ldh[p], o, inf, 1);
      });
    };
    for (int i; (i = next.fetch_add(1)) < njobs;) {
      const std::vector<int>& job = jobs[i];
      if (job.size() == 1) {
        single(job[0]);
        continue;
      }
      std::vector<int> redo;
      const int st = guarded(w, [&] {
        return run_class(w, job, m, A, lda, B, ldb, Qp, ldq, Hp, ldh, o, infos, redo);
      });
      if (st != PS_OK) {
        redo = job;   // the class could not run at all (workspace, device error)
        if (st == PS_HIP_ERROR) {
          for (int p : job) status[p] = st;
          continue;
        }
      }
      for (int p : redo) single(p);
    }
  };
  std::vector<std::thread> threads;
  for (int k = 1; k < nw; ++k) threads.emplace_back(work, k);
  work(0);
  for (auto& t : threads) t.join();
  for (int p = 0; p < batch; ++p)
    if (status[p] != PS_OK) return status[p];
  return PS_OK;
}


}  // namespace
}  // namespace ps

using namespace ps;

extern "C" {

void ps_opts_default(ps_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = PS_PREC_FP64;
  o->r = 8;
  o->max_restarts = 2;
  o->max_steps = 0;
  o->lanczos_steps = 20;
  o->timing = 0;
  o->alpha = 0.0;
  o->beta = 0.0;
  o->mixed_kappa = 20.0;
  o->step2_series = 1;
  o->basis = PS_BASIS_ALG6;
  o->iteration = PS_ITER_ZOLO;
  o->refine = PS_REFINE_RR;
}

int ps_create(ps_handle* h, void* stream) {
  if (!h) return -1;
  ps_handle_s* p = new ps_handle_s();
  p->stream = (hipStream_t)stream;
  // the device address of the static scratch area of this device, looked up once per
  // device at set-up (pseudosym_divide_static)
  if (hipGetDevice(&p->device) != hipSuccess || !static_scratch_ptr() ||
      hipHostMalloc((void**)&p->pinned, kPinned * sizeof(double), hipHostMallocDefault) !=
          hipSuccess) {
    delete p;
    return PS_HIP_ERROR;
  }
  for (auto& e : p->ev)
    if (hipEventCreate(&e) != hipSuccess) {
      delete p;
      return PS_HIP_ERROR;
    }
  p->events = true;
  if (hipEventCreateWithFlags(&p->fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&p->join, hipEventDisableTiming) != hipSuccess) {
    delete p;
    return PS_HIP_ERROR;
  }
  *h = p;
  return PS_OK;
}

int ps_destroy(ps_handle h) {
  if (!h) return -1;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  else (void)hipDeviceSynchronize();
  if (h->pinned) (void)hipHostFree(h->pinned);
  if (h->events)
    for (auto& e : h->ev) (void)hipEventDestroy(e);
  for (auto& e : h->kev) (void)hipEventDestroy(e);
  if (h->side) (void)hipStreamSynchronize(h->side);   // borrowed: the caller's stream
  if (h->fork) (void)hipEventDestroy(h->fork);
  if (h->join) (void)hipEventDestroy(h->join);
  for (auto& g : h->graphs) (void)hipGraphExecDestroy(g.exec);
  for (ps_handle w : h->workers) (void)ps_destroy(w);   // their streams are the caller's
  delete h;
  return PS_OK;
}

int ps_set_graphs(ps_handle h, int enable) {
  if (!h) return -1;
  if (enable != 0 && enable != 1) return -2;
  h->use_graphs = enable != 0;
  for (ps_handle w : h->workers) w->use_graphs = h->use_graphs;
  return PS_OK;
}

int ps_set_gemm_tuning(ps_handle h, const ps_gemm_tune* entries, int n) {
  if (!h) return -1;
  if (n < 0 || (n > 0 && !entries)) return -2;
  ps::GemmTuneTable t;
  for (int i = 0; i < n; ++i) {
    const ps_gemm_tune& e = entries[i];
    if ((e.tile != 64 && e.tile != 128) || e.ksplit < 1 || e.ksplit > ps::kMaxSplit ||
        (e.streamk != 0 && e.streamk != 1))
      return -2;
    t.keys.push_back(e.key);
    t.choices.push_back({e.tile, e.ksplit, e.streamk});
  }
  h->tuning = t;
  for (ps_handle w : h->workers) w->tuning = t;
  // captured launches follow the table in force when they were captured
  for (auto& g : h->graphs) (void)hipGraphExecDestroy(g.exec);
  h->graphs.clear();
  for (ps_handle w : h->workers) {
    for (auto& g : w->graphs) (void)hipGraphExecDestroy(g.exec);
    w->graphs.clear();
  }
  return PS_OK;
}

int ps_set_stream(ps_handle h, void* stream) {
  if (!h) return -1;
  h->stream = (hipStream_t)stream;
  return PS_OK;
}

size_t ps_workspace_size(int m, const ps_opts* o, int what) {
  ps_opts d;
  ps_opts_default(&d);
  if (m < 1) return 0;
  if (what == 4) return general_bytes(m, o ? *o : d);
  if (what == 5) return hermitian_bytes(m, o ? *o : d);
  if (what == 6) return tune_bytes(m, o ? *o : d);
  if (what == 7) return sign_bwd_iter_bytes(m, resolve_r(o ? *o : d));
  if (what >= 3) return adjoint_bytes(m);
  return workspace_bytes(m, o ? *o : d, what < 0 ? 0 : what);
}

int ps_set_workspace(ps_handle h, void* dptr, size_t bytes) {
  if (!h) return -1;
  if (dptr && ((uintptr_t)dptr % kAlign)) return -2;
  h->user_ws = dptr;
  h->user_bytes = dptr ? bytes : 0;
  return PS_OK;
}

size_t ps_workspace_size_batched(int batch, const int* m, const ps_opts* o) {
  if (batch < 1 || !m) return 0;
  for (int i = 0; i < batch; ++i)
    if (m[i] < 1) return 0;
  ps_opts d;
  ps_opts_default(&d);
  if (o) d = *o;
  d.max_steps = 0;
  d.timing = 0;
  return batched_bytes(batch, m, d, std::min(kWorkers, batch)) + kAlign;
}

int ps_set_worker_streams(ps_handle h, int count, void* const* streams) {
  if (!h) return -1;
  if (count < 0 || count > PS_MAX_WORKER_STREAMS) return -2;
  if (count > 0 && !streams) return -3;
  for (int k = 0; k < count; ++k)
    if (!streams[k] || streams[k] == (void*)h->stream) return -3;
  try {
    if (h->stream) PS_HIP(hipStreamSynchronize(h->stream));
    for (ps_handle w : h->workers) {
      if (w->stream) PS_HIP(hipStreamSynchronize(w->stream));
      (void)ps_destroy(w);
    }
  } catch (const HipError&) {
    return PS_HIP_ERROR;
  }
  h->workers.clear();
  h->wstreams.assign((hipStream_t*)streams, (hipStream_t*)streams + count);
  h->side = count > 0 ? h->wstreams[0] : nullptr;
  return PS_OK;
}

int ps_zolotarev_coeffs(double ell, int r, double* c, double* a, double* chat, double* ell_next) {
  ZoloHost z;
  if (zolotarev_host(ell, r, &z)) return -1;
  if (c)
    for (int i = 0; i < 2 * r; ++i) c[i] = z.c[i];
  if (a)
    for (int j = 0; j < r; ++j) a[j] = z.a[j];
  if (chat) *chat = z.chat;
  if (ell_next) *ell_next = z.ell_next;
  return 0;
}

int pseudosym_sign(ps_handle h, int m, const double* A, int lda, const double* B, int ldb,
                   double* SA, double* SB, int lds, const ps_opts* opts, ps_info* info) {
  int chk = check_common(h, m, A, lda, B, ldb, opts);
  if (chk) return chk;
  if (!SA) return -7;
  if (!SB) return -8;
  if (lds < m) return -9;
  ps_opts o;
  ps_opts_default(&o);
  if (opts) o = *opts;
  return guarded(h, [&] { return run(h, m, A, lda, B, ldb, SA, lds, SB, lds, o, info, 0); });
}

int pseudosym_divide(ps_handle h, int m, const double* A, int lda, const double* B, int ldb,
                     double* Qp, int ldq, double* Hp, int ldh, const ps_opts* opts,
                     ps_info* info) {
  int chk = check_common(h, m, A, lda, B, ldb, opts);
  if (chk) return chk;
  if (!Qp) return -7;
  if (ldq < 2 * m) return -8;
  if (!Hp) return -9;
  if (ldh < m) return -10;
  ps_opts o;
  ps_opts_default(&o);
  if (opts) o = *opts;
  o.max_steps = 0;
  return guarded(h, [&] { return run(h, m, A, lda, B, ldb, Qp, ldq, Hp, ldh, o, info, 1); });
}

int pseudosym_divide_static(ps_handle h, int m, const double* A, int lda, const double* B,
                            int ldb, double* Qp, int ldq, double* Hp, int ldh,
                            const ps_opts* opts, ps_info* info) {
  int chk = check_common(h, m, A, lda, B, ldb, opts);
  if (chk) return chk;
  if (!Qp) return -7;
  if (ldq < 2 * m) return -8;
  if (!Hp) return -9;
  if (ldh < m) return -10;
  ps_opts o;
  ps_opts_default(&o);
  if (opts) o = *opts;
  o.max_steps = 0;
  o.timing = 0;   // no event pool: nothing is created or allocated during the call
  if (workspace_bytes(m, o, 1) > kStaticScratchBytes) return -2;
  return guarded(h, [&] {
    char* ws = (char*)static_scratch_ptr();   // this device's copy, looked up at set-up
    if (!ws) return (int)PS_HIP_ERROR;
    return run(h, m, A, lda, B, ldb, Qp, ldq, Hp, ldh, o, info, 1, ws);
  });
}

int pseudosym_divide_general(ps_handle h, int n, const double* H, int ldh, const double* sigma,
                             double* S, int lds, double* Qp, int ldqp, double* Qm, int ldqm,
                             double* Hp, int ldhp, double* Hm, int ldhm, const ps_opts* opts,
                             ps_info* info) {
  if (!h) return -1;
  if (n < 1) return -2;
  if (!H) return -3;
  if (ldh < n) return -4;
  if (!sigma) return -5;
  int p = 0;
  for (int i = 0; i < n; ++i) {
    if (sigma[i] != 1.0 && sigma[i] != -1.0) return -5;
    p += sigma[i] > 0 ? 1 : 0;
  }
  const int q = n - p;
  if (S && lds < n) return -7;
  if (p > 0 && !Qp) return -8;
  if (p > 0 && ldqp < n) return -9;
  if (q > 0 && !Qm) return -10;
  if (q > 0 && ldqm < n) return -11;
  if (p > 0 && !Hp) return -12;
  if (p > 0 && ldhp < p) return -13;
  if (q > 0 && !Hm) return -14;
  if (q > 0 && ldhm < q) return -15;
  if (n > kPinned) return -2;
  if (opts && (opts->r < 0 || opts->r > 8 || opts->max_restarts < 0 || opts->max_steps != 0 ||
               (opts->precision != PS_PREC_FP64 && opts->precision != PS_PREC_MIXED) ||
               ((opts->basis == PS_BASIS_LDL || opts->basis == PS_BASIS_CONGRUENT) &&
                pad_to(n) > kLdlMaxN)))
    return -16;
  ps_opts o;
  ps_opts_default(&o);
  if (opts) o = *opts;
  return guarded(h, [&] {
    return run_general(h, n, H, ldh, sigma, S, lds, Qp, ldqp, Qm, ldqm, Hp, ldhp, Hm, ldhm, o,
                       info);
  });
}

// Argument checks of the complex entry points (leading dimensions in complex entries)
int check_complex(ps_handle h, int m, const double* A, int lda, const double* B, int ldb,
                  const double* O1, int ld1, const double* O2, int ld2, int ld1_min,
                  const ps_opts* o, bool divide) {
  if (!h) return -1;
  if (m < 1) return -2;
  if (!A) return -3;
  if (lda < m) return -4;
  if (!B) return -5;
  if (ldb < m) return -6;
  if (!O1) return -7;
  if (ld1 < ld1_min) return -8;
  if (!O2) return -9;
  if (ld2 < m) return -10;
  if (o && (o->r < 0 || o->r > 8 || o->max_restarts < 0 || o->max_steps != 0 ||
            (o->precision != PS_PREC_FP64 && o->precision != PS_PREC_MIXED) ||
            o->iteration != PS_ITER_ZOLO || o->refine < PS_REFINE_NONE ||
            o->refine > PS_REFINE_NS ||
            (divide && o->basis != PS_BASIS_ALG6 && o->basis != PS_BASIS_CORE)))
    return -11;
  return 0;
}

int ps_autotune_divide(ps_handle h, int m, const double* A, int lda, const double* B, int ldb,
                       const ps_opts* opts, ps_gemm_tune* out, int cap, int* count) {
  int chk = check_common(h, m, A, lda, B, ldb, opts);
  if (chk) return chk;
  if (cap < 0 || (cap > 0 && !out)) return -8;
  if (opts && opts->basis == PS_BASIS_LDL) return -7;
  ps_opts o;
  ps_opts_default(&o);
  if (opts) o = *opts;
  o.max_steps = 0;
  o.timing = 0;
  return guarded(h, [&] { return run_autotune(h, m, A, lda, B, ldb, o, out, cap, count); });
}

int pseudosym_sign_hermitian(ps_handle h, int m, const double* A, int lda, const double* B,
                             int ldb, double* SA, double* SB, int lds, const ps_opts* opts,
                             ps_info* info) {
  int chk = check_complex(h, m, A, lda, B, ldb, SA, lds, SB, lds, m, opts, false);
  if (chk) return chk;
  ps_opts o;
  ps_opts_default(&o);
  if (opts) o = *opts;
  return guarded(h, [&] {
    return run_hermitian(h, m, A, lda, B, ldb, SA, lds, SB, lds, o, info, 0, false);
  });
}

int pseudosym_divide_hermitian(ps_handle h, int m, const double* A, int lda, const double* B,
                               int ldb, double* Qp, int ldq, double* Hp, int ldh,
                               const ps_opts* opts, ps_info* info) {
  int chk = check_complex(h, m, A, lda, B, ldb, Qp, ldq, Hp, ldh, 2 * m, opts, true);
  if (chk) return chk;
  ps_opts o;
  ps_opts_default(&o);
  if (opts) o = *opts;
  o.max_steps = 0;
  return guarded(h, [&] {
    return run_hermitian(h, m, A, lda, B, ldb, Qp, ldq, Hp, ldh, o, info, 1, false);
  });
}

int pseudosym_sign_bse(ps_handle h, int m, const double* A, int lda, const double* B, int ldb,
                       double* SA, double* SB, int lds, const ps_opts* opts, ps_info* info) {
  int chk = check_complex(h, m, A, lda, B, ldb, SA, lds, SB, lds, m, opts, false);
  if (chk) return chk;
  ps_opts o;
  ps_opts_default(&o);
  if (opts) o = *opts;
  return guarded(h, [&] {
    return run_hermitian(h, m, A, lda, B, ldb, SA, lds, SB, lds, o, info, 0, true);
  });
}

int pseudosym_eig(ps_handle h, int m, const double* A, int lda, const double* B, int ldb,
                  double* lambda, double* V, int ldv, const ps_opts* opts, ps_info* info) {
  int chk = check_common(h, m, A, lda, B, ldb, opts);
  if (chk) return chk;
  if (opts && opts->basis == PS_BASIS_LDL) return -11;   // the recursion takes Alg. 4 bases
  if (!lambda) return -7;
  if (V && ldv < 2 * m) return -9;
  ps_opts o;
  ps_opts_default(&o);
  if (opts) o = *opts;
  o.max_steps = 0;
  o.timing = 0;
  return guarded(h, [&] { return run_eig(h, m, A, lda, B, ldb, lambda, V, ldv, o, info); });
}

int pseudosym_divide_batched(ps_handle h, int batch, const int* m, const double* const* A,
                             const int* lda, const double* const* B, const int* ldb,
                             double* const* Qp, const int* ldq, double* const* Hp,
                             const int* ldh, const ps_opts* opts, ps_info* infos) {
  if (!h) return -1;
  if (batch < 0) return -2;
  if (batch == 0) return PS_OK;
  if (!m) return -3;
  if (!A) return -4;
  if (!lda) return -5;
  if (!B) return -6;
  if (!ldb) return -7;
  if (!Qp) return -8;
  if (!ldq) return -9;
  if (!Hp) return -10;
  if (!ldh) return -11;
  for (int i = 0; i < batch; ++i) {
    if (m[i] < 1) return -3;
    if (!A[i]) return -4;
    if (lda[i] < m[i]) return -5;
    if (!B[i]) return -6;
    if (ldb[i] < m[i]) return -7;
    if (!Qp[i]) return -8;
    if (ldq[i] < 2 * m[i]) return -9;
    if (!Hp[i]) return -10;
    if (ldh[i] < m[i]) return -11;
  }
  if (opts && (opts->r < 0 || opts->r > 8 || opts->max_restarts < 0 || opts->max_steps < 0 ||
               opts->max_steps > 1 ||
               (opts->precision != PS_PREC_FP64 && opts->precision != PS_PREC_MIXED) ||
               (opts->basis != PS_BASIS_ALG6 && opts->basis != PS_BASIS_CORE)))
    return -12;
  ps_opts o;
  ps_opts_default(&o);
  if (opts) o = *opts;
  o.max_steps = 0;
  o.timing = o.timing >= 2 ? 2 : 0;
  return guarded(h, [&] {
    return run_batched(h, batch, m, A, lda, B, ldb, Qp, ldq, Hp, ldh, o, infos);
  });
}

int pseudosym_sign_fwd(ps_handle h, int m, const double* A, int lda, const double* B, int ldb,
                       double* SA, double* SB, int lds, double* lambda, double* V, int ldv,
                       const ps_opts* opts, ps_info* info) {
  int chk = check_common(h, m, A, lda, B, ldb, opts);
  if (chk) return chk;
  if (!SA) return -7;
  if (!SB) return -8;
  if (lds < m) return -9;
  if (!lambda) return -10;
  if (!V) return -11;
  if (ldv < 2 * m) return -12;
  ps_opts o;
  ps_opts_default(&o);
  if (opts) o = *opts;
  o.max_steps = 0;
  o.timing = 0;
  o.basis = PS_BASIS_ALG6;   // the forward returns the sign blocks of that path
  return guarded(h, [&] {
    return run_eig(h, m, A, lda, B, ldb, lambda, V, ldv, o, info, SA, SB, lds);
  });
}

int pseudosym_sign_full(ps_handle h, int m, const double* SA, const double* SB, int lds,
                        double* S, int lds2) {
  if (!h) return -1;
  if (m < 1) return -2;
  if (!SA) return -3;
  if (!SB) return -4;
  if (lds < m) return -5;
  if (!S) return -6;
  if (lds2 < 2 * m) return -7;
  return guarded(h, [&] {
    sign_full(h->stream, SA, SB, lds, m, S, lds2);
    PS_HIP(hipStreamSynchronize(h->stream));
    return PS_OK;
  });
}

size_t ps_sign_store_size(int m, const ps_opts* opts) {
  ps_opts o;
  ps_opts_default(&o);
  if (opts) o = *opts;
  if (m < 1 || o.max_restarts < 0 || 2 * (1 + o.max_restarts) > kStoreMaxSteps) return 0;
  return store_doubles(pad_to(m), resolve_r(o), 2 * (1 + o.max_restarts)) * sizeof(double);
}

int pseudosym_sign_fwd_iter(ps_handle h, int m, const double* A, int lda, const double* B,
                            int ldb, double* SA, double* SB, int lds, void* store,
                            size_t store_bytes, const ps_opts* opts, ps_info* info) {
  int chk = check_common(h, m, A, lda, B, ldb, opts);
  if (chk) return chk;
  if (!SA) return -7;
  if (!SB) return -8;
  if (lds < m) return -9;
  ps_opts o;
  ps_opts_default(&o);
  if (opts) o = *opts;
  if (!store || ((uintptr_t)store % kAlign) != 0) return -10;
  if (o.max_restarts > kStoreMaxSteps / 2 - 1) return -12;
  if (store_bytes < ps_sign_store_size(m, &o)) return -11;
  if (o.precision != PS_PREC_FP64 || o.iteration != PS_ITER_ZOLO) return -12;
  // the composition the adjoint follows: FP64 Zolotarev steps by factorizations, no
  // Newton-Schulz pass, a fixed r
  o.max_steps = 0;
  o.step2_series = 0;
  if (o.refine > PS_REFINE_RR) o.refine = PS_REFINE_RR;
  o.r = resolve_r(o);
  StepStore keep;
  keep.base = static_cast<double*>(store);
  keep.mp = pad_to(m);
  keep.r = o.r;
  keep.max_steps = 2 * (1 + o.max_restarts);
  return guarded(h, [&] {
    // the header is written last, on success: until then the store reads as empty, so a
    // backward after a failed forward is refused instead of using older factors
    std::memset(h->pinned, 0, kStoreHeader * sizeof(double));
    PS_HIP(hipMemcpyAsync(store, h->pinned, kStoreHeader * sizeof(double), hipMemcpyHostToDevice,
                          h->stream));
    PS_HIP(hipStreamSynchronize(h->stream));
    return run(h, m, A, lda, B, ldb, SA, lds, SB, lds, o, info, 0, nullptr, false, &keep);
  });
}

int pseudosym_sign_bwd_iter(ps_handle h, int m, const void* store, const double* gSA,
                            const double* gSB, int ldg, double* gA, double* gB, int ldo) {
  if (!h) return -1;
  if (m < 1) return -2;
  if (!store || ((uintptr_t)store % kAlign) != 0) return -3;
  if (!gSA) return -4;
  if (!gSB) return -5;
  if (ldg < m) return -6;
  if (!gA) return -7;
  if (!gB) return -8;
  if (ldo < m) return -9;
  return guarded(h, [&] {
    return run_sign_bwd_iter(h, m, static_cast<const double*>(store), gSA, gSB, ldg, gA, gB, ldo);
  });
}

int pseudosym_sign_bwd(ps_handle h, int m, const double* lambda, const double* V, int ldv,
                       const double* gSA, const double* gSB, int ldg, double* gA, double* gB,
                       int ldo) {
  if (!h) return -1;
  if (m < 1) return -2;
  if (!lambda) return -3;
  if (!V) return -4;
  if (ldv < 2 * m) return -5;
  if (!gSA) return -6;
  if (!gSB) return -7;
  if (ldg < m) return -8;
  if (!gA) return -9;
  if (!gB) return -10;
  if (ldo < m) return -11;
  return guarded(h, [&] { return run_sign_bwd(h, m, lambda, V, ldv, gSA, gSB, ldg, gA, gB, ldo); });
}

const char* ps_status_string(int st) {
  switch (st) {
    case PS_OK: return "ok";
    case PS_NOT_DEFINITE: return "not definite: A+B or A-B is not positive definite";
    case PS_SHIFT_BREAKDOWN: return "Cholesky of a shifted Gram matrix failed";
    case PS_NOT_CONVERGED: return "stopping test failed after the allowed restarts";
    case PS_HIP_ERROR: return "HIP runtime error";
    case PS_NO_WORKSPACE: return "workspace too small";
    case PS_BASIS_BREAKDOWN: return "Cholesky of the leading block of P_+ failed";
    default: return st < 0 ? "invalid argument" : "unknown status";
  }
}

}  // extern "C"
