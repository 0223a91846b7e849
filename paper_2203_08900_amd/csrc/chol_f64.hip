// Batched Cholesky factorization with the inverse factor, Z = R^T R, W = R^{-1}, in FP64
// or FP32 (one template).
//
// Blocked right-looking algorithm over 64 x 64 diagonal blocks with a look-ahead of one
// block row.  Per block step k, one launch applies panel k to block row k+1, factors and
// inverts diagonal block k+1 and forms its panel R(k+1, k+2:) = R^{-T} Z(k+1, k+2:) (each
// panel tile's workgroup updates and factors the block itself, and updates its own tile)
// while its other workgroups apply panel k to the rows below block row k+1.  Two
// variants of that schedule move the memory-bound K = 64 trailing updates: eight or more
// matrices of moderate size apply panels in pairs (K = 128), and large matrices go by
// outer blocks of 512 rows whose panels reach the rows below in one large GEMM.
// The full inverse factor W = R^{-1} is then assembled from the inverted diagonal
// blocks by recursive doubling, one pair of GEMM launches per level.  The batch index
// runs over independent matrices (the r shifted Gram matrices of a Zolotarev step, or
// A+B and A-B), so every launch covers all of them at once.
#include "chol_block.h"
#include "gemm_tile.h"
#include "ps_internal.h"

#include <memory>

namespace ps {

namespace {
constexpr int NB = kNb;
constexpr int NTD = 256;
constexpr int kWideBatch = 2;
constexpr int kPairedBatch = 8;  // from this many matrices, trailing updates by panel pairs
constexpr int kPairedMin = 1024; // ... and from this padded size (short chains gain nothing)
constexpr int kOuter = 512;      // outer block of the large factorizations
constexpr int kOuterMin = 4096;  // padded sizes from which they are used
}

// LDS of a step in the wide variant: the block layout, then R(k-1, tile) and the panel
// tile (row-major [64][65] each).  The narrow variant uses the block layout alone.
constexpr int kQt = blk::kLdsElems;
constexpr int kUt = kQt + NB * blk::kLdS;
constexpr int kWideElems = kUt + NB * blk::kLdS;

// A 64 x 64 column-major block (leading dimension ld) moves between memory and
// registers as coalesced 16-byte vectors: thread t holds rows [VW (t % TPC), + VW) of the
// columns t / TPC + CPI q, value q VW + u in slot u of vector q.  Block origins and
// leading dimensions are multiples of 16 bytes (checked by the launcher).
template <class T>
struct BlockVec {
  static constexpr int VW = 16 / sizeof(T);   // elements per vector
  static constexpr int TPC = NB / VW;         // threads per column
  static constexpr int CPI = NTD / TPC;       // columns per block-wide access
  static constexpr int NV = NB / CPI;         // vectors per thread
  typedef T vec_t __attribute__((ext_vector_type(VW)));
  __device__ static int row0() { return VW * ((int)threadIdx.x % TPC); }
  __device__ static int col0() { return (int)threadIdx.x / TPC; }
};
template <class T>
__device__ inline void load_block(const T* g, long long ld, T (&val)[NB * NB / NTD]) {
  using V = BlockVec<T>;
  const int e0 = V::row0(), c0 = V::col0();
#pragma unroll
  for (int q = 0; q < V::NV; ++q) {
    const auto x = *reinterpret_cast<const typename V::vec_t*>(g + e0 + (long long)(c0 + V::CPI * q) * ld);
#pragma unroll
    for (int u = 0; u < V::VW; ++u) val[q * V::VW + u] = x[u];
  }
}
template <class T>
__device__ inline void store_block(T* g, long long ld, const T (&val)[NB * NB / NTD]) {
  using V = BlockVec<T>;
  const int e0 = V::row0(), c0 = V::col0();
#pragma unroll
  for (int q = 0; q < V::NV; ++q) {
    typename V::vec_t x;
#pragma unroll
    for (int u = 0; u < V::VW; ++u) x[u] = val[q * V::VW + u];
    *reinterpret_cast<typename V::vec_t*>(g + e0 + (long long)(c0 + V::CPI * q) * ld) = x;
  }
}
// Registers to / from LDS row-major at l (leading dimension 65): entry (i, j) at
// l[i * 65 + j].
template <class T>
__device__ inline void stage_block(T* l, const T (&val)[NB * NB / NTD]) {
  using V = BlockVec<T>;
  const int e0 = V::row0(), c0 = V::col0();
#pragma unroll
  for (int q = 0; q < V::NV; ++q)
#pragma unroll
    for (int u = 0; u < V::VW; ++u) l[(e0 + u) * blk::kLdS + c0 + V::CPI * q] = val[q * V::VW + u];
}
template <class T>
__device__ inline void unstage_block(const T* l, T (&val)[NB * NB / NTD]) {
  using V = BlockVec<T>;
  const int e0 = V::row0(), c0 = V::col0();
#pragma unroll
  for (int q = 0; q < V::NV; ++q)
#pragma unroll
    for (int u = 0; u < V::VW; ++u) val[q * V::VW + u] = l[(e0 + u) * blk::kLdS + c0 + V::CPI * q];
}

// D -= P^T Q for the 16 x 16 tile (ti, tj) of row-major LDS blocks (wave-wide).
template <class T>
__device__ inline void sub_ptq(T* D, const T* P, const T* Q, int ti, int tj) {
  const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
  const auto acc = blk::tile_mm_ta(P + 16 * ti, blk::kLdS, Q + 16 * tj, blk::kLdS, NB);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    T* d = D + (16 * ti + blk::BlkMfma<T>::row(lk, v)) * blk::kLdS + 16 * tj + li;
    *d -= acc[v];
  }
}

// One step of the blocked factorization: the update of block row k by panel k-1, the
// diagonal block and the panel together.  Every workgroup (ntiles per matrix) applies
// the update to the diagonal block, factors and inverts it in LDS (the same arithmetic
// in each, so all agree; tile 0 stores R_kk^{-1} and R_kk), applies the update to its
// own 64-column tile of block row k and forms that tile of the panel
// R(k, k+1:) = R_kk^{-T} Z(k, k+1:) on the matrix cores, in place.  The redundant work
// runs side by side on otherwise idle compute units; what it saves is a dependent
// launch per step.
//
// Two variants of the LDS use.  Wide: R(k-1, tile) and the panel tile are staged in
// LDS as well (about 144 KB in FP64, one workgroup per compute unit), which gives the
// shortest diagonal chain when a step has few matrices.  Narrow: R(k-1, tile) is read
// from memory as the matrix-core operand and the panel tile stays in registers until
// the panel product (the block layout alone, two FP64 workgroups per compute unit), so
// that the trailing-update tiles of many matrices run at twice the occupancy.
template <class T, bool kWide>
__device__ __forceinline__ void diag_panel(T* lds, int bid, T* z, long long sz, T* w, long long sw,
                                           int ld, int k0, int rest, int ntiles, int fold,
                                           int* info) {
  using Acc = typename blk::BlkMfma<T>::acc_t;
  const int b = bid / ntiles, t = bid - b * ntiles;
  T* Z = z + b * sz + k0 + (long long)k0 * ld;
  T* W = w + b * sw + k0 + (long long)k0 * ld;
  T* Zt = Z + (long long)(NB + NB * t) * ld;   // panel tile t: columns k0 + 64 + 64t..
  // fold: the previous panels (0, 1 or 2, rows k0 - fold 64 .. k0 - 1) that block row k
  // still owes
  const bool tile = rest > 0;
  T* const stage = lds + blk::kStage;
  T* const Pl = lds + blk::kWl;   // a previous panel's block until the factorization
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
  // all loads in flight at once (lower triangles are staged too and ignored where they
  // do not matter); narrow: wave w's row of 16 x 16 tiles of the panel tile goes straight
  // into the accumulator layout
  constexpr int Q = NB * NB / NTD;
  T vz[Q], vp[Q];
  load_block(Z, ld, vz);
  if (fold) load_block(Z - fold * NB, ld, vp);
  Acc u[4];
  if constexpr (kWide) {
    T vt[Q], vq[Q];
    if (tile) load_block(Zt, ld, vt);
    if (fold && tile) load_block(Zt - fold * NB, ld, vq);
    if (tile) stage_block(lds + kUt, vt);
    if (fold && tile) stage_block(lds + kQt, vq);
  } else {
    if (tile) {
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          u[c][v] = Zt[(16 * wave + blk::BlkMfma<T>::row(lk, v)) + (long long)(16 * c + li) * ld];
    }
  }
  stage_block(stage, vz);
  if (fold) stage_block(Pl, vp);
  __syncthreads();
  for (int f = 0; f < fold; ++f) {
    const int off = (fold - f) * NB;   // rows of this panel above k0
    if (f > 0) {
      // the next panel's blocks (every read of the previous ones ended at its barrier)
      load_block(Z - off, ld, vp);
      if constexpr (kWide) {
        if (tile) {
          T vq[Q];
          load_block(Zt - off, ld, vq);
          stage_block(lds + kQt, vq);
        }
      }
      stage_block(Pl, vp);
      __syncthreads();
    }
    // Z_kk -= P^T P with P = R(panel, k) (the ten tiles on and above the diagonal, dealt
    // round-robin over the four waves; every LDS element is updated by one lane) and
    // Z(k, tile) -= P^T R(panel, tile)
    int n = 0;
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
      for (int tj = ti; tj < 4; ++tj, ++n)
        if ((n & 3) == wave) sub_ptq(stage, Pl, Pl, ti, tj);
    if (tile) {
      if constexpr (kWide) {
#pragma unroll
        for (int c = 0; c < 4; ++c) sub_ptq(lds + kUt, Pl, lds + kQt, wave, c);
      } else {
        const T* Qg = Zt - off;   // R(panel, tile) from memory as the B operand
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          Acc acc = {0, 0, 0, 0};
          const T* Qc = Qg + (long long)(16 * c + li) * ld + lk;
#pragma unroll
          for (int k = 0; k < NB; k += 4)
            acc = blk::BlkMfma<T>::step(Pl[(k + lk) * blk::kLdS + 16 * wave + li], Qc[k], acc);
          u[c] -= acc;
        }
      }
    }
    __syncthreads();
  }
  // The other workgroups of this matrix may still be reading the diagonal block, so
  // tile 0 leaves it untouched: R_kk goes to the (unused, zero) block below W_kk and
  // moves into place in the next step's launch, which also clears that block; the last
  // step (a single workgroup) writes it directly.
  if (t == 0 && k0 > 0) {
    T* src = W - (long long)NB * ld;              // block (k, k-1) of W
    T* dst = Z - NB - (long long)NB * ld;         // block (k-1, k-1) of Z
    // every load ahead of the stores (the compiler may not move loads past stores
    // through pointers that could alias)
    T val[Q], zero[Q];
    load_block(src, ld, val);
#pragma unroll
    for (int q = 0; q < Q; ++q) zero[q] = T(0);
    store_block(dst, ld, val);
    store_block(src, ld, zero);
  }
  blk::factor_invert_block(lds, tile ? W + NB : Z, W, ld, info, b < 30 ? b : 30, t == 0);
  if (!tile) return;
  // R(k, tile) = R_kk^{-T} Z(k, tile) = W_kk^T Z(k, tile): wave w forms column tile w
  // for the four row tiles r, each over K = 16 (r + 1) (W_kk^T is lower triangular), so
  // that every wave takes 40 matrix-core steps; the result goes to memory through the
  // staging area (narrow: the updated panel tile first goes into the staging area, free
  // again, and the result waits for every wave to finish reading it)
  const T* St = stage;
  if constexpr (kWide) {
    St = lds + kUt;
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        stage[(16 * wave + blk::BlkMfma<T>::row(lk, v)) * blk::kLdS + 16 * c + li] = u[c][v];
    __syncthreads();
  }
  const T* Wl = lds + blk::kWl;
  Acc pr[4];
  pr[0] = blk::tile_mm_ta_k<T, 16>(Wl, blk::kLdS, St + 16 * wave, blk::kLdS);
  pr[1] = blk::tile_mm_ta_k<T, 32>(Wl + 16, blk::kLdS, St + 16 * wave, blk::kLdS);
  pr[2] = blk::tile_mm_ta_k<T, 48>(Wl + 32, blk::kLdS, St + 16 * wave, blk::kLdS);
  pr[3] = blk::tile_mm_ta_k<T, 64>(Wl + 48, blk::kLdS, St + 16 * wave, blk::kLdS);
  if constexpr (!kWide) __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      stage[(16 * r + blk::BlkMfma<T>::row(lk, v)) * blk::kLdS + 16 * wave + li] = pr[r][v];
  __syncthreads();
  T val[Q];
  unstage_block(stage, val);
  store_block(Zt, ld, val);
}

// Inverse factor alongside the factorization (one or two matrices).  With
// V(i, j) = sum_{l = i}^{j - 1} W(i, l) R(l, j) for block indices i < j, the blocks of
// W = R^{-1} above the diagonal are W(i, j) = -V(i, j) W_jj.  Launch L of the chain (the
// one that factors diagonal block L) has row block L - 1 of R and W_{L-1, L-1} final, and
// V(i, L - 1) complete for i < L - 1.  Its inverse workgroup (i, j), i <= L - 1 < L <= j,
// forms T = W(i, L - 1) (= W_{L-1,L-1} for i = L - 1, else -V(i, L - 1) W_{L-1,L-1}) and
// adds T R(L - 1, j) to V(i, j) (sets it for i = L - 1); workgroup (i, L) also stores
// T as W(i, L - 1).  A last launch stores W(i, nb - 1).  V lives in a separate buffer
// (upper blocks only), so the blocks the launch reads and writes are all distinct.
struct InvPlan {
  int L;        // launch index (diagonal block being factored); L == nbk: finishing pass
  int nbk;      // number of 64-blocks
  int ncols;    // nbk - L (columns j = L .. nbk - 1), 0 in the finishing pass
  int per;      // inverse workgroups per matrix
};

template <class T>
__device__ __forceinline__ void inverse_tile(T* lds, int q, T* z, long long sz, T* w, long long sw,
                                             T* v, long long sv, int ld, const InvPlan& ip) {
  using Acc = typename blk::BlkMfma<T>::acc_t;
  constexpr int Q = NB * NB / NTD;
  const int b = q / ip.per, e = q - b * ip.per;
  const int L = ip.L;
  int i, j;
  if (ip.ncols > 0) {
    i = e / ip.ncols;
    j = L + (e - i * ip.ncols);
  } else {        // finishing pass: W(i, nbk - 1) for i < nbk - 1
    i = e;
    j = -1;
  }
  const int c = L - 1;   // the block column of W finished here
  const T* Wcc = w + b * sw + (long long)c * NB * (ld + 1);
  T* Vb = v + b * sv;
  T* const Wl = lds;                       // W_{cc}, row-major [64][65]
  T* const Tl = lds + NB * blk::kLdS;      // V(i, c) then T = W(i, c)
  T* const Rl = lds + 2 * NB * blk::kLdS;  // R(c, j)
  T* const Pl = lds + 3 * NB * blk::kLdS;  // T R(c, j)
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
  const bool diag_row = (i == c);
  T* Vij = (j >= 0) ? Vb + (long long)i * NB + (long long)j * NB * ld : nullptr;
  // every load at once, coalesced; V(i, j) stays in registers (zero for i = c, where this
  // workgroup sets it)
  T vij[Q];
  {
    T vw[Q], vt[Q], vr[Q];
    load_block(Wcc, ld, vw);
    if (!diag_row) load_block(Vb + (long long)i * NB + (long long)c * NB * ld, ld, vt);
    if (j >= 0) load_block(z + b * sz + (long long)c * NB + (long long)j * NB * ld, ld, vr);
    if (j >= 0 && !diag_row) {
      load_block(Vij, ld, vij);
    } else {
#pragma unroll
      for (int u = 0; u < Q; ++u) vij[u] = T(0);
    }
    stage_block(Wl, vw);
    if (!diag_row) stage_block(Tl, vt);
    if (j >= 0) stage_block(Rl, vr);
  }
  __syncthreads();
  // T = -V(i, c) W_cc, rows 16w.. of each wave, column tile t over K = 16 (t + 1) (W_cc is
  // upper triangular); each wave reads and then overwrites only its own rows of Tl
  const T* Trow = Wl;
  if (!diag_row) {
    const T* vr = Tl + 16 * wave * blk::kLdS;
    Acc tt[4];
    tt[0] = blk::tile_mm_k<T, 16>(vr, blk::kLdS, Wl, blk::kLdS);
    tt[1] = blk::tile_mm_k<T, 32>(vr, blk::kLdS, Wl + 16, blk::kLdS);
    tt[2] = blk::tile_mm_k<T, 48>(vr, blk::kLdS, Wl + 32, blk::kLdS);
    tt[3] = blk::tile_mm_k<T, 64>(vr, blk::kLdS, Wl + 48, blk::kLdS);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int u = 0; u < 4; ++u)
        Tl[(16 * wave + blk::BlkMfma<T>::row(lk, u)) * blk::kLdS + 16 * t + li] = -tt[t][u];
    Trow = Tl;
  }
  // V(i, j) + T R(c, j)   (T rows of this wave only), to LDS
  if (j >= 0) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const Acc pr = blk::tile_mm_k<T, 64>(Trow + 16 * wave * blk::kLdS, blk::kLdS, Rl + 16 * t, blk::kLdS);
#pragma unroll
      for (int u = 0; u < 4; ++u) Pl[(16 * wave + blk::BlkMfma<T>::row(lk, u)) * blk::kLdS + 16 * t + li] = pr[u];
    }
  }
  __syncthreads();
  // coalesced stores: W(i, c) by the first column's workgroup (or the finishing pass),
  // V(i, j)
  if (!diag_row && (j == L || j < 0)) {
    T val[Q];
    unstage_block(Tl, val);
    store_block(w + b * sw + (long long)i * NB + (long long)c * NB * ld, ld, val);
  }
  if (j >= 0) {
    T val[Q];
    unstage_block(Pl, val);
#pragma unroll
    for (int u = 0; u < Q; ++u) val[u] += vij[u];
    store_block(Vij, ld, val);
  }
}

// One 64 x 64 tile of a trailing update D = alpha op(A) op(B) + beta C with op(A) = A^T,
// op(B) = B and a short K (64 or 128, the panel rows).  Every global access is a
// coalesced 16-byte vector along the contiguous dimension (a column of C and D, a K run
// of A and B), which moves several times more bytes per compute unit than loads in the
// matrix-core fragment layout: all loads of the tile are issued at once, the operands
// go through LDS to the matrix cores, and the result goes back through LDS so that the
// stores are coalesced too.  Wave w owns the 32 x 32 sub-tile (w % 2, w / 2).  C may be
// D (it is read before any store); with kOutUpper the entries below the diagonal keep
// their C values.  Operand addresses are 16-byte aligned (checked by the launcher).
template <class T>
__device__ __forceinline__ void trail_tile(const GemmProblemT<T>& P, int bid, T* lds) {
  using Acc = typename Mfma<T>::acc_t;
  constexpr int VW = 16 / sizeof(T);     // elements per 16-byte access
  constexpr int TPC = 64 / VW;           // threads per 64-element column
  constexpr int CPI = NTD / TPC;         // columns per block-wide access
  constexpr int NV = 64 / CPI;           // accesses per 64 x 64 block
  constexpr int LDT = 64 + VW;           // LDS row length (keeps rows 16-byte aligned)
  typedef T vec_t __attribute__((ext_vector_type(VW)));
  const int z = bid / P.tiles_per_batch, t = bid - z * P.tiles_per_batch;
  int I, J;
  if (P.flags & kOutUpper) {
    tri_index(t, J, I);
  } else {
    I = t % P.tm;
    J = t / P.tm;
  }
  const int tid = threadIdx.x;
  const int i0 = 64 * I, j0 = 64 * J;
  const T* A = P.A + z * P.sA[0] + (long long)i0 * P.lda;   // op(A)(i, k) = A[k + i lda]
  const T* B = P.B + z * P.sB[0] + (long long)j0 * P.ldb;   // op(B)(k, j) = B[k + j ldb]
  const T* C = P.C + z * P.sC[0] + i0 + (long long)j0 * P.ldc;
  T* D = P.D + z * P.sD[0] + i0 + (long long)j0 * P.ldd;
  const int e0 = VW * (tid % TPC), c0 = tid / TPC;   // this thread's run: [e0, e0 + VW) of
                                                     // columns c0 + CPI q
  const int nch = P.K / 64;                          // 1 or 2 chunks of 64
  vec_t cv[NV], av[2][NV], bv[2][NV];
#pragma unroll
  for (int q = 0; q < NV; ++q)
    cv[q] = *reinterpret_cast<const vec_t*>(C + e0 + (long long)(c0 + CPI * q) * P.ldc);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (h < nch) {
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        av[h][q] = *reinterpret_cast<const vec_t*>(A + 64 * h + e0 + (long long)(c0 + CPI * q) * P.lda);
        bv[h][q] = *reinterpret_cast<const vec_t*>(B + 64 * h + e0 + (long long)(c0 + CPI * q) * P.ldb);
      }
    }
  }
  T* As = lds;                 // [i][k], row length LDT
  T* Bs = lds + 64 * LDT;      // [j][k]
  const int lane = tid & 63, wave = tid >> 6, li = lane & 15, lk = lane >> 4;
  const int ib = 32 * (wave & 1), jb = 32 * (wave >> 1);
  Acc acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = Acc{0, 0, 0, 0};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (h < nch) {
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        *reinterpret_cast<vec_t*>(As + (c0 + CPI * q) * LDT + e0) = av[h][q];
        *reinterpret_cast<vec_t*>(Bs + (c0 + CPI * q) * LDT + e0) = bv[h][q];
      }
      __syncthreads();
      // lane lk takes k = 16 lk + kk (both operands agree on the k of every slot)
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) {
        const int k = 16 * lk + kk;
        T xa[2], xb[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          xa[a] = As[(ib + 16 * a + li) * LDT + k];
          xb[a] = Bs[(jb + 16 * a + li) * LDT + k];
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) acc[a][b] = Mfma<T>::step(xa[a], xb[b], acc[a][b]);
      }
      __syncthreads();
    }
  }
  // the product to LDS as [j][i], then D = alpha acc + beta C in the coalesced layout
  T* Ds = lds;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        Ds[(jb + 16 * b + li) * LDT + ib + 16 * a + Mfma<T>::row(lk, v)] = acc[a][b][v];
  __syncthreads();
  const bool upper = (P.flags & kOutUpper) && I == J;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    const int jj = c0 + CPI * q;
    const vec_t pv = *reinterpret_cast<const vec_t*>(Ds + jj * LDT + e0);
    vec_t out;
#pragma unroll
    for (int u = 0; u < VW; ++u) {
      const T val = (T)(P.alpha * (double)pv[u] + P.beta * (double)cv[q][u]);
      out[u] = (upper && e0 + u > jj) ? cv[q][u] : val;
    }
    *reinterpret_cast<vec_t*>(D + e0 + (long long)jj * P.ldd) = out;
  }
}

// One launch of the factorization: workgroups below ndiag run diag_panel for the block
// at k0 (with the previous panel's update of block row k0 when fold is set); the others
// are tiles of the trailing update, `tp` then `tq` (np tiles of tp), that the step
// before k0 still owes to the rows below block row k0 (look-ahead: block row k0 takes
// that update inside diag_panel, so its diagonal block and panel need not wait for the
// whole trailing update).  The two roles touch disjoint parts of Z.
// Waves per SIMD the LDS of a variant allows (the register budget follows from it).
template <class T, bool kWide>
constexpr int step_waves() {
  return sizeof(T) == 8 ? (kWide ? 1 : 2) : (kWide ? 2 : 3);
}

template <class T, bool kWide>
__global__ __launch_bounds__(NTD)
__attribute__((amdgpu_waves_per_eu(step_waves<T, kWide>()))) void chol_step_kernel(
    T* z, long long sz, T* w, long long sw, int ld, int k0, int rest, int ntiles, int fold,
    int* info, GemmProblemT<T> tp, GemmProblemT<T> tq, int ndiag, int np, int ntrail, T* v,
    long long sv, InvPlan ip) {
  constexpr int kAB = 2 * 64 * (64 + 16 / (int)sizeof(T));   // trail_tile's operands
  constexpr int kElems = kWide ? kWideElems : blk::kLdsElems;
  __shared__ __attribute__((aligned(16))) T lds[kElems > kAB ? kElems : kAB];
  const int bid = blockIdx.x;
  if (bid < ndiag)
    diag_panel<T, kWide>(lds, bid, z, sz, w, sw, ld, k0, rest, ntiles, fold, info);
  else if (bid < ndiag + np)
    trail_tile<T>(tp, bid - ndiag, lds);
  else if (bid < ndiag + ntrail)
    trail_tile<T>(tq, bid - ndiag - np, lds);
  else if constexpr (kWide)
    inverse_tile<T>(lds, bid - ndiag - ntrail, z, sz, w, sw, v, sv, ld, ip);
}

inline void gemm_t(hipStream_t s, const GemmProblem* p, int n) { gemm_f64(s, p, n); }
inline void gemm_t(hipStream_t s, const GemmProblemF* p, int n) { gemm_f32(s, p, n); }

template <class T>
void potrf_inv_t(hipStream_t s, T* z, long long sz, T* w, long long sw, int mp, int batch,
                 int* info, bool inverse, LaunchList* defer, T* v = nullptr, long long sv = 0) {
  if (mp % NB) throw HipError{hipErrorInvalidValue, "potrf_inv_f64: size not a multiple of 64"};
  // the step kernel moves blocks as 16-byte vectors
  auto misaligned = [](const void* p, long long stride) {
    return (reinterpret_cast<uintptr_t>(p) % 16) != 0 || (stride * (long long)sizeof(T)) % 16 != 0;
  };
  if (misaligned(z, sz) || misaligned(w, sw) || (v && misaligned(v, sv)))
    throw HipError{hipErrorInvalidValue, "potrf_inv: factorization buffers not 16-byte aligned"};
  // every launch goes through issue (closures own copies of their arguments)
  auto issue = [defer](std::function<void()> f) {
    if (defer)
      defer->push_back(std::move(f));
    else
      f();
  };
  // the diagonal blocks and W12 blocks cover the rest
  issue([=] { zero_lower(s, w, mp, sw, batch); });
  // one or two matrices: the chain of diagonal blocks bounds the time (wide step
  // kernel); more: the trailing updates do (narrow, twice the occupancy)
  const bool wide = batch <= kWideBatch;
  // ---- blocked right-looking Cholesky with a look-ahead of one block row:
  //   C_0 = diagonal block and panel of block row 0;
  //   for k = 0, 1, ...:  C_{k+1} = update of block row k+1 by panel k, its diagonal
  //                       block and panel (in the diagonal workgroups), together with
  //                       the update by panel k of the rows below block row k+1.
  // One launch per step; the bulk of the trailing update runs beside the next diagonal
  // factorization instead of before it.
  // Large matrices (mp >= kOuterMin) go by outer blocks of kOuter rows: the steps above
  // run inside an outer block only (their trailing updates stop at its last row), and
  // the rows below it then take the update by all of its panels at once, one GEMM with
  // K = kOuter on the large tiles instead of kOuter / 64 memory-bound updates with K = 64.
  const int outer = mp >= kOuterMin ? kOuter : mp;
  // trailing problem of one launch: panel rows [pr, pr + kk) applied to rows and columns
  // [r0, r1) (upper triangle) and to rows [r0, r1) x columns [r1, mp)
  auto trailing = [&](int pr, int kk, int r0, int r1, GemmProblemT<T>* out) {
    int n = 0;
    if (r1 <= r0) return n;
    const T* a = z + pr + (long long)r0 * mp;   // R(pr:pr+kk, r0:)
    GemmProblemT<T> q = gemm_problem(r1 - r0, r1 - r0, kk, a, mp, 1, a, mp, 0,
                                     z + r0 + (long long)r0 * mp, mp, -1.0, 1.0,
                                     z + r0 + (long long)r0 * mp, mp, kOutUpper);
    out[n++] = q;
    if (r1 < mp) {
      const T* bq = z + pr + (long long)r1 * mp;   // R(pr:pr+kk, r1:)
      out[n++] = gemm_problem(r1 - r0, mp - r1, kk, a, mp, 1, bq, mp, 0,
                              z + r0 + (long long)r1 * mp, mp, -1.0, 1.0,
                              z + r0 + (long long)r1 * mp, mp, 0);
    }
    return n;
  };
  // the inverse alongside the chain: one or two matrices, no outer blocks, a V buffer
  const bool fused_inv = inverse && v && wide && mp < kOuterMin;
  const int nbk_all = mp / NB;
  auto inv_plan = [&](int L) {
    InvPlan ip{L, nbk_all, 0, 0};
    if (!fused_inv || L < 1) return ip;
    ip.ncols = nbk_all - L;
    ip.per = L < nbk_all ? L * ip.ncols : L - 1;   // (i, j) pairs, or the finishing stores
    return ip;
  };
  // Recording (per-class kernel timing): a chain without launches of other kernels
  // between its steps (no outer blocks) is one window from its first step to its last
  // launch; otherwise every step is its own window.
  struct ChainWin {
    int slot = -1, launches = 0;
    double flops = 0.0;
  };
  const auto win = std::make_shared<ChainWin>();
  const bool one_window = outer == mp;
  const int kcls = sizeof(T) == 4 ? kKcChol32 : (wide ? kKcCholWide : kKcCholNarrow);
  const bool has_finish = fused_inv && inv_plan(nbk_all).per * batch > 0;
  auto rec_begin = [win, one_window](hipStream_t st) {
    if (!one_window) return krec_begin(st);
    if (win->slot < 0) win->slot = krec_begin(st);
    return win->slot;
  };
  auto rec_end = [win, one_window, kcls](hipStream_t st, int slot, double flops, bool last) {
    if (!one_window) {
      krec_end(st, slot, kcls, flops);
      return;
    }
    win->launches += 1;
    win->flops += flops;
    if (last) krec_end(st, win->slot, kcls, win->flops, win->launches);
  };
  double outer_flops = 0.0;   // per matrix: rows [e, mp) -= K = (e - ob) outer panels
  for (int ob = 0; ob < mp; ob += outer) {
    const int obe = std::min(mp, ob + outer);
    if (obe < mp) outer_flops += (double)(mp - obe) * (mp - obe) * (obe - ob);
  }
  const double step_flops = ((double)mp * mp * mp / 3.0 - outer_flops) / (mp / NB);
  auto step = [&](int k0, int fold, const GemmProblemT<T>* tp, int ntp) {
    const int rest = mp - k0 - NB;
    const int nt = rest > 0 ? rest / NB : 1;
    const int ndiag = batch * nt;
    const InvPlan ip = inv_plan(k0 / NB);
    const int ninv = batch * ip.per;
    GemmProblemT<T> t[2] = {};
    int cnt[2] = {0, 0};
    for (int q = 0; q < ntp; ++q) {
      t[q] = tp[q];
      t[q].nb1 = batch;
      t[q].sA[0] = t[q].sB[0] = t[q].sC[0] = t[q].sD[0] = sz;
      t[q].tm = t[q].M / 64;
      t[q].tn = t[q].N / 64;
      t[q].tiles = (t[q].flags & kOutUpper) ? t[q].tm * (t[q].tm + 1) / 2 : t[q].tm * t[q].tn;
      t[q].tiles_per_batch = t[q].tiles;
      t[q].tile_begin = 0;
      cnt[q] = t[q].tiles * batch;
    }
    for (int q = 0; q < ntp; ++q) {
      // trail_tile: K a multiple of 64, 16-byte aligned operands and batch strides
      const bool ok = (t[q].K == 64 || t[q].K == 128) &&
                      (reinterpret_cast<uintptr_t>(t[q].A) % 16) == 0 &&
                      (reinterpret_cast<uintptr_t>(t[q].B) % 16) == 0 &&
                      (reinterpret_cast<uintptr_t>(t[q].C) % 16) == 0 &&
                      (reinterpret_cast<uintptr_t>(t[q].D) % 16) == 0 &&
                      (t[q].sA[0] * sizeof(T)) % 16 == 0 && t[q].lda % (16 / sizeof(T)) == 0 &&
                      t[q].ldb % (16 / sizeof(T)) == 0 && t[q].ldc % (16 / sizeof(T)) == 0 &&
                      t[q].ldd % (16 / sizeof(T)) == 0;
      if (!ok) throw HipError{hipErrorInvalidValue, "potrf_inv: misaligned factorization buffer"};
    }
    const GemmProblemT<T> t0 = t[0], t1 = t[1];
    const int np = cnt[0], ntrail = cnt[0] + cnt[1], grid = ndiag + ntrail + ninv;
    const bool last = k0 + NB >= mp && !has_finish;
    issue([=] {
      const int slot = rec_begin(s);
      if (wide)
        hipLaunchKernelGGL((chol_step_kernel<T, true>), dim3(grid), dim3(NTD), 0, s, z, sz, w, sw,
                           mp, k0, rest, nt, fold, info, t0, t1, ndiag, np, ntrail, v, sv, ip);
      else
        hipLaunchKernelGGL((chol_step_kernel<T, false>), dim3(grid), dim3(NTD), 0, s, z, sz, w,
                           sw, mp, k0, rest, nt, fold, info, t0, t1, ndiag, np, ntrail, v, sv,
                           ip);
      PS_HIP(hipGetLastError());
      // algorithmic work of a launch: the factorization's batch mp^3 / 3, less the outer
      // blocks' updates (GEMM launches, counted there), spread evenly over its mp / 64
      // block steps
      rec_end(s, slot, (double)batch * step_flops, last);
    });
  };
  // Eight or more matrices of padded size 1024 to 4095 (no outer blocks): the trailing
  // updates, bound by their memory traffic (a 64 x 64 tile with K = 64 reads and writes
  // its C tile for 64 steps of work), go by pairs of panels (2q, 2q + 1) with K = 128:
  // launch 2q + 2 takes the pair into block row 2q + 2 (diagonal workgroups) and applies
  // it to the rows [2q + 3, mid); launch 2q + 3 takes panel 2q + 2 into its block row and
  // applies the pair to the rows [mid, end).  mid splits the pair's tiles about evenly.
  const bool paired = batch >= kPairedBatch && mp >= kPairedMin && outer == mp;
  const int nbk = mp / NB;
  int mid = 0;
  if (paired) {
    for (int k = 0; k < nbk; ++k) {
      GemmProblemT<T> tp[2];
      int ntp = 0, fold = 0;
      if (k > 0 && k % 2 == 0) {
        fold = 2;
        const int n = nbk - (k + 1);   // block rows below block row k
        if (n > 0) {
          const long long half = (long long)n * (n + 1) / 4;
          int top = 1;
          while (top < n && (long long)top * n - (long long)top * (top - 1) / 2 < half) ++top;
          mid = (k + 1 + top) * NB;
          ntp = trailing((k - 2) * NB, 2 * NB, (k + 1) * NB, mid, tp);
        } else {
          mid = mp;
        }
      } else if (k % 2 == 1) {
        fold = 1;
        if (k >= 3) {
          ntp = trailing((k - 3) * NB, 2 * NB, mid, mp, tp);   // (upper square only)
        }
      }
      step(k * NB, fold, tp, ntp);
    }
  }
  for (int ob = 0; ob < mp && !paired; ob += outer) {
    const int obe = std::min(mp, ob + outer);
    for (int k0 = ob; k0 < obe; k0 += NB) {
      // the launch for block k0 carries the previous panel's update of the rows below
      // block row k0 + 1 within this outer block (none for the outer block's first
      // block: its rows took every earlier panel in the outer update)
      GemmProblemT<T> tp[2];
      const int ntp = k0 > ob ? trailing(k0 - NB, NB, k0 + NB, obe, tp) : 0;
      step(k0, k0 > ob ? 1 : 0, tp, ntp);
    }
    if (obe < mp) {
      // rows and columns [obe, mp) -= R(ob:obe, obe:)^T R(ob:obe, obe:)  (upper triangle)
      const T* a = z + ob + (long long)obe * mp;
      GemmProblemT<T> pu = gemm_problem(mp - obe, mp - obe, obe - ob, a, mp, 1, a, mp, 0,
                                        z + obe + (long long)obe * mp, mp, -1.0, 1.0,
                                        z + obe + (long long)obe * mp, mp, kOutUpper);
      pu.nb1 = batch;
      pu.sA[0] = pu.sB[0] = pu.sC[0] = pu.sD[0] = sz;
      issue([=] { gemm_t(s, &pu, 1); });
    }
  }
  if (!inverse) return;   // W then holds only the inverted diagonal blocks
  if (fused_inv) {
    // the finishing pass: W(i, nbk - 1) = -V(i, nbk - 1) W_{nbk-1, nbk-1}
    const InvPlan ip = inv_plan(nbk_all);
    const int ninv = batch * ip.per;
    if (ninv > 0) {
      const GemmProblemT<T> none{};
      issue([=] {
        const int slot = rec_begin(s);
        hipLaunchKernelGGL((chol_step_kernel<T, true>), dim3(ninv), dim3(NTD), 0, s, z, sz, w, sw,
                           mp, 0, 0, 1, 0, info, none, none, 0, 0, 0, v, sv, ip);
        PS_HIP(hipGetLastError());
        rec_end(s, slot, 0.0, true);
      });
    }
    return;
  }
  // ---- W = R^{-1} by recursive doubling over the block diagonal: at level S every
  // diagonal block of size S is already inverted, and for each pair of neighbours
  //   W12 = -W11 R12 W22.
  // T = R12 W22 is kept transposed in the (still unused) strictly lower block W21 and
  // cleared right after use: the triangle-aware GEMMs of the next levels read whole
  // diagonal tiles of W11 and W22 and rely on zeros below the diagonal.
  for (int S = NB; S < mp; S *= 2) {
    const int full = mp / (2 * S);               // pairs whose right block has size S
    const int rem = mp - full * 2 * S;           // leftover rows after the full pairs
    const long long pstride = (long long)2 * S * (mp + 1);
    GemmProblemT<T> t1[2], t2[2];
    int n1 = 0;
    auto add_pair = [&](long long off, int sr, int nb2) {
      T* w11 = w + off;
      T* w22 = w + off + (long long)S * (mp + 1);
      T* w21 = w + off + S;                  // rows right, cols left (sr x S)
      T* w12 = w + off + (long long)S * mp;  // rows left, cols right (S x sr)
      const T* r12 = z + off + (long long)S * mp;
      GemmProblemT<T> a = gemm_problem(sr, S, sr, w22, mp, 1, r12, mp, 1, w21, mp, 1.0, 0.0, nullptr,
                                   0, kALower);
      GemmProblemT<T> b = gemm_problem(S, sr, S, w11, mp, 0, w21, mp, 1, w12, mp, -1.0, 0.0, nullptr,
                                   0, kAUpper);
      for (GemmProblemT<T>* q : {&a, &b}) {
        q->nb1 = batch;
        q->sA[0] = (q == &a) ? sw : sw;
        q->sB[0] = (q == &a) ? sz : sw;
        q->sC[0] = sw;
        q->sD[0] = sw;
        q->nb2 = nb2;
        q->sA[1] = q->sB[1] = q->sC[1] = q->sD[1] = pstride;
      }
      t1[n1] = a;
      t2[n1] = b;
      ++n1;
    };
    if (full > 0) add_pair(0, S, full);
    if (rem > S) add_pair((long long)full * pstride, rem - S, 1);
    if (n1) {
      issue([=] { gemm_t(s, t1, n1); });
      issue([=] { gemm_t(s, t2, n1); });
      for (int q = 0; q < n1; ++q) {
        const GemmProblemT<T> u = t2[q];
        issue([=] { zero_block(s, const_cast<T*>(u.B), u.N, u.K, mp, batch, sw, u.nb2, pstride); });
      }
    }
  }
}

void potrf_inv_f64(hipStream_t s, double* z, long long sz, double* w, long long sw,
                   double* /*tmp*/, int mp, int batch, int* info, bool inverse,
                   LaunchList* defer, double* v, long long sv) {
  potrf_inv_t(s, z, sz, w, sw, mp, batch, info, inverse, defer, v, sv);
}

void potrf_inv_f32(hipStream_t s, float* z, long long sz, float* w, long long sw, int mp,
                   int batch, int* info, LaunchList* defer) {
  potrf_inv_t(s, z, sz, w, sw, mp, batch, info, true, defer);
}

void issue_interleaved(LaunchList& a, LaunchList& b) {
  const size_t n = std::max(a.size(), b.size());
  for (size_t i = 0; i < n; ++i) {
    if (i < a.size()) a[i]();
    if (i < b.size()) b[i]();
  }
  a.clear();
  b.clear();
}

}  // namespace ps
