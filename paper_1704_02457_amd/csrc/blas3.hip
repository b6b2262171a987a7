// Generic panel-major level-3 routines: gemm_nt, gemm_nn, syrk_ln, trmm_rlnn,
// trsm_rltn, potrf_l, potrf_l_mn, syrk_potrf_ln, getrf and gelqf on
// arbitrary sub-matrices (any (ai, aj), any
// sizes), single instance or uniform batch (one batch index per grid row).
//
// These are the generic kernel variant of §4.4.2: every 16x16 block is
// computed as a full register tile and stored through a masked store that
// also handles sub-matrices not aligned to a panel top.  Operands are read
// straight from the caller's panel-major buffers; nothing is repacked (§4.3).
#include "common.hpp"

namespace bh {

constexpr int GW = 4;  // waves per workgroup in the generic kernels

__device__ __forceinline__ View at_batch(View v, long long stride) {
  v.p += (long long)blockIdx.y * stride;
  return v;
}

// ---------------------------------------------------------------- gemm/syrk
// One wave per 16x16 block of D.  The wave accumulates the transposed block
// D^T(j,i) = sum_k B_j[:,k] A_i[:,k]^T with one MFMA per 4-wide k-step (the
// gemm_nt k-loop of §4.4.1: both factors are read along panels), then
// applies alpha/beta and stores with the generic masked store.
// B^T fragment read column-wise from a k-by-n B (the NN variant, §4.4: B is
// read across panels): lane (c, g) holds B[k0 + g][j0 + c]
__device__ __forceinline__ double load_fragT(const View &v, int j0, int k0) {
  const int l = lane_id();
  const int j = j0 + (l & 15), k = k0 + (l >> 4);
  const bool ok = k < v.rows && j < v.cols;
  const double x = v.p[ok ? pm_off(v.ai + k, v.aj + j, v.cn) : pm_off(v.ai, v.aj, v.cn)];
  return ok ? x : 0.0;
}

constexpr int kGemmKU = 8;

// Fragment loads without the final select (elements outside the view come
// from its origin), for loops that issue a group of loads and mask after.
__device__ __forceinline__ double load_frag_raw(const View &v, int i0, int k0) {
  const int l = lane_id();
  const int i = i0 + (l & 15), k = k0 + (l >> 4);
  const bool ok = i < v.rows && k < v.cols;
  return v.p[ok ? pm_off(v.ai + i, v.aj + k, v.cn) : pm_off(v.ai, v.aj, v.cn)];
}

__device__ __forceinline__ double load_fragT_raw(const View &v, int j0, int k0) {
  const int l = lane_id();
  const int j = j0 + (l & 15), k = k0 + (l >> 4);
  const bool ok = k < v.rows && j < v.cols;
  return v.p[ok ? pm_off(v.ai + k, v.aj + j, v.cn) : pm_off(v.ai, v.aj, v.cn)];
}

template <bool SYRK, bool NN = false>
__global__ __launch_bounds__(64 * GW) void k_gemm_nt(
    int m, int n, int k, double alpha, View A, View B, double beta, View C,
    View D, long long sA, long long sB, long long sC, long long sD) {
  A = at_batch(A, sA);
  B = at_batch(B, sB);
  C = at_batch(C, sC);
  D = at_batch(D, sD);
  const int w = wave_id();
  const int tm = (m + 15) >> 4, tn = (n + 15) >> 4;
  const int tile = blockIdx.x * GW + w;
  int ti, tj;
  if (SYRK) {
    // lower block triangle, row-major enumeration: tile = ti*(ti+1)/2 + tj
    if (tile >= tm * (tm + 1) / 2) return;
    ti = 0;
    while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
    tj = tile - ti * (ti + 1) / 2;
  } else {
    if (tile >= tm * tn) return;
    ti = tile / tn;
    tj = tile - ti * tn;
  }
  // The k-loop in groups of kGemmKU steps whose fragment loads are all in
  // flight together: the loads come first, a scheduling barrier keeps the
  // compiler from interleaving them with their masks and the products, and
  // the k index is masked afterwards on both operands (rows past m or n only
  // reach accumulator rows or columns that are never stored).
  const int g = lane_id() >> 4;
  d4 acc = zero4();
  for (int k0 = 0; k0 < k; k0 += 4 * kGemmKU) {
    double fa[kGemmKU], fb[kGemmKU];
#pragma unroll
    for (int u = 0; u < kGemmKU; ++u) {
      fb[u] = NN ? load_fragT_raw(B, 16 * tj, k0 + 4 * u) : load_frag_raw(B, 16 * tj, k0 + 4 * u);
      fa[u] = load_frag_raw(A, 16 * ti, k0 + 4 * u);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < kGemmKU; ++u) {
      const bool kin = k0 + 4 * u + g < k;
      acc = mfma(kin ? fb[u] : 0.0, kin ? fa[u] : 0.0, acc);
    }
  }
  const d4 ct = load_tileT(C, 16 * ti, 16 * tj, SYRK);
  d4 out;
#pragma unroll
  for (int r = 0; r < 4; ++r) out[r] = beta * ct[r] + alpha * acc[r];
  store_tileT(D, 16 * ti, 16 * tj, out, SYRK);
}

// ---------------------------------------------------------------- trmm_rlnn
// D = alpha * B * A with A lower triangular (§5.2.2, trmm paragraph; the
// C step of the Riccati recursion, §5.3).  One wave per 16x16 block (i, j)
// of D: D(i,j) = sum_{k >= j} B(i,k) A(k,j), i.e. a gemm_nt against A^T
// whose k-loop starts at the block's first column (A(k,j) = 0 for k < j);
// the A^T fragment of rows 16j..16j+15 is read column-wise from A and masked
// to the lower triangle, so the diagonal block needs no special case.  (The
// grouped loads of gemm_nt do not pay here: the k-loops are 4-8 steps long.)
__device__ __forceinline__ double load_fragT_lower(const View &v, int j0, int k0) {
  const int l = lane_id();
  const int j = j0 + (l & 15), k = k0 + (l >> 4);  // A(k, j)
  const bool ok = k < v.rows && j < v.cols && k >= j;
  const double x = v.p[ok ? pm_off(v.ai + k, v.aj + j, v.cn) : pm_off(v.ai, v.aj, v.cn)];
  return ok ? x : 0.0;
}

__global__ __launch_bounds__(64 * GW) void k_trmm_rlnn(int m, int n, double alpha,
                                                       View A, View B, View D,
                                                       long long sA, long long sB,
                                                       long long sD) {
  A = at_batch(A, sA);
  B = at_batch(B, sB);
  D = at_batch(D, sD);
  const int w = wave_id();
  const int tm = (m + 15) >> 4, tn = (n + 15) >> 4;
  const int tile = blockIdx.x * GW + w;
  if (tile >= tm * tn) return;
  const int ti = tile / tn, tj = tile - ti * tn;
  d4 acc = zero4();
  for (int k0 = 16 * tj; k0 < n; k0 += 4) {
    const double fa = load_fragT_lower(A, 16 * tj, k0);  // A^T rows 16tj.., cols k0..k0+3
    const double fb = load_frag(B, 16 * ti, k0);
    acc = mfma(fa, fb, acc);
  }
  d4 out;
#pragma unroll
  for (int r = 0; r < 4; ++r) out[r] = alpha * acc[r];
  store_tileT(D, 16 * ti, 16 * tj, out, false);
}

// ---------------------------------------------------------------- trsm_rltn
// D = alpha * B * A^{-T}, A lower.  In the transposed view Y = D^T solves
// A*Y = alpha*B^T by block forward substitution; each wave owns 16 rows of B
// (16 columns of Y) and walks the block rows of A.  For block row j:
//   Z = alpha*B^T(j) - sum_{l<j} A(j,l) Y(l)          (MFMA downdate)
//   Y(j) = A(j,j)^{-1} Z                               (MFMA with the
//          register-computed inverse of the diagonal block)
// The gemm downdate and the substitution run in one kernel (§4.6, "trsm as
// one kernel").  Earlier Y(l) are re-read from D, which this wave wrote.
__device__ __forceinline__ void diag_inverse_lower(const View &A, int j0,
                                                   int nv, WaveLds &s,
                                                   d4 &V) {
  // W^T (upper) of the lower diagonal block W = A(j0:j0+16, j0:j0+16)
  d4 Wt = load_tileT(A, j0, j0, true);
  pad_identity(Wt, nv);
  const int l = lane_id();
  if (l < 16) {
    const double d = (l < nv) ? A.p[pm_off(A.ai + j0 + l, A.aj + j0 + l, A.cn)]
                              : 1.0;
    s.inv[l] = 1.0 / d;
  }
  wave_sync();
  V = trtri_tile_upper(Wt, s.inv, s.ulds, s.row);
}

// One wave per 16-row strip of B, GW strips per workgroup.  For n <= 16 *
// kTrsmLdsBlocks the inverses of A's diagonal blocks do not depend on the
// strip: the workgroup's waves form them first, in parallel, into LDS, and
// every strip then reads them there (otherwise each wave forms each inverse
// where it needs it).
constexpr int kTrsmLdsBlocks = 8;

__global__ __launch_bounds__(64 * GW) void k_trsm_rltn(
    int m, int n, double alpha, View A, View B, View D, long long sA,
    long long sB, long long sD) {
  A = at_batch(A, sA);
  B = at_batch(B, sB);
  D = at_batch(D, sD);
  __shared__ WaveLds lds[GW];
  __shared__ double vinv[kTrsmLdsBlocks][256];  // T-tiles of the diagonal-block inverses
  const int w = wave_id();
  const int lane = lane_id();
  const int strip = blockIdx.x * GW + w;  // 16 rows of B
  WaveLds &s = lds[w];
  const int nb = (n + 15) >> 4;
  const bool pre = nb <= kTrsmLdsBlocks;
  if (pre) {
    for (int j = w; j < nb; j += GW) {
      d4 V;
      diag_inverse_lower(A, 16 * j, min(16, n - 16 * j), s, V);
#pragma unroll
      for (int r = 0; r < 4; ++r) vinv[j][64 * r + lane] = V[r];
    }
    __syncthreads();
  }
  if (strip * 16 >= m) return;
  for (int j = 0; j < nb; ++j) {
    d4 z = load_tileT(B, 16 * strip, 16 * j, false);
#pragma unroll
    for (int r = 0; r < 4; ++r) z[r] *= alpha;
    for (int l = 0; l < j; ++l) {
      const d4 a = load_tileT(A, 16 * j, 16 * l, false);  // A(j,l)^T
      const d4 y = load_tileT(D, 16 * strip, 16 * l, false);  // Y(l)
      z = mfma_tn(neg4(a), y, z);
    }
    d4 V;
    if (pre) {
#pragma unroll
      for (int r = 0; r < 4; ++r) V[r] = vinv[j][64 * r + lane];
    } else {
      diag_inverse_lower(A, 16 * j, min(16, n - 16 * j), s, V);
    }
    const d4 y = mfma_tn(V, z, zero4());
    store_tileT(D, 16 * strip, 16 * j, y, false);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    wave_sync();
  }
}

// ---------------------------------------------------------------- potrf_l
// Lower Cholesky of C (+ A*B^T when k > 0), one workgroup per instance.
// Left-looking over block columns j of L, i.e. block rows j of U = L^T: every
// 16x16 block is produced once by one kernel pass -- the gemm_nt downdate
// over the already computed blocks, then either the register-resident
// factorization (diagonal block) or the triangular solve with the diagonal
// block's inverse (off-diagonal blocks) -- and stored (§4.6: LAPACK routines
// written as BLAS-like kernels, block size = kernel size).
struct PotrfLds {
  DiagLds d;
  double V[64 * 4];  // inverse of the current diagonal block (T-tile)
  int info;
};

__global__ __launch_bounds__(64 * GW) void k_potrf_l(
    int m, int n, int k, View A, View B, View C, View D, double *dA, int *info,
    long long sA, long long sB, long long sC, long long sD, long long sdA) {
  A = at_batch(A, sA);
  B = at_batch(B, sB);
  C = at_batch(C, sC);
  D = at_batch(D, sD);
  const long long b = blockIdx.y;
  double *dAb = dA ? dA + b * sdA : nullptr;
  __shared__ PotrfLds s;
  const int w = wave_id();
  const int l = lane_id();
  const int nb = (n + 15) >> 4, nbr = (m + 15) >> 4;
  if (threadIdx.x == 0) s.info = 0;
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    const int nv = min(16, n - 16 * j);
    if (w == 0) {
      d4 t = load_tileT(C, 16 * j, 16 * j, true);
      for (int k0 = 0; k0 < k; k0 += 4)
        t = mfma(load_frag(B, 16 * j, k0), load_frag(A, 16 * j, k0), t);
      for (int q = 0; q < j; ++q) {
        const d4 u = load_tileT(D, 16 * j, 16 * q, false);  // U(q,j)
        t = mfma_tn(neg4(u), u, t);
      }
      // stacked rows below column n that share this tile (the last block
      // column of a non-square factorization): they are solved with the
      // block's inverse like any off-diagonal block
      const int l16 = l & 15, g4 = l >> 4;
      const bool stacked = min(16, m - 16 * j) > nv;
      d4 tb = zero4();
      if (stacked) {
#pragma unroll
        for (int r = 0; r < 4; ++r) tb[r] = (l16 >= nv && g4 + 4 * r < nv) ? t[r] : 0.0;
      }
      pad_identity(t, nv);
      d4 v;
      const int inf = potrf_inv_tile_upper(t, v, s.d, nullptr, (nv + 3) >> 2);
      if (inf && l == 0 && s.info == 0) s.info = 16 * j + inf;
      if (stacked) {
        const d4 ub = mfma_tn(v, tb, zero4());
#pragma unroll
        for (int r = 0; r < 4; ++r) t[r] = l16 >= nv ? ub[r] : t[r];
      }
      store_tileT(D, 16 * j, 16 * j, t, true);
      if (dAb && l < nv) dAb[16 * j + l] = s.d.inv[l];
#pragma unroll
      for (int r = 0; r < 4; ++r) s.V[l * 4 + r] = v[r];
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __syncthreads();
    d4 v;
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = s.V[l * 4 + r];
    for (int i = j + 1 + w; i < nbr; i += GW) {
      d4 t = load_tileT(C, 16 * i, 16 * j, false);  // M(j,i) = C(i,j)^T
      for (int k0 = 0; k0 < k; k0 += 4)
        t = mfma(load_frag(B, 16 * j, k0), load_frag(A, 16 * i, k0), t);
      for (int q = 0; q < j; ++q) {
        const d4 uj = load_tileT(D, 16 * j, 16 * q, false);  // U(q,j)
        const d4 ui = load_tileT(D, 16 * i, 16 * q, false);  // U(q,i)
        t = mfma_tn(neg4(uj), ui, t);
      }
      const d4 u = mfma_tn(v, t, zero4());  // U(j,i) = V^T M(j,i)
      store_tileT(D, 16 * i, 16 * j, u, false);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __syncthreads();
  }
  if (info && threadIdx.x == 0) info[b] = s.info;
}

// m <= 16*NB <= 64: one wavefront per instance with the whole factor in
// registers (the fused kernel's scheme on generic views): T(j,i) = C(i,j)^T
// (+ the syrk term of syrk_potrf), then for each block row the diagonal
// subroutine, U(j,i) = V^T T(j,i) and the trailing MFMA downdates; every
// block is read and written once, with no barrier.
template <int NB>
__global__ __launch_bounds__(64) void k_potrf_reg(
    int m, int n, int k, View A, View B, View C, View D, double *dA, int *info,
    long long sA, long long sB, long long sC, long long sD, long long sdA) {
  A = at_batch(A, sA);
  B = at_batch(B, sB);
  C = at_batch(C, sC);
  D = at_batch(D, sD);
  const long long b = blockIdx.y;
  double *dAb = dA ? dA + b * sdA : nullptr;
  __shared__ DiagLds s;
  const int l = lane_id();
  constexpr int NT = NB * (NB + 1) / 2;
  d4 T[NT];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) T[tix_up(j, i)] = load_tileT(C, 16 * i, 16 * j, i == j);
  for (int k0 = 0; k0 < k; k0 += 4) {
    double fa[NB], fb[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      fa[i] = load_frag(A, 16 * i, k0);
      fb[i] = load_frag(B, 16 * i, k0);
    }
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int j = 0; j <= i; ++j) T[tix_up(j, i)] = mfma(fb[j], fa[i], T[tix_up(j, i)]);
  }
  int inf0 = 0;
  const int c16 = l & 15, g4 = l >> 4;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int nv = min(16, n - 16 * j);
    if (nv <= 0) break;
    d4 &Dj = T[tix_up(j, j)];
    // stacked rows below column n inside this tile (m > n, last block
    // column): solved with the block's inverse like an off-diagonal block
    const bool stacked = min(16, m - 16 * j) > nv;
    d4 tb = zero4();
    if (stacked) {
#pragma unroll
      for (int r = 0; r < 4; ++r) tb[r] = (c16 >= nv && g4 + 4 * r < nv) ? Dj[r] : 0.0;
    }
    pad_identity(Dj, nv);
    d4 V;
    const int inf = potrf_inv_tile_upper(Dj, V, s, nullptr, (nv + 3) >> 2);
    if (inf && inf0 == 0) inf0 = 16 * j + inf;
    if (stacked) {
      const d4 ub = mfma_tn(V, tb, zero4());
#pragma unroll
      for (int r = 0; r < 4; ++r) Dj[r] = c16 >= nv ? ub[r] : Dj[r];
    }
    store_tileT(D, 16 * j, 16 * j, Dj, true);
    if (dAb && l < nv) dAb[16 * j + l] = s.inv[l];
#pragma unroll
    for (int i = j + 1; i < NB; ++i) {
      T[tix_up(j, i)] = mfma_tn(V, T[tix_up(j, i)], zero4());
      store_tileT(D, 16 * i, 16 * j, T[tix_up(j, i)], false);
    }
#pragma unroll
    for (int q = j + 1; q < NB; ++q) {
      const d4 nu = neg4(T[tix_up(j, q)]);
#pragma unroll
      for (int i = q; i < NB; ++i) T[tix_up(q, i)] = mfma_tn(nu, T[tix_up(j, i)], T[tix_up(q, i)]);
    }
  }
  if (info && l == 0) info[b] = inf0;
}

__global__ void k_fill_int(int *p, int count, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

// One step of a wave argmax by data-parallel primitives (DPP): every lane
// that receives a (key, position) pair from the lane the control selects
// keeps the better of the two (larger key, ties to the smaller position);
// lanes without a source, or outside the rows of RM, receive an element
// below every candidate.  The selection is a total order, so the result does
// not depend on the reduction order.
template <int CTRL, int RM>
__device__ __forceinline__ void argmax_step(double &key, int &pos) {
  const long long kb = __builtin_bit_cast(long long, key);
  const long long ib = __builtin_bit_cast(long long, -3.0);
  const int lo = __builtin_amdgcn_update_dpp((int)ib, (int)kb, CTRL, RM, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(ib >> 32), (int)(kb >> 32), CTRL, RM, 0xf, false);
  const int p2 = __builtin_amdgcn_update_dpp(0x7fffffff, pos, CTRL, RM, 0xf, false);
  const double k2 = __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
  const bool take = k2 > key || (k2 == key && p2 < pos);
  key = take ? k2 : key;
  pos = take ? p2 : pos;
}

// ---------------------------------------------------------------- getrf
// LU with (PIVOT) or without partial pivoting of an m-by-n matrix, m, n <=
// 64 (§5.2.2, getrf): one wave per instance with lane i holding row i of
// the matrix in NC registers (n rounded up to 16), the right-looking
// unblocked sweep of the oracle.  Rows are never moved: each lane keeps the current position of its
// row, an interchange swaps two positions, and the rows are stored to their
// final positions at the end.  Step k: the pivot is the row of largest
// magnitude in column k among positions >= k, ties to the smallest position
// (a wave argmax on DPP, the result in lane 63), the multipliers are formed
// with the pivot's reciprocal and the pivot row's entries reach the other
// lanes by readlane for the rank-1 update (NaN entries in column k are
// ranked as the oracle's scan ranks them).  Contraction into fused multiply-adds is off, so every operation
// rounds as the oracle's does and the pivot choices agree.  Column k lives
// in register 16*qb + kk: the 16 steps of a block of columns select it from
// the block's 16 registers, and the update runs over the columns from the
// block on, so registers are indexed at compile time.
template <bool PIVOT, int NC>
__global__ __launch_bounds__(64) void k_getrf(int m, int n, View C, View D, double *dA,
                                              int *ipiv, int *info, long long sC,
                                              long long sD, long long sdA, long long sip) {
#pragma clang fp contract(off)
  C = at_batch(C, sC);
  D = at_batch(D, sD);
  const long long b = blockIdx.y;
  double *dAb = dA ? dA + b * sdA : nullptr;
  int *ipb = ipiv ? ipiv + b * sip : nullptr;
  const int l = lane_id();
  const bool live = l < m;
  const int lr = min(l, m - 1);
  double r[NC];  // NC: n rounded up to a multiple of 16
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double x = C.p[pm_off(C.ai + lr, C.aj + min(c, n - 1), C.cn)];  // clamped: no branch
    r[c] = (live && c < n) ? x : 0.0;
  }
  int pos = l;
  int inf = 0;
  const int mn = min(m, n);
#pragma unroll
  for (int qb = 0; qb < NC / 16; ++qb) {
    for (int kk = 0; kk < 16; ++kk) {
      const int k = 16 * qb + kk;
      if (k >= mn) break;
      double v = r[16 * qb];
#pragma unroll
      for (int e = 1; e < 16; ++e) v = kk == e ? r[16 * qb + e] : v;
      int pl = k, ppos = k;
      if (PIVOT) {
        // the oracle's scan keeps position k unless a later row is strictly
        // larger, so a NaN there wins and a NaN elsewhere never does
        const double av = __builtin_isnan(v) ? (pos == k ? __builtin_inf() : -0.5) : fabs(v);
        double key = (live && pos >= k) ? av : -1.0;
        int kp = pos;
        argmax_step<0x111, 0xf>(key, kp);  // row_shr:1
        argmax_step<0x112, 0xf>(key, kp);  // row_shr:2
        argmax_step<0x114, 0xf>(key, kp);  // row_shr:4
        argmax_step<0x118, 0xf>(key, kp);  // row_shr:8: lane 15 of a row holds its best
        argmax_step<0x142, 0xa>(key, kp);  // row_bcast:15 into rows 1 and 3
        argmax_step<0x143, 0xc>(key, kp);  // row_bcast:31 into rows 2 and 3
        ppos = __builtin_amdgcn_readlane(kp, 63);
        pl = __ffsll((unsigned long long)__ballot(live && pos == ppos)) - 1;
        const int kl = __ffsll((unsigned long long)__ballot(live && pos == k)) - 1;
        if (l == kl) pos = ppos;
        if (l == pl) pos = k;
      }
      if (ipb && l == 0) ipb[k] = ppos;
      const double piv = readlane_d(v, pl);
      if (piv == 0.0 && inf == 0) inf = k + 1;
      const double inv = 1.0 / piv;
      if (dAb && l == 0) dAb[k] = inv;
      const bool below = live && pos > k;
      const double mult = v * inv;
#pragma unroll
      for (int e = 0; e < 16; ++e) r[16 * qb + e] = (below && kk == e) ? mult : r[16 * qb + e];
#pragma unroll
      for (int c = 16 * qb; c < NC; ++c) {
        if (c < n) {
          const double pc = readlane_d(r[c], pl);
          const double upd = r[c] - mult * pc;
          r[c] = (below && c > k) ? upd : r[c];
        }
      }
    }
  }
  if (live) {
#pragma unroll
    for (int c = 0; c < NC; ++c)
      if (c < n) D.p[pm_off(D.ai + pos, D.aj + c, D.cn)] = r[c];
  }
  if (info && l == 0) info[b] = inf;
}

// ---------------------------------------------------------------- getrf, one wave, MFMA
// LU of an m-by-n matrix with 32 < max(m, n) <= 64, blocked by panels of 16
// columns as in §5.2.2 (getrf), one wave per instance with the whole matrix
// in registers as 16 T-tiles (register r of lane (c, g) of tile (t, J) holds
// A[16t + g + 4r][16J + c]).  Rows are never moved: row i keeps its
// registers, pos(i) is its current position, and the rows are stored to
// their final positions at the end.  Per panel of columns k0..k0+15:
//   (a) the panel's column tile goes through LDS to one row per lane (16
//       registers) and the oracle's unblocked sweep runs over it: the pivot
//       is the row of largest magnitude among positions >= k (a wave max on
//       DPP, ties to the smallest position), the pivot row's entries reach
//       the other lanes by readlane, and each row below forms its
//       multiplier and updates the panel's remaining columns (a full,
//       finite panel is swept first without branches and swept again with
//       them only if a pivot or a tie rules the first sweep out); the
//       finished panel then stays in its tile's registers as one row per
//       lane;
//   (b) the pivot rows' entries right of the panel (A12, written to LDS by
//       the lanes holding them) give U12 = L11^{-1} A12 by forward
//       substitution, one lane per column;
//   (c) the trailing update on the f64 MFMA: every row takes the
//       multipliers of the steps before its own position times U12, so that
//       the rows below the pivot rows take the whole update, the pivot rows
//       their rows of U12 and the rows finished by earlier panels nothing
//       (a non-finite U12 is handled by selects instead).
// The oracle's operations with the updates right of a panel delayed to (c)
// and fused multiply-adds: the factors agree to rounding, the interchanges
// wherever the pivot candidates differ by more than the rounding, and on
// data whose every intermediate value is exact the results are the oracle's
// bit for bit.
// One step of a wave max of non-negative, non-NaN doubles: lanes without a
// source lane read 0 (bound_ctrl), which never exceeds the maximum.  The max
// is a single v_max_f64 (the operands are never signalling NaNs, so the
// quieting that fmax adds is not needed).
template <int CTRL>
__device__ __forceinline__ double dpp_max_step(double x) {
  const long long xb = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_mov_dpp((int)xb, CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(xb >> 32), CTRL, 0xf, 0xf, true);
  const double y = __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
  double r;
  asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(x), "v"(y));
  return r;
}

template <int CTRL, int RM>
__device__ __forceinline__ int dpp_min_step(int x) {
  return min(x, __builtin_amdgcn_update_dpp(0x7fffffff, x, CTRL, RM, 0xf, false));
}

// A byte offset past the end of every descriptor the kernel below builds (a
// descriptor covers one instance's matrix, far below 2 GiB): buffer loads at
// it read zero.
constexpr int kOobOffset = 0x7ffffff0;

template <bool PIVOT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_getrf_mf(
    int m, int n, View C, View D, double *dA, int *ipiv, int *info, long long sC, long long sD,
    long long sdA, long long sip) {
  C = at_batch(C, sC);
  D = at_batch(D, sD);
  const long long b = blockIdx.y;
  double *dAb = dA ? dA + b * sdA : nullptr;
  int *ipb = ipiv ? ipiv + b * sip : nullptr;
  __shared__ double sp[64][17];  // one column tile, a row per line
  __shared__ double su[20][49];  // A12 of the panel's pivot rows, then U12 (rows 16..19: discarded writes)
  __shared__ __align__(16) double slT[16][16];  // L11 transposed (below its diagonal)
  __shared__ int spos[64];       // position of each row (-1 beyond m)
  __shared__ int sipv[64];       // ipiv and dA, stored at the end
  __shared__ double sdav[64];
  __shared__ double szero;       // a zero that masked reads read (the select
                                 // is on the address, so no read waits under a branch)
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
  const int mn = min(m, n);
  const int tr = (m + 15) >> 4, tc = (n + 15) >> 4;
  const brsrc rC = make_rsrc(C.p, 8LL * ((C.ai + m + 15) & ~15) * C.cn);
  const brsrc rD = make_rsrc(D.p, 8LL * ((D.ai + m + 15) & ~15) * D.cn);
  // The loads go out column tile by column tile, the first panel's first,
  // so that its sweep starts while the others are in flight; an element
  // outside the matrix is read at an offset past the end of the buffer,
  // which reads as zero (no select waiting on the load).
  d4 A[4][4];
#pragma unroll
  for (int J = 0; J < 4; ++J)
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * t + g + 4 * r, j = 16 * J + c;
        const int off = (i < m && j < n) ? 8 * (int)pm_off(C.ai + i, C.aj + j, C.cn) : kOobOffset;
        A[t][J][r] = bload(rC, off, 0);
      }
  const bool live = l < m;
  int pos = l;
  int inf = 0;
  if (l == 0) szero = 0.0;
  // The panel loop runs as a loop (its body once in the code, which keeps
  // the kernel within the instruction cache): the current panel's column
  // tile is always A[.][0], the trailing ones A[.][1..ntr], and the tile
  // columns rotate by one at the end of each panel, by four in all.
  const int np = (mn + 15) >> 4;
#pragma unroll 1
  for (int p = 0; p < np; ++p) {
    const int k0 = 16 * p;
    const int wd = min(16, mn - k0);
    const int ntr = tc - 1 - p;  // trailing column tiles
    // (a) the panel, one row per lane
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) sp[16 * t + g + 4 * r][c] = A[t][0][r];
    wave_sync();
    double pr[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) pr[j] = sp[l][j];
    wave_sync();
    // A full panel whose entries are all finite and below 2^1000 in
    // magnitude first takes a sweep without branches (its steps overlap in
    // the instruction schedule): partial pivoting keeps every multiplier at
    // most 1, so the panel stays finite unless a pivot is zero, and a row
    // that is not below the pivot may take a zero update.  A zero, tiny or
    // huge pivot or a tie for the maximum (in binary32) marks the sweep as
    // unusable; the panel is then read again from LDS and swept with the
    // branches below.
    bool safe = true;
    if (PIVOT && wd == 16) {
      bool okl = true;
#pragma unroll
      for (int j = 0; j < 16; ++j) okl = okl && fabs(pr[j]) < 0x1p1000;
      if (__ballot(!okl) == 0) {
        const int pos0 = pos;
        bool bad = false;
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
          const int k = k0 + kk;
          const double v = pr[kk];
          const bool cand = live && pos >= k;
          const float kf = cand ? (float)fabs(v) : -1.0f;
          float x = kf;
          asm volatile(
              "s_nop 1\n\tv_max_f32_dpp %0, %0, %0 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
              "s_nop 1\n\tv_max_f32_dpp %0, %0, %0 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
              "s_nop 1\n\tv_max_f32_dpp %0, %0, %0 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
              "s_nop 1\n\tv_max_f32_dpp %0, %0, %0 row_shr:8 row_mask:0xf bank_mask:0xf\n\t"
              "s_nop 1\n\tv_max_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
              "s_nop 1\n\tv_max_f32_dpp %0, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
              "s_nop 1"
              : "+v"(x));
          const float mxf = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), 63));
          const unsigned long long hit = __ballot(cand && kf == mxf);
          const int pl = __builtin_ctzll(hit);
          const int ppos = __builtin_amdgcn_readlane(pos, pl);
          pos = pos == k ? ppos : pos;
          pos = l == pl ? k : pos;
          const double piv = readlane_d(v, pl);
          const unsigned int pex = (unsigned int)(__builtin_bit_cast(unsigned long long, piv) >> 52) & 0x7ffu;
          bad = bad || (hit & (hit - 1)) != 0 || pex <= 23u || pex >= 2023u;
          double r = __builtin_amdgcn_rcp(piv);
          r = fma(r, fma(-piv, r, 1.0), r);
          const double invp = fma(r, fma(-piv, r, 1.0), r);
          sipv[k] = ppos;  // (every lane stores the same value)
          sdav[k] = invp;
          double pc[16];
#pragma unroll
          for (int j = kk + 1; j < 16; ++j) pc[j] = readlane_d(pr[j], pl);
          const bool below = live && pos > k;
          const double mult = v * invp;
          const double mm = below ? mult : 0.0;
          pr[kk] = below ? mult : pr[kk];
#pragma unroll
          for (int j = kk + 1; j < 16; ++j) pr[j] = fma(-mm, pc[j], pr[j]);
        }
        safe = bad;
        if (bad) {
          pos = pos0;
#pragma unroll
          for (int j = 0; j < 16; ++j) pr[j] = sp[l][j];
        }
      }
    }
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      if (!safe || kk >= wd) continue;
      const int k = k0 + kk;
      const double v = pr[kk];
      int pl = k, ppos = k;
      if (PIVOT) {
        // the oracle's scan keeps position k unless a later row is strictly
        // larger: a NaN at position k is the pivot, a NaN elsewhere never
        // is.  Otherwise the wave max runs on |v| rounded to binary32 (a
        // rounding that keeps the order, ties aside; NaN keys drop out of
        // the max): a single lane at the maximum is the pivot, several are
        // resolved by their binary64 values, then by position.
        const int kl = __builtin_ctzll(__ballot(live && pos == k));
        const bool knan = __builtin_isnan(readlane_d(v, kl));
        {
          const bool cand = live && pos >= k;
          const float kf = cand ? (float)fabs(v) : -1.0f;
          float x = kf;
          asm volatile(
              "s_nop 1\n\tv_max_f32_dpp %0, %0, %0 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
              "s_nop 1\n\tv_max_f32_dpp %0, %0, %0 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
              "s_nop 1\n\tv_max_f32_dpp %0, %0, %0 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
              "s_nop 1\n\tv_max_f32_dpp %0, %0, %0 row_shr:8 row_mask:0xf bank_mask:0xf\n\t"
              "s_nop 1\n\tv_max_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
              "s_nop 1\n\tv_max_f32_dpp %0, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
              "s_nop 1"
              : "+v"(x));
          const float mxf = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), 63));
          unsigned long long hit = __ballot(cand && kf == mxf);
          if (hit & (hit - 1)) {
            const bool h = (hit >> l) & 1;
            double y = h ? fabs(v) : -1.0;
            y = dpp_max_step<0x111>(y);
            y = dpp_max_step<0x112>(y);
            y = dpp_max_step<0x114>(y);
            y = dpp_max_step<0x118>(y);
            y = dpp_max_step<0x142>(y);
            y = dpp_max_step<0x143>(y);
            const double mx = readlane_d(y, 63);
            hit = __ballot(h && fabs(v) == mx);
          }
          pl = __builtin_ctzll(hit);
          if (hit & (hit - 1)) {
            int q = (hit >> l) & 1 ? pos : 0x7fffffff;
            q = dpp_min_step<0x111, 0xf>(q);
            q = dpp_min_step<0x112, 0xf>(q);
            q = dpp_min_step<0x114, 0xf>(q);
            q = dpp_min_step<0x118, 0xf>(q);
            q = dpp_min_step<0x142, 0xa>(q);
            q = dpp_min_step<0x143, 0xc>(q);
            const int best = __builtin_amdgcn_readlane(q, 63);
            pl = __builtin_ctzll(__ballot(live && pos == best));
          }
        }
        if (knan) pl = kl;
        ppos = __builtin_amdgcn_readlane(pos, pl);
        if (pos == k) pos = ppos;
        if (l == pl) pos = k;
      }
      const double piv = readlane_d(v, pl);
      if (piv == 0.0 && inf == 0) inf = k + 1;
      // 1/piv: the hardware reciprocal and two Newton steps (within an ulp)
      // for pivots of moderate magnitude (binary exponent within +-1000),
      // the division otherwise (zero, infinite, NaN or extreme pivots keep
      // the oracle's special values)
      double invp;
      const unsigned int pex = (unsigned int)(__builtin_bit_cast(unsigned long long, piv) >> 52) & 0x7ffu;
      if (pex > 23u && pex < 2023u) {
        double r = __builtin_amdgcn_rcp(piv);
        r = fma(r, fma(-piv, r, 1.0), r);
        invp = fma(r, fma(-piv, r, 1.0), r);
      } else {
        invp = 1.0 / piv;
      }
      if (l == 0) {
        sipv[k] = ppos;
        sdav[k] = invp;
      }
      double pc[16];
#pragma unroll
      for (int j = kk + 1; j < 16; ++j) pc[j] = readlane_d(pr[j], pl);
      if (live && pos > k) {
        const double mult = v * invp;
        pr[kk] = mult;
#pragma unroll
        for (int j = kk + 1; j < 16; ++j) pr[j] = fma(-mult, pc[j], pr[j]);
      }
    }
    // the panel back into its column tile; the multipliers (transposed, for
    // the MFMA's left operand), the pivot rows and the positions to LDS
    spos[l] = live ? pos : -1;
#pragma unroll
    for (int j = 0; j < 16; ++j) sp[l][j] = pr[j];
    const int kp = pos - k0;
    if (live && kp >= 0 && kp < wd) {
#pragma unroll
      for (int j = 0; j < 16; ++j) slT[j][kp] = pr[j];
    }
    wave_sync();
    // the finished panel stays in its column tile's registers as the lane's
    // row (register r of tile t holds column 4t + r): rows are what the
    // final stores take
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) A[t][0][r] = pr[4 * t + r];
    if (ntr > 0) {
    // (b) A12 of the pivot rows: each lane writes the entries of its rows,
    // a pivot row's to its row of su and the others' to a row past the
    // sixteenth (unconditional stores, distinct addresses per lane)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (t >= tr) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int q = spos[16 * t + g + 4 * r] - k0;
        const int qd = (q >= 0 && q < wd) ? q : 16 + g;
#pragma unroll
        for (int J = 1; J < 4; ++J)
          if (J <= ntr) su[qd][16 * (J - 1) + c] = A[t][J][r];
      }
    }
    wave_sync();
    // U12 = L11^{-1} A12 by columns of L11 (rows wd..15 of the result zero)
    if (l < 16 * ntr) {
      double x[16];
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) x[kk] = su[kk][l];
#pragma unroll
      for (int j = 0; j < 15; ++j) {
        const double xj = x[j];
#pragma unroll
        for (int kk = j + 1; kk < 16; ++kk) x[kk] = fma(-slT[j][kk], xj, x[kk]);
      }
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) su[kk][l] = kk < wd ? x[kk] : 0.0;
    }
    wave_sync();
    // (c) the trailing update.  With a finite U12 (the usual case) every
    // row's multipliers of the steps before its own position go into X, so
    // that the rows below the pivot rows take the whole update, each pivot
    // row the updates of the steps before its own (its row of U12, to
    // rounding) and every other row a zero update (its values kept, up to
    // the sign of a zero).  Otherwise only the rows below the pivot rows are
    // updated, by a select, and the pivot rows take U12 from LDS, as in the
    // oracle a non-finite U12 entry never reaches a finished row.
    d4 Y[4];
    bool fin = true;
#pragma unroll
    for (int J = 1; J < 4; ++J)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        Y[J][r] = -su[g + 4 * r][16 * (J - 1) + c];
        fin = fin && (J > ntr || __builtin_isfinite(Y[J][r]));
      }
    const bool allfin = __ballot(!fin) == 0;
    // X: row i's multipliers of the steps j it takes (rows at positions
    // above k0 + j with a finite U12, rows below the pivot rows otherwise)
    const int xlo = allfin ? k0 : k0 + wd - 1;
    d4 X[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int ps = spos[16 * t + c];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = g + 4 * r;
        X[t][r] = *((j < wd && ps > xlo + (allfin ? j : 0)) ? &sp[16 * t + c][j] : &szero);
      }
    }
    const unsigned long long act = __ballot(live && pos >= k0 + wd);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (t >= tr) continue;
#pragma unroll
      for (int J = 1; J < 4; ++J) {
        if (J > ntr) continue;
        d4 acc = A[t][J];
#pragma unroll
        for (int r = 0; r < 4; ++r) acc = mfma(X[t][r], Y[J][r], acc);
        if (allfin) {
          A[t][J] = acc;
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if ((act >> (16 * t + g + 4 * r)) & 1) A[t][J][r] = acc[r];
        }
      }
    }
    if (!allfin) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (t >= tr) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int q = spos[16 * t + g + 4 * r] - k0;
          const bool pv = q >= 0 && q < wd;
          const int qq = pv ? q : 0;
#pragma unroll
          for (int J = 1; J < 4; ++J) {
            if (J > ntr) continue;
            const double u = su[qq][16 * (J - 1) + c];
            if (pv) A[t][J][r] = u;
          }
        }
      }
    }
    wave_sync();
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const d4 f = A[t][0];
      A[t][0] = A[t][1];
      A[t][1] = A[t][2];
      A[t][2] = A[t][3];
      A[t][3] = f;
    }
  }
#pragma unroll 1
  for (int q = np; q < 4; ++q) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const d4 f = A[t][0];
      A[t][0] = A[t][1];
      A[t][1] = A[t][2];
      A[t][2] = A[t][3];
      A[t][3] = f;
    }
  }
  // rows to their final positions, one column per store so that the
  // lanes' rows fill whole panel columns: the factored column tiles hold
  // rows already, the others (columns right of the last panel) go through
  // LDS
#pragma unroll
  for (int J = 0; J < 4; ++J) {
    if (J >= tc) continue;
    if (J < np) {
      if (live) {
#pragma unroll
        for (int j = 0; j < 16; ++j)
          if (16 * J + j < n)
            bstore(rD, 8 * (int)pm_off(D.ai + pos, D.aj + 16 * J + j, D.cn), 0, A[j >> 2][J][j & 3]);
      }
    } else {
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) sp[16 * t + g + 4 * r][c] = A[t][J][r];
      wave_sync();
      if (live) {
#pragma unroll
        for (int j = 0; j < 16; ++j)
          if (16 * J + j < n) bstore(rD, 8 * (int)pm_off(D.ai + pos, D.aj + 16 * J + j, D.cn), 0, sp[l][j]);
      }
      wave_sync();
    }
  }
  if (l < mn) {
    if (ipb) ipb[l] = sipv[l];
    if (dAb) dAb[l] = sdav[l];
  }
  if (info && l == 0) info[b] = inf;
}

// ---------------------------------------------------------------- getrf, blocked
// LU with partial pivoting of an m-by-n matrix with max(m, n) > 64 (up to
// 256), blocked by panels of 16 columns as in §5.2.2 (getrf: a panel
// factorization, the row interchanges, the triangular solve for the block
// row of U, then the trailing matrix updated by a gemm), one workgroup of 256
// threads per instance, D updated in place after a copy of C:
//   (a) the panel's rows k0..m-1 are held one per thread (16 registers);
//       for each of its columns the pivot is the first row of largest
//       magnitude (a wave argmax on DPP, then over the four waves through
//       LDS), row k and the pivot row trade places through LDS, which also
//       broadcasts the pivot row, and the rows below form their multipliers
//       and update the panel's remaining columns;
//   (b) the panel's interchanges are applied to every column outside the
//       panel (one thread per column, in order);
//   (c) U12 = L11^{-1} A12 by forward substitution with the unit lower L11,
//       one thread per column, the result also kept in LDS;
//   (d) A22 -= L21 U12 on the f64 MFMA, one wave per 16x16 block of A22
//       (the transposed product, so that each lane's accumulator is one
//       element of D).
// These are the oracle's operations with the updates of the columns right
// of a panel delayed to (d), so the factors agree to rounding and the
// interchanges agree wherever the pivot candidates differ by more than the
// rounding; on data whose every intermediate value is exact the results are
// the oracle's bit for bit.
constexpr int kGetrfBigT = 256;  // threads per instance = the largest m
constexpr int kGetrfBigN = 256;  // the largest n

template <bool PIVOT>
__global__ __launch_bounds__(kGetrfBigT) __attribute__((amdgpu_waves_per_eu(4))) void k_getrf_big(int m, int n, View C, View D, double *dA,
                                                          int *ipiv, int *info, long long sC,
                                                          long long sD, long long sdA, long long sip) {
  C = at_batch(C, sC);
  D = at_batch(D, sD);
  const long long b = blockIdx.y;
  double *dAb = dA ? dA + b * sdA : nullptr;
  int *ipb = ipiv ? ipiv + b * sip : nullptr;
  __shared__ double u12[16][kGetrfBigN + 1];  // block row of U right of the panel
  __shared__ double l11[16][17];              // the panel's unit lower block
  __shared__ double prow[2][2][16];           // [parity][row k, pivot row][column]
  __shared__ double wkey[2][4];
  __shared__ int wpos[2][4];
  __shared__ int spiv[16];
  __shared__ int cont[kGetrfBigT];  // row contents while composing interchanges
  __shared__ int pdst[32], psrc[32];
  __shared__ int npair;
  const int w = wave_id();
  const int mn = min(m, n);
  // D through a buffer descriptor: a 32-bit byte offset per access (the
  // panels holding rows 0..ai+m-1 of D)
  const brsrc rD = make_rsrc(D.p, 8LL * ((D.ai + m + 15) & ~15) * D.cn);
  auto doff = [&](int i, int j) { return 8 * (int)pm_off(D.ai + i, D.aj + j, D.cn); };
  auto dld = [&](int i, int j) { return bload(rD, doff(i, j), 0); };
  auto dst = [&](int i, int j, double x) { bstore(rD, doff(i, j), 0, x); };
  for (int e = threadIdx.x; e < m * n; e += kGetrfBigT) {
    const int i = e % m, j = e / m;
    dst(i, j, C.p[pm_off(C.ai + i, C.aj + j, C.cn)]);
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __syncthreads();
  int inf = 0;
  for (int k0 = 0; k0 < mn; k0 += 16) {
    const int wd = min(16, mn - k0);
    // the thread index passes through an empty asm each panel, so that what
    // is derived from it is recomputed here rather than kept live (and
    // spilled) across the whole panel loop
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    const int l = t & 63;
    // (a) the panel, one row per thread
    const int row = k0 + t;
    const bool live = row < m;
    const int rc = min(row, m - 1);
    double r[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const double x = dld(rc, min(k0 + c, n - 1));  // clamped: no branch
      r[c] = (live && c < wd) ? x : 0.0;
    }
    for (int kk = 0; kk < wd; ++kk) {
      const int k = k0 + kk;
      const int par = kk & 1;
      double v = r[0];
#pragma unroll
      for (int e = 1; e < 16; ++e) v = kk == e ? r[e] : v;
      int pt = kk;  // panel-local index of the pivot row
      if (PIVOT) {
        // the oracle's scan keeps row k unless a later row is strictly
        // larger: a NaN in row k wins, a NaN elsewhere never does
        const double av = __builtin_isnan(v) ? (t == kk ? __builtin_inf() : -0.5) : fabs(v);
        double key = (live && t >= kk) ? av : -1.0;
        int kp = t;
        argmax_step<0x111, 0xf>(key, kp);  // row_shr:1
        argmax_step<0x112, 0xf>(key, kp);  // row_shr:2
        argmax_step<0x114, 0xf>(key, kp);  // row_shr:4
        argmax_step<0x118, 0xf>(key, kp);  // row_shr:8: lane 15 of a row holds its best
        argmax_step<0x142, 0xa>(key, kp);  // row_bcast:15 into rows 1 and 3
        argmax_step<0x143, 0xc>(key, kp);  // row_bcast:31 into rows 2 and 3
        if (l == 63) {
          wkey[par][w] = key;
          wpos[par][w] = kp;
        }
        __syncthreads();
        double bk = wkey[par][0];
        pt = wpos[par][0];
#pragma unroll
        for (int q = 1; q < 4; ++q) {
          const double k2 = wkey[par][q];
          const int p2 = wpos[par][q];
          if (k2 > bk || (k2 == bk && p2 < pt)) {
            bk = k2;
            pt = p2;
          }
        }
      }
      // rows k and k0 + pt trade places; prow[par][1] is the pivot row
      if (t == kk) {
#pragma unroll
        for (int c = 0; c < 16; ++c) prow[par][0][c] = r[c];
      }
      if (t == pt) {
#pragma unroll
        for (int c = 0; c < 16; ++c) prow[par][1][c] = r[c];
      }
      __syncthreads();
      if (pt != kk && (t == kk || t == pt)) {
        const int src = t == kk ? 1 : 0;
#pragma unroll
        for (int c = 0; c < 16; ++c) r[c] = prow[par][src][c];
      }
      const double piv = prow[par][1][kk];
      const double invp = 1.0 / piv;
      if (t == 0) {
        spiv[kk] = k0 + pt;
        if (ipb) ipb[k] = k0 + pt;
        if (dAb) dAb[k] = invp;
        if (piv == 0.0 && inf == 0) inf = k + 1;
      }
      if (live && t > kk) {
        double vk = r[0];
#pragma unroll
        for (int e = 1; e < 16; ++e) vk = kk == e ? r[e] : vk;
        const double mult = vk * invp;
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          const double upd = r[c] - mult * prow[par][1][c];
          r[c] = c == kk ? mult : (c > kk && c < wd) ? upd : r[c];
        }
      }
    }
    if (live) {
#pragma unroll
      for (int c = 0; c < 16; ++c)
        if (c < wd) dst(row, k0 + c, r[c]);
    }
    if (t < wd) {
#pragma unroll
      for (int c = 0; c < 16; ++c) l11[t][c] = r[c];
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __syncthreads();
    // (b) the interchanges in the columns outside the panel, composed into
    // one permutation of the (at most 32) rows they touch: one thread lists
    // (destination, source) pairs, then every column moves its values with
    // all loads in flight at once
    if (PIVOT) {
      if (t == 0) {
        for (int kk = 0; kk < wd; ++kk) {
          cont[k0 + kk] = k0 + kk;
          cont[spiv[kk]] = spiv[kk];
        }
        for (int kk = 0; kk < wd; ++kk) {
          const int ra = k0 + kk, rb = spiv[kk];
          const int x = cont[ra];
          cont[ra] = cont[rb];
          cont[rb] = x;
        }
        int np2 = 0;
        for (int kk = 0; kk < wd; ++kk)
          for (int h = 0; h < 2; ++h) {
            const int rr = h == 0 ? k0 + kk : spiv[kk];
            if (cont[rr] != rr) {
              pdst[np2] = rr;
              psrc[np2] = cont[rr];
              ++np2;
              cont[rr] = rr;  // listed
            }
          }
        npair = np2;
      }
      __syncthreads();
      const int j = t, np2 = npair;
      if (np2 > 0 && j < n && (j < k0 || j >= k0 + wd)) {
        // pairs past the last are the last again (the same value to the
        // same place), so that every access is unconditional
        double vals[32];
#pragma unroll
        for (int q = 0; q < 32; ++q) vals[q] = dld(psrc[min(q, np2 - 1)], j);
#pragma unroll
        for (int q = 0; q < 32; ++q) dst(pdst[min(q, np2 - 1)], j, vals[q]);
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      __syncthreads();
    }
    // (c) U12 = L11^{-1} A12, one thread per column right of the panel
    const int c0 = k0 + wd, nc = n - c0;
    if (t < nc) {
      const int j = c0 + t;
      double x[16];
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) {
        const double y = dld(k0 + min(kk, wd - 1), j);
        x[kk] = kk < wd ? y : 0.0;
      }
#pragma unroll
      for (int jj = 0; jj < 15; ++jj)
#pragma unroll
        for (int kk = jj + 1; kk < 16; ++kk) x[kk] -= l11[kk][jj] * x[jj];
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) u12[kk][t] = kk < wd ? x[kk] : 0.0;
      // stored from LDS (the thread's own entries) in a loop over the
      // panel's rows: a store per register under a condition each made the
      // compiler keep every register and address live at once
      for (int kk = 0; kk < wd; ++kk) dst(k0 + kk, j, u12[kk][t]);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __syncthreads();
    // (d) A22 -= L21 U12 for rows c0..m-1 (the rows below the panel start at
    // k0 + wd = c0) and columns c0..n-1
    const int nr = m - c0;
    if (nr > 0 && nc > 0) {
      // work item: one 16-row block of A22 and four 16-column blocks; the
      // row block's L21 fragments are loaded once, then all 16 accumulator
      // loads are in flight together
      const int tr = (nr + 15) >> 4, tcn = (nc + 15) >> 4, tg = (tcn + 3) >> 2;
      const int i = l & 15, g = l >> 4;
      for (int item = w; item < tr * tg; item += kGetrfBigT / 64) {
        const int I0 = c0 + 16 * (item % tr), Jg = 64 * (item / tr);
        const int ii = I0 + i;
        double bv[4];
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const int kidx = 4 * st + g;
          const double y = dld(min(ii, m - 1), k0 + min(kidx, wd - 1));
          bv[st] = (kidx < wd && ii < m) ? y : 0.0;
        }
        d4 acc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int jj = c0 + Jg + 16 * u + 4 * q + g;
            const double x = dld(min(ii, m - 1), min(jj, n - 1));
            acc[u][q] = (ii < m && jj < n) ? x : 0.0;
          }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int jl = Jg + 16 * u + i;
#pragma unroll
          for (int st = 0; st < 4; ++st) {
            const double a = u12[4 * st + g][min(jl, kGetrfBigN)];
            acc[u] = mfma(-(jl < nc ? a : 0.0), bv[st], acc[u]);
          }
        }
        if (ii < m) {
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int jj = c0 + Jg + 16 * u + 4 * q + g;
              if (jj < n) dst(ii, jj, acc[u][q]);
            }
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __syncthreads();
  }
  if (info && threadIdx.x == 0) info[b] = inf;
}

// ---------------------------------------------------------------- gelqf, one wave, MFMA
// LQ factorization (LAPACK's compact form, as the oracle's) of an m-by-n
// matrix with 32 < max(m, n) <= 64, blocked by panels of 16 rows as in
// §5.2.2 (gelqf), one wave per instance.  The matrix is held transposed in
// registers, as 16 T-tiles of A^T (register r of lane (c, g) of tile AT[j][i]
// holds A[16i + c][16j + g + 4r]), so that the block update of the rows below
// a panel is three T-tile products on the f64 MFMA.  Per panel of rows
// k0..k0+15:
//   (a) the panel goes through LDS to lane i + 16q holding row k0 + i,
//       columns 16q..16q+15 (16 registers); for each of its rows k: the
//       squared norm right of column k and every row's product with the
//       reflector are sums of four lanes' parts (row swaps), the
//       oracle's scalars follow, and the reflector reaches the lanes of each
//       column quarter by a DPP row broadcast; the rows below it in the panel
//       subtract; the finished rows are stored at once (later panels do not
//       touch them);
//   (b) the reflectors V (unit leading entry) go to LDS, their Gram matrix
//       V V^T is formed on the MFMA and T (H_0 ... H_15 = I - V^T T V) by the
//       forward recurrence, one lane per row of T;
//   (c) every row tile below: A2 -= ((A2 V^T) T) V, as W^T = V A2^T,
//       Z^T = T^T W^T and A2^T -= V^T Z^T on the MFMA.
// The row tiles rotate by one per panel so that the panel is always AT[.][0]
// (the loop's body once in the code).  The oracle's reflectors with the sums
// in another order: the factors agree to rounding.
__device__ __forceinline__ int newbcast_i(int x, int kk) {
  switch (kk) {  // kk is a constant where this is called
    case 0: return __builtin_amdgcn_update_dpp(0, x, 0x150, 0xf, 0xf, false);
    case 1: return __builtin_amdgcn_update_dpp(0, x, 0x151, 0xf, 0xf, false);
    case 2: return __builtin_amdgcn_update_dpp(0, x, 0x152, 0xf, 0xf, false);
    case 3: return __builtin_amdgcn_update_dpp(0, x, 0x153, 0xf, 0xf, false);
    case 4: return __builtin_amdgcn_update_dpp(0, x, 0x154, 0xf, 0xf, false);
    case 5: return __builtin_amdgcn_update_dpp(0, x, 0x155, 0xf, 0xf, false);
    case 6: return __builtin_amdgcn_update_dpp(0, x, 0x156, 0xf, 0xf, false);
    case 7: return __builtin_amdgcn_update_dpp(0, x, 0x157, 0xf, 0xf, false);
    case 8: return __builtin_amdgcn_update_dpp(0, x, 0x158, 0xf, 0xf, false);
    case 9: return __builtin_amdgcn_update_dpp(0, x, 0x159, 0xf, 0xf, false);
    case 10: return __builtin_amdgcn_update_dpp(0, x, 0x15a, 0xf, 0xf, false);
    case 11: return __builtin_amdgcn_update_dpp(0, x, 0x15b, 0xf, 0xf, false);
    case 12: return __builtin_amdgcn_update_dpp(0, x, 0x15c, 0xf, 0xf, false);
    case 13: return __builtin_amdgcn_update_dpp(0, x, 0x15d, 0xf, 0xf, false);
    case 14: return __builtin_amdgcn_update_dpp(0, x, 0x15e, 0xf, 0xf, false);
    default: return __builtin_amdgcn_update_dpp(0, x, 0x15f, 0xf, 0xf, false);
  }
}

// lane kk's value of each row of 16 lanes, to that row's every lane
__device__ __forceinline__ double newbcast_d(double x, int kk) {
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = newbcast_i((int)b, kk), hi = newbcast_i((int)(b >> 32), kk);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// sum over the four lanes l, l^16, l^32, l^48 with the row swaps of gfx950:
// permlane16_swap of (x, x) leaves rows (0,0,2,2) in one register and
// (1,1,3,3) in the other, whose sum is x + x[l^16]; permlane32_swap does the
// same with rows (0,1,0,1) and (2,3,2,3)
__device__ __forceinline__ double swap_sum(double x, bool by32) {
  const long long b = __builtin_bit_cast(long long, x);
  const unsigned lo = (unsigned)b, hi = (unsigned)(b >> 32);
  unsigned a0, a1, h0, h1;
  if (by32) {
    const auto pl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto ph = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    a0 = pl[0]; a1 = pl[1]; h0 = ph[0]; h1 = ph[1];
  } else {
    const auto pl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto ph = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    a0 = pl[0]; a1 = pl[1]; h0 = ph[0]; h1 = ph[1];
  }
  const double u = __builtin_bit_cast(double, ((unsigned long long)h0 << 32) | a0);
  const double v = __builtin_bit_cast(double, ((unsigned long long)h1 << 32) | a1);
  return u + v;
}

__device__ __forceinline__ double quarter_sum(double x) {
  return swap_sum(swap_sum(x, false), true);
}

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_gelqf_mf(
    int m, int n, View C, View D, double *tau, long long sC, long long sD, long long stau) {
  C = at_batch(C, sC);
  D = at_batch(D, sD);
  const long long b = blockIdx.y;
  double *taub = tau + b * stau;
  __shared__ double sp[64][17];  // the panel: [column][row]
  __shared__ double sv[16][65];  // V: [reflector][column]
  __shared__ double sg[16][17];  // the Gram matrix, then T
  __shared__ double stk[16];     // tau of the panel's steps
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;  // also (row i, column quarter q) of the panel sweep
  const int mn = min(m, n);
  const int tr = (m + 15) >> 4;
  const brsrc rC = make_rsrc(C.p, 8LL * ((C.ai + m + 15) & ~15) * C.cn);
  const brsrc rD = make_rsrc(D.p, 8LL * ((D.ai + m + 15) & ~15) * D.cn);
  // A^T in registers; an element outside the matrix reads as zero (an
  // offset past the end of the buffer)
  d4 AT[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * i + c, col = 16 * j + g + 4 * r;
        const int off = (row < m && col < n) ? 8 * (int)pm_off(C.ai + row, C.aj + col, C.cn) : kOobOffset;
        AT[j][i][r] = bload(rC, off, 0);
      }
  const int np = (mn + 15) >> 4;
  // the panel loop is unrolled: a row tile's registers are dead once it has
  // been a panel (its rows are stored from the sweep) or, below the last
  // panel (m > n), once it is stored
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    if (p >= np) {
      if (p < tr) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = 16 * p + c, col = 16 * j + g + 4 * r;
            if (row < m && col < n) bstore(rD, 8 * (int)pm_off(D.ai + row, D.aj + col, D.cn), 0, AT[j][p][r]);
          }
      }
      continue;
    }
    const int k0 = 16 * p;
    const int wd = min(16, mn - k0);
    const int ntr = tr - 1 - p;  // row tiles below the panel
    // (a) the panel, lane i + 16q holding row k0 + i, columns 16q + jj
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
      for (int r = 0; r < 4; ++r) sp[16 * j + g + 4 * r][c] = AT[j][p][r];
    }
    wave_sync();
    double pr[16];
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) pr[jj] = sp[16 * g + jj][c];
    wave_sync();
    const bool qgt = g > p, qge = g >= p;  // quarter right of / holding the diagonal
    const bool liverow = k0 + c < m;
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      if (kk >= wd) continue;
      // row kk's squared norm right of column k0 + kk
      double ps = 0.0;
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        const bool in = jj > kk ? qge : qgt;
        ps = in ? fma(pr[jj], pr[jj], ps) : ps;
      }
      ps = quarter_sum(ps);
      const double xn2 = readlane_d(ps, kk);
      const double alpha = readlane_d(pr[kk], kk + 16 * p);
      double tk = 0.0, scale = 0.0, beta = alpha;
      if (sqrt(xn2) != 0.0) {
        beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
        tk = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      if (l == 0) stk[kk] = tk;
      // the reflector (v = 0 left of column k, 1 at it) from row kk's lanes
      // to every lane of the same column quarter
      double vb[16];
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        const bool right = jj > kk ? qge : qgt, at = jj == kk && g == p;
        const double vv = right ? pr[jj] * scale : (at ? 1.0 : 0.0);
        vb[jj] = newbcast_d(vv, kk);
      }
      if (c == kk) {
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
          const bool right = jj > kk ? qge : qgt, at = jj == kk && g == p;
          pr[jj] = right ? vb[jj] : (at ? beta : pr[jj]);
        }
      }
      // the rows below: w = tau (row . v), row -= w v
      double d = 0.0;
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) d = fma(pr[jj], vb[jj], d);
      d = quarter_sum(d);
      if (liverow && c > kk) {
        const double w = tk * d;
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) pr[jj] = fma(-w, vb[jj], pr[jj]);
      }
    }
    // the finished rows to D (one column per store: whole panel columns),
    // tau, and the reflectors to LDS for the block update
    if (liverow) {
#pragma unroll
      for (int jj = 0; jj < 16; ++jj)
        if (16 * g + jj < n) bstore(rD, 8 * (int)pm_off(D.ai + k0 + c, D.aj + 16 * g + jj, D.cn), 0, pr[jj]);
    }
    wave_sync();
    if (l < wd) taub[k0 + l] = stk[l];
    if (ntr > 0) {
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        const int col = 16 * g + jj, kc = k0 + c;
        sv[c][col] = (c < wd && col > kc) ? pr[jj] : ((c < wd && col == kc) ? 1.0 : 0.0);
      }
      wave_sync();
      // (b) G = V V^T, then T, one lane per row
      d4 G = zero4();
#pragma unroll
      for (int J = p; J < 4; ++J) {
        d4 VT;
#pragma unroll
        for (int r = 0; r < 4; ++r) VT[r] = sv[c][16 * J + g + 4 * r];
        G = mfma_tn(VT, VT, G);
      }
      // T = (I + diag(tau) striu(G))^{-1} diag(tau): the inverse of T is
      // diag(1/tau) + striu(G) (the forward recurrence in closed form),
      // written without dividing by tau so that a zero tau (an identity
      // reflector) needs no care; the unit upper triangular inverse by the
      // register back substitution (sp as its staging area)
      d4 U;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = g + 4 * r;
        U[r] = c > a ? stk[a] * G[r] : (c == a ? 1.0 : 0.0);
      }
      if (l < 16) sg[1][l] = 1.0;
      wave_sync();
      const d4 Vi = trtri_tile_upper(U, &sg[1][0], &sp[0][0], &sg[0][0]);
      d4 TT;
      const double tc = stk[c];
#pragma unroll
      for (int r = 0; r < 4; ++r) TT[r] = Vi[r] * tc;
      // (c) W^T = V A2^T and Z^T = T^T W^T for every row tile below
      d4 Zt[3];
#pragma unroll
      for (int i = p + 1; i < 4; ++i) {
        if (i >= tr) continue;
        d4 Wt = zero4();
#pragma unroll
        for (int J = p; J < 4; ++J) {
          d4 VT;
#pragma unroll
          for (int r = 0; r < 4; ++r) VT[r] = sv[c][16 * J + g + 4 * r];
          Wt = mfma_tn(VT, AT[J][i], Wt);
        }
        Zt[i - p - 1] = -mfma_tn(TT, Wt, zero4());
      }
      // A2^T -= V^T Z^T, one column tile of V at a time
#pragma unroll
      for (int J = p; J < 4; ++J) {
        d4 VN;
#pragma unroll
        for (int r = 0; r < 4; ++r) VN[r] = sv[g + 4 * r][16 * J + c];
#pragma unroll
        for (int i = p + 1; i < 4; ++i) {
          if (i >= tr) continue;
          AT[J][i] = mfma_tn(VN, Zt[i - p - 1], AT[J][i]);
        }
      }
      wave_sync();
    }
  }
}

// ---------------------------------------------------------------- gelqf, blocked
// LQ factorization (Householder reflectors, LAPACK's compact form) of an
// m-by-n matrix with max(m, n) > 64 (up to 256), blocked by panels of 16
// rows (§5.2.2: the paper's gelqf blocks its reflectors), one workgroup of
// 256 threads per instance, D updated in place after a copy of C:
//   (a) the panel's rows are held one column per thread (16 registers);
//       each reflector's squared norm and each remaining row's product with
//       it are workgroup sums (a shuffle tree per wave, then the four
//       partial sums through LDS in a fixed order), and the reflector is
//       applied to the panel's remaining rows;
//   (b) the reflectors V (unit leading entry) go to LDS, their Gram matrix
//       V V^T is formed on the f64 MFMA, and the upper triangular T with
//       H_0 H_1 ... H_{w-1} = I - V^T T V by the forward recurrence
//       T[0:k,k] = -tau_k T[0:k,0:k] (V V^T)[0:k,k], one lane per row of T;
//   (c) every 16-row block below the panel: A2 -= ((A2 V^T) T) V, as
//       W^T = V A2^T, Z^T = T^T W^T and A2 -= Z V on the MFMA.
// The oracle's reflectors with the products in another order: the factors
// agree to rounding.
constexpr int kGelqfBigT = 256;  // threads per instance = the largest n
constexpr int kGelqfBigN = 256;

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

__global__ __launch_bounds__(kGelqfBigT) __attribute__((amdgpu_waves_per_eu(4)))
void k_gelqf_big(int m, int n, View C, View D, double *tau, long long sC, long long sD,
                 long long stau) {
  C = at_batch(C, sC);
  D = at_batch(D, sD);
  const long long b = blockIdx.y;
  double *taub = tau + b * stau;
  __shared__ double vl[16][kGelqfBigN + 1];  // the panel's reflectors, columns r0..n-1
  __shared__ double tt[16][17];              // T
  __shared__ double gg[16][17];              // V V^T
  __shared__ double red[2][16][4];           // [parity][sum][wave]
  __shared__ double bc[2];                   // the diagonal entry alpha
  __shared__ double stk[16];                 // the panel's tau
  const int w = wave_id();
  const int mn = min(m, n);
  const brsrc rD = make_rsrc(D.p, 8LL * ((D.ai + m + 15) & ~15) * D.cn);
  auto doff = [&](int i, int j) { return 8 * (int)pm_off(D.ai + i, D.aj + j, D.cn); };
  auto dld = [&](int i, int j) { return bload(rD, doff(i, j), 0); };
  auto dst = [&](int i, int j, double x) { bstore(rD, doff(i, j), 0, x); };
  for (int e = threadIdx.x; e < m * n; e += kGelqfBigT) {
    const int i = e % m, j = e / m;
    dst(i, j, C.p[pm_off(C.ai + i, C.aj + j, C.cn)]);
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __syncthreads();
  for (int r0 = 0; r0 < mn; r0 += 16) {
    const int wd = min(16, mn - r0);
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));  // recomputed per panel, not kept live
    const int l = t & 63;
    const int j = t;  // this thread's column
    const bool col = j >= r0 && j < n;
    const int jc = min(max(j, r0), n - 1);
    // (a) the panel's rows
    double P[16];
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const double x = dld(r0 + min(kk, wd - 1), jc);
      P[kk] = (col && kk < wd) ? x : 0.0;
    }
    for (int kk = 0; kk < wd; ++kk) {
      const int k = r0 + kk;
      const int par = kk & 1;
      double pk = P[0];
#pragma unroll
      for (int e = 1; e < 16; ++e) pk = kk == e ? P[e] : pk;
      const double sw = wave_sum((col && j > k) ? pk * pk : 0.0);
      if (l == 0) red[par][0][w] = sw;
      if (j == k) bc[par] = pk;
      __syncthreads();
      const double ss = ((red[par][0][0] + red[par][0][1]) + red[par][0][2]) + red[par][0][3];
      const double alpha = bc[par];
      const double xn = sqrt(ss);
      double tk = 0.0, sc = 1.0, beta = alpha;
      if (xn != 0.0) {
        beta = -copysign(sqrt(alpha * alpha + ss), alpha);
        tk = (beta - alpha) / beta;
        sc = 1.0 / (alpha - beta);
      }
      // the reflector (v_k = 1, zero left of k) and row k of the panel
      const double v = j > k ? pk * sc : (j == k ? 1.0 : 0.0);
      const double rowk = j > k ? v : (j == k ? beta : pk);
#pragma unroll
      for (int e = 0; e < 16; ++e) P[e] = (kk == e && col) ? rowk : P[e];
      if (t == 0) {
        taub[k] = tk;
        stk[kk] = tk;
      }
      if (tk != 0.0) {
        // w_i = sum_{j >= k} P[i][j] v_j for the panel rows below k, then
        // P[i][j] -= tau w_i v_j
        double part[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) part[e] = (col && e > kk && e < wd && j >= k) ? P[e] * v : 0.0;
#pragma unroll
        for (int e = 1; e < 16; ++e) part[e] = wave_sum(part[e]);
        if (l == 0) {
#pragma unroll
          for (int e = 1; e < 16; ++e) red[par][e][w] = part[e];
        }
        __syncthreads();
#pragma unroll
        for (int e = 1; e < 16; ++e) {
          if (e > kk && e < wd) {
            const double wi = tk * (((red[par][e][0] + red[par][e][1]) + red[par][e][2]) + red[par][e][3]);
            P[e] = (col && j >= k) ? P[e] - wi * v : P[e];
          }
        }
      }
    }
    // the panel's rows back to D; the reflectors to LDS
    if (col) {
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) {
        const int k = r0 + kk;
        vl[kk][j - r0] = kk < wd ? (j > k ? P[kk] : (j == k ? 1.0 : 0.0)) : 0.0;
      }
      for (int kk = 0; kk < wd; ++kk) {
        double x = P[0];
#pragma unroll
        for (int e = 1; e < 16; ++e) x = kk == e ? P[e] : x;
        dst(r0 + kk, j, x);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __syncthreads();
    const int ncv = n - r0;  // columns of V
    const int rb0 = r0 + wd, nrow = m - rb0;
    if (nrow > 0) {
      const int i = l & 15, g = l >> 4;
      // (b) V V^T (wave 0), then T (lanes 0..15 of wave 0)
      if (w == 0) {
        d4 G = zero4();
        for (int J = 0; J < ncv; J += 4) {
          const int jj = J + g;
          const double x = jj < ncv ? vl[i][min(jj, kGelqfBigN)] : 0.0;
          G = mfma(x, x, G);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) gg[g + 4 * r][i] = G[r];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (l < 16) {
          const int a = l;
          double trow[16];
#pragma unroll
          for (int kk = 0; kk < 16; ++kk) {
            const double tk = kk < wd ? stk[kk] : 0.0;
            double sm = 0.0;
#pragma unroll
            for (int bb = 0; bb < kk; ++bb) sm = (bb >= a) ? sm + trow[bb] * gg[bb][kk] : sm;
            trow[kk] = kk == a ? tk : (kk > a ? -tk * sm : 0.0);
          }
#pragma unroll
          for (int kk = 0; kk < 16; ++kk) tt[a][kk] = (a < wd && kk < wd) ? trow[kk] : 0.0;
        }
      }
      __syncthreads();
      // (c) A2 -= ((A2 V^T) T) V, one 16-row block per wave at a time
      const int nrb = (nrow + 15) >> 4;
      for (int rb = w; rb < nrb; rb += kGelqfBigT / 64) {
        const int ii = rb0 + 16 * rb + i;
        const int iic = min(ii, m - 1);
        d4 Wt = zero4();  // W^T = V A2^T, T-tile [reflector][row]
        for (int J = 0; J < ncv; J += 16) {
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            const int jj = J + 4 * s4 + g;
            const double a = jj < ncv ? vl[i][min(jj, kGelqfBigN)] : 0.0;
            const double y = dld(iic, r0 + min(jj, ncv - 1));
            Wt = mfma(a, (ii < m && jj < ncv) ? y : 0.0, Wt);
          }
        }
        d4 Zt = zero4();  // Z^T = T^T W^T
#pragma unroll
        for (int r = 0; r < 4; ++r) Zt = mfma(tt[g + 4 * r][i], Wt[r], Zt);
        for (int J = 0; J < ncv; J += 16) {
          d4 acc;
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            const int jj = J + 4 * s4 + g;
            const double y = dld(iic, r0 + min(jj, ncv - 1));
            acc[s4] = (ii < m && jj < ncv) ? y : 0.0;
          }
          const int jv = J + i;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const double vt = jv < ncv ? vl[g + 4 * r][min(jv, kGelqfBigN)] : 0.0;
            acc = mfma(-vt, Zt[r], acc);
          }
          if (ii < m) {
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
              const int jj = J + 4 * s4 + g;
              if (jj < ncv) dst(ii, r0 + jj, acc[s4]);
            }
          }
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __syncthreads();
  }
}

// ---------------------------------------------------------------- gelqf
// LQ factorization by Householder reflectors of an m-by-n matrix, m, n <= 64
// (§5.2.2, gelqf; unblocked): one wave per instance with lane i holding row
// i in NC registers (n rounded up to 16).  Step k: every lane forms the squared norm of its row
// right of column k in ascending column order (the oracle's order; lane k's
// is the one used), the oracle's scalars follow, lane k scales its row into
// the reflector, whose entries reach the other lanes by readlane, and every
// row below forms its product with the reflector and subtracts.  tau goes
// to dA.  Contraction is off, as in the oracle, so each operation rounds as
// the oracle's does.  Column k is register 16*qb + kk, selected as in getrf.
template <int NC>
__global__ __launch_bounds__(64) void k_gelqf(int m, int n, View C, View D, double *tau,
                                              long long sC, long long sD, long long stau) {
#pragma clang fp contract(off)
  C = at_batch(C, sC);
  D = at_batch(D, sD);
  const long long b = blockIdx.y;
  double *taub = tau + b * stau;
  const int l = lane_id();
  const bool live = l < m;
  const int lr = min(l, m - 1);
  double r[NC];  // NC: n rounded up to a multiple of 16
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double x = C.p[pm_off(C.ai + lr, C.aj + min(c, n - 1), C.cn)];  // clamped: no branch
    r[c] = (live && c < n) ? x : 0.0;
  }
  const int mn = min(m, n);
#pragma unroll
  for (int qb = 0; qb < NC / 16; ++qb) {
    for (int kk = 0; kk < 16; ++kk) {
      const int k = 16 * qb + kk;
      if (k >= mn) break;
      double rk = r[16 * qb];
#pragma unroll
      for (int e = 1; e < 16; ++e) rk = kk == e ? r[16 * qb + e] : rk;
      double ss = 0.0;
#pragma unroll
      for (int c = 16 * qb; c < NC; ++c)
        if (c < n) ss = c > k ? ss + r[c] * r[c] : ss;
      const double alpha = readlane_d(rk, k);
      const double ssk = readlane_d(ss, k);
      double t = 0.0;
      if (sqrt(ssk) != 0.0) {
        const double beta = -copysign(sqrt(alpha * alpha + ssk), alpha);
        t = (beta - alpha) / beta;
        const double sc = 1.0 / (alpha - beta);
        const bool me = l == k;
#pragma unroll
        for (int c = 16 * qb; c < NC; ++c)
          if (c < n) r[c] = (me && c > k) ? r[c] * sc : r[c];
#pragma unroll
        for (int e = 0; e < 16; ++e) r[16 * qb + e] = (me && kk == e) ? beta : r[16 * qb + e];
      }
      if (l == 0) taub[k] = t;
      if (t == 0.0) continue;
      // rows below: w = (r[k] + sum_{c>k} r[c] v[c]) t, then r -= w v (v[k] = 1)
      // (the reflector's entries are read twice by readlane rather than
      // held: 48 of them would not fit next to the row)
      const bool below = live && l > k;
      double w = rk;
#pragma unroll
      for (int c = 16 * qb; c < NC; ++c)
        if (c < n) w = c > k ? w + r[c] * readlane_d(r[c], k) : w;
      w *= t;
#pragma unroll
      for (int c = 16 * qb; c < NC; ++c) {
        if (c < n) {
          const bool diag = c - 16 * qb == kk;
          const double upd = diag ? r[c] - w : r[c] - w * readlane_d(r[c], k);
          r[c] = (below && c >= k) ? upd : r[c];
        }
      }
    }
  }
  if (live) {
#pragma unroll
    for (int c = 0; c < NC; ++c)
      if (c < n) D.p[pm_off(D.ai + l, D.aj + c, D.cn)] = r[c];
  }
}

int launch_gelqf(int batch, int m, int n, const blasfeo_dmat *sC, int ci, int cj,
                 const blasfeo_dmat *sD, int di, int dj, hipStream_t st) {
  if (batch == 0 || m == 0 || n == 0) return 0;
  View C = make_view(sC, ci, cj, m, n);
  View D = make_view(sD, di, dj, m, n);
  // the one-wave kernel addresses C and D through 32-bit buffer offsets
  const bool small_bufs = 8LL * ((C.ai + m + 15) & ~15) * C.cn < kOobOffset &&
                          8LL * ((D.ai + m + 15) & ~15) * D.cn < kOobOffset;
  if (m > 64 || n > 64)
    hipLaunchKernelGGL(k_gelqf_big, dim3(1, batch), dim3(kGelqfBigT), 0, st, m, n, C, D, sD->dA,
                       batch_stride(sC), batch_stride(sD), batch_stride(sD));
  else if ((m > 32 || n > 32) && small_bufs)
    hipLaunchKernelGGL(k_gelqf_mf, dim3(1, batch), dim3(64), 0, st, m, n, C, D, sD->dA,
                       batch_stride(sC), batch_stride(sD), batch_stride(sD));
  else
    hipLaunchKernelGGL(n <= 16 ? k_gelqf<16> : n <= 32 ? k_gelqf<32> : k_gelqf<64>, dim3(1, batch), dim3(64), 0,
                       st, m, n, C, D, sD->dA, batch_stride(sC), batch_stride(sD), batch_stride(sD));
  return launch_status();
}

int launch_getrf(int batch, int m, int n, const blasfeo_dmat *sC, int ci, int cj,
                 const blasfeo_dmat *sD, int di, int dj, bool pivot, int *ipiv,
                 int *info, hipStream_t st) {
  if (batch == 0) return 0;
  if (m == 0 || n == 0) {
    if (info) hipLaunchKernelGGL(k_fill_int, dim3((batch + 255) / 256), dim3(256), 0, st, info, batch, 0);
    return info ? launch_status() : 0;
  }
  View C = make_view(sC, ci, cj, m, n);
  View D = make_view(sD, di, dj, m, n);
  const dim3 g(1, batch);
  const long long sdA = batch_stride(sD), sip = m < n ? m : n;
  // the one-wave kernel addresses C and D through 32-bit buffer offsets
  const bool small_bufs = 8LL * ((C.ai + m + 15) & ~15) * C.cn < kOobOffset &&
                          8LL * ((D.ai + m + 15) & ~15) * D.cn < kOobOffset;
  if ((m > 32 || n > 32) && (m > 64 || n > 64 || small_bufs)) {
    if (m <= 64 && n <= 64) {
      if (pivot)
        hipLaunchKernelGGL(k_getrf_mf<true>, g, dim3(64), 0, st, m, n, C, D, sD->dA, ipiv, info,
                           batch_stride(sC), batch_stride(sD), sdA, sip);
      else
        hipLaunchKernelGGL(k_getrf_mf<false>, g, dim3(64), 0, st, m, n, C, D, sD->dA, ipiv, info,
                           batch_stride(sC), batch_stride(sD), sdA, sip);
      return launch_status();
    }
    if (pivot)
      hipLaunchKernelGGL(k_getrf_big<true>, g, dim3(kGetrfBigT), 0, st, m, n, C, D, sD->dA, ipiv,
                         info, batch_stride(sC), batch_stride(sD), sdA, sip);
    else
      hipLaunchKernelGGL(k_getrf_big<false>, g, dim3(kGetrfBigT), 0, st, m, n, C, D, sD->dA, ipiv,
                         info, batch_stride(sC), batch_stride(sD), sdA, sip);
    return launch_status();
  }
  // the unblocked kernel, compiled for the column count rounded up to 16
  auto kern = pivot ? (n <= 16 ? k_getrf<true, 16> : n <= 32 ? k_getrf<true, 32> : k_getrf<true, 64>)
                    : (n <= 16 ? k_getrf<false, 16> : n <= 32 ? k_getrf<false, 32> : k_getrf<false, 64>);
  hipLaunchKernelGGL(kern, g, dim3(64), 0, st, m, n, C, D, sD->dA, ipiv, info, batch_stride(sC),
                     batch_stride(sD), sdA, sip);
  return launch_status();
}

// ---------------------------------------------------------------- launchers

int launch_gemm(bool syrk, int batch, int m, int n, int k, double alpha,
                const blasfeo_dmat *sA, int ai, int aj, const blasfeo_dmat *sB,
                int bi, int bj, double beta, const blasfeo_dmat *sC, int ci,
                int cj, const blasfeo_dmat *sD, int di, int dj,
                hipStream_t st, bool nn = false) {
  if (batch == 0 || m == 0 || n == 0) return 0;
  const int tm = (m + 15) / 16, tn = (n + 15) / 16;
  const int tiles = syrk ? tm * (tm + 1) / 2 : tm * tn;
  dim3 grid((tiles + GW - 1) / GW, batch);
  View A = make_view(sA, ai, aj, m, k);
  View B = nn ? make_view(sB, bi, bj, k, n) : make_view(sB, bi, bj, n, k);
  View C = make_view(sC, ci, cj, m, n);
  View D = make_view(sD, di, dj, m, n);
  if (nn)
    hipLaunchKernelGGL((k_gemm_nt<false, true>), grid, dim3(64 * GW), 0, st, m, n,
                       k, alpha, A, B, beta, C, D, batch_stride(sA),
                       batch_stride(sB), batch_stride(sC), batch_stride(sD));
  else if (syrk)
    hipLaunchKernelGGL(k_gemm_nt<true>, grid, dim3(64 * GW), 0, st, m, n, k,
                       alpha, A, B, beta, C, D, batch_stride(sA),
                       batch_stride(sB), batch_stride(sC), batch_stride(sD));
  else
    hipLaunchKernelGGL(k_gemm_nt<false>, grid, dim3(64 * GW), 0, st, m, n,
                       k, alpha, A, B, beta, C, D, batch_stride(sA),
                       batch_stride(sB), batch_stride(sC), batch_stride(sD));
  return launch_status();
}

int launch_trsm(int batch, int m, int n, double alpha, const blasfeo_dmat *sA,
                int ai, int aj, const blasfeo_dmat *sB, int bi, int bj,
                const blasfeo_dmat *sD, int di, int dj, hipStream_t st) {
  if (batch == 0 || m == 0 || n == 0) return 0;
  const int strips = (m + 15) / 16;
  dim3 grid((strips + GW - 1) / GW, batch);
  View A = make_view(sA, ai, aj, n, n);
  View B = make_view(sB, bi, bj, m, n);
  View D = make_view(sD, di, dj, m, n);
  hipLaunchKernelGGL(k_trsm_rltn, grid, dim3(64 * GW), 0, st, m, n, alpha,
                     A, B, D, batch_stride(sA), batch_stride(sB),
                     batch_stride(sD));
  return launch_status();
}

int launch_trmm(int batch, int m, int n, double alpha, const blasfeo_dmat *sA,
                int ai, int aj, const blasfeo_dmat *sB, int bi, int bj,
                const blasfeo_dmat *sD, int di, int dj, hipStream_t st) {
  if (batch == 0 || m == 0 || n == 0) return 0;
  const int tiles = ((m + 15) / 16) * ((n + 15) / 16);
  dim3 grid((tiles + GW - 1) / GW, batch);
  View A = make_view(sA, ai, aj, n, n);
  View B = make_view(sB, bi, bj, m, n);
  View D = make_view(sD, di, dj, m, n);
  hipLaunchKernelGGL(k_trmm_rlnn, grid, dim3(64 * GW), 0, st, m, n, alpha, A, B, D,
                     batch_stride(sA), batch_stride(sB), batch_stride(sD));
  return launch_status();
}

// True if the two sub-matrices share storage: same panel buffer and
// intersecting row and column ranges.
static bool overlaps(const blasfeo_dmat *x, int xi, int xj, int xr, int xc,
                     const blasfeo_dmat *y, int yi, int yj, int yr, int yc) {
  if (x->pA != y->pA || xr == 0 || xc == 0 || yr == 0 || yc == 0) return false;
  return xi < yi + yr && yi < xi + xr && xj < yj + yc && yj < xj + xc;
}

int launch_potrf(int batch, int m, int k, const blasfeo_dmat *sA, int ai,
                 int aj, const blasfeo_dmat *sB, int bi, int bj,
                 const blasfeo_dmat *sC, int ci, int cj,
                 const blasfeo_dmat *sD, int di, int dj, int *info,
                 hipStream_t st, int n = -1) {
  // n < 0: square (n = m); otherwise the stacked m-by-n factorization
  // (rows m <= 64: one wave with the factor in registers; else the
  // left-looking workgroup kernel), the same kernels in both cases
  const bool square = n < 0 || n == m;
  if (n < 0) n = m;
  if (batch == 0) return 0;
  if (n == 0) {
    // a fill kernel rather than a memset node, so that the call can be
    // captured into a graph
    if (info) hipLaunchKernelGGL(k_fill_int, dim3((batch + 255) / 256), dim3(256), 0, st, info, batch, 0);
    return info ? launch_status() : 0;
  }
  View A{}, B{};
  if (k > 0) {
    A = make_view(sA, ai, aj, m, k);
    B = make_view(sB, bi, bj, m, k);
  }
  View C = make_view(sC, ci, cj, m, n);
  View D = make_view(sD, di, dj, m, n);
  const long long ssA = k > 0 ? batch_stride(sA) : 0, ssB = k > 0 ? batch_stride(sB) : 0;
  const long long ssC = batch_stride(sC), ssD = batch_stride(sD);
  const dim3 g(1, batch);
  (void)square;
  switch ((m + 15) / 16) {
    case 1: hipLaunchKernelGGL(k_potrf_reg<1>, g, dim3(64), 0, st, m, n, k, A, B, C, D, sD->dA, info, ssA, ssB, ssC, ssD, ssD); break;
    case 2: hipLaunchKernelGGL(k_potrf_reg<2>, g, dim3(64), 0, st, m, n, k, A, B, C, D, sD->dA, info, ssA, ssB, ssC, ssD, ssD); break;
    case 3: hipLaunchKernelGGL(k_potrf_reg<3>, g, dim3(64), 0, st, m, n, k, A, B, C, D, sD->dA, info, ssA, ssB, ssC, ssD, ssD); break;
    case 4: hipLaunchKernelGGL(k_potrf_reg<4>, g, dim3(64), 0, st, m, n, k, A, B, C, D, sD->dA, info, ssA, ssB, ssC, ssD, ssD); break;
    default:
      hipLaunchKernelGGL(k_potrf_l, g, dim3(64 * GW), 0, st, m, n, k, A, B, C, D, sD->dA, info,
                         ssA, ssB, ssC, ssD, ssD);
  }
  return launch_status();
}

}  // namespace bh

using namespace bh;

extern "C" {

void blasfeo_dgemm_nt(int m, int n, int k, double alpha,
                      struct blasfeo_dmat *sA, int ai, int aj,
                      struct blasfeo_dmat *sB, int bi, int bj, double beta,
                      struct blasfeo_dmat *sC, int ci, int cj,
                      struct blasfeo_dmat *sD, int di, int dj) {
  if (m < 0) return set_error(-1);
  if (n < 0) return set_error(-2);
  if (k < 0) return set_error(-3);
  if (!operand_ok(sA, ai, aj, m, k)) return set_error(-5);
  if (!operand_ok(sB, bi, bj, n, k)) return set_error(-8);
  if (!operand_ok(sC, ci, cj, m, n)) return set_error(-12);
  if (!operand_ok(sD, di, dj, m, n)) return set_error(-15);
  set_error(launch_gemm(false, 1, m, n, k, alpha, sA, ai, aj, sB, bi, bj,
                        beta, sC, ci, cj, sD, di, dj, tl_stream()));
}

void blasfeo_dgemm_nn(int m, int n, int k, double alpha,
                      struct blasfeo_dmat *sA, int ai, int aj,
                      struct blasfeo_dmat *sB, int bi, int bj, double beta,
                      struct blasfeo_dmat *sC, int ci, int cj,
                      struct blasfeo_dmat *sD, int di, int dj) {
  if (m < 0) return set_error(-1);
  if (n < 0) return set_error(-2);
  if (k < 0) return set_error(-3);
  if (!operand_ok(sA, ai, aj, m, k)) return set_error(-5);
  if (!operand_ok(sB, bi, bj, k, n)) return set_error(-8);
  if (!operand_ok(sC, ci, cj, m, n)) return set_error(-12);
  if (!operand_ok(sD, di, dj, m, n)) return set_error(-15);
  set_error(launch_gemm(false, 1, m, n, k, alpha, sA, ai, aj, sB, bi, bj,
                        beta, sC, ci, cj, sD, di, dj, tl_stream(), true));
}

void blasfeo_dgetrf_pivot(int m, int n, struct blasfeo_dmat *sC, int ci,
                          int cj, struct blasfeo_dmat *sD, int di, int dj,
                          int *ipiv) {
  if (m < 0 || m > 256) return set_error(-1);
  if (n < 0 || n > 256) return set_error(-2);
  if (!operand_ok(sC, ci, cj, m, n)) return set_error(-3);
  if (!operand_ok(sD, di, dj, m, n)) return set_error(-6);
  if (m > 0 && n > 0 && !sD->dA) return set_error(-6);
  if (m > 0 && n > 0 && !ipiv) return set_error(-9);
  const int e = launch_getrf(1, m, n, sC, ci, cj, sD, di, dj, true, ipiv, nullptr, tl_stream());
  if (e == 0) sD->use_dA = (di == 0 && dj == 0);
  set_error(e);
}

void blasfeo_dgetrf_nopivot(int m, int n, struct blasfeo_dmat *sC, int ci,
                            int cj, struct blasfeo_dmat *sD, int di, int dj) {
  if (m < 0 || m > 256) return set_error(-1);
  if (n < 0 || n > 256) return set_error(-2);
  if (!operand_ok(sC, ci, cj, m, n)) return set_error(-3);
  if (!operand_ok(sD, di, dj, m, n)) return set_error(-6);
  if (m > 0 && n > 0 && !sD->dA) return set_error(-6);
  const int e = launch_getrf(1, m, n, sC, ci, cj, sD, di, dj, false, nullptr, nullptr, tl_stream());
  if (e == 0) sD->use_dA = (di == 0 && dj == 0);
  set_error(e);
}

void blasfeo_dgelqf(int m, int n, struct blasfeo_dmat *sC, int ci, int cj,
                    struct blasfeo_dmat *sD, int di, int dj) {
  if (m < 0 || m > 256) return set_error(-1);
  if (n < 0 || n > 256) return set_error(-2);
  if (!operand_ok(sC, ci, cj, m, n)) return set_error(-3);
  if (!operand_ok(sD, di, dj, m, n)) return set_error(-6);
  if (m > 0 && n > 0 && !sD->dA) return set_error(-6);
  set_error(launch_gelqf(1, m, n, sC, ci, cj, sD, di, dj, tl_stream()));
}

void blasfeo_dsyrk_ln(int m, int k, double alpha, struct blasfeo_dmat *sA,
                      int ai, int aj, struct blasfeo_dmat *sB, int bi,
                      int bj, double beta, struct blasfeo_dmat *sC, int ci,
                      int cj, struct blasfeo_dmat *sD, int di, int dj) {
  if (m < 0) return set_error(-1);
  if (k < 0) return set_error(-2);
  if (!operand_ok(sA, ai, aj, m, k)) return set_error(-4);
  if (!operand_ok(sB, bi, bj, m, k)) return set_error(-7);
  if (!operand_ok(sC, ci, cj, m, m)) return set_error(-11);
  if (!operand_ok(sD, di, dj, m, m)) return set_error(-14);
  set_error(launch_gemm(true, 1, m, m, k, alpha, sA, ai, aj, sB, bi, bj,
                        beta, sC, ci, cj, sD, di, dj, tl_stream()));
}

void blasfeo_dtrsm_rltn(int m, int n, double alpha, struct blasfeo_dmat *sA,
                        int ai, int aj, struct blasfeo_dmat *sB, int bi,
                        int bj, struct blasfeo_dmat *sD, int di, int dj) {
  if (m < 0) return set_error(-1);
  if (n < 0) return set_error(-2);
  if (!operand_ok(sA, ai, aj, n, n)) return set_error(-4);
  if (!operand_ok(sB, bi, bj, m, n)) return set_error(-7);
  if (!operand_ok(sD, di, dj, m, n)) return set_error(-10);
  set_error(launch_trsm(1, m, n, alpha, sA, ai, aj, sB, bi, bj, sD, di, dj,
                        tl_stream()));
}

void blasfeo_dtrmm_rlnn(int m, int n, double alpha, struct blasfeo_dmat *sA,
                        int ai, int aj, struct blasfeo_dmat *sB, int bi,
                        int bj, struct blasfeo_dmat *sD, int di, int dj) {
  if (m < 0) return set_error(-1);
  if (n < 0) return set_error(-2);
  if (!operand_ok(sA, ai, aj, n, n)) return set_error(-4);
  if (!operand_ok(sB, bi, bj, m, n)) return set_error(-7);
  if (!operand_ok(sD, di, dj, m, n)) return set_error(-10);
  if (overlaps(sD, di, dj, m, n, sB, bi, bj, m, n) ||
      overlaps(sD, di, dj, m, n, sA, ai, aj, n, n))
    return set_error(-10);
  set_error(launch_trmm(1, m, n, alpha, sA, ai, aj, sB, bi, bj, sD, di, dj,
                        tl_stream()));
}

void blasfeo_hip_dpotrf_l_info(int m, struct blasfeo_dmat *sC, int ci,
                               int cj, struct blasfeo_dmat *sD, int di,
                               int dj, int *info) {
  if (m < 0) return set_error(-1);
  if (!operand_ok(sC, ci, cj, m, m)) return set_error(-2);
  if (!operand_ok(sD, di, dj, m, m)) return set_error(-5);
  if (m > 0 && !sD->dA) return set_error(-5);
  int e = launch_potrf(1, m, 0, nullptr, 0, 0, nullptr, 0, 0, sC, ci, cj, sD,
                       di, dj, info, tl_stream());
  if (e == 0) sD->use_dA = (di == 0 && dj == 0);
  set_error(e);
}

void blasfeo_dpotrf_l(int m, struct blasfeo_dmat *sC, int ci, int cj,
                      struct blasfeo_dmat *sD, int di, int dj) {
  blasfeo_hip_dpotrf_l_info(m, sC, ci, cj, sD, di, dj, nullptr);
}

void blasfeo_dpotrf_l_mn(int m, int n, struct blasfeo_dmat *sC, int ci,
                         int cj, struct blasfeo_dmat *sD, int di, int dj) {
  if (m < 0) return set_error(-1);
  if (n < 0 || n > m) return set_error(-2);
  if (!operand_ok(sC, ci, cj, m, n)) return set_error(-3);
  if (!operand_ok(sD, di, dj, m, n)) return set_error(-6);
  if (n > 0 && !sD->dA) return set_error(-6);
  int e = launch_potrf(1, m, 0, nullptr, 0, 0, nullptr, 0, 0, sC, ci, cj, sD,
                       di, dj, nullptr, tl_stream(), n);
  if (e == 0) sD->use_dA = (di == 0 && dj == 0);
  set_error(e);
}

void blasfeo_hip_dsyrk_dpotrf_ln_info(int m, int k, struct blasfeo_dmat *sA,
                                      int ai, int aj,
                                      struct blasfeo_dmat *sB, int bi,
                                      int bj, struct blasfeo_dmat *sC,
                                      int ci, int cj,
                                      struct blasfeo_dmat *sD, int di,
                                      int dj, int *info) {
  if (m < 0) return set_error(-1);
  if (k < 0) return set_error(-2);
  if (!operand_ok(sA, ai, aj, m, k)) return set_error(-3);
  if (!operand_ok(sB, bi, bj, m, k)) return set_error(-6);
  if (!operand_ok(sC, ci, cj, m, m)) return set_error(-9);
  if (!operand_ok(sD, di, dj, m, m)) return set_error(-12);
  if (m > 0 && !sD->dA) return set_error(-12);
  int e = launch_potrf(1, m, k, sA, ai, aj, sB, bi, bj, sC, ci, cj, sD, di,
                       dj, info, tl_stream());
  if (e == 0) sD->use_dA = (di == 0 && dj == 0);
  set_error(e);
}

void blasfeo_dsyrk_dpotrf_ln(int m, int k, struct blasfeo_dmat *sA, int ai,
                             int aj, struct blasfeo_dmat *sB, int bi,
                             int bj, struct blasfeo_dmat *sC, int ci,
                             int cj, struct blasfeo_dmat *sD, int di,
                             int dj) {
  blasfeo_hip_dsyrk_dpotrf_ln_info(m, k, sA, ai, aj, sB, bi, bj, sC, ci, cj,
                                   sD, di, dj, nullptr);
}

int blasfeo_hip_dgemm_nt_batched(int batch, int m, int n, int k,
                                 double alpha,
                                 const struct blasfeo_dmat *sA, int ai,
                                 int aj, const struct blasfeo_dmat *sB,
                                 int bi, int bj, double beta,
                                 const struct blasfeo_dmat *sC, int ci,
                                 int cj, const struct blasfeo_dmat *sD,
                                 int di, int dj, void *stream) {
  if (batch < 0 || batch > 65535) return -1;
  if (m < 0) return -2;
  if (n < 0) return -3;
  if (k < 0) return -4;
  if (!operand_ok(sA, ai, aj, m, k)) return -6;
  if (!operand_ok(sB, bi, bj, n, k)) return -9;
  if (!operand_ok(sC, ci, cj, m, n)) return -13;
  if (!operand_ok(sD, di, dj, m, n)) return -16;
  return launch_gemm(false, batch, m, n, k, alpha, sA, ai, aj, sB, bi, bj,
                     beta, sC, ci, cj, sD, di, dj, (hipStream_t)stream);
}

int blasfeo_hip_dgemm_nn_batched(int batch, int m, int n, int k,
                                 double alpha,
                                 const struct blasfeo_dmat *sA, int ai,
                                 int aj, const struct blasfeo_dmat *sB,
                                 int bi, int bj, double beta,
                                 const struct blasfeo_dmat *sC, int ci,
                                 int cj, const struct blasfeo_dmat *sD,
                                 int di, int dj, void *stream) {
  if (batch < 0 || batch > 65535) return -1;
  if (m < 0) return -2;
  if (n < 0) return -3;
  if (k < 0) return -4;
  if (!operand_ok(sA, ai, aj, m, k)) return -6;
  if (!operand_ok(sB, bi, bj, k, n)) return -9;
  if (!operand_ok(sC, ci, cj, m, n)) return -13;
  if (!operand_ok(sD, di, dj, m, n)) return -16;
  return launch_gemm(false, batch, m, n, k, alpha, sA, ai, aj, sB, bi, bj,
                     beta, sC, ci, cj, sD, di, dj, (hipStream_t)stream, true);
}

int blasfeo_hip_dgetrf_batched(int batch, int m, int n,
                               const struct blasfeo_dmat *sC, int ci, int cj,
                               const struct blasfeo_dmat *sD, int di, int dj,
                               int pivot, int *ipiv, int *info, void *stream) {
  if (batch < 0 || batch > 65535) return -1;
  if (m < 0 || m > 256) return -2;
  if (n < 0 || n > 256) return -3;
  if (!operand_ok(sC, ci, cj, m, n)) return -4;
  if (!operand_ok(sD, di, dj, m, n)) return -7;
  if (m > 0 && n > 0 && !sD->dA) return -7;
  if (pivot != 0 && pivot != 1) return -10;
  if (pivot && m > 0 && n > 0 && !ipiv) return -11;
  return launch_getrf(batch, m, n, sC, ci, cj, sD, di, dj, pivot != 0, ipiv, info,
                      (hipStream_t)stream);
}

int blasfeo_hip_dgelqf_batched(int batch, int m, int n,
                               const struct blasfeo_dmat *sC, int ci, int cj,
                               const struct blasfeo_dmat *sD, int di, int dj,
                               void *stream) {
  if (batch < 0 || batch > 65535) return -1;
  if (m < 0 || m > 256) return -2;
  if (n < 0 || n > 256) return -3;
  if (!operand_ok(sC, ci, cj, m, n)) return -4;
  if (!operand_ok(sD, di, dj, m, n)) return -7;
  if (m > 0 && n > 0 && !sD->dA) return -7;
  return launch_gelqf(batch, m, n, sC, ci, cj, sD, di, dj, (hipStream_t)stream);
}

int blasfeo_hip_dsyrk_ln_batched(int batch, int m, int k, double alpha,
                                 const struct blasfeo_dmat *sA, int ai,
                                 int aj, const struct blasfeo_dmat *sB,
                                 int bi, int bj, double beta,
                                 const struct blasfeo_dmat *sC, int ci,
                                 int cj, const struct blasfeo_dmat *sD,
                                 int di, int dj, void *stream) {
  if (batch < 0 || batch > 65535) return -1;
  if (m < 0) return -2;
  if (k < 0) return -3;
  if (!operand_ok(sA, ai, aj, m, k)) return -5;
  if (!operand_ok(sB, bi, bj, m, k)) return -8;
  if (!operand_ok(sC, ci, cj, m, m)) return -12;
  if (!operand_ok(sD, di, dj, m, m)) return -15;
  return launch_gemm(true, batch, m, m, k, alpha, sA, ai, aj, sB, bi, bj,
                     beta, sC, ci, cj, sD, di, dj, (hipStream_t)stream);
}

int blasfeo_hip_dtrsm_rltn_batched(int batch, int m, int n, double alpha,
                                   const struct blasfeo_dmat *sA, int ai,
                                   int aj, const struct blasfeo_dmat *sB,
                                   int bi, int bj,
                                   const struct blasfeo_dmat *sD, int di,
                                   int dj, void *stream) {
  if (batch < 0 || batch > 65535) return -1;
  if (m < 0) return -2;
  if (n < 0) return -3;
  if (!operand_ok(sA, ai, aj, n, n)) return -5;
  if (!operand_ok(sB, bi, bj, m, n)) return -8;
  if (!operand_ok(sD, di, dj, m, n)) return -11;
  return launch_trsm(batch, m, n, alpha, sA, ai, aj, sB, bi, bj, sD, di, dj,
                     (hipStream_t)stream);
}

int blasfeo_hip_dtrmm_rlnn_batched(int batch, int m, int n, double alpha,
                                   const struct blasfeo_dmat *sA, int ai,
                                   int aj, const struct blasfeo_dmat *sB,
                                   int bi, int bj,
                                   const struct blasfeo_dmat *sD, int di,
                                   int dj, void *stream) {
  if (batch < 0 || batch > 65535) return -1;
  if (m < 0) return -2;
  if (n < 0) return -3;
  if (!operand_ok(sA, ai, aj, n, n)) return -6;
  if (!operand_ok(sB, bi, bj, m, n)) return -9;
  if (!operand_ok(sD, di, dj, m, n)) return -12;
  if (overlaps(sD, di, dj, m, n, sB, bi, bj, m, n) ||
      overlaps(sD, di, dj, m, n, sA, ai, aj, n, n))
    return -12;
  return launch_trmm(batch, m, n, alpha, sA, ai, aj, sB, bi, bj, sD, di, dj,
                     (hipStream_t)stream);
}

int blasfeo_hip_dpotrf_l_batched(int batch, int m,
                                 const struct blasfeo_dmat *sC, int ci,
                                 int cj, const struct blasfeo_dmat *sD,
                                 int di, int dj, int *info, void *stream) {
  if (batch < 0 || batch > 65535) return -1;
  if (m < 0) return -2;
  if (!operand_ok(sC, ci, cj, m, m)) return -3;
  if (!operand_ok(sD, di, dj, m, m)) return -6;
  if (m > 0 && !sD->dA) return -6;
  return launch_potrf(batch, m, 0, nullptr, 0, 0, nullptr, 0, 0, sC, ci, cj,
                      sD, di, dj, info, (hipStream_t)stream);
}

int blasfeo_hip_dpotrf_l_mn_batched(int batch, int m, int n,
                                    const struct blasfeo_dmat *sC, int ci,
                                    int cj, const struct blasfeo_dmat *sD,
                                    int di, int dj, int *info, void *stream) {
  if (batch < 0 || batch > 65535) return -1;
  if (m < 0) return -2;
  if (n < 0 || n > m) return -3;
  if (!operand_ok(sC, ci, cj, m, n)) return -4;
  if (!operand_ok(sD, di, dj, m, n)) return -7;
  if (n > 0 && !sD->dA) return -7;
  return launch_potrf(batch, m, 0, nullptr, 0, 0, nullptr, 0, 0, sC, ci, cj,
                      sD, di, dj, info, (hipStream_t)stream, n);
}

}  // extern "C"
