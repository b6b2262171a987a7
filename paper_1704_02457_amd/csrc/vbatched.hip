// Uneven batches of SPD solves A_i X_i = B_i (potrf_l + forward/back
// substitution), driven by a host-side plan: instances are bucketed by order,
// every bucket is one launch of a kernel specialised for its size class, the
// launches are captured once into a hipGraph and replayed.
//
//   n <= 64  : one wavefront per instance, the whole factor register
//              resident (the fused kernel's scheme with the right-hand sides
//              staged in LDS); forward substitution interleaved with the
//              factorization, back substitution on the register tiles.
//   n >  64  : one workgroup per instance, left-looking over block columns
//              (each block of L is produced once: gemm downdate, then the
//              diagonal subroutine or the solve with the diagonal block's
//              inverse -- §4.6), forward substitution fused into the
//              diagonal step, back substitution at the end; instances in
//              longest-first order.
//
// Layout (fixed by the plan): instance i's matrix is a blasfeo_dmat(n_i, n_i)
// chunk; its right-hand sides are a column-major n_i x nrhs block with leading
// dimension round_up(n_i, 16).  The factor L (with its dA) goes to a second
// arena of the same layout, the solutions to a second vector arena.
#include <cstdint>
#include <algorithm>
#include <mutex>
#include <vector>

#include "plan.hpp"

namespace bh {

struct VbArgs {
  const int *ids;          // instances of this bucket
  int count;
  const int *n;            // order of every instance
  const long long *moff;   // matrix chunk offsets (doubles)
  const long long *voff;   // right-hand-side block offsets (doubles)
  const double *A;
  double *L;
  const double *B;
  double *X;
  int nrhs;
  int *info;
  const int *only;  // if not null, instance id runs only where only[id] != 0
  double *wsw;             // n > 64: W_j = V_j^T tiles of instance id at
  const long long *wwoff;  //   wsw + wwoff[id] (256 doubles per block)
};

__device__ __forceinline__ int cn_of(int n) { return (n + 3) & ~3; }
__device__ __forceinline__ int ld_of(int n) { return (n + 15) & ~15; }

// Right-hand-side block j as a T-tile: logical (row p, column c) =
// B[16j + p][c] for c < nrhs, p < n (zero elsewhere).
__device__ __forceinline__ d4 load_rhs(const double *Bb, int ld, int n,
                                       int nrhs, int j) {
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
  d4 z;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int p = 16 * j + g + 4 * r;
    z[r] = (c < nrhs && p < n) ? Bb[(long long)c * ld + p] : 0.0;
  }
  return z;
}

__device__ __forceinline__ void store_rhs(double *Xb, int ld, int n, int nrhs,
                                          int j, const d4 &x) {
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int p = 16 * j + g + 4 * r;
    if (c < nrhs && p < n) Xb[(long long)c * ld + p] = x[r];
  }
}

// ---------------------------------------------------------------- n <= 64

template <int NB, int VW>
__global__ __launch_bounds__(64 * VW) void k_vb_small(VbArgs a) {
  __shared__ DiagLds lds[VW];
  __shared__ double zl[VW][NB][256];  // right-hand sides, then y, then x
  const int w = wave_id();
  const int t = blockIdx.x * VW + w;
  if (t >= a.count) return;
  DiagLds &s = lds[w];
  const int id = a.ids[t];
  if (a.only && a.only[id] == 0) return;
  const int n = a.n[id];
  const int cn = cn_of(n), ld = ld_of(n), pm = (n + 15) >> 4;
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
  constexpr int NT = NB * (NB + 1) / 2;
  const double *Ab = a.A + a.moff[id];
  double *Lb = a.L + a.moff[id];
  const long long panel_doubles = (long long)pm * 16 * cn;
  const brsrc rA = make_rsrc(Ab, 8 * panel_doubles);
  const brsrc rL = make_rsrc(Lb, 8 * (panel_doubles + n));
  const int vo = 8 * l, pS = 8 * 16 * cn;

  d4 T[NT];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * i + c, col = 16 * j + g + 4 * r;
        const bool ok = row < n && col < n && (i != j || c >= g + 4 * r);
        const double x = ok ? bload(rA, vo, i * pS + 8 * (256 * j + 64 * r)) : 0.0;
        T[tix_up(j, i)][r] = x;
      }
  const bool has_rhs = a.nrhs > 0;
  if (has_rhs) {
    const double *Bb = a.B + a.voff[id];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const d4 z = load_rhs(Bb, ld, n, a.nrhs, j);
#pragma unroll
      for (int r = 0; r < 4; ++r) zl[w][j][64 * r + l] = z[r];
    }
  }

  int info = 0;
  d4 Wk[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int nv = min(16, n - 16 * j);
    d4 &D = T[tix_up(j, j)];
    if (nv < 16) pad_identity(D, nv);
    d4 V;
    const int inf = potrf_inv_tile_upper(D, V, s, &Wk[j], (nv + 3) >> 2);
    if (inf && info == 0) info = 16 * j + inf;
    if (l < nv) bstore(rL, vo, 8 * (int)(panel_doubles + 16 * j), s.inv[l]);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * j + c, col = 16 * j + g + 4 * r;
      if (row < n && col < n && c >= g + 4 * r) bstore(rL, vo, j * pS + 8 * (256 * j + 64 * r), D[r]);
    }
#pragma unroll
    for (int i = j + 1; i < NB; ++i) {
      d4 &Ti = T[tix_up(j, i)];
      Ti = mfma_tn(V, Ti, zero4());
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * i + c, col = 16 * j + g + 4 * r;
        if (row < n && col < n) bstore(rL, vo, i * pS + 8 * (256 * j + 64 * r), Ti[r]);
      }
    }
    d4 y;
    if (has_rhs) {  // forward substitution: y(j) = V^T z(j)
      d4 z;
#pragma unroll
      for (int r = 0; r < 4; ++r) z[r] = zl[w][j][64 * r + l];
      y = mfma_tn(V, z, zero4());
#pragma unroll
      for (int r = 0; r < 4; ++r) zl[w][j][64 * r + l] = y[r];
    }
#pragma unroll
    for (int q = j + 1; q < NB; ++q) {
      const d4 nu = neg4(T[tix_up(j, q)]);
#pragma unroll
      for (int i = q; i < NB; ++i)
        T[tix_up(q, i)] = mfma_tn(nu, T[tix_up(j, i)], T[tix_up(q, i)]);
      if (has_rhs) {
        d4 z;
#pragma unroll
        for (int r = 0; r < 4; ++r) z[r] = zl[w][q][64 * r + l];
        z = mfma_tn(nu, y, z);
#pragma unroll
        for (int r = 0; r < 4; ++r) zl[w][q][64 * r + l] = z[r];
      }
    }
  }
  if (has_rhs) {
    // back substitution: x(j) = V_j (y(j) - sum_{i>j} U(j,i) x(i)), with
    // U(j,i) x(i) = (U(j,i)^T)^T x(i) and V_j = W_j^T
    double *Xb = a.X + a.voff[id];
#pragma unroll
    for (int j = NB - 1; j >= 0; --j) {
      d4 acc;
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] = zl[w][j][64 * r + l];
#pragma unroll
      for (int i = j + 1; i < NB; ++i) {
        const d4 ut = transpose_tile(T[tix_up(j, i)], s.tr);
        d4 xi;
#pragma unroll
        for (int r = 0; r < 4; ++r) xi[r] = zl[w][i][64 * r + l];
        acc = mfma_tn(neg4(ut), xi, acc);
      }
      const d4 x = mfma_tn(Wk[j], acc, zero4());
#pragma unroll
      for (int r = 0; r < 4; ++r) zl[w][j][64 * r + l] = x[r];
      store_rhs(Xb, ld, n, a.nrhs, j, x);
    }
  }
  if (a.info && l == 0) a.info[id] = info;
}

// ---------------------------------------------------------------- n > 64

// off-diagonal blocks of a column: block rows per downdate group of a wave,
// and steps of the downdate sum loaded together
constexpr int kVbGroupRows = 2;
constexpr int kVbGroupSteps = 1;
// back substitution: tiles loaded together
constexpr int kVbBackSteps = 1;
// diagonal downdate: steps loaded together
constexpr int kVbDiagSteps = 2;

// Dynamic LDS of k_vb_large: W_j tiles (nbmax x 256), compact y/x blocks
// (nbmax x 16 x nrhs), the current V (256), diagonal scratch.

// Gemm downdate of the upper block T(j,i) of the transposed factor:
//   acc -= sum_{q<j} U(q,j)^T U(q,i),  U(q,x) read back from L,
// UNR block pairs per round so that 2*UNR tile loads are in flight.
template <int UNR>
__device__ __forceinline__ d4 downdate(const PMat &L, int j, int i, d4 acc) {
  int q = 0;
  for (; q + UNR <= j; q += UNR) {
    d4 uj[UNR], ui[UNR];
#pragma unroll
    for (int t = 0; t < UNR; ++t) {
      uj[t] = pm_ldT(L, j, q + t, false);
      ui[t] = i == j ? uj[t] : pm_ldT(L, i, q + t, false);
    }
#pragma unroll
    for (int t = 0; t < UNR; ++t) acc = mfma_tn(neg4(uj[t]), ui[t], acc);
  }
  for (; q < j; ++q) {
    const d4 uj = pm_ldT(L, j, q, false);
    const d4 ui = i == j ? uj : pm_ldT(L, i, q, false);
    acc = mfma_tn(neg4(uj), ui, acc);
  }
  return acc;
}

// Two block rows i0, i1 of column j at once: each U(q,j) is loaded once for
// both, and twice as many independent loads are in flight per step.
__device__ __forceinline__ void downdate_pair(const PMat &L, int j, int i0, int i1,
                                              d4 &acc0, d4 &acc1) {
  for (int q = 0; q < j; ++q) {
    const d4 uj = pm_ldT(L, j, q, false);
    const d4 ua = pm_ldT(L, i0, q, false);
    const d4 ub = pm_ldT(L, i1, q, false);
    acc0 = mfma_tn(neg4(uj), ua, acc0);
    acc1 = mfma_tn(neg4(uj), ub, acc1);
  }
}

// R block rows i0 + r * stride (r < R) of column j at once: one load of
// each U(q,j) serves the whole group, and the tiles of QU steps of q are
// loaded together (steps past j - 1 reload the last one and are multiplied
// by zero; rows past the last block row repeat it and their results are
// dropped by the caller).
template <int R, int QU>
__device__ __forceinline__ void downdate_rows(const PMat &L, int j, int i0,
                                              int stride, int nb, d4 (&acc)[R]) {
  int ir[R];
#pragma unroll
  for (int r = 0; r < R; ++r) ir[r] = min(i0 + r * stride, nb - 1);
  for (int q = 0; q < j; q += QU) {
    d4 uj[QU], ui[QU][R];
#pragma unroll
    for (int u = 0; u < QU; ++u) {
      const int qq = min(q + u, j - 1);
      uj[u] = pm_ldT(L, j, qq, false);
#pragma unroll
      for (int r = 0; r < R; ++r) ui[u][r] = pm_ldT(L, ir[r], qq, false);
    }
#pragma unroll
    for (int u = 0; u < QU; ++u) {
      const d4 m = (u == 0 || q + u < j) ? neg4(uj[u]) : zero4();
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] = mfma_tn(m, ui[u][r], acc[r]);
    }
  }
}

// Gemm downdate as above with the U(q,j) tiles of the column staged in LDS
// (ul, one 16x16 T-tile per 256 doubles): one global tile load per update.
template <int DU>
__device__ __forceinline__ d4 downdate_staged(const double *ul, const PMat &L, int j,
                                              int i, d4 acc) {
  const int l = lane_id();
  int q = 0;
  for (; q + DU <= j; q += DU) {
    d4 ui[DU];
#pragma unroll
    for (int e = 0; e < DU; ++e) ui[e] = pm_ldT(L, i, q + e, false);
#pragma unroll
    for (int e = 0; e < DU; ++e) {
      d4 uj;
#pragma unroll
      for (int r = 0; r < 4; ++r) uj[r] = ul[(q + e) * 256 + 64 * r + l];
      acc = mfma_tn(neg4(uj), ui[e], acc);
    }
  }
  for (; q < j; ++q) {
    d4 uj;
#pragma unroll
    for (int r = 0; r < 4; ++r) uj[r] = ul[q * 256 + 64 * r + l];
    acc = mfma_tn(neg4(uj), pm_ldT(L, i, q, false), acc);
  }
  return acc;
}

// One workgroup of LW waves per instance.  Block column j of L: wave 0
// downdates and factors the diagonal block (and advances the forward
// substitution); then all waves share the off-diagonal blocks of the column:
// gemm downdate and U(j,i) = V_j^T T(j,i).  With ST, the column's U(q,j)
// tiles are first copied to LDS by all waves, so that every later use (the
// diagonal downdate, the forward substitution, every off-diagonal downdate)
// reads them there: the re-reads of the left part of the factor, which
// mostly miss the L2, are halved.
template <int LW, bool ST, bool PAIR = true>
__global__ __launch_bounds__(64 * LW) __attribute__((amdgpu_waves_per_eu(3))) void k_vb_large(VbArgs a, int nbmax) {
  constexpr int DU = ST ? 4 : kVbDiagSteps;
  constexpr int GR = kVbGroupRows, GQ = kVbGroupSteps, BQ = kVbBackSteps;
  extern __shared__ double dyn[];
  __shared__ DiagLds s;
  __shared__ double vsh[256];
  __shared__ int sinfo;
  const int nr = a.nrhs > 0 ? a.nrhs : 1;
  double *yl = dyn;                                // nbmax * 16 * nr
  double *ul = dyn + (long long)nbmax * 16 * nr;   // ST: nbmax * 256
  const int t = blockIdx.x;
  if (t >= a.count) return;
  const int id = a.ids[t];
  if (a.only && a.only[id] == 0) return;
  const int n = a.n[id];
  const int cn = cn_of(n), ld = ld_of(n), pm = (n + 15) >> 4;
  const int nb = pm;
  const int w = wave_id();
  const int l = lane_id();
  const PMat A = make_pmat(a.A + a.moff[id], n, cn);
  const PMat L = make_pmat(a.L + a.moff[id], n, cn);
  double *dAb = a.L + a.moff[id] + (long long)pm * 16 * cn;
  const bool has_rhs = a.nrhs > 0;
  const double *Bb = has_rhs ? a.B + a.voff[id] : nullptr;
  double *wl = a.wsw + a.wwoff[id];
  if (threadIdx.x == 0) sinfo = 0;
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    const int nv = min(16, n - 16 * j);
    if constexpr (ST) {
      for (int q = w; q < j; q += LW) {
        const d4 u = pm_ldT(L, j, q, false);
#pragma unroll
        for (int r = 0; r < 4; ++r) ul[q * 256 + 64 * r + l] = u[r];
      }
      __syncthreads();
    }
    auto ujq = [&](int q) {
      if constexpr (ST) {
        d4 u;
#pragma unroll
        for (int r = 0; r < 4; ++r) u[r] = ul[q * 256 + 64 * r + l];
        return u;
      } else {
        return pm_ldT(L, j, q, false);
      }
    };
    if (w == 0) {
      // diagonal downdate and forward substitution, one load of U(q,j) each
      d4 t0 = pm_ldT(A, j, j, true);
      d4 z = has_rhs ? load_rhs(Bb, ld, n, a.nrhs, j) : zero4();
      int q = 0;
      if constexpr (!ST) {
        for (; q + DU <= j; q += DU) {
          d4 u[DU];
#pragma unroll
          for (int e = 0; e < DU; ++e) u[e] = ujq(q + e);
#pragma unroll
          for (int e = 0; e < DU; ++e) {
            t0 = mfma_tn(neg4(u[e]), u[e], t0);
            if (has_rhs)
              z = mfma_tn(neg4(u[e]), load_compact(yl + (long long)(q + e) * 16 * nr, nr), z);
          }
        }
      }
      for (; q < j; ++q) {
        const d4 u = ujq(q);
        t0 = mfma_tn(neg4(u), u, t0);
        if (has_rhs) z = mfma_tn(neg4(u), load_compact(yl + (long long)q * 16 * nr, nr), z);
      }
      pad_identity(t0, nv);
      d4 V, W;
      const int inf = potrf_inv_tile_upper(t0, V, s, &W, (nv + 3) >> 2);
      if (inf && l == 0 && sinfo == 0) sinfo = 16 * j + inf;
      pm_stT(L, j, j, t0, true);
      if (l < nv) dAb[16 * j + l] = s.inv[l];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        wl[(long long)j * 256 + 64 * r + l] = W[r];
        vsh[64 * r + l] = V[r];
      }
      if (has_rhs) save_compact(yl + (long long)j * 16 * nr, mfma_tn(V, z, zero4()), nr);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __syncthreads();
    d4 V;
#pragma unroll
    for (int r = 0; r < 4; ++r) V[r] = vsh[64 * r + l];
    int i = j + 1 + w;
    if constexpr (!ST && PAIR) {
      // groups of GR rows of this wave; the blocks of A are added after the
      // downdate sum so that their loads overlap it
      for (; i < nb; i += GR * LW) {
        d4 av[GR], acc[GR];
#pragma unroll
        for (int r = 0; r < GR; ++r) {
          av[r] = pm_ldT(A, min(i + r * LW, nb - 1), j, false);
          acc[r] = zero4();
        }
        downdate_rows<GR, GQ>(L, j, i, LW, nb, acc);
#pragma unroll
        for (int r = 0; r < GR; ++r) {
          if (i + r * LW < nb) {
            pm_stT(L, i + r * LW, j, mfma_tn(V, av[r] + acc[r], zero4()), false);
          }
        }
      }
    }
    for (; i < nb; i += LW) {
      const d4 a0 = pm_ldT(A, i, j, false);
      d4 t1;
      if constexpr (ST)
        t1 = downdate_staged<DU>(ul, L, j, i, a0);
      else
        t1 = downdate<DU>(L, j, i, a0);
      pm_stT(L, i, j, mfma_tn(V, t1, zero4()), false);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __syncthreads();
  }
  if (has_rhs && w == 0) {
    double *Xb = a.X + a.voff[id];
    for (int j = nb - 1; j >= 0; --j) {
      d4 acc = load_compact(yl + (long long)j * 16 * nr, nr);
      // BQ tiles L(i,j) = U(j,i)^T in flight at a time (indices past the
      // last block row reload it and are multiplied by zero)
      for (int i = j + 1; i < nb; i += BQ) {
        d4 ut[BQ];
#pragma unroll
        for (int u = 0; u < BQ; ++u) ut[u] = pm_ldN(L, min(i + u, nb - 1), j);
#pragma unroll
        for (int u = 0; u < BQ; ++u) {
          const d4 m = (u == 0 || i + u < nb) ? neg4(ut[u]) : zero4();
          acc = mfma_tn(m, load_compact(yl + (long long)min(i + u, nb - 1) * 16 * nr, nr), acc);
        }
      }
      d4 W;
#pragma unroll
      for (int r = 0; r < 4; ++r) W[r] = wl[(long long)j * 256 + 64 * r + l];
      const d4 x = mfma_tn(W, acc, zero4());
      save_compact(yl + (long long)j * 16 * nr, x, nr);
      store_rhs(Xb, ld, n, a.nrhs, j, x);
    }
  }
  if (a.info && threadIdx.x == 0) a.info[id] = sinfo;
}

// Two block columns j, j+1 at once: acc0[r] -= sum_{q<j} U(q,j)^T U(q,i_r)
// and acc1[r] -= sum_{q<j} U(q,j+1)^T U(q,i_r) for the R rows
// i_r = i0 + r * stride (rows past the last block row repeat it); each
// U(q,i_r) is loaded once for both columns and each U(q,j), U(q,j+1) once
// for all R rows: 2 + R tile loads per 2R products.
template <int R>
__device__ __forceinline__ void downdate_cols2(const PMat &L, int j, int i0,
                                               int stride, int nb, d4 (&acc0)[R],
                                               d4 (&acc1)[R]) {
  int ir[R];
#pragma unroll
  for (int r = 0; r < R; ++r) ir[r] = min(i0 + r * stride, nb - 1);
  for (int q = 0; q < j; ++q) {
    const d4 u0 = pm_ldT(L, j, q, false), u1 = pm_ldT(L, j + 1, q, false);
    d4 ui[R];
#pragma unroll
    for (int r = 0; r < R; ++r) ui[r] = pm_ldT(L, ir[r], q, false);
    const d4 m0 = neg4(u0), m1 = neg4(u1);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      acc0[r] = mfma_tn(m0, ui[r], acc0[r]);
      acc1[r] = mfma_tn(m1, ui[r], acc1[r]);
    }
  }
}

// Left-looking over pairs of block columns (the blocked form of §4.6 with a
// panel two blocks wide), one workgroup of LW waves per instance.  Wave 0
// downdates the 2x2 diagonal blocks and the two right-hand-side blocks with
// one load of U(q,j), U(q,j+1) per step, factors block j, forms U(j,j+1),
// downdates and factors block j+1; then the waves share the remaining block
// rows, each row's left part read once for both columns.  Against the
// one-column kernel this halves the serial diagonal steps and barriers, and
// with R = 2 rows per group cuts the re-reads of the factor's left part by a
// third.  Same outputs and workspace use.
template <int LW, int R>
__global__ __launch_bounds__(64 * LW) __attribute__((amdgpu_waves_per_eu(3))) void k_vb_large_cp(VbArgs a, int nbmax) {
  extern __shared__ double dyn[];
  __shared__ DiagLds s;
  __shared__ double vsh[3][256];  // V_j, V_{j+1}, U(j,j+1)
  __shared__ int sinfo;
  const int nr = a.nrhs > 0 ? a.nrhs : 1;
  double *yl = dyn;  // nbmax * 16 * nr
  const int t = blockIdx.x;
  if (t >= a.count) return;
  const int id = a.ids[t];
  if (a.only && a.only[id] == 0) return;
  const int n = a.n[id];
  const int cn = cn_of(n), ld = ld_of(n), pm = (n + 15) >> 4;
  const int nb = pm;
  const int w = wave_id();
  const int l = lane_id();
  const PMat A = make_pmat(a.A + a.moff[id], n, cn);
  const PMat L = make_pmat(a.L + a.moff[id], n, cn);
  double *dAb = a.L + a.moff[id] + (long long)pm * 16 * cn;
  const bool has_rhs = a.nrhs > 0;
  const double *Bb = has_rhs ? a.B + a.voff[id] : nullptr;
  double *wl = a.wsw + a.wwoff[id];
  if (threadIdx.x == 0) sinfo = 0;
  __syncthreads();
  for (int j = 0; j < nb; j += 2) {
    const bool two = j + 1 < nb;
    const int jb = two ? j + 1 : j;
    if (w == 0) {
      d4 t00 = pm_ldT(A, j, j, true);
      d4 t01 = pm_ldT(A, jb, j, false);
      d4 t11 = pm_ldT(A, jb, jb, true);
      d4 z0 = has_rhs ? load_rhs(Bb, ld, n, a.nrhs, j) : zero4();
      d4 z1 = has_rhs ? load_rhs(Bb, ld, n, a.nrhs, jb) : zero4();
      for (int q = 0; q < j; ++q) {
        const d4 u0 = pm_ldT(L, j, q, false), u1 = pm_ldT(L, jb, q, false);
        const d4 m0 = neg4(u0), m1 = neg4(u1);
        t00 = mfma_tn(m0, u0, t00);
        t01 = mfma_tn(m0, u1, t01);
        t11 = mfma_tn(m1, u1, t11);
        if (has_rhs) {
          const d4 y = load_compact(yl + (long long)q * 16 * nr, nr);
          z0 = mfma_tn(m0, y, z0);
          z1 = mfma_tn(m1, y, z1);
        }
      }
      // block j
      pad_identity(t00, min(16, n - 16 * j));
      d4 V0, W0;
      int inf = potrf_inv_tile_upper(t00, V0, s, &W0, (min(16, n - 16 * j) + 3) >> 2);
      if (inf && l == 0 && sinfo == 0) sinfo = 16 * j + inf;
      pm_stT(L, j, j, t00, true);
      if (l < min(16, n - 16 * j)) dAb[16 * j + l] = s.inv[l];
      const d4 y0 = mfma_tn(V0, z0, zero4());
      if (has_rhs) save_compact(yl + (long long)j * 16 * nr, y0, nr);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        wl[(long long)j * 256 + 64 * r + l] = W0[r];
        vsh[0][64 * r + l] = V0[r];
      }
      if (two) {
        // U(j,j+1), then block j+1
        const d4 u01 = mfma_tn(V0, t01, zero4());
        pm_stT(L, j + 1, j, u01, false);
        t11 = mfma_tn(neg4(u01), u01, t11);
        z1 = mfma_tn(neg4(u01), y0, z1);
        const int nv1 = min(16, n - 16 * (j + 1));
        pad_identity(t11, nv1);
        d4 V1, W1;
        inf = potrf_inv_tile_upper(t11, V1, s, &W1, (nv1 + 3) >> 2);
        if (inf && l == 0 && sinfo == 0) sinfo = 16 * (j + 1) + inf;
        pm_stT(L, j + 1, j + 1, t11, true);
        if (l < nv1) dAb[16 * (j + 1) + l] = s.inv[l];
        if (has_rhs) save_compact(yl + (long long)(j + 1) * 16 * nr, mfma_tn(V1, z1, zero4()), nr);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          wl[(long long)(j + 1) * 256 + 64 * r + l] = W1[r];
          vsh[1][64 * r + l] = V1[r];
          vsh[2][64 * r + l] = u01[r];
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __syncthreads();
    if (two && j + 2 < nb) {
      d4 V0, V1, U01;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        V0[r] = vsh[0][64 * r + l];
        V1[r] = vsh[1][64 * r + l];
        U01[r] = vsh[2][64 * r + l];
      }
      const d4 mU01 = neg4(U01);
      for (int i = j + 2 + w; i < nb; i += R * LW) {
        d4 acc0[R], acc1[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          acc0[r] = zero4();
          acc1[r] = zero4();
        }
        downdate_cols2<R>(L, j, i, LW, nb, acc0, acc1);
        d4 a0[R], a1[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int ii = min(i + r * LW, nb - 1);
          a0[r] = pm_ldT(A, ii, j, false);
          a1[r] = pm_ldT(A, ii, j + 1, false);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int ii = i + r * LW;
          if (ii < nb) {
            const d4 uji = mfma_tn(V0, a0[r] + acc0[r], zero4());
            pm_stT(L, ii, j, uji, false);
            const d4 t1 = mfma_tn(mU01, uji, a1[r] + acc1[r]);
            pm_stT(L, ii, j + 1, mfma_tn(V1, t1, zero4()), false);
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      __syncthreads();
    }
  }
  if (has_rhs && w == 0) {
    double *Xb = a.X + a.voff[id];
    for (int j = nb - 1; j >= 0; --j) {
      d4 acc = load_compact(yl + (long long)j * 16 * nr, nr);
      for (int i = j + 1; i < nb; ++i) {
        const d4 ut = pm_ldN(L, i, j);  // L(i,j) = U(j,i)^T
        acc = mfma_tn(neg4(ut), load_compact(yl + (long long)i * 16 * nr, nr), acc);
      }
      d4 W;
#pragma unroll
      for (int r = 0; r < 4; ++r) W[r] = wl[(long long)j * 256 + 64 * r + l];
      const d4 x = mfma_tn(W, acc, zero4());
      save_compact(yl + (long long)j * 16 * nr, x, nr);
      store_rhs(Xb, ld, n, a.nrhs, j, x);
    }
  }
  if (a.info && threadIdx.x == 0) a.info[id] = sinfo;
}

size_t large_lds_bytes(int nbmax, int nrhs, bool staged) {
  const int nr = nrhs > 0 ? nrhs : 1;
  return sizeof(double) * ((size_t)nbmax * 16 * nr + (staged ? (size_t)nbmax * 256 : 0));
}

}  // namespace bh

// ---------------------------------------------------------------- plan

using namespace bh;


// orders above this go to the second n > 64 class
static const int kLargeSplit = 192;

static void drop_graph(blasfeo_hip_plan *p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
  p->have_graph = false;
}

template <int NB>
static void launch_small(const VbArgs &a, int vw, hipStream_t st) {
  switch (vw) {
    case 1: hipLaunchKernelGGL((k_vb_small<NB, 1>), dim3((a.count + 0) / 1), dim3(64), 0, st, a); break;
    case 2: hipLaunchKernelGGL((k_vb_small<NB, 2>), dim3((a.count + 1) / 2), dim3(128), 0, st, a); break;
    default: hipLaunchKernelGGL((k_vb_small<NB, 4>), dim3((a.count + 3) / 4), dim3(256), 0, st, a); break;
  }
}

static int launch_bucket(const blasfeo_hip_plan *p, const blasfeo_hip_plan::Bucket &bk,
                         const double *A, double *L, const double *B, double *X,
                         int *info, double *W, hipStream_t st, const int *only = nullptr) {
  if (bk.count == 0) return 0;
  VbArgs a;
  a.ids = p->d_ids + bk.first;
  a.count = bk.count;
  a.n = p->d_n;
  a.moff = p->d_moff;
  a.voff = p->d_voff;
  a.A = A;
  a.L = L;
  a.B = B;
  a.X = X;
  a.nrhs = p->nrhs;
  a.info = info;
  a.only = only;
  a.wsw = W;
  a.wwoff = p->d_wwoff;
  switch (bk.kind) {
    case 1: launch_small<1>(a, bk.cfg, st); break;
    case 2: launch_small<2>(a, bk.cfg, st); break;
    case 3: launch_small<3>(a, bk.cfg, st); break;
    case 4: launch_small<4>(a, bk.cfg, st); break;
    default: {
      const bool pair = bk.cfg >= 200;
      const bool staged = !pair && bk.cfg >= 100;
      const int lw = bk.cfg % 100;
      const size_t lds = large_lds_bytes(bk.nbmax, p->nrhs, staged);
      const dim3 g(bk.count), b(64 * lw);
      if (pair) {
        const int lwp = bk.cfg % 10;
        if (bk.cfg >= 210) {
          if (lwp == 4) hipLaunchKernelGGL((k_vb_large_cp<4, 2>), g, dim3(256), lds, st, a, bk.nbmax);
          else if (lwp == 2) hipLaunchKernelGGL((k_vb_large_cp<2, 2>), g, dim3(128), lds, st, a, bk.nbmax);
          else hipLaunchKernelGGL((k_vb_large_cp<1, 2>), g, dim3(64), lds, st, a, bk.nbmax);
        } else {
          if (lwp == 4) hipLaunchKernelGGL((k_vb_large_cp<4, 1>), g, dim3(256), lds, st, a, bk.nbmax);
          else if (lwp == 2) hipLaunchKernelGGL((k_vb_large_cp<2, 1>), g, dim3(128), lds, st, a, bk.nbmax);
          else hipLaunchKernelGGL((k_vb_large_cp<1, 1>), g, dim3(64), lds, st, a, bk.nbmax);
        }
      } else if (staged) {
        if (lw == 16) hipLaunchKernelGGL((k_vb_large<16, true>), g, b, lds, st, a, bk.nbmax);
        else if (lw == 8) hipLaunchKernelGGL((k_vb_large<8, true>), g, b, lds, st, a, bk.nbmax);
        else hipLaunchKernelGGL((k_vb_large<4, true>), g, b, lds, st, a, bk.nbmax);
      } else {
        if (lw == 16) hipLaunchKernelGGL((k_vb_large<16, false>), g, b, lds, st, a, bk.nbmax);
        else if (lw == 8) hipLaunchKernelGGL((k_vb_large<8, false>), g, b, lds, st, a, bk.nbmax);
        else if (lw == 4) hipLaunchKernelGGL((k_vb_large<4, false>), g, b, lds, st, a, bk.nbmax);
        else if (lw == 2) hipLaunchKernelGGL((k_vb_large<2, false>), g, b, lds, st, a, bk.nbmax);
        else hipLaunchKernelGGL((k_vb_large<1, false>), g, b, lds, st, a, bk.nbmax);
      }
    }
  }
  return launch_status();
}

int bh::launch_all(const blasfeo_hip_plan *p, const double *A, double *L,
                   const double *B, double *X, int *info, double *W,
                   hipStream_t st, const int *only) {
  // the large instances first: they are the longest (LPT)
  for (int pass = 0; pass < 2; ++pass)
    for (const auto &bk : p->buckets) {
      if ((pass == 0) != (bk.kind == 0)) continue;
      int e = launch_bucket(p, bk, A, L, B, X, info, W, st, only);
      if (e) return e;
    }
  return 0;
}

extern "C" {

int blasfeo_hip_dposv_vbatched_plan(int batch, const int *n_host, int nrhs,
                                    blasfeo_hip_plan **plan,
                                    long long *workspace_bytes) {
  if (batch < 0) return -1;
  if (batch > 0 && !n_host) return -2;
  if (nrhs < 0 || nrhs > 16) return -3;
  if (!plan) return -4;
  for (int i = 0; i < batch; ++i)
    if (n_host[i] < 1 || n_host[i] > 512) return -2;
  auto *p = new blasfeo_hip_plan();
  p->batch = batch;
  p->nrhs = nrhs;
  p->n.assign(n_host, n_host + batch);
  p->moff.resize(batch);
  p->voff.resize(batch);
  long long mo = 0, vo = 0;
  for (int i = 0; i < batch; ++i) {
    p->moff[i] = mo;
    p->voff[i] = vo;
    mo += blasfeo_memsize_dmat(p->n[i], p->n[i]);
    vo += ((long long)(p->n[i] + 15) / 16 * 16 * (nrhs > 0 ? nrhs : 1) * 8 + 255) / 256 * 256;
  }
  p->mat_bytes = mo;
  p->vec_bytes = vo;
  // buckets: small kernels by number of 16-blocks, one large bucket
  std::vector<int> ids;
  ids.reserve(batch);
  for (int kind = 1; kind <= 4; ++kind) {
    const int first = (int)ids.size();
    for (int i = 0; i < batch; ++i)
      if ((p->n[i] + 15) / 16 == kind) ids.push_back(i);
    p->buckets.push_back({kind, first, (int)ids.size() - first, kind, 2});
  }
  // n > 64: two classes (n <= 192 and n > 192), each largest first and each
  // with its own launch configuration (the larger instances favour more
  // waves per instance)
  for (int part = 0; part < 2; ++part) {
    const int first = (int)ids.size();
    std::vector<int> big;
    for (int i = 0; i < batch; ++i)
      if (p->n[i] > 64 && ((p->n[i] > kLargeSplit) == (part == 0))) big.push_back(i);
    std::stable_sort(big.begin(), big.end(),
                     [&](int x, int y) { return p->n[x] > p->n[y]; });
    ids.insert(ids.end(), big.begin(), big.end());
    const int nbmax = big.empty() ? 0 : (p->n[big[0]] + 15) / 16;
    p->buckets.push_back({0, first, (int)big.size(), nbmax, part == 0 ? 2 : 1});
  }
  p->ids = ids;
  std::vector<long long> wwo(batch, 0);
  long long wtot = 0;
  for (int i = 0; i < batch; ++i)
    if (p->n[i] > 64) {
      wwo[i] = wtot;
      wtot += 256LL * ((p->n[i] + 15) / 16);
    }
  p->ws64_bytes = wtot * (long long)sizeof(double);
  std::vector<long long> md(batch), vd(batch);
  for (int i = 0; i < batch; ++i) {
    md[i] = p->moff[i] / 8;
    vd[i] = p->voff[i] / 8;
  }
  hipError_t e = hipSuccess;
  const size_t nb = (size_t)(batch > 0 ? batch : 1);
  if (e == hipSuccess) e = hipMalloc(&p->d_n, nb * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&p->d_moff, nb * sizeof(long long));
  if (e == hipSuccess) e = hipMalloc(&p->d_voff, nb * sizeof(long long));
  if (e == hipSuccess) e = hipMalloc(&p->d_ids, nb * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&p->d_wwoff, nb * sizeof(long long));
  if (e == hipSuccess && batch > 0)
    e = hipMemcpy(p->d_wwoff, wwo.data(), batch * sizeof(long long), hipMemcpyHostToDevice);
  if (e == hipSuccess && batch > 0) {
    e = hipMemcpy(p->d_n, p->n.data(), batch * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_moff, md.data(), batch * sizeof(long long), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_voff, vd.data(), batch * sizeof(long long), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_ids, ids.data(), batch * sizeof(int), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming);
  for (int i = 0; i < (int)p->buckets.size() && i < blasfeo_hip_plan::kMaxAux && e == hipSuccess; ++i) {
    e = hipStreamCreateWithFlags(&p->aux[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_join[i], hipEventDisableTiming);
  }
  int nbm = 0;
  for (const auto &bk : p->buckets)
    if (bk.kind == 0) nbm = std::max(nbm, bk.nbmax);
  if (e == hipSuccess && nbm > 0) {
    // the large kernel's dynamic LDS may exceed the default limit
    const void *ks[8] = {(const void *)k_vb_large<4, true>, (const void *)k_vb_large<8, true>,
                         (const void *)k_vb_large<16, true>, (const void *)k_vb_large<1, false>,
                         (const void *)k_vb_large<2, false>, (const void *)k_vb_large<4, false>,
                         (const void *)k_vb_large<8, false>, (const void *)k_vb_large<16, false>};
    for (int k = 0; k < 8 && e == hipSuccess; ++k)
      e = hipFuncSetAttribute(ks[k], hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)large_lds_bytes(nbm, nrhs, k < 3));
    const void *kp[6] = {(const void *)k_vb_large_cp<1, 1>, (const void *)k_vb_large_cp<2, 1>,
                         (const void *)k_vb_large_cp<4, 1>, (const void *)k_vb_large_cp<1, 2>,
                         (const void *)k_vb_large_cp<2, 2>, (const void *)k_vb_large_cp<4, 2>};
    for (int k = 0; k < 6 && e == hipSuccess; ++k)
      e = hipFuncSetAttribute(kp[k], hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)large_lds_bytes(nbm, nrhs, false));
  }
  int me = e == hipSuccess ? mx_plan_setup(p) : 0;
  if (e != hipSuccess || me) {
    blasfeo_hip_plan_destroy(p);
    return e != hipSuccess ? (int)e : me;
  }
  if (workspace_bytes) *workspace_bytes = p->ws64_bytes;
  *plan = p;
  return 0;
}

int blasfeo_hip_plan_workspace(const blasfeo_hip_plan *p, long long *fp64_bytes,
                               long long *mixed_bytes) {
  if (!p) return -1;
  if (fp64_bytes) *fp64_bytes = p->ws64_bytes;
  if (mixed_bytes) *mixed_bytes = p->mx_ok ? mixed_ws_bytes(p) : 0;
  return 0;
}

int blasfeo_hip_plan_layout(const blasfeo_hip_plan *p, long long *mat_off,
                            long long *vec_off, long long *mat_bytes,
                            long long *vec_bytes) {
  if (!p) return -1;
  if (mat_off) std::copy(p->moff.begin(), p->moff.end(), mat_off);
  if (vec_off) std::copy(p->voff.begin(), p->voff.end(), vec_off);
  if (mat_bytes) *mat_bytes = p->mat_bytes;
  if (vec_bytes) *vec_bytes = p->vec_bytes;
  return 0;
}

int blasfeo_hip_plan_set_graph(blasfeo_hip_plan *p, int on) {
  if (!p) return -1;
  p->use_graph = on ? 1 : 0;
  drop_graph(p);
  return 0;
}

static bool cfg_valid(int kind, int cfg) { return tune_cfg_valid(kind, cfg); }

int blasfeo_hip_plan_set_config(blasfeo_hip_plan *p, const int *cfg, int count) {
  if (!p) return -1;
  if (!cfg) return -2;
  if (count != (int)p->buckets.size()) return -3;
  for (int i = 0; i < count; ++i)
    if (!cfg_valid(p->buckets[i].kind, cfg[i])) return -2;
  for (int i = 0; i < count; ++i) p->buckets[i].cfg = cfg[i];
  drop_graph(p);
  return 0;
}

int blasfeo_hip_plan_config(const blasfeo_hip_plan *p, int *cfg_out) {
  if (!p) return -1;
  if (cfg_out)
    for (size_t i = 0; i < p->buckets.size(); ++i) cfg_out[i] = p->buckets[i].cfg;
  return (int)p->buckets.size();
}

// Argument checks shared by execution and capture (positions as in
// blasfeo_hip_dposv_vbatched).
static int operands_ok(const blasfeo_hip_plan *p, const void *A, const void *L,
                       const void *B, const void *X) {
  if (!A) return -2;
  if (!L) return -3;
  if (p->nrhs > 0 && !B) return -4;
  if (p->nrhs > 0 && !X) return -5;
  return 0;
}

static int exec_args_ok(const blasfeo_hip_plan *p, const void *A, const void *L,
                        const void *B, const void *X, const void *W) {
  if (const int e = operands_ok(p, A, L, B, X)) return e;
  if (p->ws64_bytes > 0 && (!W || ((uintptr_t)W & 255))) return -7;
  return 0;
}

int blasfeo_hip_plan_capture(blasfeo_hip_plan *p, const void *A, void *L,
                             const void *B, void *X, int *info, void *work) {
  if (!p) return -1;
  if (p->batch == 0) return 0;
  if (const int e = exec_args_ok(p, A, L, B, X, work)) return e;
  drop_graph(p);
  hipError_t e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return (int)e;
  // the classes touch disjoint instances (and disjoint parts of the
  // workspace): each becomes its own branch of the graph, so that one
  // class's last workgroups overlap the others' instead of each launch
  // draining the GPU before the next starts; the n > 64 classes first
  int le = (int)hipEventRecord(p->ev_fork, p->cap);
  int nbr = 0;
  for (int pass = 0; pass < 2 && !le; ++pass)
    for (const auto &bk : p->buckets) {
      if ((pass == 0) != (bk.kind == 0) || bk.count == 0 || le) continue;
      hipStream_t s = nbr < blasfeo_hip_plan::kMaxAux && p->aux[nbr] ? p->aux[nbr] : p->cap;
      if (s != p->cap) le = (int)hipStreamWaitEvent(s, p->ev_fork, 0);
      if (!le)
        le = launch_bucket(p, bk, (const double *)A, (double *)L, (const double *)B,
                           (double *)X, info, (double *)work, s);
      if (!le && s != p->cap) {
        le = (int)hipEventRecord(p->ev_join[nbr], s);
        if (!le) le = (int)hipStreamWaitEvent(p->cap, p->ev_join[nbr], 0);
      }
      ++nbr;
    }
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(p->cap, &g);
  if (le) {
    if (g) (void)hipGraphDestroy(g);
    return le;
  }
  if (e != hipSuccess) return (int)e;
  e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    p->exec = nullptr;
    return (int)e;
  }
  p->graph = g;
  p->have_graph = true;
  const void *key[6] = {A, L, B, X, info, work};
  for (int i = 0; i < 6; ++i) p->key[i] = key[i];
  return 0;
}

int blasfeo_hip_dposv_vbatched(blasfeo_hip_plan *p, const void *A, void *L,
                               const void *B, void *X, int *info, void *work,
                               void *stream) {
  if (!p) return -1;
  if (p->batch == 0) return 0;
  if (const int e = exec_args_ok(p, A, L, B, X, work)) return e;
  hipStream_t st = (hipStream_t)stream;
  const void *key[6] = {A, L, B, X, info, work};
  bool same = p->use_graph && p->have_graph;
  for (int i = 0; i < 6 && same; ++i) same = key[i] == p->key[i];
  if (same) {
    const hipError_t e = hipGraphLaunch(p->exec, st);
    return e == hipSuccess ? 0 : (int)e;
  }
  return launch_all(p, (const double *)A, (double *)L, (const double *)B,
                    (double *)X, info, (double *)work, st);
}

}  // extern "C"

// Workspace of blasfeo_hip_dposv_vbatched_noalloc: a fixed device array in
// the code object, one copy per GPU, held until the process ends.  Host code
// never uses the symbol itself as an address (it is a host-side stand-in):
// each device's address is read once with hipGetSymbolAddress while that
// device is current, and only that address is passed to kernels.
static __device__ __align__(256) double scratch[BLASFEO_HIP_NOALLOC_SCRATCH_BYTES / 8];

namespace {
std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;  // per device ordinal, null until looked up
}  // namespace

// Address of this device's scratch array; 0 or a HIP error.
static int scratch_address(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    if (!ptr || ((uintptr_t)ptr & 255)) return (int)hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return 0;
}

extern "C" {

int blasfeo_hip_noalloc_init(void) {
  void *ptr = nullptr;
  return scratch_address(&ptr);
}

int blasfeo_hip_dposv_vbatched_noalloc(const blasfeo_hip_plan *p, const void *A,
                                       void *L, const void *B, void *X,
                                       int *info, void *stream) {
  if (!p) return -1;
  if (p->batch == 0) return 0;
  if (const int e = operands_ok(p, A, L, B, X)) return e;
  if (p->ws64_bytes > BLASFEO_HIP_NOALLOC_SCRATCH_BYTES) return -1;
  void *w = nullptr;
  if (p->ws64_bytes > 0) {
    if (const int e = scratch_address(&w)) return e;
  }
  return launch_all(p, (const double *)A, (double *)L, (const double *)B,
                    (double *)X, info, (double *)w, (hipStream_t)stream);
}

int blasfeo_hip_plan_autotune(blasfeo_hip_plan *p, const void *A, void *L,
                              const void *B, void *X, int *info, void *work,
                              void *stream) {
  if (!p) return -1;
  if (p->batch == 0) return 0;
  if (const int e = exec_args_ok(p, A, L, B, X, work)) return e;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -8;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -8;
  }
  TuneKey key;
  int err = tune_key_device(key) ? -8 : 0;
  for (auto &bk : p->buckets) {
    if (bk.count == 0 || err) continue;
    key.kind = bk.kind;
    key.nrhs = p->nrhs;
    key.count = bk.count;
    key.nmin = 1 << 30;
    key.nmax = 0;
    key.nsum = 0;
    for (int t = 0; t < bk.count; ++t) {
      const int nn = p->n[p->ids[bk.first + t]];
      key.nmin = std::min(key.nmin, nn);
      key.nmax = std::max(key.nmax, nn);
      key.nsum += nn;
    }
    int cached = 0;
    if (tune_lookup(key, &cached)) {
      bk.cfg = cached;
      continue;
    }
    const int cands_small[3] = {1, 2, 4};
    const int cands_large[11] = {1, 2, 4, 8, 104, 108, 201, 202, 204, 211, 212};
    const int *cands = bk.kind ? cands_small : cands_large;
    const int nc = bk.kind ? 3 : 11;
    auto timed = [&](float &ms) {
      (void)hipEventRecord(e0, st);
      err = launch_bucket(p, bk, (const double *)A, (double *)L, (const double *)B, (double *)X,
                          info, (double *)work, st);
      (void)hipEventRecord(e1, st);
      (void)hipEventSynchronize(e1);
      ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
    };
    // the GPU's clocks settle only after tens of milliseconds under load:
    // run the class until it has been busy 30 ms before timing candidates
    {
      float busy = 0.f, ms = 0.f;
      for (int w = 0; w < 1000 && busy < 30.f && !err; ++w) {
        timed(ms);
        busy += ms;
      }
    }
    float best = 1e30f;
    int best_cfg = bk.cfg;
    for (int ci = 0; ci < nc && !err; ++ci) {
      bk.cfg = cands[ci];
      float t[4] = {0.f, 0.f, 0.f, 0.f};
      for (int rep = 0; rep < 4 && !err; ++rep) timed(t[rep]);  // rep 0 warms up
      // median of the three timed runs
      const float med = std::max(std::min(t[1], t[2]), std::min(std::max(t[1], t[2]), t[3]));
      if (med < best) {
        best = med;
        best_cfg = cands[ci];
      }
    }
    bk.cfg = best_cfg;
    if (!err) tune_store(key, best_cfg, best);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  drop_graph(p);
  return err;
}

void blasfeo_hip_plan_destroy(blasfeo_hip_plan *p) {
  if (!p) return;
  drop_graph(p);
  if (p->d_n) (void)hipFree(p->d_n);
  if (p->d_moff) (void)hipFree(p->d_moff);
  if (p->d_voff) (void)hipFree(p->d_voff);
  if (p->d_ids) (void)hipFree(p->d_ids);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  for (int i = 0; i < blasfeo_hip_plan::kMaxAux; ++i) {
    if (p->aux[i]) (void)hipStreamDestroy(p->aux[i]);
    if (p->ev_join[i]) (void)hipEventDestroy(p->ev_join[i]);
  }
  if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
  if (p->d_woff) (void)hipFree(p->d_woff);
  if (p->d_mx_ids) (void)hipFree(p->d_mx_ids);
  if (p->d_wwoff) (void)hipFree(p->d_wwoff);
  delete p;
}

}  // extern "C"
