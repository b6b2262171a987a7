// Device building blocks shared by all kernels: the counterpart of the
// paper's assembly subroutines (§4.4.1) -- fragment loads from panel-major
// storage, the MFMA k-loop, the register-resident 16x16 factorization and
// inversion, masked/unaligned stores -- written as forceinline device
// functions that pass 16x16 tiles in registers.
//
// Register tile ("T-tile") convention.  A 16x16 FP64 tile lives in the
// result layout of v_mfma_f64_16x16x4f64 on gfx950: lane l = c + 16*g
// (c = l & 15, g = l >> 4) holds in register r the element in row g + 4r,
// column c.  Two facts make this layout the work-horse of the library:
//   * register r of a T-tile X is exactly the B operand of the k-step
//     covering rows 4r..4r+3 of X, and the A operand of the same k-step of
//     X^T, so  sum_r mfma(X[r], Y[r])  =  X^T * Y  for T-tiles X, Y;
//   * loading the TRANSPOSE of a 16x16 block of a panel-major matrix into a
//     T-tile reads, for register r, the 64 consecutive doubles
//     [64r, 64r+64) of the block's 16 panel columns: one contiguous 512-byte
//     wave transaction (the panel-wise reads of §4.3).
// The kernels therefore work on transposed blocks: a lower factor L is held
// as its transpose U = L^T, and every trailing update, triangular solve and
// product is a chain of MFMAs on register tiles.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bh {

constexpr int PS = 16;  // panel height (rows per panel), double precision

typedef double d4 __attribute__((ext_vector_type(4)));

// Offset of element (i, j) in a panel-major buffer with panel length cn
// (§4.3): (i - i % ps) * cn + j * ps + i % ps.
__host__ __device__ __forceinline__ long long pm_off(int i, int j, int cn) {
  return (long long)(i & ~(PS - 1)) * cn + (long long)j * PS + (i & (PS - 1));
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
// Index of the wavefront in its workgroup, read from the first lane so that
// the compiler knows it is uniform: values derived from it (an instance
// index, a block index used as a buffer offset) stay in scalar registers
// instead of forcing a loop over lanes around every buffer access.
__device__ __forceinline__ int wave_id() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

// Orders LDS traffic of one wavefront (no hardware barrier needed: a wave's
// LDS instructions execute in issue order; this stops compiler reordering).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ d4 zero4() { return (d4){0.0, 0.0, 0.0, 0.0}; }

// Index of the upper block (j, i), j <= i, in a column-packed list of the
// upper block triangle (U = L^T view of a lower factor).
__host__ __device__ constexpr int tix_up(int j, int i) { return i * (i + 1) / 2 + j; }

// acc += X^T * Y for T-tiles X, Y (four chained MFMAs).
__device__ __forceinline__ d4 mfma_tn(const d4 &X, const d4 &Y, d4 acc) {
  acc = mfma(X[0], Y[0], acc);
  acc = mfma(X[1], Y[1], acc);
  acc = mfma(X[2], Y[2], acc);
  acc = mfma(X[3], Y[3], acc);
  return acc;
}

__device__ __forceinline__ d4 neg4(const d4 &x) { return -x; }

// ---------------------------------------------------------------------------
// Buffer-resource accesses: a 128-bit descriptor (base, size in bytes) in
// SGPRs plus a 32-bit per-lane byte offset and a uniform byte offset.  The
// kernels address every operand of an instance through one descriptor, so
// an access costs one VGPR offset instead of a 64-bit address.
// ---------------------------------------------------------------------------
typedef __amdgpu_buffer_rsrc_t brsrc;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// dword 3 of a raw (untyped, stride 0) buffer descriptor on gfx9-family GPUs
constexpr int kBufferWord3 = 0x00020000;

__device__ __forceinline__ brsrc make_rsrc(const void *base, long long bytes) {
  const int n = bytes > 0x7fffffffLL ? 0x7fffffff : (int)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, n,
                                           kBufferWord3);
}

__device__ __forceinline__ double bload(brsrc r, int voff, int soff) {
  return __builtin_bit_cast(double,
                            __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

__device__ __forceinline__ void bstore(brsrc r, int voff, int soff, double x) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, voff, soff, 0);
}

// A square panel-major matrix of order n (origin at its first element)
// addressed through a buffer descriptor: block (i, j) of 16x16 starts at
// byte i * pst + j * 2048 (pst = 16 cn 8 bytes per panel), so the lane part
// of a T-tile access is the same 8 * lane for every block.
struct PMat {
  brsrc r;
  int pst;
  int n;
};

__device__ __forceinline__ PMat make_pmat(const double *p, int n, int cn) {
  const int pm = (n + 15) >> 4;
  return PMat{make_rsrc(p, 8LL * (pm * 16LL * cn + n)), 16 * cn * 8, n};
}

// T-tile of block (i, j)^T: register r of lane (c, g) = M[16i + c][16j + g + 4r];
// zero outside the matrix and, if lower, above its diagonal.
__device__ __forceinline__ d4 pm_ldT(const PMat &m, int i, int j, bool lower) {
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
  const int row = 16 * i + c;
  const int base = i * m.pst + j * 2048;
  d4 t;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int col = 16 * j + g + 4 * r;
    const bool ok = row < m.n && col < m.n && (!lower || row >= col);
    const double x = bload(m.r, 8 * l, base + 512 * r);
    t[r] = ok ? x : 0.0;
  }
  return t;
}

// T-tile of block (i, j) itself: register r of lane (c, g) = M[16i + g + 4r][16j + c].
__device__ __forceinline__ d4 pm_ldN(const PMat &m, int i, int j) {
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
  const int col = 16 * j + c;
  const int base = i * m.pst + j * 2048;
  d4 t;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 16 * i + g + 4 * r;
    const double x = bload(m.r, 128 * c + 8 * g, base + 32 * r);
    t[r] = (row < m.n && col < m.n) ? x : 0.0;
  }
  return t;
}

// Stores a T-tile holding block (i, j)^T, masked to the matrix and, if
// lower, to its lower triangle.
__device__ __forceinline__ void pm_stT(const PMat &m, int i, int j, const d4 &t, bool lower) {
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
  const int row = 16 * i + c;
  const int base = i * m.pst + j * 2048;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int col = 16 * j + g + 4 * r;
    if (row < m.n && col < m.n && (!lower || row >= col)) bstore(m.r, 8 * l, base + 512 * r, t[r]);
  }
}

// ---------------------------------------------------------------------------
// Generic (any offset, any bounds) accesses.  A "view" is a panel-major
// matrix with its sub-matrix origin (ai, aj) and the sub-matrix extent.
// ---------------------------------------------------------------------------
struct View {
  double *p;
  int cn;
  int ai, aj;
  int rows, cols;  // extent of the sub-matrix
};

// The loads below are unconditional: an element outside the sub-matrix is
// read from the sub-matrix origin and replaced by zero, so that the loads of
// a tile are all in flight at once (a load under a branch is waited for
// inside the branch).  The sub-matrix must therefore be non-empty, which
// every caller guarantees by only addressing blocks that exist.

// A/B operand fragment of the 16x4 block X = S[i0:i0+16, k0:k0+4] of the
// sub-matrix S: lane l holds X[l & 15][l >> 4] (zero outside S).  Used as
// the A operand it supplies X; used as the B operand it supplies X^T.
__device__ __forceinline__ double load_frag(const View &v, int i0, int k0) {
  const int l = lane_id();
  const int i = i0 + (l & 15), k = k0 + (l >> 4);
  const bool ok = i < v.rows && k < v.cols;
  const double x = v.p[ok ? pm_off(v.ai + i, v.aj + k, v.cn) : pm_off(v.ai, v.aj, v.cn)];
  return ok ? x : 0.0;
}

// T-tile holding the transpose of the block S[i0:i0+16, j0:j0+16]:
// register r of lane (c, g) = S[i0 + c][j0 + g + 4r].  Elements outside S,
// and, if lower_only, elements above the diagonal of S (i < j), read as 0.
__device__ __forceinline__ d4 load_tileT(const View &v, int i0, int j0,
                                         bool lower_only) {
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
  const int o0 = pm_off(v.ai, v.aj, v.cn);
  double x[4];
  bool ok[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + c, j = j0 + g + 4 * r;
    ok[r] = i < v.rows && j < v.cols && (!lower_only || i >= j);
    x[r] = v.p[ok[r] ? pm_off(v.ai + i, v.aj + j, v.cn) : o0];
  }
  d4 t;
#pragma unroll
  for (int r = 0; r < 4; ++r) t[r] = ok[r] ? x[r] : 0.0;
  return t;
}

// T-tile holding the block S[i0:i0+16, j0:j0+16] itself (not transposed):
// register r of lane (c, g) = S[i0 + g + 4r][j0 + c].  Zero outside S.
__device__ __forceinline__ d4 load_tileN(const View &v, int i0, int j0) {
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
  const int o0 = pm_off(v.ai, v.aj, v.cn);
  double x[4];
  bool ok[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + g + 4 * r, j = j0 + c;
    ok[r] = i < v.rows && j < v.cols;
    x[r] = v.p[ok[r] ? pm_off(v.ai + i, v.aj + j, v.cn) : o0];
  }
  d4 t;
#pragma unroll
  for (int r = 0; r < 4; ++r) t[r] = ok[r] ? x[r] : 0.0;
  return t;
}

// Transpose of a T-tile through 16x17 doubles of wave-private LDS.
__device__ __forceinline__ d4 transpose_tile(const d4 &x, double *tr) {
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) tr[(g + 4 * r) * 17 + c] = x[r];
  wave_sync();
  d4 y;
#pragma unroll
  for (int r = 0; r < 4; ++r) y[r] = tr[c * 17 + g + 4 * r];
  wave_sync();
  return y;
}

// Stores the T-tile t (holding the transpose of a block) into
// S[i0:i0+16, j0:j0+16], masked to S and, if lower_only, to i >= j.
__device__ __forceinline__ void store_tileT(const View &v, int i0, int j0,
                                            const d4 &t, bool lower_only) {
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + c, j = j0 + g + 4 * r;
    if (i < v.rows && j < v.cols && (!lower_only || i >= j))
      v.p[pm_off(v.ai + i, v.aj + j, v.cn)] = t[r];
  }
}

// ---------------------------------------------------------------------------
// Register-resident 16x16 Cholesky and triangular inversion (§4.6: the
// unblocked part of the LAPACK-style routines is a subroutine that works on a
// block held in registers).
// ---------------------------------------------------------------------------

// V = U^{-1} for an upper triangular T-tile U with inv[k] = 1/U[k][k]
// (back substitution, one column per lane group column).  `ulds` is 256
// doubles of wave-private LDS (U is staged there row-major), `row` is 16.
// The strictly lower part of V is exactly zero.
__device__ __forceinline__ d4 trtri_tile_upper(const d4 &U, const double *inv,
                                               double *ulds, double *row) {
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) ulds[(g + 4 * r) * 16 + c] = U[r];
  wave_sync();
  d4 s = zero4();
  d4 V = zero4();
#pragma unroll
  for (int p = 15; p >= 0; --p) {
    const int rp = p >> 2, gp = p & 3;
    if (g == gp) {
      const double v = ((p == c) ? 1.0 : 0.0) - s[rp];
      V[rp] = v * inv[p];
      row[c] = V[rp];
    }
    wave_sync();
    const double vpc = row[c];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int q = g + 4 * r;
      if (q < p) s[r] = s[r] + ulds[q * 16 + p] * vpc;
    }
    wave_sync();
  }
  return V;
}

// Wave-private LDS scratch of the diagonal-block subroutines.
struct WaveLds {
  double ulds[256];
  double row[16];
  double inv[16];
};

// Scratch of potrf_inv_tile_upper: the reciprocals, the pivots and a padded
// 16x17 transpose buffer (the pivot rows go through its first 128 doubles).
struct DiagLds {
  double inv[16];
  double piv[16];
  double tr[16 * 17];
};

__device__ __forceinline__ double readlane_d(double x, int lane) {
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// 1/sqrt(d) for d > 0: the hardware estimate (about 25 correct bits), one
// Newton step (about 50) and one residual correction (Markstein): within an
// ulp of the exact value and exact when it is representable (d a power of 4);
// both measured on the device over 2^20 arguments spanning 2^-100..2^100.
__device__ __forceinline__ double rsqrt_refined(double d) {
  double r = __builtin_amdgcn_rsq(d);
  const double h = 0.5 * d;
  r = r * fma(-h * r, r, 1.5);
  return fma(0.5 * r, fma(-d * r, r, 1.0), r);
}

// Reciprocal square root of a pivot: iv = 1/sqrt(d) if d > 0 (ok), else 0
// (for d <= 0 or NaN the refinement yields NaN or an infinity, which the
// final selection drops).
__device__ __forceinline__ void pivot_rsqrt(double d, bool &ok, double &iv) {
  ok = d > 0.0;
  const double r = rsqrt_refined(d);
  iv = ok ? r : 0.0;
}

// Upper Cholesky factorization of a T-tile together with the inverse of the
// factor, in one sweep over the 16 pivots.
//   In:  T holds a symmetric block in its upper triangle (rows <= cols);
//        padding rows/cols >= nv must hold the identity.
//   Out: T = U (upper, exact zeros below), V = U^{-1} (upper, T-tile),
//        s.inv[k] = 1/U[k][k].  Returns 0 or k+1 for the first pivot that is
//        not > 0; that pivot's reciprocal is set to 0, which keeps every entry of
//        the earlier rows exact and finite; later entries are unspecified.
// Pivot k is U[k][k] = sqrt(d_k), U[k][c] = T[k][c]*(1/U[k][k]); at the same
// time row k of W = L^{-1} = U^{-T} follows from forward substitution,
//   W[k][c] = (delta_kc - S[k][c]) / U[k][k],  S[p][c] = sum_{q<p} U[q][p] W[q][c].
// The 16 pivots are processed in four panels of four rows (one register of
// the T-tile each).  Inside a panel the rank-1 downdates of T and updates of
// S touch only the panel's rows; the panel's contribution to the rows below
// is then one rank-4 MFMA for T and one for S (register b of a T-tile is the
// MFMA operand of rows 4b..4b+3).  Each pivot row of U and W crosses lanes
// through LDS (every lane group writes its own copy, the pivot's group is
// read back; a wave's LDS operations execute in order).
// The serial chain from pivot to pivot is shortened by a one-step look-ahead:
// the next pivot inside the panel, d_{k+1} = T[k+1][k+1] - (T[k][k+1]/U[k][k])^2,
// is formed from two values read with readlane before this pivot's row
// broadcast, so its reciprocal square root (rsqrt_refined) runs while the
// broadcast is in flight.  The product and the downdate are the same
// roundings as the downdate of the whole row, so the result does not depend
// on the look-ahead.  The diagonal sqrt(d) is formed for all 16 columns after
// the sweep; V is W^T (one LDS transpose at the end).
// With np < 4 (the caller's block holds the identity in rows and columns
// 4 np..15, as pad_identity leaves it) only the first np panels are swept;
// the rest of U, V and W is the identity.
__device__ __forceinline__ int potrf_inv_tile_upper(d4 &T, d4 &V,
                                                    DiagLds &s,
                                                    d4 *Wout = nullptr,
                                                    int np = 4) {
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
  int info = 0;
  d4 S = zero4(), W = zero4();
  double *rowU = s.tr, *rowW = s.tr + 64;  // one 16-entry row per lane group
  double d = readlane_d(T[0], 0);
  double t01 = readlane_d(T[0], 1), t11 = readlane_d(T[0], 1 + 16);
  bool ok;
  double iv;
  pivot_rsqrt(d, ok, iv);
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    if (b >= np) {  // identity rows
      W[b] = (c == g + 4 * b) ? 1.0 : 0.0;
      continue;
    }
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int k = 4 * b + kk;
      if (!ok && info == 0) info = k + 1;
      if (l == k) {
        s.inv[k] = iv;
        s.piv[k] = d;
      }
      // row k of U (off the diagonal) and of W, valid in lane group kk
      const double ukc = (c > k) ? T[b] * iv : 0.0;
      const double wkc = (((c == k) ? 1.0 : 0.0) - S[b]) * iv;
      rowU[16 * g + c] = ukc;
      rowW[16 * g + c] = wkc;
      const bool mine = g == kk;
      T[b] = mine ? ukc : T[b];
      W[b] = mine ? wkc : W[b];
      wave_sync();
      const double rc = rowU[16 * kk + c];
      const double rp = rowU[16 * kk + 4 * b + g];
      const double rw = rowW[16 * kk + c];
      // the next pivot of this panel while the reads are in flight
      __builtin_amdgcn_sched_barrier(0);
      double dn = 0.0, ivn = 0.0;
      bool okn = true;
      if (kk < 3) {
        const double u = t01 * iv;
        dn = fma(-u, u, t11);
        pivot_rsqrt(dn, okn, ivn);
      }
      __builtin_amdgcn_sched_barrier(0);
      // rank-1 downdate of the panel rows below the pivot (groups g > kk).
      // rp is zero in the other groups (it is row k of U left of column
      // k + 1), so S needs no selection: its rows up to the pivot's are not
      // used again.  T keeps one, so that a non-finite pivot row cannot
      // reach the finished rows through 0 * inf.
      const bool below = g > kk;
      T[b] = (below && c > k) ? fma(-rp, rc, T[b]) : T[b];
      S[b] = fma(rp, rw, S[b]);
      wave_sync();
      if (kk < 3) {
        d = dn;
        ok = okn;
        iv = ivn;
      }
      if (kk < 2) {  // T[k+1][k+2] and T[k+2][k+2] for the next look-ahead
        t01 = readlane_d(T[b], (k + 2) + 16 * (kk + 1));
        t11 = readlane_d(T[b], (k + 2) + 16 * (kk + 2));
      }
    }
    if (b < 3 && b + 1 < np) {
      const double ub = T[b], wb = W[b];
      const d4 Tn = mfma(-ub, ub, T);
      const d4 Sn = mfma(ub, wb, S);
#pragma unroll
      for (int r = b + 1; r < 4; ++r) {
        T[r] = Tn[r];
        S[r] = Sn[r];
      }
      const int k1 = 4 * (b + 1);
      d = readlane_d(T[b + 1], k1);
      t01 = readlane_d(T[b + 1], k1 + 1);
      t11 = readlane_d(T[b + 1], k1 + 1 + 16);
      pivot_rsqrt(d, ok, iv);
    }
  }
  if (l >= 4 * np && l < 16) {
    s.inv[l] = 1.0;
    s.piv[l] = 1.0;
  }
  // the diagonal of U: sqrt(d_c), correctly rounded (exact for squares)
  wave_sync();
  const double uc = sqrt(s.piv[c]);
#pragma unroll
  for (int r = 0; r < 4; ++r) T[r] = (c == g + 4 * r) ? uc : T[r];
  if (Wout) *Wout = W;  // W = L^{-1} = V^T, itself a T-tile
  // V = W^T through a padded LDS transpose
#pragma unroll
  for (int r = 0; r < 4; ++r) s.tr[(g + 4 * r) * 17 + c] = W[r];
  wave_sync();
#pragma unroll
  for (int r = 0; r < 4; ++r) V[r] = s.tr[c * 17 + g + 4 * r];
  wave_sync();
  return info;
}

// Sets padding rows/columns (index >= nv) of a diagonal T-tile to the
// identity so that the factorization of the padded block is blockdiag(U, I).
__device__ __forceinline__ void pad_identity(d4 &T, int nv) {
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int p = g + 4 * r;
    if (p >= nv || c >= nv) T[r] = (p == c) ? 1.0 : 0.0;
  }
}

// Block of right-hand sides kept compact in LDS (16 rows x nrhs, row-major)
// <-> T-tile with the right-hand side index as the column: register r of lane
// (c, g) = buf[(g + 4r) * nrhs + c], zero for c >= nrhs.
__device__ __forceinline__ void save_compact(double *buf, const d4 &y, int nrhs) {
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
  if (c < nrhs) {
#pragma unroll
    for (int r = 0; r < 4; ++r) buf[(g + 4 * r) * nrhs + c] = y[r];
  }
}

__device__ __forceinline__ d4 load_compact(const double *buf, int nrhs) {
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
  d4 y;
#pragma unroll
  for (int r = 0; r < 4; ++r) y[r] = (c < nrhs) ? buf[(g + 4 * r) * nrhs + c] : 0.0;
  return y;
}

}  // namespace bh
