// Mixed-precision solves of an uneven batch A_i X_i = B_i (A_i SPD): the
// Cholesky factor is computed in single precision on the FP32 matrix cores
// (or with binary16 operands and FP32 accumulation), and FP64 iterative
// refinement recovers a solution whose backward error meets a tolerance;
// instances that do not get there are flagged and solved again by the FP64
// plan kernels.  Not part of the paper: its FP64 panel-major building blocks
// (§4.3 storage, §4.6 blocked factorization) carry over unchanged.
//
// Per instance (one workgroup of LW waves, instances longest first):
//   S     = diag(s), s_p = 2^-floor(e_p/2) for a_pp = m 2^e_p, m in [0.5, 1):
//           S A S has its diagonal in [0.5, 2) and is formed without rounding;
//   L32   = Cholesky factor of fl32(S A S), left-looking over block columns:
//           gemm downdate on the FP32 (or FP16-operand) MFMA, the 16x16
//           diagonal block factored and inverted in FP64 registers
//           (potrf_inv_tile_upper) and rounded back, off-diagonal blocks by
//           multiplication with the FP32 inverse;
//   solve d = S L32^-T L32^-1 fl32(S r), FP32 MFMA, right-looking over
//           blocks with one barrier per block;
//   x0    = solve(b); then r = b - A x (FP64 MFMA over the lower triangle of
//           A, each tile read once and applied as A(i,j) and A(i,j)^T),
//           backward error eta_c = |r_c|_inf / (|A|_inf |x_c|_inf + |b_c|_inf)
//           per right-hand side, stop when every eta_c <= tol, give up at
//           max_iter corrections or when an eta_c stops decreasing;
//           x_c += d_c for the columns not yet converged.
//
// The factor of each instance lives in a plan-owned workspace as 16x16 FP32
// tiles in MFMA register order ("T32 tiles": register r of lane (c, g) holds
// element [4g + r][c]; a tile is 1 KiB, one 16-byte load per lane):
//   U(j,i) = L(i,j)^T for i >= j      at tile  tix_up(j, i)
//   U(j,i)^T (i > j)                  at tile  NT + tix_up(j, i)
//   V_j = U(j,j)^-1, W_j = V_j^T      at tiles 2 NT + j, 2 NT + nb + j
// with NT = nb (nb + 1) / 2, nb = ceil(n / 16).
#include <algorithm>
#include <cstdint>
#include <cmath>
#include <vector>

#include "plan.hpp"

namespace bh {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));

struct MxArgs {
  const int *ids;
  int count;
  const int *n;
  const long long *moff, *voff, *woff;  // doubles, doubles, floats
  const double *A;
  const double *B;
  double *X;
  float *ws;
  int nrhs;
  double tol;
  int max_iter;
  int *iters;
  double *berr;
  int *fallback;
  int *info;
};

__device__ __forceinline__ f4 zero4f() { return (f4){0.f, 0.f, 0.f, 0.f}; }

// sum over the four registers of 16x16x4 products: X^T Y for T32 tiles
__device__ __forceinline__ f4 mfma32_tn(const f4 &X, const f4 &Y, f4 acc) {
#pragma unroll
  for (int r = 0; r < 4; ++r)
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(X[r], Y[r], acc, 0, 0, 0);
  return acc;
}

// X^T Y with both operands rounded to binary16: the four registers of a T32
// tile are exactly the k-slice of the 16x16x16 f16 operand of their lane.
__device__ __forceinline__ f4 mfma16_tn(const f4 &X, const f4 &Y, f4 acc) {
  const h4 xh = {(_Float16)X[0], (_Float16)X[1], (_Float16)X[2], (_Float16)X[3]};
  const h4 yh = {(_Float16)Y[0], (_Float16)Y[1], (_Float16)Y[2], (_Float16)Y[3]};
  return __builtin_amdgcn_mfma_f32_16x16x16f16(xh, yh, acc, 0, 0, 0);
}

template <bool H>
__device__ __forceinline__ f4 upd_tn(const f4 &X, const f4 &Y, f4 acc) {
  if constexpr (H)
    return mfma16_tn(X, Y, acc);
  else
    return mfma32_tn(X, Y, acc);
}

__device__ __forceinline__ f4 ld_tile(const float *t) {
  return *reinterpret_cast<const f4 *>(t + 4 * lane_id());
}
__device__ __forceinline__ void st_tile(float *t, const f4 &x) {
  *reinterpret_cast<f4 *>(t + 4 * lane_id()) = x;
}

// Blocks A(i0 + r, j), r < R, as they enter the U view: element k of lane
// (c, g) is a_pq with p = 16(i0 + r) + c, q = 16j + 4g + k.  Block rows past
// the last one repeat it.  Every lane loads unconditionally (masked elements
// read a_00), so all 4R loads are in flight together.
template <int R>
__device__ __forceinline__ void load_a64(const View &A, int i0, int j, int nb,
                                         double (&v)[R][4]) {
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int p = 16 * min(i0 + r, nb - 1) + c;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int q = 16 * j + 4 * g + k;
      const bool ok = p < A.rows && q < A.rows && p >= q;
      v[r][k] = A.p[ok ? pm_off(p, q, A.cn) : 0];
    }
  }
}

// acc[r] += fl32(s_p s_q a_pq) on the elements of the lower triangle of A
// (T32 tiles of the scaled A(i0 + r, j)^T; zero elsewhere)
template <int R>
__device__ __forceinline__ void add_a32(const View &A, const double *sc, int i0,
                                        int j, int nb, const double (&v)[R][4],
                                        f4 (&acc)[R]) {
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int p = 16 * min(i0 + r, nb - 1) + c;
    const double sp = sc[p];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int q = 16 * j + 4 * g + k;
      const bool ok = p < A.rows && q < A.rows && p >= q;
      const float x = (float)(v[r][k] * sp * sc[q]);
      acc[r][k] = ok ? acc[r][k] + x : acc[r][k];
    }
  }
}

// T-tile of A(i,j)^T in FP64: register r of lane (c, g) = a_pq with
// p = 16i + c, q = 16j + g + 4r; zero outside the matrix and, with lower,
// above the diagonal.  Unconditional loads (masked elements read a_00).
__device__ __forceinline__ d4 load_a64T(const View &A, int i, int j, bool lower) {
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
  const int p = 16 * i + c;
  double v[4];
  bool ok[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int q = 16 * j + g + 4 * r;
    ok[r] = p < A.rows && q < A.rows && (!lower || p >= q);
    v[r] = A.p[ok[r] ? pm_off(p, q, A.cn) : 0];
  }
  d4 t;
#pragma unroll
  for (int r = 0; r < 4; ++r) t[r] = ok[r] ? v[r] : 0.0;
  return t;
}

// T-tile of A(i,j) itself in FP64: register r of lane (c, g) = a_pq with
// p = 16i + g + 4r, q = 16j + c; zero outside the matrix and, with strict,
// on and above the diagonal.  Unconditional loads (masked elements read
// a_00).
__device__ __forceinline__ d4 load_a64N(const View &A, int i, int j, bool strict) {
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
  const int q = 16 * j + c;
  double v[4];
  bool ok[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int p = 16 * i + g + 4 * r;
    ok[r] = p < A.rows && q < A.rows && (!strict || p > q);
    v[r] = A.p[ok[r] ? pm_off(p, q, A.cn) : 0];
  }
  d4 t;
#pragma unroll
  for (int r = 0; r < 4; ++r) t[r] = ok[r] ? v[r] : 0.0;
  return t;
}

// k-th tile (i, j), i >= j, of step st of the residual sweep: the tiles with
// i + j = st (mod nb) touch pairwise distinct block rows (k < step_tiles)
__device__ __forceinline__ int step_tiles(int st, int nb) {
  return st / 2 + 1 + max(0, (st + nb) / 2 - st);
}
__device__ __forceinline__ void step_tile(int st, int nb, int k, int &i, int &j) {
  const int h = st / 2;
  if (k <= h) {
    j = k;
    i = st - k;
  } else {
    j = st + 1 + (k - h - 1);
    i = st - j + nb;
  }
}

// T32 tile (row 4g + r) <-> FP64 T-tile (row g + 4r), through 16x17 doubles
__device__ __forceinline__ d4 t32_to_t64(const f4 &x, double *tr) {
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) tr[(4 * g + r) * 17 + c] = (double)x[r];
  wave_sync();
  d4 y;
#pragma unroll
  for (int r = 0; r < 4; ++r) y[r] = tr[(g + 4 * r) * 17 + c];
  wave_sync();
  return y;
}

__device__ __forceinline__ f4 t64_to_t32(const d4 &x, double *tr) {
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) tr[(g + 4 * r) * 17 + c] = x[r];
  wave_sync();
  f4 y;
#pragma unroll
  for (int r = 0; r < 4; ++r) y[r] = (float)tr[(4 * g + r) * 17 + c];
  wave_sync();
  return y;
}

// transpose of a T32 tile through 16x17 floats
__device__ __forceinline__ f4 transpose32(const f4 &x, float *tr) {
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) tr[(4 * g + r) * 17 + c] = x[r];
  wave_sync();
  f4 y;
#pragma unroll
  for (int r = 0; r < 4; ++r) y[r] = tr[c * 17 + 4 * g + r];
  wave_sync();
  return y;
}

// compact FP32 vector block (16 rows x nrhs) <-> T32 tile, column = rhs
__device__ __forceinline__ f4 load_v32(const float *buf, int nrhs) {
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
  f4 y;
#pragma unroll
  for (int r = 0; r < 4; ++r) y[r] = (c < nrhs) ? buf[(4 * g + r) * nrhs + c] : 0.f;
  return y;
}

__device__ __forceinline__ void save_v32(float *buf, const f4 &y, int nrhs) {
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
  if (c < nrhs) {
#pragma unroll
    for (int r = 0; r < 4; ++r) buf[(4 * g + r) * nrhs + c] = y[r];
  }
}

// acc[r] -= sum_{q<j} U(q,j)^T U(q,i0 + r), r < R: one load of each U(q,j)
// serves the whole group of R block rows, and the tiles of QU steps of q are
// loaded together (indices past j - 1 are clamped, their products zeroed).
// Rows past the last block row repeat the last one (their results are
// dropped).  With DIAG the group starts at the diagonal block, whose second
// operand is U(q,j) itself.
template <bool H, int R, int QU, bool DIAG>
__device__ __forceinline__ void downdate32_rows(const float *Ut, int j, int i0,
                                                int nb, f4 (&acc)[R]) {
  int ti[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = min(i0 + r, nb - 1);
    ti[r] = i * (i + 1) / 2;
  }
  const float *uj = Ut + 256 * (j * (j + 1) / 2);
  for (int q = 0; q < j; q += QU) {
    f4 a[QU], b[QU][R];
#pragma unroll
    for (int u = 0; u < QU; ++u) {
      const int qq = min(q + u, j - 1);
      a[u] = ld_tile(uj + 256 * qq);
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (!(DIAG && r == 0)) b[u][r] = ld_tile(Ut + 256 * (ti[r] + qq));
    }
#pragma unroll
    for (int u = 0; u < QU; ++u) {
      // a skipped step multiplies by zero instead of branching, so that the
      // compiler keeps its loads with the others
      const f4 m = (u == 0 || q + u < j) ? -a[u] : zero4f();
#pragma unroll
      for (int r = 0; r < R; ++r)
        acc[r] = upd_tn<H>(m, (DIAG && r == 0) ? a[u] : b[u][r], acc[r]);
    }
  }
}

// maximum that propagates NaN (a NaN residual must never pass the test)
__device__ __forceinline__ double nmax(double a, double b) {
  return (b > a || b != b) ? b : a;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = nmax(v, __shfl_xor(v, o));
  return v;
}

// diagonal scaling s_p = 2^-floor(e/2) for a_pp = m 2^e (1 if a_pp is not
// positive and finite): s_p^2 a_pp lies in [0.5, 2), the scaling is exact
__device__ __forceinline__ double pow2_scale(double d) {
  if (!(d > 0.0 && d <= 1.79769313486231570815e308)) return 1.0;
  int e;
  (void)frexp(d, &e);
  return ldexp(1.0, -(e >> 1));
}

template <int LW>
struct FacLds {
  DiagLds diag;            // wave 0: diagonal block
  double tr[LW][16 * 17];  // per wave: transposes
  float vsh[256];          // V_j for all waves
  double sc[512];          // scaling
  int info;
};

// Factorization of fl32(S A S) into the workspace tiles, one workgroup of LW
// waves per instance, left-looking over block columns, block rows in groups
// of R (one load of the column's tiles per group; a block's entries of
// fl32(S A S) are added after its downdate sum, so that their loads overlap
// it): wave 0 takes the group
// that starts at the diagonal block, factors and inverts that block (FP64
// registers, rounded back to FP32) and finishes the rest of its group; the
// waves share the column's remaining groups.  Little LDS, so that many
// instances run on a CU at once.  fallback[id] = 1 if a pivot is not
// positive, else 0.
template <int LW, int R, int QU, bool ZA, bool H>
__global__ __launch_bounds__(64 * LW) void k_mx_fac(MxArgs a) {
  __shared__ FacLds<LW> s;
  const int t = blockIdx.x;
  if (t >= a.count) return;
  const int id = a.ids[t];
  const int n = a.n[id];
  const int nb = (n + 15) >> 4, cn = (n + 3) & ~3;
  const int nt = nb * (nb + 1) / 2;
  const int w = wave_id();
  const int l = lane_id();
  const int tid = threadIdx.x;
  constexpr int NTH = 64 * LW;
  const View A{const_cast<double *>(a.A + a.moff[id]), cn, 0, 0, n, n};
  float *Ut = a.ws + a.woff[id];
  float *Lt = Ut + 256LL * nt;
  float *Vt = Ut + 512LL * nt;
  float *Wt = Vt + 256LL * nb;
  double *tr = s.tr[w];
  float *trf = reinterpret_cast<float *>(tr);
  double *sc = s.sc;
  for (int p = tid; p < 16 * nb; p += NTH) sc[p] = p < n ? pow2_scale(A.p[pm_off(p, p, cn)]) : 1.0;
  if (tid == 0) s.info = 0;
  __syncthreads();
  // ---------------------------------------------------------------- factor
  for (int j = 0; j < nb; ++j) {
    f4 Vj = zero4f();
    if (w == 0) {
      double av[R][4];
      load_a64<R>(A, j, j, nb, av);
      f4 acc[R];
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] = zero4f();
      if (!ZA) add_a32<R>(A, sc, j, j, nb, av, acc);
      downdate32_rows<H, R, QU, true>(Ut, j, j, nb, acc);
      if (ZA) add_a32<R>(A, sc, j, j, nb, av, acc);
      d4 T = t32_to_t64(acc[0], tr);
      pad_identity(T, min(16, n - 16 * j));
      d4 V, W;
      const int inf = potrf_inv_tile_upper(T, V, s.diag, &W, (min(16, n - 16 * j) + 3) >> 2);
      if (inf && l == 0 && s.info == 0) s.info = 16 * j + inf;
      const f4 u32 = t64_to_t32(T, tr);
      const f4 v32 = t64_to_t32(V, tr);
      const f4 w32 = t64_to_t32(W, tr);
      st_tile(Ut + 256 * tix_up(j, j), u32);
      st_tile(Vt + 256 * j, v32);
      st_tile(Wt + 256 * j, w32);
      if (LW > 1) *reinterpret_cast<f4 *>(s.vsh + 4 * l) = v32;
      Vj = v32;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        if (j + r < nb) {
          const f4 u = mfma32_tn(v32, acc[r], zero4f());
          st_tile(Ut + 256 * tix_up(j, j + r), u);
          st_tile(Lt + 256 * tix_up(j, j + r), transpose32(u, trf));
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __syncthreads();
    if (s.info) break;
    if (j + R < nb) {
      const f4 V = w ? *reinterpret_cast<const f4 *>(s.vsh + 4 * l) : Vj;
      for (int i0 = j + R * (1 + w); i0 < nb; i0 += R * LW) {
        double av[R][4];
        load_a64<R>(A, i0, j, nb, av);
        f4 acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = zero4f();
        if (!ZA) add_a32<R>(A, sc, i0, j, nb, av, acc);
        downdate32_rows<H, R, QU, false>(Ut, j, i0, nb, acc);
        if (ZA) add_a32<R>(A, sc, i0, j, nb, av, acc);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (i0 + r < nb) {
            const f4 u = mfma32_tn(V, acc[r], zero4f());
            st_tile(Ut + 256 * tix_up(j, i0 + r), u);
            st_tile(Lt + 256 * tix_up(j, i0 + r), transpose32(u, trf));
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      __syncthreads();
    }
  }
  if (tid == 0) {
    a.fallback[id] = s.info ? 1 : 0;
    if (s.info) {
      a.iters[id] = 0;
      a.berr[id] = __builtin_inf();
      if (a.info) a.info[id] = 0;
    }
  }
}

template <int LW>
struct MxLds {
  double eprev[16];             // backward error per right-hand side
  double rmax[16], xmax[16], bmax[16];
  double anorm;
};

// FP64 iterative refinement on the factor that k_mx_fac left in the
// workspace (instances with fallback[id] == 1 are skipped): one workgroup of
// LW waves per instance, the iterate, residual and solve vectors in LDS.
template <int LW, int RT>
__global__ __launch_bounds__(64 * LW) void k_mx_ir(MxArgs a, int nbmax) {
  extern __shared__ double dyn[];
  __shared__ MxLds<LW> s;
  const int t = blockIdx.x;
  if (t >= a.count) return;
  const int id = a.ids[t];
  if (a.fallback[id] == 1) return;
  const int n = a.n[id];
  const int nb = (n + 15) >> 4, cn = (n + 3) & ~3, ld = (n + 15) & ~15;
  const int nt = nb * (nb + 1) / 2;
  const int nr = a.nrhs;
  const int w = wave_id();
  const int l = lane_id();
  const int tid = threadIdx.x;
  constexpr int NTH = 64 * LW;
  const int nv16 = 16 * nb;

  // dynamic LDS: x, r (FP64, compact n16 x nr), row sums of |A|, scaling,
  // the FP32 vector of the solve
  double *x64 = dyn;
  double *r64 = x64 + (long long)nbmax * 16 * nr;
  double *arow = r64 + (long long)nbmax * 16 * nr;
  double *sc = arow + nbmax * 16;
  float *vz = reinterpret_cast<float *>(sc + nbmax * 16);

  const View A{const_cast<double *>(a.A + a.moff[id]), cn, 0, 0, n, n};
  const double *Bb = a.B + a.voff[id];
  float *Ut = a.ws + a.woff[id];
  float *Lt = Ut + 256LL * nt;
  float *Vt = Ut + 512LL * nt;
  float *Wt = Vt + 256LL * nb;
  for (int p = tid; p < nv16; p += NTH) {
    sc[p] = p < n ? pow2_scale(A.p[pm_off(p, p, cn)]) : 1.0;
    arow[p] = 0.0;
  }
  __syncthreads();

  // |b_c|_inf
  for (int c = w; c < nr; c += LW) {
    double m = 0.0;
    for (int p = l; p < n; p += 64) m = nmax(m, fabs(Bb[(long long)c * ld + p]));
    m = wave_max(m);
    if (l == 0) {
      s.bmax[c] = m;
      s.eprev[c] = __builtin_inf();
    }
  }
  // x = 0 and the first right-hand side of the solve: fl32(S b)
  for (int e = tid; e < nv16 * nr; e += NTH) {
    const int p = e / nr, c = e - p * nr;
    x64[e] = 0.0;
    vz[e] = p < n ? (float)(sc[p] * Bb[(long long)c * ld + p]) : 0.f;
  }
  __syncthreads();

  int it = 0, fb = 0;
  double worst = 0.0;
  for (;;) {
    // ------------------------------------------------ solve in FP32, in place
    // block row i is updated by wave i % LW, which also takes its diagonal
    // step; the inverse of the next diagonal block is loaded a step early
    // and each wave loads its tiles of a step in groups of RT
    f4 Dn = w == 0 ? ld_tile(Vt) : zero4f();
    for (int j = 0; j < nb; ++j) {
      if (w == j % LW) {
        const f4 z = load_v32(vz + 16 * j * nr, nr);
        save_v32(vz + 16 * j * nr, mfma32_tn(Dn, z, zero4f()), nr);
      }
      __syncthreads();
      if (j + 1 < nb && w == (j + 1) % LW) Dn = ld_tile(Vt + 256 * (j + 1));
      const f4 y = load_v32(vz + 16 * j * nr, nr);
      const int i0 = j + 1 + ((w - (j + 1) % LW) + LW) % LW;
      for (int ib = i0; ib < nb; ib += RT * LW) {
        f4 Us[RT];
#pragma unroll
        for (int m = 0; m < RT; ++m) Us[m] = ld_tile(Ut + 256 * tix_up(j, min(ib + m * LW, nb - 1)));
#pragma unroll
        for (int m = 0; m < RT; ++m) {
          const int i = ib + m * LW;
          if (i >= nb) break;
          f4 z = load_v32(vz + 16 * i * nr, nr);
          z = mfma32_tn(-Us[m], y, z);
          save_v32(vz + 16 * i * nr, z, nr);
        }
      }
    }
    Dn = w == (nb - 1) % LW ? ld_tile(Wt + 256 * (nb - 1)) : zero4f();
    for (int i = nb - 1; i >= 0; --i) {
      if (w == i % LW) {
        const f4 z = load_v32(vz + 16 * i * nr, nr);
        save_v32(vz + 16 * i * nr, mfma32_tn(Dn, z, zero4f()), nr);
      }
      __syncthreads();
      if (i > 0 && w == (i - 1) % LW) Dn = ld_tile(Wt + 256 * (i - 1));
      const f4 xi = load_v32(vz + 16 * i * nr, nr);
      for (int jb = w; jb < i; jb += RT * LW) {
        f4 Ls[RT];
#pragma unroll
        for (int m = 0; m < RT; ++m) Ls[m] = ld_tile(Lt + 256 * tix_up(min(jb + m * LW, i - 1), i));
#pragma unroll
        for (int m = 0; m < RT; ++m) {
          const int j = jb + m * LW;
          if (j >= i) break;
          f4 z = load_v32(vz + 16 * j * nr, nr);
          z = mfma32_tn(-Ls[m], xi, z);
          save_v32(vz + 16 * j * nr, z, nr);
        }
      }
    }
    __syncthreads();
    // x += S d (columns already converged carry d = 0)
    for (int e = tid; e < nv16 * nr; e += NTH) {
      const int p = e / nr;
      x64[e] += sc[p] * (double)vz[e];
    }
    __syncthreads();

    // ------------------------------------------ r = b - A x in FP64, |A|_inf
    for (int e = tid; e < nv16 * nr; e += NTH) {
      const int p = e / nr, c = e - p * nr;
      r64[e] = p < n ? Bb[(long long)c * ld + p] : 0.0;
    }
    __syncthreads();
    const bool first = it == 0;
    // step st: the tiles (i, j), i >= j, i + j = st (mod nb) touch distinct
    // block rows, so their updates of r (and of the row sums) do not collide;
    // each wave loads its tiles of a step in groups of RT before using them
    for (int st = 0; st < nb; ++st) {
      const int cnt = step_tiles(st, nb);
      for (int k0 = w; k0 < cnt; k0 += RT * LW) {
        d4 Xs[RT], Ns[RT];
#pragma unroll
        for (int m = 0; m < RT; ++m) {
          int i, j;
          step_tile(st, nb, min(k0 + m * LW, cnt - 1), i, j);
          Xs[m] = load_a64T(A, i, j, i == j);  // A(i,j)^T
          Ns[m] = load_a64N(A, i, j, i == j);  // A(i,j), strictly lower if i == j
        }
#pragma unroll
        for (int m = 0; m < RT; ++m) {
          if (k0 + m * LW >= cnt) break;
          int i, j;
          step_tile(st, nb, k0 + m * LW, i, j);
          d4 X = Xs[m];
          const int c = l & 15, g = l >> 4;
          d4 ri = load_compact(r64 + 16 * i * nr, nr);
          ri = mfma_tn(neg4(X), load_compact(x64 + 16 * j * nr, nr), ri);
          // row sums of |A(i,j)| (rows 16i + c); on a diagonal block, of its
          // lower part including the diagonal
          double rs = fabs(X[0]) + fabs(X[1]) + fabs(X[2]) + fabs(X[3]);
          if (i == j) {  // keep the strictly lower part: it also acts as the upper
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (c == g + 4 * r) X[r] = 0.0;
          }
          if (first) {
            rs += __shfl_xor(rs, 16);
            rs += __shfl_xor(rs, 32);
            if (g == 0) arow[16 * i + c] += rs;
            // column sums (rows 16j + g + 4r of the symmetric matrix)
            d4 cs;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              double v = fabs(X[r]);
              v += __shfl_xor(v, 1);
              v += __shfl_xor(v, 2);
              v += __shfl_xor(v, 4);
              v += __shfl_xor(v, 8);
              cs[r] = v;
            }
            if (c == 0) {
#pragma unroll
              for (int r = 0; r < 4; ++r) arow[16 * j + g + 4 * r] += cs[r];
            }
          }
          const d4 Xt = Ns[m];  // the same block in the other layout (an L1/L2 hit)
          if (i != j) {
            save_compact(r64 + 16 * i * nr, ri, nr);
            d4 rj = load_compact(r64 + 16 * j * nr, nr);
            rj = mfma_tn(neg4(Xt), load_compact(x64 + 16 * i * nr, nr), rj);
            save_compact(r64 + 16 * j * nr, rj, nr);
          } else {
            ri = mfma_tn(neg4(Xt), load_compact(x64 + 16 * i * nr, nr), ri);
            save_compact(r64 + 16 * i * nr, ri, nr);
          }
        }
      }
      __syncthreads();
    }

    // ------------------------------------------------ backward errors
    if (first && w == 0) {
      double m = 0.0;
      for (int p = l; p < n; p += 64) m = nmax(m, arow[p]);
      m = wave_max(m);
      if (l == 0) s.anorm = m;
    }
    for (int c = w; c < nr; c += LW) {
      double mr = 0.0, mx = 0.0;
      for (int p = l; p < n; p += 64) {
        mr = nmax(mr, fabs(r64[p * nr + c]));
        mx = nmax(mx, fabs(x64[p * nr + c]));
      }
      mr = wave_max(mr);
      mx = wave_max(mx);
      if (l == 0) {
        s.rmax[c] = mr;
        s.xmax[c] = mx;
      }
    }
    __syncthreads();
    bool done = true, stalled = false;
    worst = 0.0;
    unsigned active = 0;
    for (int c = 0; c < nr; ++c) {
      const double den = s.anorm * s.xmax[c] + s.bmax[c];
      const double eta = den > 0.0 ? s.rmax[c] / den : s.rmax[c];
      worst = (eta > worst || eta != eta) ? eta : worst;
      if (!(eta <= a.tol)) {
        done = false;
        active |= 1u << c;
        if (!(eta < s.eprev[c])) stalled = true;
      }
    }
    __syncthreads();
    if (tid < nr) {
      const int c = tid;
      const double den = s.anorm * s.xmax[c] + s.bmax[c];
      s.eprev[c] = den > 0.0 ? s.rmax[c] / den : s.rmax[c];
    }
    if (done) break;
    if (it >= a.max_iter || stalled) {
      fb = 2;
      break;
    }
    // next right-hand side of the solve: fl32(S r) on the active columns
    for (int e = tid; e < nv16 * nr; e += NTH) {
      const int p = e / nr, c = e - p * nr;
      const double v = ((active >> c) & 1u) ? sc[p] * r64[e] : 0.0;
      vz[e] = (float)v;
    }
    __syncthreads();
    ++it;
  }

  double *Xb = a.X + a.voff[id];
  for (int e = tid; e < n * nr; e += NTH) {
    const int p = e / nr, c = e - p * nr;
    Xb[(long long)c * ld + p] = x64[e];
  }
  if (tid == 0) {
    a.iters[id] = it;
    a.berr[id] = worst;
    a.fallback[id] = fb;
    if (a.info) a.info[id] = 0;
  }
}

size_t mx_lds_bytes(int nbmax, int nrhs) {
  return (size_t)nbmax * 16 * (sizeof(double) * (2 * nrhs + 2) + sizeof(float) * nrhs);
}

template <int LW, int RT>
static hipError_t mx_prepare(size_t lds) {
  return hipFuncSetAttribute((const void *)k_mx_ir<LW, RT>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

// FP32 factor tiles of instance `id` -> column-major lower triangle
__global__ void k_mx_factor(const float *ws, long long woff, int n, float *dst,
                            int ldd) {
  const int q = blockIdx.y;  // column
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n || q >= n) return;
  float v = 0.f;
  if (p >= q) {
    const int i = p >> 4, b = p & 15, j = q >> 4, aa = q & 15;
    const int g = aa >> 2, r = aa & 3, ln = b + 16 * g;
    v = ws[woff + 256LL * tix_up(j, i) + 4 * ln + r];
  }
  dst[(long long)q * ldd + p] = v;
}

}  // namespace bh

using namespace bh;

static const int kMxLW = 4;     // waves per instance, refinement
static const int kMxRT = 2;     // residual tiles per wave loaded together
static const int kMxFacLW = 1;  // waves per instance, factorization
static const int kMxFacR = 4;   // block rows per downdate group, factorization
static const int kMxFacQU = 2;  // steps of the downdate sum loaded together
static const bool kMxFacZA = true;  // A added after the downdate sum

int bh::mx_plan_setup(blasfeo_hip_plan *p) {
  p->mx_ok = false;
  if (p->nrhs < 1) return 0;
  std::vector<long long> woff(p->batch);
  long long wo = 0;
  int nbmax = 0;
  for (int i = 0; i < p->batch; ++i) {
    const int nb = (p->n[i] + 15) / 16;
    nbmax = std::max(nbmax, nb);
    woff[i] = wo;
    wo += 256LL * (nb * (nb + 1) + 2 * nb);
  }
  const size_t lds = mx_lds_bytes(nbmax, p->nrhs);
  if (lds + sizeof(MxLds<kMxLW>) > 160 * 1024) return 0;  // mixed solves unavailable
  std::vector<int> ids(p->batch);
  for (int i = 0; i < p->batch; ++i) ids[i] = i;
  std::stable_sort(ids.begin(), ids.end(),
                   [&](int x, int y) { return p->n[x] > p->n[y]; });
  const size_t nbt = (size_t)std::max(p->batch, 1);
  hipError_t e = hipMalloc(&p->d_woff, nbt * sizeof(long long));
  if (e == hipSuccess) e = hipMalloc(&p->d_mx_ids, nbt * sizeof(int));
  if (e == hipSuccess && p->batch > 0) {
    e = hipMemcpy(p->d_woff, woff.data(), p->batch * sizeof(long long), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(p->d_mx_ids, ids.data(), p->batch * sizeof(int), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = mx_prepare<kMxLW, kMxRT>(lds);
  if (e != hipSuccess) return (int)e;  // the caller destroys the plan
  p->ws32_bytes = wo * (long long)sizeof(float);
  p->mx_nbmax = nbmax;
  p->mx_ok = true;
  return 0;
}

extern "C" {

int blasfeo_hip_dposv_mixed_vbatched(blasfeo_hip_plan *p, int prec, double tol,
                                     int max_iter, const void *A, const void *B,
                                     void *X, void *L, int *info, int *iters,
                                     double *berr, int *fallback, void *work,
                                     void *stream) {
  if (!p || !p->mx_ok) return -1;
  if (prec != 1 && prec != 2) return -2;
  if (!(tol >= 0.0)) return -3;
  if (max_iter < 0) return -4;
  if (p->batch == 0) return 0;
  if (!A) return -5;
  if (!B) return -6;
  if (!X) return -7;
  if (!iters) return -10;
  if (!berr) return -11;
  if (!fallback) return -12;
  if (!work || ((uintptr_t)work & 255)) return -13;
  hipStream_t st = (hipStream_t)stream;
  MxArgs a;
  a.ids = p->d_mx_ids;
  a.count = p->batch;
  a.n = p->d_n;
  a.moff = p->d_moff;
  a.voff = p->d_voff;
  a.woff = p->d_woff;
  a.A = (const double *)A;
  a.B = (const double *)B;
  a.X = (double *)X;
  a.ws = (float *)((char *)work + round256(p->ws64_bytes));
  a.nrhs = p->nrhs;
  a.tol = tol;
  a.max_iter = max_iter;
  a.iters = iters;
  a.berr = berr;
  a.fallback = fallback;
  a.info = info;
  const size_t lds = mx_lds_bytes(p->mx_nbmax, p->nrhs);
  if (prec == 2)
    hipLaunchKernelGGL((k_mx_fac<kMxFacLW, kMxFacR, kMxFacQU, kMxFacZA, true>), dim3(p->batch), dim3(64 * kMxFacLW), 0, st, a);
  else
    hipLaunchKernelGGL((k_mx_fac<kMxFacLW, kMxFacR, kMxFacQU, kMxFacZA, false>), dim3(p->batch), dim3(64 * kMxFacLW), 0, st, a);
  hipLaunchKernelGGL((k_mx_ir<kMxLW, kMxRT>), dim3(p->batch), dim3(64 * kMxLW), lds, st, a, p->mx_nbmax);
  int e = launch_status();
  if (e) return e;
  // FP64 solve of the instances that fell back (workspace: the FP64 part)
  if (L) e = launch_all(p, (const double *)A, (double *)L, (const double *)B,
                        (double *)X, info, (double *)work, st, fallback);
  return e;
}

int blasfeo_hip_plan_mixed_factor(const blasfeo_hip_plan *p, int i,
                                  const void *work, float *dst, int ldd,
                                  void *stream) {
  if (!p || !p->mx_ok) return -1;
  if (i < 0 || i >= p->batch) return -2;
  if (!work || ((uintptr_t)work & 255)) return -3;
  if (!dst) return -4;
  const int n = p->n[i];
  if (ldd < n) return -5;
  long long wo = 0;
  for (int k = 0; k < i; ++k) {
    const int nb = (p->n[k] + 15) / 16;
    wo += 256LL * (nb * (nb + 1) + 2 * nb);
  }
  const float *ws = (const float *)((const char *)work + round256(p->ws64_bytes));
  hipLaunchKernelGGL(k_mx_factor, dim3((n + 63) / 64, n), dim3(64), 0,
                     (hipStream_t)stream, ws, wo, n, dst, ldd);
  return launch_status();
}

}  // extern "C"
