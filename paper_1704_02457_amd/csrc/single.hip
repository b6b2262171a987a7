// Single-precision public routines.  The routine list of Appendix A.3 comes
// in single and double precision; §4.8 fixes the panel size per precision
// so that one panel column fills a cache line.  struct blasfeo_smat stores
// panels of 32 floats (one 128-byte line per panel column, as the 16-double
// panels of blasfeo_dmat); element (i, j) is at
//   pA[(i - i % 32) * cn + j * 32 + i % 32],  cn = round_up(n, 4).
// Memory handling and packing mirror the double-precision ones; the
// compute kernels run on the FP32 matrix cores (16x16x4 f32 MFMA), and the
// 16x16 diagonal blocks of the Cholesky factorization are factored and
// inverted by the FP64 register routine and rounded back to single.
//
// FP32 register tile ("T32"): register r of lane (c, g) holds row 4g + r,
// column c of a 16x16 block; sum_r mfma_f32(X[r], Y[r]) = X^T Y for two such
// tiles, and mfma_f32 on two 16x4 fragments F1 (rows i, k) and F2 (rows j,
// k) accumulates F1 F2^T in the same layout.
#include "common.hpp"

namespace bh {

constexpr int PSS = 32;  // single-precision panel size

typedef float f4s __attribute__((ext_vector_type(4)));

__host__ __device__ inline long long pm_off_s(int i, int j, int cn) {
  return (long long)(i & ~(PSS - 1)) * cn + (long long)j * PSS + (i & (PSS - 1));
}

struct SView {
  float *p;
  int cn;
  int ai, aj;
  int rows, cols;
};

inline SView make_sview(const blasfeo_smat *s, int ai, int aj, int rows, int cols) {
  return SView{s->pA, s->cn, ai, aj, rows, cols};
}

inline bool soperand_ok(const blasfeo_smat *s, int ai, int aj, int rows, int cols) {
  if (!s) return false;
  if (ai < 0 || aj < 0 || rows < 0 || cols < 0) return false;
  if ((long long)ai + rows > s->m || (long long)aj + cols > s->n) return false;
  if (rows > 0 && cols > 0 && !s->pA) return false;
  if (s->cn < s->n || s->pm * PSS < s->m) return false;
  return true;
}

inline long long sbatch_stride(const blasfeo_smat *s) { return s->memsize / 4; }

__device__ __forceinline__ SView sat_batch(SView v, long long stride) {
  v.p += (long long)blockIdx.y * stride;
  return v;
}

// 16x4 fragment S[i0:i0+16, k0:k0+4]: lane (c, g) holds S[i0 + c][k0 + g]
// (zero outside S; unconditional load from a clamped address)
__device__ __forceinline__ float sload_frag(const SView &v, int i0, int k0) {
  const int l = lane_id();
  const int i = i0 + (l & 15), k = k0 + (l >> 4);
  const bool ok = i < v.rows && k < v.cols;
  const float x = v.p[ok ? pm_off_s(v.ai + i, v.aj + k, v.cn) : pm_off_s(v.ai, v.aj, v.cn)];
  return ok ? x : 0.0f;
}

// The same fragment without the final select: elements outside S come from
// S's origin (any finite value), for callers that mask later.
__device__ __forceinline__ float sload_frag_raw(const SView &v, int i0, int k0) {
  const int l = lane_id();
  const int i = i0 + (l & 15), k = k0 + (l >> 4);
  const bool ok = i < v.rows && k < v.cols;
  return v.p[ok ? pm_off_s(v.ai + i, v.aj + k, v.cn) : pm_off_s(v.ai, v.aj, v.cn)];
}

// T32 tile of block S(i0.., j0..): register r of lane (c, g) = S[i0 + 4g + r][j0 + c]
// (trans: S[i0 + c][j0 + 4g + r]); zero outside S and, with lower, where
// the block's row index is below its column index
__device__ __forceinline__ f4s sload_tile(const SView &v, int i0, int j0, bool trans, bool lower) {
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
  f4s t;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = trans ? i0 + c : i0 + 4 * g + r, j = trans ? j0 + 4 * g + r : j0 + c;
    const bool ok = i < v.rows && j < v.cols && (!lower || i - i0 >= j - j0);
    const float x = v.p[ok ? pm_off_s(v.ai + i, v.aj + j, v.cn) : pm_off_s(v.ai, v.aj, v.cn)];
    t[r] = ok ? x : 0.0f;
  }
  return t;
}

__device__ __forceinline__ void sstore_tile(const SView &v, int i0, int j0, const f4s &t,
                                            bool trans, bool lower) {
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = trans ? i0 + c : i0 + 4 * g + r, j = trans ? j0 + 4 * g + r : j0 + c;
    if (i < v.rows && j < v.cols && (!lower || i - i0 >= j - j0))
      v.p[pm_off_s(v.ai + i, v.aj + j, v.cn)] = t[r];
  }
}

__device__ __forceinline__ f4s smfma(float a, float b, f4s acc) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
}

__device__ __forceinline__ f4s smfma_tn(const f4s &X, const f4s &Y, f4s acc) {
#pragma unroll
  for (int r = 0; r < 4; ++r) acc = smfma(X[r], Y[r], acc);
  return acc;
}

// T32 (row 4g + r) <-> FP64 T-tile (row g + 4r) through 16x17 doubles
__device__ __forceinline__ d4 st32_to_t64(const f4s &x, double *tr) {
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

__device__ __forceinline__ f4s st64_to_t32(const d4 &x, double *tr) {
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) tr[(g + 4 * r) * 17 + c] = x[r];
  wave_sync();
  f4s y;
#pragma unroll
  for (int r = 0; r < 4; ++r) y[r] = (float)tr[(4 * g + r) * 17 + c];
  wave_sync();
  return y;
}

// ---------------------------------------------------------------- pack
__global__ void k_spack(int batch, int m, int n, const float *__restrict__ A, int lda,
                        long long sa, float *__restrict__ B, int cn, int bi, int bj,
                        long long sb, int to_panel) {
  const long long per = (long long)m * n;
  const long long total = per * batch;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const long long b = t / per, e = t - b * per;
    const int i = (int)(e % m), j = (int)(e / m);
    const long long po = b * sb + pm_off_s(bi + i, bj + j, cn);
    const long long co = b * sa + (long long)i + (long long)j * lda;
    if (to_panel)
      B[po] = A[co];
    else
      ((float *)A)[co] = B[po];
  }
}

static int launch_spack(int batch, int m, int n, const float *A, int lda, long long sa,
                        float *B, int cn, int bi, int bj, long long sb, int to_panel,
                        hipStream_t st) {
  if (batch == 0 || m == 0 || n == 0) return 0;
  const long long total = (long long)m * n * batch;
  long long blocks = (total + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_spack, dim3((unsigned)blocks), dim3(256), 0, st, batch, m, n, A, lda,
                     sa, B, cn, bi, bj, sb, to_panel);
  return launch_status();
}

// ---------------------------------------------------------------- gemm/syrk
// One wave per 64x64 block of D (4x4 tiles of 16x16): per 4-wide k-step it
// loads four fragments of A and four of B and issues the 16 FP32 MFMAs of
// their outer product, D = beta C + alpha sum_k A B^T.  The accumulators hold
// D^T (B fragment first) so that the lanes of a store run down a panel
// column: 64-byte contiguous segments instead of scattered words.  syrk_ln takes the
// blocks on and below the diagonal and stores the lower triangle only.
template <bool SYRK>
__global__ __launch_bounds__(256) void k_sgemm_nt(int m, int n, int k, float alpha, SView A,
                                                  SView B, float beta, SView C, SView D,
                                                  long long sA, long long sB, long long sC,
                                                  long long sD) {
  A = sat_batch(A, sA);
  B = sat_batch(B, sB);
  C = sat_batch(C, sC);
  D = sat_batch(D, sD);
  const int bm = (m + 63) >> 6, bn = (n + 63) >> 6;
  const int blk = blockIdx.x * 4 + wave_id();
  int bi, bj;
  if (SYRK) {
    if (blk >= bm * (bm + 1) / 2) return;
    bi = 0;
    while ((bi + 1) * (bi + 2) / 2 <= blk) ++bi;
    bj = blk - bi * (bi + 1) / 2;
  } else {
    if (blk >= bm * bn) return;
    bi = blk / bn;
    bj = blk - bi * bn;
  }
  const int i0 = 64 * bi, j0 = 64 * bj;
  f4s acc[4][4];
#pragma unroll
  for (int ti = 0; ti < 4; ++ti)
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) acc[ti][tj] = (f4s){0.f, 0.f, 0.f, 0.f};
  // Fragments of step k0 + 4 are loaded before the MFMAs of step k0, and
  // scheduling barriers keep the compiler from moving them (or the waits for
  // them) back.  Rows of A or B beyond m or n only reach rows or columns of
  // the accumulators that are never stored, so only the k index is masked,
  // on both fragments (a non-finite element read in place of a missing
  // column would otherwise reach every output through 0 * inf).
  const int g = lane_id() >> 4;
  float fa[4] = {0.f, 0.f, 0.f, 0.f}, fb[4] = {0.f, 0.f, 0.f, 0.f};
  if (k > 0) {  // k == 0: A and B are empty views without storage
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const float xa = sload_frag_raw(A, i0 + 16 * t, 0);
      const float x = sload_frag_raw(B, j0 + 16 * t, 0);
      fa[t] = g < k ? xa : 0.f;
      fb[t] = g < k ? x : 0.f;
    }
  }
  for (int k0 = 0; k0 < k; k0 += 4) {
    float na[4], nb[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      na[t] = sload_frag_raw(A, i0 + 16 * t, k0 + 4);
      nb[t] = sload_frag_raw(B, j0 + 16 * t, k0 + 4);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) acc[ti][tj] = smfma(fb[tj], fa[ti], acc[ti][tj]);
    __builtin_amdgcn_sched_barrier(0);
    const bool kin = k0 + 4 + g < k;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      fa[t] = kin ? na[t] : 0.f;
      fb[t] = kin ? nb[t] : 0.f;
    }
  }
#pragma unroll
  for (int ti = 0; ti < 4; ++ti)
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) {
      const int r0 = i0 + 16 * ti, c0 = j0 + 16 * tj;
      if (r0 >= m || c0 >= n || (SYRK && c0 > r0)) continue;
      const bool diag = SYRK && r0 == c0;
      const f4s ct = sload_tile(C, r0, c0, true, diag);
      f4s out;
#pragma unroll
      for (int r = 0; r < 4; ++r) out[r] = beta * ct[r] + alpha * acc[ti][tj][r];
      sstore_tile(D, r0, c0, out, true, diag);
    }
}

// ---------------------------------------------------------------- potrf_l
// Left-looking over block columns, one workgroup of 4 waves per instance:
// wave 0 forms M = C(j,j) - sum_q L(j,q) L(j,q)^T (as its transpose, in the
// upper triangle), factors and inverts it in FP64 registers and keeps
// V = U^{-1} (U = L(j,j)^T) as a T32 tile in LDS; then every wave takes
// block rows i > j: L(i,j)^T = V^T (C(i,j) - sum_q L(i,q) L(j,q)^T)^T.
struct SPotrfLds {
  DiagLds d;
  double tr[16 * 17];
  float V[256];
  int info;
};

__global__ __launch_bounds__(256) void k_spotrf_l(int m, SView C, SView D, float *dA, int *info,
                                                  long long sC, long long sD, long long sdA) {
  __shared__ SPotrfLds s;
  C = sat_batch(C, sC);
  D = sat_batch(D, sD);
  const long long b = blockIdx.y;
  float *dAb = dA ? dA + b * sdA : nullptr;
  const int w = wave_id();
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
  const int nb = (m + 15) >> 4;
  if (threadIdx.x == 0) s.info = 0;
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    const int nv = min(16, m - 16 * j);
    if (w == 0) {
      // M^T: register r of lane (c, g) = C[16j + c][16j + 4g + r] - (L_j L_j^T)
      f4s t = sload_tile(C, 16 * j, 16 * j, true, true);
      for (int k0 = 0; k0 < 16 * j; k0 += 4) {
        const float fj = sload_frag(D, 16 * j, k0);
        t = smfma(-fj, fj, t);
      }
      d4 T = st32_to_t64(t, s.tr);
      pad_identity(T, nv);
      d4 V, W;
      const int inf = potrf_inv_tile_upper(T, V, s.d, &W, (nv + 3) >> 2);
      if (inf && l == 0 && s.info == 0) s.info = 16 * j + inf;
      // L(j,j) = U^T: row 16j + c, column 16j + g + 4r holds U[g + 4r][c]
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * j + c, col = 16 * j + g + 4 * r;
        if (row < m && c >= g + 4 * r) D.p[pm_off_s(D.ai + row, D.aj + col, D.cn)] = (float)T[r];
      }
      if (dAb && l < nv) dAb[16 * j + l] = (float)s.d.inv[l];
      const f4s v32 = st64_to_t32(V, s.tr);
      *reinterpret_cast<f4s *>(s.V + 4 * l) = v32;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __syncthreads();
    const f4s V = *reinterpret_cast<const f4s *>(s.V + 4 * l);
    for (int i = j + 1 + w; i < nb; i += 4) {
      // M(i,j)^T: register r of lane (c, g) = C[16i + c][16j + 4g + r] - (L_j L_i^T)
      f4s t = sload_tile(C, 16 * i, 16 * j, true, false);
      for (int k0 = 0; k0 < 16 * j; k0 += 4)
        t = smfma(-sload_frag(D, 16 * j, k0), sload_frag(D, 16 * i, k0), t);
      const f4s u = smfma_tn(V, t, (f4s){0.f, 0.f, 0.f, 0.f});  // L(i,j)^T = V^T M^T
      sstore_tile(D, 16 * i, 16 * j, u, true, false);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __syncthreads();
  }
  if (info && threadIdx.x == 0) info[b] = s.info;
}

// m <= 16*NB <= 64: one wave per instance with the whole lower triangle in
// registers as T32 tiles T(j,i) = C(i,j)^T, right-looking: for each block
// column the FP64 diagonal routine, T(j,i) = V^T T(j,i) = L(i,j)^T for the
// blocks below, and the trailing downdates T(q,i) -= T(j,q)^T T(j,i) on the
// FP32 MFMA.  Every block is read and written once, with no barrier.
template <int NB>
__global__ __launch_bounds__(64) void k_spotrf_reg(int m, SView C, SView D, float *dA, int *info,
                                                   long long sC, long long sD, long long sdA) {
  struct Lds {
    DiagLds d;
    double tr[16 * 17];
  };
  __shared__ Lds s;
  C = sat_batch(C, sC);
  D = sat_batch(D, sD);
  const long long b = blockIdx.y;
  float *dAb = dA ? dA + b * sdA : nullptr;
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
  constexpr int NT = NB * (NB + 1) / 2;
  f4s T[NT];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) T[tix_up(j, i)] = sload_tile(C, 16 * i, 16 * j, true, i == j);
  int inf0 = 0;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int nv = min(16, m - 16 * j);
    d4 Dj = st32_to_t64(T[tix_up(j, j)], s.tr);
    pad_identity(Dj, nv);
    d4 V;
    const int inf = potrf_inv_tile_upper(Dj, V, s.d, nullptr, (nv + 3) >> 2);
    if (inf && inf0 == 0) inf0 = 16 * j + inf;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * j + c, col = 16 * j + g + 4 * r;
      if (row < m && c >= g + 4 * r) D.p[pm_off_s(D.ai + row, D.aj + col, D.cn)] = (float)Dj[r];
    }
    if (dAb && l < nv) dAb[16 * j + l] = (float)s.d.inv[l];
    const f4s V32 = st64_to_t32(V, s.tr);
#pragma unroll
    for (int i = j + 1; i < NB; ++i) {
      T[tix_up(j, i)] = smfma_tn(V32, T[tix_up(j, i)], (f4s){0.f, 0.f, 0.f, 0.f});
      sstore_tile(D, 16 * i, 16 * j, T[tix_up(j, i)], true, false);
    }
#pragma unroll
    for (int q = j + 1; q < NB; ++q) {
      const f4s nq = -T[tix_up(j, q)];
#pragma unroll
      for (int i = q; i < NB; ++i) T[tix_up(q, i)] = smfma_tn(nq, T[tix_up(j, i)], T[tix_up(q, i)]);
    }
  }
  if (info && l == 0) info[b] = inf0;
}

__global__ void k_sfill_int(int *p, int count, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

static int launch_sgemm(bool syrk, int batch, int m, int n, int k, float alpha,
                        const blasfeo_smat *sA, int ai, int aj, const blasfeo_smat *sB, int bi,
                        int bj, float beta, const blasfeo_smat *sC, int ci, int cj,
                        const blasfeo_smat *sD, int di, int dj, hipStream_t st) {
  if (batch == 0 || m == 0 || n == 0) return 0;
  const int bm = (m + 63) / 64, bn = (n + 63) / 64;
  const int blocks = syrk ? bm * (bm + 1) / 2 : bm * bn;
  const dim3 grid((blocks + 3) / 4, batch);
  const SView A = k > 0 ? make_sview(sA, ai, aj, m, k) : SView{};
  const SView B = k > 0 ? make_sview(sB, bi, bj, n, k) : SView{};
  const SView C = make_sview(sC, ci, cj, m, n), D = make_sview(sD, di, dj, m, n);
  const long long ssA = k > 0 ? sbatch_stride(sA) : 0, ssB = k > 0 ? sbatch_stride(sB) : 0;
  if (syrk)
    hipLaunchKernelGGL(k_sgemm_nt<true>, grid, dim3(256), 0, st, m, n, k, alpha, A, B, beta, C,
                       D, ssA, ssB, sbatch_stride(sC), sbatch_stride(sD));
  else
    hipLaunchKernelGGL(k_sgemm_nt<false>, grid, dim3(256), 0, st, m, n, k, alpha, A, B, beta, C,
                       D, ssA, ssB, sbatch_stride(sC), sbatch_stride(sD));
  return launch_status();
}

static int launch_spotrf(int batch, int m, const blasfeo_smat *sC, int ci, int cj,
                         const blasfeo_smat *sD, int di, int dj, int *info, hipStream_t st) {
  if (batch == 0) return 0;
  if (m == 0) {
    if (info) hipLaunchKernelGGL(k_sfill_int, dim3((batch + 255) / 256), dim3(256), 0, st, info, batch, 0);
    return launch_status();
  }
  const SView C = make_sview(sC, ci, cj, m, m), D = make_sview(sD, di, dj, m, m);
  const long long ssC = sbatch_stride(sC), ssD = sbatch_stride(sD);
  const dim3 g(1, batch);
  switch ((m + 15) / 16) {
    case 1: hipLaunchKernelGGL(k_spotrf_reg<1>, g, dim3(64), 0, st, m, C, D, sD->dA, info, ssC, ssD, ssD); break;
    case 2: hipLaunchKernelGGL(k_spotrf_reg<2>, g, dim3(64), 0, st, m, C, D, sD->dA, info, ssC, ssD, ssD); break;
    case 3: hipLaunchKernelGGL(k_spotrf_reg<3>, g, dim3(64), 0, st, m, C, D, sD->dA, info, ssC, ssD, ssD); break;
    case 4: hipLaunchKernelGGL(k_spotrf_reg<4>, g, dim3(64), 0, st, m, C, D, sD->dA, info, ssC, ssD, ssD); break;
    default:
      hipLaunchKernelGGL(k_spotrf_l, g, dim3(256), 0, st, m, C, D, sD->dA, info, ssC, ssD, ssD);
  }
  return launch_status();
}

}  // namespace bh

using namespace bh;

extern "C" {

int blasfeo_memsize_smat(int m, int n) {
  if (m < 0 || n < 0) return -1;
  const long long cn = ((long long)n + 3) / 4 * 4;
  const long long pm = ((long long)m + PSS - 1) / PSS;
  long long bytes = pm * PSS * cn * 4 + (long long)(m > n ? m : n) * 4;
  bytes = (bytes + 255) / 256 * 256;
  if (bytes > 0x7fffffffLL) return -1;
  return (int)bytes;
}

void blasfeo_create_smat(int m, int n, struct blasfeo_smat *sA, void *memory) {
  if (!sA || m < 0 || n < 0) {
    set_error(!sA ? -3 : -1);
    return;
  }
  const int cn = (n + 3) / 4 * 4;
  const int pm = (m + PSS - 1) / PSS;
  sA->m = m;
  sA->n = n;
  sA->cn = cn;
  sA->pm = pm;
  sA->pA = (float *)memory;
  sA->dA = memory ? (float *)memory + (size_t)pm * PSS * cn : nullptr;
  sA->use_dA = 0;
  sA->memsize = blasfeo_memsize_smat(m, n);
}

void blasfeo_allocate_smat(int m, int n, struct blasfeo_smat *sA) {
  const int bytes = blasfeo_memsize_smat(m, n);
  if (!sA || bytes < 0) {
    set_error(!sA ? -3 : -1);
    return;
  }
  void *p = nullptr;
  if (bytes > 0) {
    const hipError_t e = hipMalloc(&p, (size_t)bytes);
    if (e != hipSuccess) {
      set_error((int)e);
      p = nullptr;
    }
  }
  blasfeo_create_smat(m, n, sA, p);
}

void blasfeo_free_smat(struct blasfeo_smat *sA) {
  if (!sA) return;
  if (sA->pA) {
    const hipError_t e = hipFree(sA->pA);
    if (e != hipSuccess) set_error((int)e);
  }
  sA->pA = nullptr;
  sA->dA = nullptr;
}

void blasfeo_pack_smat(int m, int n, const float *A, int lda, struct blasfeo_smat *sB, int bi,
                       int bj) {
  if (m < 0) return set_error(-1);
  if (n < 0) return set_error(-2);
  if (!A && m > 0 && n > 0) return set_error(-3);
  if (lda < (m > 1 ? m : 1)) return set_error(-4);
  if (!soperand_ok(sB, bi, bj, m, n)) return set_error(-5);
  set_error(launch_spack(1, m, n, A, lda, 0, sB->pA, sB->cn, bi, bj, 0, 1, tl_stream()));
}

void blasfeo_unpack_smat(int m, int n, struct blasfeo_smat *sA, int ai, int aj, float *B,
                         int ldb) {
  if (m < 0) return set_error(-1);
  if (n < 0) return set_error(-2);
  if (!soperand_ok(sA, ai, aj, m, n)) return set_error(-3);
  if (!B && m > 0 && n > 0) return set_error(-6);
  if (ldb < (m > 1 ? m : 1)) return set_error(-7);
  set_error(launch_spack(1, m, n, B, ldb, 0, sA->pA, sA->cn, ai, aj, 0, 0, tl_stream()));
}

int blasfeo_hip_pack_smat_batched(int batch, int m, int n, const float *A, int lda,
                                  long long strideA, const struct blasfeo_smat *sB, int bi,
                                  int bj, void *stream) {
  if (batch < 0) return -1;
  if (m < 0) return -2;
  if (n < 0) return -3;
  if (!A && batch > 0 && m > 0 && n > 0) return -4;
  if (lda < (m > 1 ? m : 1)) return -5;
  if (strideA < 0) return -6;
  if (!soperand_ok(sB, bi, bj, m, n)) return -7;
  return launch_spack(batch, m, n, A, lda, strideA, sB->pA, sB->cn, bi, bj, sbatch_stride(sB),
                      1, (hipStream_t)stream);
}

int blasfeo_hip_unpack_smat_batched(int batch, int m, int n, const struct blasfeo_smat *sA,
                                    int ai, int aj, float *B, int ldb, long long strideB,
                                    void *stream) {
  if (batch < 0) return -1;
  if (m < 0) return -2;
  if (n < 0) return -3;
  if (!soperand_ok(sA, ai, aj, m, n)) return -4;
  if (!B && batch > 0 && m > 0 && n > 0) return -7;
  if (ldb < (m > 1 ? m : 1)) return -8;
  if (strideB < 0) return -9;
  return launch_spack(batch, m, n, B, ldb, strideB, sA->pA, sA->cn, ai, aj, sbatch_stride(sA),
                      0, (hipStream_t)stream);
}

void blasfeo_sgemm_nt(int m, int n, int k, float alpha, struct blasfeo_smat *sA, int ai, int aj,
                      struct blasfeo_smat *sB, int bi, int bj, float beta,
                      struct blasfeo_smat *sC, int ci, int cj, struct blasfeo_smat *sD, int di,
                      int dj) {
  if (m < 0) return set_error(-1);
  if (n < 0) return set_error(-2);
  if (k < 0) return set_error(-3);
  if (!soperand_ok(sA, ai, aj, m, k)) return set_error(-5);
  if (!soperand_ok(sB, bi, bj, n, k)) return set_error(-8);
  if (!soperand_ok(sC, ci, cj, m, n)) return set_error(-12);
  if (!soperand_ok(sD, di, dj, m, n)) return set_error(-15);
  set_error(launch_sgemm(false, 1, m, n, k, alpha, sA, ai, aj, sB, bi, bj, beta, sC, ci, cj, sD,
                         di, dj, tl_stream()));
}

void blasfeo_ssyrk_ln(int m, int k, float alpha, struct blasfeo_smat *sA, int ai, int aj,
                      struct blasfeo_smat *sB, int bi, int bj, float beta,
                      struct blasfeo_smat *sC, int ci, int cj, struct blasfeo_smat *sD, int di,
                      int dj) {
  if (m < 0) return set_error(-1);
  if (k < 0) return set_error(-2);
  if (!soperand_ok(sA, ai, aj, m, k)) return set_error(-4);
  if (!soperand_ok(sB, bi, bj, m, k)) return set_error(-7);
  if (!soperand_ok(sC, ci, cj, m, m)) return set_error(-11);
  if (!soperand_ok(sD, di, dj, m, m)) return set_error(-14);
  set_error(launch_sgemm(true, 1, m, m, k, alpha, sA, ai, aj, sB, bi, bj, beta, sC, ci, cj, sD,
                         di, dj, tl_stream()));
}

void blasfeo_spotrf_l(int m, struct blasfeo_smat *sC, int ci, int cj, struct blasfeo_smat *sD,
                      int di, int dj) {
  if (m < 0) return set_error(-1);
  if (!soperand_ok(sC, ci, cj, m, m)) return set_error(-2);
  if (!soperand_ok(sD, di, dj, m, m)) return set_error(-5);
  if (m > 0 && !sD->dA) return set_error(-5);
  const int e = launch_spotrf(1, m, sC, ci, cj, sD, di, dj, nullptr, tl_stream());
  if (e == 0) sD->use_dA = (di == 0 && dj == 0);
  set_error(e);
}

int blasfeo_hip_sgemm_nt_batched(int batch, int m, int n, int k, float alpha,
                                 const struct blasfeo_smat *sA, int ai, int aj,
                                 const struct blasfeo_smat *sB, int bi, int bj, float beta,
                                 const struct blasfeo_smat *sC, int ci, int cj,
                                 const struct blasfeo_smat *sD, int di, int dj, void *stream) {
  if (batch < 0 || batch > 65535) return -1;
  if (m < 0) return -2;
  if (n < 0) return -3;
  if (k < 0) return -4;
  if (!soperand_ok(sA, ai, aj, m, k)) return -6;
  if (!soperand_ok(sB, bi, bj, n, k)) return -9;
  if (!soperand_ok(sC, ci, cj, m, n)) return -13;
  if (!soperand_ok(sD, di, dj, m, n)) return -16;
  return launch_sgemm(false, batch, m, n, k, alpha, sA, ai, aj, sB, bi, bj, beta, sC, ci, cj, sD,
                      di, dj, (hipStream_t)stream);
}

int blasfeo_hip_ssyrk_ln_batched(int batch, int m, int k, float alpha,
                                 const struct blasfeo_smat *sA, int ai, int aj,
                                 const struct blasfeo_smat *sB, int bi, int bj, float beta,
                                 const struct blasfeo_smat *sC, int ci, int cj,
                                 const struct blasfeo_smat *sD, int di, int dj, void *stream) {
  if (batch < 0 || batch > 65535) return -1;
  if (m < 0) return -2;
  if (k < 0) return -3;
  if (!soperand_ok(sA, ai, aj, m, k)) return -5;
  if (!soperand_ok(sB, bi, bj, m, k)) return -8;
  if (!soperand_ok(sC, ci, cj, m, m)) return -12;
  if (!soperand_ok(sD, di, dj, m, m)) return -15;
  return launch_sgemm(true, batch, m, m, k, alpha, sA, ai, aj, sB, bi, bj, beta, sC, ci, cj, sD,
                      di, dj, (hipStream_t)stream);
}

int blasfeo_hip_spotrf_l_batched(int batch, int m, const struct blasfeo_smat *sC, int ci, int cj,
                                 const struct blasfeo_smat *sD, int di, int dj, int *info,
                                 void *stream) {
  if (batch < 0 || batch > 65535) return -1;
  if (m < 0) return -2;
  if (!soperand_ok(sC, ci, cj, m, m)) return -3;
  if (!soperand_ok(sD, di, dj, m, m)) return -6;
  if (m > 0 && !sD->dA) return -6;
  return launch_spotrf(batch, m, sC, ci, cj, sD, di, dj, info, (hipStream_t)stream);
}

}  // extern "C"
