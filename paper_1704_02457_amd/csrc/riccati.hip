// Backward Riccati recursion in square-root form (§5.3), a batch of
// independent problems, one wavefront per problem, all N stages with the
// stage matrices register resident (no host round trip between stages).
//
// With dynamics x+ = A x + B u (A nx-by-nx, B nx-by-nu), cost blocks Q, R
// (S = 0) and terminal P_N, for n = N-1 down to 0:
//   C   = [B^T; A^T] Lc_{n+1}                 (Lc lower, nx-by-nx)
//   M   = blockdiag(R, Q) + C C^T
//   F_n = chol(M) = [[Lambda_n, 0], [L_n, Lc_n]],   Lc_N = chol(P_N).
// The control block is padded from nu to a whole number of 16-row blocks
// with an identity block, so Lc_n always starts on a block boundary of the
// padded factor and no realignment is needed between stages; the padding is
// dropped when F_n is stored.  In the T-tile view (blocks.hpp):
//   Ct(k,j)  = sum_m Ln(m,k)^T X^T(m,j)        (Ct = C^T, X = [B^T; 0; A^T])
//   T(j,i)   = RQ(j,i) + sum_k Ct(k,j)^T Ct(k,i)
// then the register factorization of T, and Ln(m,k) = U(k+nub, m+nub)^T
// for the next stage (one LDS transpose per block).
#include "common.hpp"

namespace bh {

struct RicArgs {
  int batch, nx, nu, N;
  View A, B, Q, R, P;  // instance 0; offsets are per-instance strides below
  long long sA, sB, sQ, sR, sP;
  double *F;  // stage factors, chunk (b*N + n) at F + (b*N + n)*sF
  int cnF;
  long long sF;
  int *info;
};

// padded index (u block padded to 16*NUB rows) -> unpadded index, or -1
template <int NUB>
__device__ __forceinline__ int unpad(int x, int nu) {
  if (x < nu) return x;
  if (x < 16 * NUB) return -1;
  return x - 16 * NUB + nu;
}

// load_tileT split in two: the loads (elements outside the view, or above
// its diagonal with lower, come from the view's origin) and the masking, so
// that a group of tiles can be in flight before any is used.
__device__ __forceinline__ d4 tile_raw(const View &v, int i0, int j0, bool lower) {
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
  const int o0 = pm_off(v.ai, v.aj, v.cn);
  d4 t;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + c, j = j0 + g + 4 * r;
    const bool ok = i < v.rows && j < v.cols && (!lower || i >= j);
    t[r] = v.p[ok ? pm_off(v.ai + i, v.aj + j, v.cn) : o0];
  }
  return t;
}

__device__ __forceinline__ d4 tile_mask(d4 t, const View &v, int i0, int j0, bool lower) {
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + c, j = j0 + g + 4 * r;
    t[r] = (i < v.rows && j < v.cols && (!lower || i >= j)) ? t[r] : 0.0;
  }
  return t;
}

template <int NUB, int NXB>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_ric_trf(RicArgs a) {
  constexpr int NB = NUB + NXB;
  constexpr int NT = NB * (NB + 1) / 2;
  constexpr int NLT = NXB * (NXB + 1) / 2;
  __shared__ DiagLds s;
  __shared__ double xs[NXB * NB][256];  // X^T tiles, constant over the stages
  const long long b = blockIdx.x;
  if (b >= a.batch) return;
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
  const int nu = a.nu, nx = a.nx;
  View A = a.A, B = a.B, Q = a.Q, R = a.R, P = a.P;
  A.p += b * a.sA;
  B.p += b * a.sB;
  Q.p += b * a.sQ;
  R.p += b * a.sR;
  P.p += b * a.sP;

  // X^T tiles: logical X^T(m, j) block, X = [B^T; 0; A^T] (padded rows),
  // kept in LDS (they are read once per stage and would otherwise hold
  // registers through the whole recursion)
#pragma unroll
  for (int m = 0; m < NXB; ++m) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      // X(16j + q, 16m + p) = B(16m + p, 16j + q) for 16j + q < nu
      const d4 x = (j < NUB) ? load_tileN(B, 16 * m, 16 * j) : load_tileN(A, 16 * m, 16 * (j - NUB));
#pragma unroll
      for (int r = 0; r < 4; ++r) xs[m * NB + j][64 * r + l] = x[r];
    }
  }
  auto Xt = [&](int m, int j) {
    d4 x;
#pragma unroll
    for (int r = 0; r < 4; ++r) x[r] = xs[m * NB + j][64 * r + l];
    return x;
  };

  // Lc_N = chol(P_N): register factorization of the NXB x NXB block
  d4 Ln[NLT];  // Ln(m,k), m >= k, logical Lc(m,k), index tix_up(k, m)
  int info = 0;
  {
    d4 T[NLT];
#pragma unroll
    for (int i = 0; i < NXB; ++i)
#pragma unroll
      for (int j = 0; j <= i; ++j) T[tix_up(j, i)] = load_tileT(P, 16 * i, 16 * j, i == j);
#pragma unroll
    for (int j = 0; j < NXB; ++j) {
      d4 &D = T[tix_up(j, j)];
      const int nv = min(16, nx - 16 * j);
      if (nv < 16) pad_identity(D, nv);
      d4 V;
      const int inf = potrf_inv_tile_upper(D, V, s, nullptr, (nv + 3) >> 2);
      if (inf && info == 0) info = 1000 * (a.N + 1) + 16 * j + inf;
#pragma unroll
      for (int i = j + 1; i < NXB; ++i) T[tix_up(j, i)] = mfma_tn(V, T[tix_up(j, i)], zero4());
#pragma unroll
      for (int q = j + 1; q < NXB; ++q) {
        const d4 nu4 = neg4(T[tix_up(j, q)]);
#pragma unroll
        for (int i = q; i < NXB; ++i)
          T[tix_up(q, i)] = mfma_tn(nu4, T[tix_up(j, i)], T[tix_up(q, i)]);
      }
    }
#pragma unroll
    for (int m = 0; m < NXB; ++m)
#pragma unroll
      for (int k = 0; k <= m; ++k) Ln[tix_up(k, m)] = transpose_tile(T[tix_up(k, m)], s.tr);
  }

  for (int n = a.N - 1; n >= 0; --n) {
    // the constant R and Q blocks of this stage's matrix: their loads go out
    // first so that they are in flight during the Ct products (placed at
    // their use, each tile's loads were waited for one after another)
    d4 RQ[NT];
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int j = 0; j <= i; ++j) {
        if (i < NUB)
          RQ[tix_up(j, i)] = tile_raw(R, 16 * i, 16 * j, i == j);
        else if (j >= NUB)
          RQ[tix_up(j, i)] = tile_raw(Q, 16 * (i - NUB), 16 * (j - NUB), i == j);
        else
          RQ[tix_up(j, i)] = zero4();
      }
    __builtin_amdgcn_sched_barrier(0);
    // Ct(k, j) = sum_{m >= k} Ln(m,k)^T X^T(m,j)
    d4 T[NT];
    {
      d4 Ct[NXB][NB];
#pragma unroll
      for (int k = 0; k < NXB; ++k)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          d4 acc = zero4();
#pragma unroll
          for (int m = k; m < NXB; ++m) acc = mfma_tn(Ln[tix_up(k, m)], Xt(m, j), acc);
          Ct[k][j] = acc;
        }
      // T(j,i) = blockdiag(R, I, Q)(j,i) + sum_k Ct(k,j)^T Ct(k,i)
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) {
          d4 acc = RQ[tix_up(j, i)];
          if (i < NUB)
            acc = tile_mask(acc, R, 16 * i, 16 * j, i == j);
          else if (j >= NUB)
            acc = tile_mask(acc, Q, 16 * (i - NUB), 16 * (j - NUB), i == j);
          if (i < NUB) {
            if (i == j) {  // identity on the padding rows nu..16*NUB-1
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int p = 16 * j + g + 4 * r, q = 16 * i + c;
                if (p >= nu || q >= nu) acc[r] = (p == q) ? 1.0 : 0.0;
              }
            }
          } else if (j >= NUB) {
            if (i == j) {
              const int nv = min(16, nx - 16 * (j - NUB));
              if (nv < 16) pad_identity(acc, nv);
            }
          }
#pragma unroll
          for (int k = 0; k < NXB; ++k) acc = mfma_tn(Ct[k][j], Ct[k][i], acc);
          T[tix_up(j, i)] = acc;
        }
    }
    // F_n = chol(M): register factorization, stored without the padding
    double *Fb = a.F + (b * a.N + n) * a.sF;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      d4 &D = T[tix_up(j, j)];
      d4 V;
      // rows past the control block's nu (or the state block's nx) are identity
      const int nvj = j < NUB ? min(16, nu - 16 * j) : min(16, nx - 16 * (j - NUB));
      const int inf = potrf_inv_tile_upper(D, V, s, nullptr, (nvj + 3) >> 2);
      if (inf && info == 0) {
        // report the pivot as an index of the unpadded stage matrix
        const int pv = unpad<NUB>(16 * j + inf - 1, nu);
        info = 1000 * (n + 1) + (pv >= 0 ? pv + 1 : 16 * j + inf);
      }
#pragma unroll
      for (int i = j + 1; i < NB; ++i) T[tix_up(j, i)] = mfma_tn(V, T[tix_up(j, i)], zero4());
#pragma unroll
      for (int q = j + 1; q < NB; ++q) {
        const d4 nu4 = neg4(T[tix_up(j, q)]);
#pragma unroll
        for (int i = q; i < NB; ++i)
          T[tix_up(q, i)] = mfma_tn(nu4, T[tix_up(j, i)], T[tix_up(q, i)]);
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int j = 0; j <= i; ++j) {
        const d4 &t = T[tix_up(j, i)];  // U(j,i) = F(i,j)^T
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ro = unpad<NUB>(16 * i + c, nu), co = unpad<NUB>(16 * j + g + 4 * r, nu);
          if (ro >= 0 && co >= 0 && ro < nu + nx && co < nu + nx && ro >= co)
            Fb[pm_off(ro, co, a.cnF)] = t[r];
        }
      }
    // Lc_n = trailing NXB x NXB blocks of the padded factor
#pragma unroll
    for (int m = 0; m < NXB; ++m)
#pragma unroll
      for (int k = 0; k <= m; ++k)
        Ln[tix_up(k, m)] = transpose_tile(T[tix_up(k + NUB, m + NUB)], s.tr);
  }
  if (a.info && l == 0) a.info[b] = info;
}

template <int NUB, int NXB>
static void launch_ric(const RicArgs &a, hipStream_t st) {
  hipLaunchKernelGGL((k_ric_trf<NUB, NXB>), dim3(a.batch), dim3(64), 0, st, a);
}

// ---------------------------------------------------------------- solve
// The solution of the linear-quadratic problem whose KKT matrix the
// recursion above factors (the standard substitution of the square-root
// form): a backward pass for the linear term p_n of the value function,
//   w = P_{n+1} b_n + p_{n+1},  m = [r_n + B'w; q_n + A'w],
//   l_n = Lambda_n^{-1} m_u,    p_n = m_x - L_n l_n,   p_N = q_N,
// with P_{n+1} = Lc_{n+1} Lc_{n+1}' taken from the next stage's factor
// (P_N itself for the last stage), then a forward pass
//   u_n = -Lambda_n^{-T} (L_n' x_n + l_n),   x_{n+1} = A x_n + B u_n + b_n.
// All of it is matrix-vector work on order <= 48: one wave per problem,
// lane i owning row i of every vector, vectors broadcast through LDS and
// the two nu-by-nu triangular solves column by column.
struct RicSolveArgs {
  int batch, nx, nu, N;
  View A, B, P;
  long long sA, sB, sP;
  const double *F;  // stage factors as written by k_ric_trf
  int cnF;
  long long sF;
  const double *b, *r, *q, *x0;
  double *u, *x;
};

__device__ __forceinline__ double vel(const View &v, int i, int j) {
  return v.p[pm_off(v.ai + i, v.aj + j, v.cn)];
}

// Copy of the rows x cols matrix v into LDS (row i at dst + i * ld), the lanes
// running down the panel columns.
__device__ __forceinline__ void stage_lds(const View &v, int rows, int cols, double *dst, int ld) {
  for (int t = lane_id(); t < rows * cols; t += 64) {
    const int i = t % rows, j = t / rows;
    dst[i * ld + j] = vel(v, i, j);
  }
}

// The stage factor F_n (nm x nm, nm <= 48) in flight in registers: element
// t = lane + 64 s of the column-major enumeration in pf[s].
constexpr int kRicPf = 36;  // 48 * 48 / 64

struct RicPf {
  double v[kRicPf];
};

__device__ __forceinline__ void ric_pf_load(RicPf &pf, const double *F, int cn, int nm) {
  // buffer loads: element offsets past the descriptor's range read 0
  const int pm = (nm + 15) >> 4;
  const brsrc rs = make_rsrc(F, 8LL * pm * 16 * cn);
  const int l = lane_id();
  int i = l % nm, j = l / nm;
  const int di = 64 % nm, dj = 64 / nm;
#pragma unroll
  for (int s = 0; s < kRicPf; ++s) {
    const int off = j < nm ? 8 * ((i & ~15) * cn + j * 16 + (i & 15)) : 0x7ffffff0;
    pf.v[s] = bload(rs, off, 0);
    i += di;
    j += dj;
    if (i >= nm) {
      i -= nm;
      ++j;
    }
  }
}

__device__ __forceinline__ void ric_pf_store(const RicPf &pf, double *Fs, int nm) {
  const int l = lane_id();
  int i = l % nm, j = l / nm;
  const int di = 64 % nm, dj = 64 / nm;
#pragma unroll
  for (int s = 0; s < kRicPf; ++s) {
    if (j < nm) Fs[i * (nm + 1) + j] = pf.v[s];
    i += di;
    j += dj;
    if (i >= nm) {
      i -= nm;
      ++j;
    }
  }
}

size_t ric_trs_lds_bytes(int nx, int nu) {
  const int nm = nx + nu;
  return sizeof(double) * ((size_t)nx * (nx + 1) + (size_t)nx * (nu + 1) + (size_t)nm * (nm + 1) + 4 * 64);
}

// Solve of the Riccati problem on the stored stage factors, one wave per
// problem, lane = vector row.  A and B are copied to LDS once and each stage
// factor once per pass (padded rows, so that row- and column-wise reads are
// both free of bank conflicts); every matrix-vector product reads LDS.  The
// global loads that a stage waits for go out early: the factor's while the
// previous factor is still in use, the stage vectors (b, r, q, and l in the
// forward pass) one stage ahead.
__global__ __launch_bounds__(64) void k_ric_trs(RicSolveArgs a) {
  extern __shared__ double lds[];
  const long long pb = blockIdx.x;
  if (pb >= a.batch) return;
  const int l = lane_id();
  const int nx = a.nx, nu = a.nu, N = a.N, nm = nu + nx;
  View A = a.A, B = a.B, P = a.P;
  A.p += pb * a.sA;
  B.p += pb * a.sB;
  P.p += pb * a.sP;
  const int la = nx + 1, lb = nu + 1, lf = nm + 1;
  double *As = lds, *Bs = As + nx * la, *Fs = Bs + nx * lb;
  double *vt = Fs + nm * lf, *vm = vt + 64, *vp = vm + 64, *vx = vp + 64;
  auto Fp = [&](int n) { return a.F + (pb * N + n) * a.sF; };
  const double *bv = a.b + pb * N * nx, *rv = a.r + pb * N * nu;
  const double *qv = a.q + pb * (N + 1) * nx, *x0 = a.x0 + pb * nx;
  double *u = a.u + pb * N * nu, *x = a.x + pb * (N + 1) * nx;
  auto F = [&](int i, int j) { return Fs[i * lf + j]; };

  RicPf pf;
  stage_lds(A, nx, nx, As, la);
  stage_lds(B, nx, nu, Bs, lb);
  // ------------------------------------------------ backward: p_n and l_n
  if (l < nx) vp[l] = qv[(long long)N * nx + l];
  // the stage vectors are loaded one stage ahead
  const int lx = min(l, nx - 1), lu = min(l, nu - 1), lq = min(max(l - nu, 0), nx - 1);
  double bnx = bv[(long long)(N - 1) * nx + lx], rnx = rv[(long long)(N - 1) * nu + lu];
  double qnx = qv[(long long)(N - 1) * nx + lq];
  for (int n = N - 1; n >= 0; --n) {
    const double bcur = bnx, rcur = rnx, qcur = qnx;
    if (n > 0) {
      bnx = bv[(long long)(n - 1) * nx + lx];
      rnx = rv[(long long)(n - 1) * nu + lu];
      qnx = qv[(long long)(n - 1) * nx + lq];
    }
    ric_pf_load(pf, Fp(n), a.cnF, nm);  // F_n's loads go out while F_{n+1} is used
    if (l < nx) vt[l] = bcur;
    wave_sync();
    double w = 0.0;
    if (n == N - 1) {
      // P_N b (lower triangle of P_N read)
      if (l < nx)
        #pragma unroll 8
        for (int k = 0; k < nx; ++k) w += vel(P, max(l, k), min(l, k)) * vt[k];
    } else {
      // Fs holds F_{n+1}: s = Lc' b, Lc = its trailing block, then w = Lc s
      double sj = 0.0;
      if (l < nx)
        #pragma unroll 8
        for (int i = l; i < nx; ++i) sj += F(nu + i, nu + l) * vt[i];
      wave_sync();
      if (l < nx) vt[l] = sj;
      wave_sync();
      if (l < nx)
        #pragma unroll 8
        for (int k = 0; k <= l; ++k) w += F(nu + l, nu + k) * vt[k];
    }
    if (l < nx) w += vp[l];
    wave_sync();
    if (l < nx) vt[l] = w;
    wave_sync();
    // m = [r_n + B'w; q_n + A'w], lane = row of m
    double mv = 0.0;
    if (l < nu) {
      mv = rcur;
      #pragma unroll 8
      for (int i = 0; i < nx; ++i) mv += Bs[i * lb + l] * vt[i];
    } else if (l < nm) {
      mv = qcur;
      #pragma unroll 8
      for (int i = 0; i < nx; ++i) mv += As[i * la + l - nu] * vt[i];
    }
    if (l < nm) vm[l] = mv;
    wave_sync();
    // F_n replaces F_{n+1}; the loads of F_{n-1} go out
    ric_pf_store(pf, Fs, nm);
    wave_sync();
    // l_n = Lambda_n^{-1} m_u, column by column
    for (int k = 0; k < nu; ++k) {
      const double lk = vm[k] / F(k, k);
      wave_sync();
      if (l == k) vm[l] = lk;
      if (l > k && l < nu) vm[l] -= F(l, k) * lk;
      wave_sync();
    }
    if (l < nu) u[(long long)n * nu + l] = vm[l];  // l_n, overwritten by u_n below
    double pn = 0.0;
    if (l >= nu && l < nm) {
      pn = vm[l];
      #pragma unroll 8
      for (int k = 0; k < nu; ++k) pn -= F(l, k) * vm[k];
    }
    wave_sync();
    if (l >= nu && l < nm) vp[l - nu] = pn;
    wave_sync();
  }

  // ------------------------------------------------ forward: u_n and x_n
  // (Fs holds F_0)
  if (l < nx) {
    vx[l] = x0[l];
    x[l] = x0[l];
  }
  double unx = u[lu], bfx = bv[lx];
  for (int n = 0; n < N; ++n) {
    const double ucur = unx, bfc = bfx;
    if (n + 1 < N) ric_pf_load(pf, Fp(n + 1), a.cnF, nm);  // used from the next stage on
    if (n + 1 < N) {
      unx = u[(long long)(n + 1) * nu + lu];
      bfx = bv[(long long)(n + 1) * nx + lx];
    }
    wave_sync();
    double v = 0.0;  // L_n' x_n + l_n
    if (l < nu) {
      #pragma unroll 8
      for (int i = 0; i < nx; ++i) v += F(nu + i, l) * vx[i];
      v += ucur;
      vm[l] = v;
    }
    wave_sync();
    for (int k = nu - 1; k >= 0; --k) {  // Lambda_n^T y = v, row by row from the bottom
      const double yk = vm[k] / F(k, k);
      wave_sync();
      if (l == k) vm[l] = yk;
      if (l < k) vm[l] -= F(k, l) * yk;
      wave_sync();
    }
    if (l < nu) {
      const double un = -vm[l];
      u[(long long)n * nu + l] = un;
      vm[l] = un;
    }
    wave_sync();
    double xn = 0.0;
    if (l < nx) {
      #pragma unroll 8
      for (int k = 0; k < nx; ++k) xn += As[l * la + k] * vx[k];
      #pragma unroll 8
      for (int k = 0; k < nu; ++k) xn += Bs[l * lb + k] * vm[k];
      xn += bfc;
    }
    wave_sync();
    if (l < nx) {
      vx[l] = xn;
      x[(long long)(n + 1) * nx + l] = xn;
    }
    if (n + 1 < N) ric_pf_store(pf, Fs, nm);
  }
}

}  // namespace bh

using namespace bh;

extern "C" int blasfeo_hip_dric_trf_batched(
    int batch, int nx, int nu, int N, const struct blasfeo_dmat *sA,
    const struct blasfeo_dmat *sB, const struct blasfeo_dmat *sQ,
    const struct blasfeo_dmat *sR, const struct blasfeo_dmat *sP,
    const struct blasfeo_dmat *sF, int *info, void *stream) {
  if (batch < 0) return -1;
  if (nx < 1 || nx > 32) return -2;
  if (nu < 1 || nu > 16) return -3;
  if (N < 1) return -4;
  if (!operand_ok(sA, 0, 0, nx, nx)) return -5;
  if (!operand_ok(sB, 0, 0, nx, nu)) return -6;
  if (!operand_ok(sQ, 0, 0, nx, nx)) return -7;
  if (!operand_ok(sR, 0, 0, nu, nu)) return -8;
  if (!operand_ok(sP, 0, 0, nx, nx)) return -9;
  if (!operand_ok(sF, 0, 0, nu + nx, nu + nx)) return -10;
  if (batch == 0) return 0;
  RicArgs a;
  a.batch = batch;
  a.nx = nx;
  a.nu = nu;
  a.N = N;
  a.A = make_view(sA, 0, 0, nx, nx);
  a.B = make_view(sB, 0, 0, nx, nu);
  a.Q = make_view(sQ, 0, 0, nx, nx);
  a.R = make_view(sR, 0, 0, nu, nu);
  a.P = make_view(sP, 0, 0, nx, nx);
  a.sA = batch_stride(sA);
  a.sB = batch_stride(sB);
  a.sQ = batch_stride(sQ);
  a.sR = batch_stride(sR);
  a.sP = batch_stride(sP);
  a.F = sF->pA;
  a.cnF = sF->cn;
  a.sF = batch_stride(sF);
  a.info = info;
  hipStream_t st = (hipStream_t)stream;
  if (nx <= 16)
    launch_ric<1, 1>(a, st);
  else
    launch_ric<1, 2>(a, st);
  return launch_status();
}

extern "C" int blasfeo_hip_dric_trs_batched(
    int batch, int nx, int nu, int N, const struct blasfeo_dmat *sA,
    const struct blasfeo_dmat *sB, const struct blasfeo_dmat *sP,
    const struct blasfeo_dmat *sF, const double *b, const double *r,
    const double *q, const double *x0, double *u, double *x, void *stream) {
  if (batch < 0) return -1;
  if (nx < 1 || nx > 32) return -2;
  if (nu < 1 || nu > 16) return -3;
  if (N < 1) return -4;
  if (!operand_ok(sA, 0, 0, nx, nx)) return -5;
  if (!operand_ok(sB, 0, 0, nx, nu)) return -6;
  if (!operand_ok(sP, 0, 0, nx, nx)) return -7;
  if (!operand_ok(sF, 0, 0, nu + nx, nu + nx)) return -8;
  if (batch == 0) return 0;
  if (!b) return -9;
  if (!r) return -10;
  if (!q) return -11;
  if (!x0) return -12;
  if (!u) return -13;
  if (!x) return -14;
  RicSolveArgs a;
  a.batch = batch;
  a.nx = nx;
  a.nu = nu;
  a.N = N;
  a.A = make_view(sA, 0, 0, nx, nx);
  a.B = make_view(sB, 0, 0, nx, nu);
  a.P = make_view(sP, 0, 0, nx, nx);
  a.sA = batch_stride(sA);
  a.sB = batch_stride(sB);
  a.sP = batch_stride(sP);
  a.F = sF->pA;
  a.cnF = sF->cn;
  a.sF = batch_stride(sF);
  a.b = b;
  a.r = r;
  a.q = q;
  a.x0 = x0;
  a.u = u;
  a.x = x;
  hipLaunchKernelGGL(k_ric_trs, dim3(batch), dim3(64), ric_trs_lds_bytes(nx, nu), (hipStream_t)stream, a);
  return launch_status();
}
