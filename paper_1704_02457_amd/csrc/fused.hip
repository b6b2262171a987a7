// Fused syrk_ln + potrf_l + trsm_rltn for uniform batches of small matrices
// (the range-space pair of §4.7.2, "concatenating updates/downdates"), one
// wavefront per instance, every intermediate register resident.
//
// Per instance (m <= 16*NB):
//   M = Q + A*A^T  (lower),  L = chol(M),  X = E * L^{-T}.
// The wave holds the transposed problem: U = L^T block row by block row,
// Y = X^T.  With T-tiles (see blocks.hpp) the whole algorithm is
//   T(j,i) = Q(i,j)^T + sum_k A_j[:,k] A_i[:,k]^T        (MFMA syrk)
//   for j = 0..NB-1:
//     U(j,j) = chol(T(j,j)), V = U(j,j)^{-1}             (register subroutine)
//     U(j,i) = V^T T(j,i),  Y(j) = V^T Z(j)                (MFMA solves)
//     T(l,i) -= U(j,l)^T U(j,i),  Z(i) -= U(j,i)^T Y(j)    (MFMA downdates)
// so the only non-MFMA work is the 16x16 diagonal factorization/inversion.
// Every global load and store is a contiguous 512-byte wave transaction
// along a panel (aligned operands only).
#include "common.hpp"

namespace bh {

constexpr int FW = 1;  // independent waves (instances) per workgroup

struct FusedArgs {
  int batch, m, k, nrhs;
  const double *A;  // update factor, m x k
  int cnA;
  long long sA;
  const double *Q;  // m x m, lower read
  int cnQ;
  long long sQ;
  const double *E;  // nrhs x m
  int cnE;
  long long sE;
  double *L;  // m x m, lower written
  int cnL;
  long long sL;
  double *dA;  // inverse diagonal of L, instance stride sL
  double *X;   // nrhs x m
  int cnX;
  long long sX;
  int *info;
};


// FULL: m == 16*NB, k % 16 == 0 and nrhs in {0, 16}: no masking at all.
// All accesses go through buffer descriptors of the instance's chunks; the
// per-lane byte offset is 8*l (+ a uniform part), so a load or store of one
// register of a T-tile or one MFMA fragment is a single 512-byte wave
// transaction.
template <int NB, bool FULL>
__device__ __forceinline__ void fused_instance(const FusedArgs &a, long long b,
                                               DiagLds &s, double (*zl)[256]) {
  const int l = lane_id();
  const int c = l & 15, g = l >> 4;
  const int m = FULL ? 16 * NB : a.m;
  constexpr int NT = NB * (NB + 1) / 2;
  const int vo = 8 * l;  // per-lane byte offset

  const brsrc rA = make_rsrc(a.A + b * a.sA, 8 * a.sA);
  const brsrc rQ = make_rsrc(a.Q + b * a.sQ, 8 * a.sQ);
  const brsrc rL = make_rsrc(a.L + b * a.sL, 8 * a.sL);  // L panels and dA
  const brsrc rX = make_rsrc(a.X + b * a.sX, 8 * a.sX);
  const int dA_off = (int)(8 * (a.dA - a.L));
  const int pQ = 8 * 16 * a.cnQ, pA = 8 * 16 * a.cnA, pL = 8 * 16 * a.cnL;

  // T(j,i) = Q(i,j)^T (lower part of Q only; zero outside the matrix)
  d4 T[NT];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
#pragma unroll
    for (int j = 0; j <= i; ++j) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * i + c, col = 16 * j + g + 4 * r;
        const bool ok = (FULL || (row < m && col < m)) && (i != j || c >= g + 4 * r);
        const double x = bload(rQ, vo, i * pQ + 8 * (256 * j + 64 * r));
        T[tix_up(j, i)][r] = ok ? x : 0.0;
      }
    }
  }

  // right-hand sides Z(j) = E(:, 16j:16j+16)^T, staged in LDS: they are
  // read-modify-written once per block row, so they need no registers
  // during the factorization.
  const bool has_rhs = a.nrhs > 0;
  if (has_rhs) {
    const brsrc rE = make_rsrc(a.E + b * a.sE, 8 * a.sE);
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = 16 * j + g + 4 * r;
        const bool ok = FULL || (c < a.nrhs && col < m);
        const double x = bload(rE, vo, 8 * (256 * j + 64 * r));
        zl[j][64 * r + l] = ok ? x : 0.0;
      }
  }

  // syrk: T(j,i) += A_j A_i^T, one MFMA per block pair per 4-wide k-step.
  // The k-loop is software pipelined in chunks of KC k-steps: the loads of
  // chunk c+1 are in flight while chunk c feeds the MFMAs.
  {
    constexpr int KC = 4;
    const int nch = (a.k + 4 * KC - 1) / (4 * KC);
    double fa[KC][NB], fb[KC][NB];
    auto load_chunk = [&](double(&f)[KC][NB], int k0) {
#pragma unroll
      for (int t = 0; t < KC; ++t) {
        const bool kok = FULL || (k0 + 4 * t + g < a.k);
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          const bool ok = kok && (FULL || 16 * i + c < m);
          const double x = bload(rA, vo, i * pA + 8 * 16 * (k0 + 4 * t));
          f[t][i] = ok ? x : 0.0;
        }
      }
    };
    auto mma_chunk = [&](const double(&f)[KC][NB]) {
#pragma unroll
      for (int t = 0; t < KC; ++t)
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
          for (int j = 0; j <= i; ++j)
            T[tix_up(j, i)] = mfma(f[t][j], f[t][i], T[tix_up(j, i)]);
    };
    if (nch > 0) load_chunk(fa, 0);
    for (int ch = 0; ch < nch; ch += 2) {
      if (ch + 1 < nch) load_chunk(fb, (ch + 1) * 4 * KC);
      mma_chunk(fa);
      if (ch + 1 < nch) {
        if (ch + 2 < nch) load_chunk(fa, (ch + 2) * 4 * KC);
        mma_chunk(fb);
      }
    }
  }

  int info = 0;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int nv = FULL ? 16 : min(16, m - 16 * j);
    d4 &D = T[tix_up(j, j)];
    // Diagonal blocks of L are written as whole 128-byte panel columns: the
    // part above the diagonal is rewritten with the values it already holds
    // (read while the block is factored), because a line written only partly
    // costs the memory a read-modify-write.  Only where every line of the
    // block lies inside the matrix (FULL); elsewhere the store is masked.
    d4 Lold;
    if (FULL) {
#pragma unroll
      for (int r = 0; r < 4; ++r) Lold[r] = bload(rL, vo, j * pL + 8 * (256 * j + 64 * r));
    }
    if (!FULL && nv < 16) pad_identity(D, nv);
    d4 V;
    const int inf = potrf_inv_tile_upper(D, V, s, nullptr, (nv + 3) >> 2);
    if (inf && info == 0) info = 16 * j + inf;
    if (l < nv) bstore(rL, vo, dA_off + 8 * 16 * j, s.inv[l]);
    // store L(j,j) (lower part of the diagonal block)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * j + c, col = 16 * j + g + 4 * r;
      if (FULL)
        bstore(rL, vo, j * pL + 8 * (256 * j + 64 * r), c >= g + 4 * r ? D[r] : Lold[r]);
      else if (row < m && col < m && c >= g + 4 * r)
        bstore(rL, vo, j * pL + 8 * (256 * j + 64 * r), D[r]);
    }
#pragma unroll
    for (int i = j + 1; i < NB; ++i) {
      d4 &Ti = T[tix_up(j, i)];
      Ti = mfma_tn(V, Ti, zero4());
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * i + c, col = 16 * j + g + 4 * r;
        if (FULL || (row < m && col < m)) bstore(rL, vo, i * pL + 8 * (256 * j + 64 * r), Ti[r]);
      }
    }
    d4 Y;
    if (has_rhs) {
      // Y(j) = V^T Z(j), the block of X = E L^-T for columns 16j..16j+15
      d4 z;
#pragma unroll
      for (int r = 0; r < 4; ++r) z[r] = zl[j][64 * r + l];
      Y = mfma_tn(V, z, zero4());
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = 16 * j + g + 4 * r;
        if (FULL || (c < a.nrhs && col < m)) bstore(rX, vo, 8 * (256 * j + 64 * r), Y[r]);
      }
    }
    // trailing downdate of the remaining block rows and right-hand sides
#pragma unroll
    for (int q = j + 1; q < NB; ++q) {
      const d4 nu = neg4(T[tix_up(j, q)]);
#pragma unroll
      for (int i = q; i < NB; ++i)
        T[tix_up(q, i)] = mfma_tn(nu, T[tix_up(j, i)], T[tix_up(q, i)]);
      if (has_rhs) {
        d4 z;
#pragma unroll
        for (int r = 0; r < 4; ++r) z[r] = zl[q][64 * r + l];
        z = mfma_tn(nu, Y, z);
#pragma unroll
        for (int r = 0; r < 4; ++r) zl[q][64 * r + l] = z[r];
      }
    }
  }
  if (a.info && l == 0) a.info[b] = info;

}

// One wavefront per instance; the occupancy hint keeps the register
// footprint of the largest variant at three waves per SIMD.
template <int NB, bool FULL>
__global__ __launch_bounds__(64 * FW) __attribute__((amdgpu_waves_per_eu(3)))
void k_syrk_potrf_trsm(FusedArgs a) {
  __shared__ DiagLds lds[FW];
  __shared__ double zl[FW][NB][256];  // right-hand-side blocks, T-tile order
  const int w = wave_id();
  const long long b = (long long)blockIdx.x * FW + w;
  if (b < a.batch) fused_instance<NB, FULL>(a, b, lds[w], zl[w]);
}

template <int NB>
static void launch_nb(const FusedArgs &a, hipStream_t st) {
  dim3 grid((unsigned)((a.batch + FW - 1) / FW));
  const bool full = a.m == 16 * NB && a.k % 16 == 0 && (a.nrhs == 0 || a.nrhs == 16);
  if (full)
    hipLaunchKernelGGL((k_syrk_potrf_trsm<NB, true>), grid, dim3(64 * FW), 0, st, a);
  else
    hipLaunchKernelGGL((k_syrk_potrf_trsm<NB, false>), grid, dim3(64 * FW), 0, st, a);
}

int launch_fused(const FusedArgs &a, hipStream_t st) {
  if (a.batch == 0) return 0;
  const int nb = (a.m + 15) / 16;
  switch (nb) {
    case 1: launch_nb<1>(a, st); break;
    case 2: launch_nb<2>(a, st); break;
    case 3: launch_nb<3>(a, st); break;
    case 4: launch_nb<4>(a, st); break;
    default: return -2;
  }
  return launch_status();
}

}  // namespace bh

using namespace bh;

extern "C" int blasfeo_hip_dsyrk_dpotrf_trsm_batched(
    int batch, int m, int k, int nrhs, const struct blasfeo_dmat *sA,
    const struct blasfeo_dmat *sQ, const struct blasfeo_dmat *sE,
    const struct blasfeo_dmat *sL, const struct blasfeo_dmat *sX, int *info,
    void *stream) {
  if (batch < 0) return -1;
  if (m < 1 || m > 64) return -2;
  if (k < 0) return -3;
  if (nrhs < 0 || nrhs > 16) return -4;
  if (k > 0 && !operand_ok(sA, 0, 0, m, k)) return -5;
  if (!operand_ok(sQ, 0, 0, m, m)) return -6;
  if (nrhs > 0 && !operand_ok(sE, 0, 0, nrhs, m)) return -7;
  if (!operand_ok(sL, 0, 0, m, m) || !sL->dA) return -8;
  if (nrhs > 0 && !operand_ok(sX, 0, 0, nrhs, m)) return -9;
  FusedArgs a;
  a.batch = batch;
  a.m = m;
  a.k = k;
  a.nrhs = nrhs;
  a.A = k > 0 ? sA->pA : nullptr;
  a.cnA = k > 0 ? sA->cn : 0;
  a.sA = k > 0 ? batch_stride(sA) : 0;
  a.Q = sQ->pA;
  a.cnQ = sQ->cn;
  a.sQ = batch_stride(sQ);
  a.E = nrhs > 0 ? sE->pA : nullptr;
  a.cnE = nrhs > 0 ? sE->cn : 0;
  a.sE = nrhs > 0 ? batch_stride(sE) : 0;
  a.L = sL->pA;
  a.cnL = sL->cn;
  a.sL = batch_stride(sL);
  a.dA = sL->dA;
  a.X = nrhs > 0 ? sX->pA : nullptr;
  a.cnX = nrhs > 0 ? sX->cn : 0;
  a.sX = nrhs > 0 ? batch_stride(sX) : 0;
  a.info = info;
  return launch_fused(a, (hipStream_t)stream);
}
