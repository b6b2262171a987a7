// Memory handling (Appendix A.1.2), per-thread state and the packing
// routines (col-major <-> panel-major) of the C ABI.
#include <stdint.h>
#include <string.h>

#include "common.hpp"

namespace bh {

hipStream_t &tl_stream() {
  static thread_local hipStream_t s = nullptr;
  return s;
}
int &tl_error() {
  static thread_local int e = 0;
  return e;
}

// One thread per element; i (row) fastest so that both the column-major
// source and the panel-major destination (rows of a panel are contiguous)
// are walked in address order.
__global__ void k_pack(int batch, int m, int n, const double *__restrict__ A,
                       int lda, long long sa, double *__restrict__ B, int cn,
                       int bi, int bj, long long sb, int to_panel) {
  const long long per = (long long)m * n;
  const long long total = per * batch;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
       t < total; t += (long long)gridDim.x * blockDim.x) {
    const long long b = t / per, e = t - b * per;
    const int i = (int)(e % m), j = (int)(e / m);
    const long long po = b * sb + pm_off(bi + i, bj + j, cn);
    const long long co = b * sa + (long long)i + (long long)j * lda;
    if (to_panel)
      B[po] = A[co];
    else
      ((double *)A)[co] = B[po];
  }
}

static int launch_pack(int batch, int m, int n, const double *A, int lda,
                       long long sa, double *B, int cn, int bi, int bj,
                       long long sb, int to_panel, hipStream_t st) {
  if (batch == 0 || m == 0 || n == 0) return 0;
  long long total = (long long)m * n * batch;
  int threads = 256;
  long long blocks = (total + threads - 1) / threads;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_pack, dim3((unsigned)blocks), dim3(threads), 0, st,
                     batch, m, n, A, lda, sa, B, cn, bi, bj, sb, to_panel);
  return launch_status();
}

// Pack/unpack of `count` m x n column-major matrices (instance b at A +
// b*sa) to/from panel-major chunks at arbitrary offsets of an arena.
__global__ void k_pack_indexed(int count, int m, int n, const double *__restrict__ A,
                               int lda, long long sa, const long long *__restrict__ off,
                               double *__restrict__ arena, int cn, int to_panel) {
  const long long per = (long long)m * n;
  const long long total = per * count;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
       t < total; t += (long long)gridDim.x * blockDim.x) {
    const long long b = t / per, e = t - b * per;
    const int i = (int)(e % m), j = (int)(e / m);
    const long long po = off[b] + pm_off(i, j, cn);
    const long long co = b * sa + (long long)i + (long long)j * lda;
    if (to_panel)
      arena[po] = A[co];
    else
      ((double *)A)[co] = arena[po];
  }
}

}  // namespace bh

using namespace bh;

extern "C" {

int blasfeo_memsize_dmat(int m, int n) {
  if (m < 0 || n < 0) return -1;
  long long cn = ((long long)n + 3) / 4 * 4;
  long long pm = ((long long)m + PS - 1) / PS;
  long long bytes = pm * PS * cn * 8 + (long long)(m > n ? m : n) * 8;
  bytes = (bytes + 255) / 256 * 256;
  if (bytes > 0x7fffffffLL) return -1;
  return (int)bytes;
}

int blasfeo_memsize_dvec(int m) {
  if (m < 0) return -1;
  long long pm = ((long long)m + PS - 1) / PS;
  long long bytes = (pm * PS * 8 + 255) / 256 * 256;
  if (bytes > 0x7fffffffLL) return -1;
  return (int)bytes;
}

void blasfeo_create_dmat(int m, int n, struct blasfeo_dmat *sA,
                         void *memory) {
  if (!sA || m < 0 || n < 0) {
    set_error(!sA ? -3 : -1);
    return;
  }
  int cn = (n + 3) / 4 * 4;
  int pm = (m + PS - 1) / PS;
  sA->m = m;
  sA->n = n;
  sA->cn = cn;
  sA->pm = pm;
  sA->pA = (double *)memory;
  sA->dA = memory ? (double *)memory + (size_t)pm * PS * cn : nullptr;
  sA->use_dA = 0;
  sA->memsize = blasfeo_memsize_dmat(m, n);
}

void blasfeo_create_dvec(int m, struct blasfeo_dvec *sx, void *memory) {
  if (!sx || m < 0) {
    set_error(!sx ? -2 : -1);
    return;
  }
  sx->m = m;
  sx->pm = (m + PS - 1) / PS;
  sx->pa = (double *)memory;
  sx->memsize = blasfeo_memsize_dvec(m);
}

void blasfeo_allocate_dmat(int m, int n, struct blasfeo_dmat *sA) {
  int bytes = blasfeo_memsize_dmat(m, n);
  if (!sA || bytes < 0) {
    set_error(!sA ? -3 : -1);
    return;
  }
  void *p = nullptr;
  if (bytes > 0) {
    hipError_t e = hipMalloc(&p, (size_t)bytes);
    if (e != hipSuccess) {
      set_error((int)e);
      p = nullptr;
    }
  }
  blasfeo_create_dmat(m, n, sA, p);
}

void blasfeo_free_dmat(struct blasfeo_dmat *sA) {
  if (!sA) return;
  if (sA->pA) {
    hipError_t e = hipFree(sA->pA);
    if (e != hipSuccess) set_error((int)e);
  }
  sA->pA = nullptr;
  sA->dA = nullptr;
}

void blasfeo_allocate_dvec(int m, struct blasfeo_dvec *sx) {
  int bytes = blasfeo_memsize_dvec(m);
  if (!sx || bytes < 0) {
    set_error(!sx ? -2 : -1);
    return;
  }
  void *p = nullptr;
  if (bytes > 0) {
    hipError_t e = hipMalloc(&p, (size_t)bytes);
    if (e != hipSuccess) {
      set_error((int)e);
      p = nullptr;
    }
  }
  blasfeo_create_dvec(m, sx, p);
}

void blasfeo_free_dvec(struct blasfeo_dvec *sx) {
  if (!sx) return;
  if (sx->pa) {
    hipError_t e = hipFree(sx->pa);
    if (e != hipSuccess) set_error((int)e);
  }
  sx->pa = nullptr;
}

void blasfeo_pack_dmat(int m, int n, const double *A, int lda,
                       struct blasfeo_dmat *sB, int bi, int bj) {
  if (m < 0) return set_error(-1);
  if (n < 0) return set_error(-2);
  if (!A && m > 0 && n > 0) return set_error(-3);
  if (lda < (m > 1 ? m : 1)) return set_error(-4);
  if (!operand_ok(sB, bi, bj, m, n)) return set_error(-5);
  set_error(launch_pack(1, m, n, A, lda, 0, sB->pA, sB->cn, bi, bj, 0, 1,
                        tl_stream()));
}

void blasfeo_unpack_dmat(int m, int n, struct blasfeo_dmat *sA, int ai,
                         int aj, double *B, int ldb) {
  if (m < 0) return set_error(-1);
  if (n < 0) return set_error(-2);
  if (!operand_ok(sA, ai, aj, m, n)) return set_error(-3);
  if (!B && m > 0 && n > 0) return set_error(-6);
  if (ldb < (m > 1 ? m : 1)) return set_error(-7);
  set_error(launch_pack(1, m, n, B, ldb, 0, sA->pA, sA->cn, ai, aj, 0, 0,
                        tl_stream()));
}

void blasfeo_pack_dvec(int m, const double *x, struct blasfeo_dvec *sy,
                       int yi) {
  if (m < 0) return set_error(-1);
  if (!x && m > 0) return set_error(-2);
  if (!sy || yi < 0 || yi + m > sy->m || (m > 0 && !sy->pa))
    return set_error(-3);
  if (m == 0) return;
  hipError_t e = hipMemcpyAsync(sy->pa + yi, x, (size_t)m * 8,
                                hipMemcpyDeviceToDevice, tl_stream());
  set_error(e == hipSuccess ? 0 : (int)e);
}

void blasfeo_unpack_dvec(int m, struct blasfeo_dvec *sx, int xi, double *y) {
  if (m < 0) return set_error(-1);
  if (!sx || xi < 0 || xi + m > sx->m || (m > 0 && !sx->pa))
    return set_error(-2);
  if (!y && m > 0) return set_error(-4);
  if (m == 0) return;
  hipError_t e = hipMemcpyAsync(y, sx->pa + xi, (size_t)m * 8,
                                hipMemcpyDeviceToDevice, tl_stream());
  set_error(e == hipSuccess ? 0 : (int)e);
}

void blasfeo_hip_set_stream(void *stream) {
  tl_stream() = (hipStream_t)stream;
}
void *blasfeo_hip_get_stream(void) { return (void *)tl_stream(); }

int blasfeo_hip_get_last_error(void) {
  int e = tl_error();
  tl_error() = 0;
  return e;
}

const char *blasfeo_hip_strerror(int code) {
  if (code == 0) return "success";
  if (code < 0) {
    static const char *msg[] = {
        "invalid argument", "invalid argument 1", "invalid argument 2",
        "invalid argument 3", "invalid argument 4", "invalid argument 5",
        "invalid argument 6", "invalid argument 7", "invalid argument 8",
        "invalid argument 9", "invalid argument 10", "invalid argument 11",
        "invalid argument 12", "invalid argument 13", "invalid argument 14",
        "invalid argument 15", "invalid argument 16", "invalid argument 17",
        "invalid argument 18", "invalid argument 19", "invalid argument 20"};
    int i = -code;
    return i <= 20 ? msg[i] : msg[0];
  }
  return hipGetErrorString((hipError_t)code);
}

int blasfeo_hip_version(void) { return 100; }

int blasfeo_hip_pack_dmat_batched(int batch, int m, int n, const double *A,
                                  int lda, long long strideA,
                                  const struct blasfeo_dmat *sB, int bi,
                                  int bj, void *stream) {
  if (batch < 0) return -1;
  if (m < 0) return -2;
  if (n < 0) return -3;
  if (!A && batch > 0 && m > 0 && n > 0) return -4;
  if (lda < (m > 1 ? m : 1)) return -5;
  if (strideA < 0) return -6;
  if (!operand_ok(sB, bi, bj, m, n)) return -7;
  return launch_pack(batch, m, n, A, lda, strideA, sB->pA, sB->cn, bi, bj,
                     batch_stride(sB), 1, (hipStream_t)stream);
}

int blasfeo_hip_unpack_dmat_batched(int batch, int m, int n,
                                    const struct blasfeo_dmat *sA, int ai,
                                    int aj, double *B, int ldb,
                                    long long strideB, void *stream) {
  if (batch < 0) return -1;
  if (m < 0) return -2;
  if (n < 0) return -3;
  if (!operand_ok(sA, ai, aj, m, n)) return -4;
  if (!B && batch > 0 && m > 0 && n > 0) return -7;
  if (ldb < (m > 1 ? m : 1)) return -8;
  if (strideB < 0) return -9;
  return launch_pack(batch, m, n, B, ldb, strideB, sA->pA, sA->cn, ai, aj,
                     batch_stride(sA), 0, (hipStream_t)stream);
}

int blasfeo_hip_pack_dmat_indexed(int count, int m, int n, const double *A,
                                  int lda, long long strideA,
                                  const long long *dst_off, double *arena,
                                  int to_panel, void *stream) {
  if (count < 0) return -1;
  if (m < 0) return -2;
  if (n < 0) return -3;
  if (!A && count > 0 && m > 0 && n > 0) return -4;
  if (lda < (m > 1 ? m : 1)) return -5;
  if (strideA < 0) return -6;
  if (!dst_off && count > 0) return -7;
  if (!arena && count > 0) return -8;
  if (count == 0 || m == 0 || n == 0) return 0;
  const int cn = (n + 3) / 4 * 4;
  long long total = (long long)m * n * count;
  long long blocks = (total + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_pack_indexed, dim3((unsigned)blocks), dim3(256), 0,
                     (hipStream_t)stream, count, m, n, A, lda, strideA, dst_off,
                     arena, cn, to_panel);
  return launch_status();
}

}  // extern "C"
