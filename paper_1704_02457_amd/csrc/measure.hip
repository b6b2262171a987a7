// Measurement probes: the attainable FP64 matrix-core rate and HBM streaming
// rate of the device, the denominators a roofline of the library's kernels is
// read against next to the published peaks.  Not part of the paper's API.
#include <cstdint>

#include "common.hpp"

namespace bh {

constexpr int kProbeChains = 4;  // independent accumulator chains per wave

// Every wave runs `iters` rounds of kProbeChains independent
// v_mfma_f64_16x16x4f64 (2 * 16 * 16 * 4 flop each), enough independent
// work to keep the matrix pipe of its SIMD busy.
__global__ __launch_bounds__(256) void k_probe_dmfma(int iters, double *sink) {
  const int l = lane_id();
  const double x = 1.0 + 1e-3 * l, y = 1.0 - 1e-3 * l;
  d4 a[kProbeChains];
#pragma unroll
  for (int q = 0; q < kProbeChains; ++q) a[q] = (d4){1e-3 * q, 0.0, 0.0, 0.0};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < kProbeChains; ++q) a[q] = mfma(x, y, a[q]);
  }
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < kProbeChains; ++q) s += a[q][0] + a[q][1] + a[q][2] + a[q][3];
  // a data-dependent store the compiler cannot drop (never taken for finite s)
  if (s == -1.0) sink[blockIdx.x] = s;
}

typedef double d2 __attribute__((ext_vector_type(2)));

// Grid-stride copy with 16-byte accesses per lane.
__global__ __launch_bounds__(256) void k_probe_copy(const d2 *__restrict__ src,
                                                    d2 *__restrict__ dst,
                                                    long long n) {
  const long long step = (long long)gridDim.x * blockDim.x;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += step)
    dst[i] = src[i];
}

}  // namespace bh

using namespace bh;

extern "C" {

long long blasfeo_hip_probe_dmfma(int blocks, int iters, double *sink, void *stream) {
  if (blocks < 1) return -1;
  if (iters < 1) return -2;
  if (!sink) return -3;
  hipLaunchKernelGGL(k_probe_dmfma, dim3(blocks), dim3(256), 0, (hipStream_t)stream, iters, sink);
  const int e = launch_status();
  if (e) return e;
  return (long long)blocks * 4 * iters * kProbeChains * (2LL * 16 * 16 * 4);
}

int blasfeo_hip_probe_copy(const void *src, void *dst, long long bytes, void *stream) {
  if (!src) return -1;
  if (!dst) return -2;
  if (bytes < 0 || (bytes & 15) || ((uintptr_t)src & 15) || ((uintptr_t)dst & 15)) return -3;
  if (bytes == 0) return 0;
  const long long n = bytes / 16;
  const long long want = (n + 255) / 256;
  const int grid = (int)(want < 32768 ? want : 32768);
  hipLaunchKernelGGL(k_probe_copy, dim3(grid), dim3(256), 0, (hipStream_t)stream,
                     (const d2 *)src, (d2 *)dst, n);
  return launch_status();
}

}  // extern "C"
