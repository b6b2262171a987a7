// Host-side plan of an uneven batch (shared by the FP64 and the
// mixed-precision solvers).
#pragma once
#include <vector>

#include "common.hpp"

struct blasfeo_hip_plan {
  int batch = 0, nrhs = 0;
  std::vector<int> n;
  std::vector<long long> moff, voff;  // bytes
  long long mat_bytes = 0, vec_bytes = 0;
  int *d_n = nullptr;
  long long *d_moff = nullptr, *d_voff = nullptr;
  int *d_ids = nullptr;
  struct Bucket {
    int kind;   // 1..4: small kernel with NB = kind; 0: large kernel
    int first;  // into the id list
    int count;
    int nbmax;  // large kernel: blocks of the largest instance
    int cfg;    // small: waves per block (1, 2, 4); large: waves per instance (4, 8)
  };
  std::vector<Bucket> buckets;
  int use_graph = 1;
  bool have_graph = false;
  const void *key[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;
  double *wsw = nullptr;          // n > 64: inverse diagonal blocks (W_j tiles)
  long long *d_wwoff = nullptr;   // per instance offset into wsw (doubles)
  // mixed-precision solves (allocated on first use)
  float *ws = nullptr;          // low-precision factors, per instance
  long long ws_bytes = 0;
  long long *d_woff = nullptr;  // per instance offset into ws (floats)
  int *d_mx_ids = nullptr;      // all instances, longest first
  int mx_nbmax = 0;
};

namespace bh {
// Launches every size-class kernel of the FP64 solver; with `only` set, an
// instance id is processed only where only[id] != 0.
int launch_all(const blasfeo_hip_plan *p, const double *A, double *L,
               const double *B, double *X, int *info, hipStream_t st,
               const int *only = nullptr);
}  // namespace bh
