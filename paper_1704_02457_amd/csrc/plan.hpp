// Host-side plan of an uneven batch (shared by the FP64 and the
// mixed-precision solvers).  The plan owns only host data and a small device
// table (orders, offsets, class lists); every byte of scratch memory the
// kernels use comes from the caller's workspace.
#pragma once
#include <string>
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
  std::vector<int> ids;  // host copy of the class lists (d_ids)
  int use_graph = 1;
  bool have_graph = false;
  const void *key[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;
  // captured graphs run the size classes as parallel branches: one stream
  // per class forked from and joined to the capturing stream by events
  static constexpr int kMaxAux = 8;
  hipStream_t aux[kMaxAux] = {};
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[kMaxAux] = {};
  // Workspace of an FP64 execution: for the instances with n > 64, the
  // inverses W_j of the diagonal blocks (256 doubles per 16-row block), kept
  // for the back substitution, at W + wwoff[id] doubles.
  long long ws64_bytes = 0;
  long long *d_wwoff = nullptr;
  // Workspace of a mixed-precision call: the FP64 part above (rounded up to
  // 256 bytes), then the low-precision factor tiles of every instance at
  // + woff[id] floats.
  long long ws32_bytes = 0;
  long long *d_woff = nullptr;  // per instance offset into the FP32 part (floats)
  int *d_mx_ids = nullptr;      // all instances, longest first
  int mx_nbmax = 0;
  bool mx_ok = false;           // right-hand sides present and the LDS fits
};

namespace bh {

inline long long round256(long long b) { return (b + 255) / 256 * 256; }

// Bytes of the workspace of a mixed-precision call.
inline long long mixed_ws_bytes(const blasfeo_hip_plan *p) {
  return round256(p->ws64_bytes) + p->ws32_bytes;
}

// Launches every size-class kernel of the FP64 solver with workspace W; with
// `only` set, an instance id is processed only where only[id] != 0.
int launch_all(const blasfeo_hip_plan *p, const double *A, double *L,
               const double *B, double *X, int *info, double *W,
               hipStream_t st, const int *only = nullptr);

// Launch configuration values valid for a size class (kind 1..4: small
// kernel; 0: n > 64).
inline bool tune_cfg_valid(int kind, int cfg) {
  if (kind >= 1 && kind <= 4) return cfg == 1 || cfg == 2 || cfg == 4;
  if (kind != 0) return false;
  return cfg == 1 || cfg == 2 || cfg == 4 || cfg == 8 || cfg == 16 || cfg == 104 ||
         cfg == 108 || cfg == 116 || cfg == 201 || cfg == 202 || cfg == 204 ||
         cfg == 211 || cfg == 212 || cfg == 214;
}

// What identifies a size class in the tuning cache.
struct TuneKey {
  std::string arch;
  int cus = 0, kind = 0, nrhs = 0, count = 0, nmin = 0, nmax = 0;
  long long nsum = 0;
};
int tune_key_device(TuneKey &k);  // fills arch and cus of the current device
bool tune_lookup(const TuneKey &k, int *cfg);
void tune_store(const TuneKey &k, int cfg, float ms);

// Mixed-precision part of plan creation: the FP32 tile offsets, the
// longest-first order and the launch attributes (device tables allocated
// here, never in a compute call).
int mx_plan_setup(blasfeo_hip_plan *p);
}  // namespace bh
