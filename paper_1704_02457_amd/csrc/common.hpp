// Host-side helpers shared by the library's translation units: argument
// checks, per-thread stream / last-error state, launch error capture.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/blasfeo_hip.h"
#include "blocks.hpp"

namespace bh {

// Per-thread library state (stream of the single-instance routines and the
// last error they recorded).
hipStream_t &tl_stream();
int &tl_error();

inline void set_error(int e) {
  if (e != 0 && tl_error() == 0) tl_error() = e;
}

// Validates an operand (sA, ai, aj) covering rows x cols; returns true if ok.
inline bool operand_ok(const blasfeo_dmat *s, int ai, int aj, int rows,
                       int cols) {
  if (!s) return false;
  if (ai < 0 || aj < 0 || rows < 0 || cols < 0) return false;
  if ((long long)ai + rows > s->m || (long long)aj + cols > s->n) return false;
  if ((rows > 0 && cols > 0) && !s->pA) return false;
  if (s->cn < s->n || s->pm * PS < s->m) return false;
  return true;
}

inline View make_view(const blasfeo_dmat *s, int ai, int aj, int rows,
                      int cols) {
  View v;
  v.p = s->pA;
  v.cn = s->cn;
  v.ai = ai;
  v.aj = aj;
  v.rows = rows;
  v.cols = cols;
  return v;
}

// Doubles between consecutive instances of a uniform batch.
inline long long batch_stride(const blasfeo_dmat *s) {
  return s ? (long long)s->memsize / 8 : 0;
}

inline int launch_status() {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : (int)e;
}

}  // namespace bh
