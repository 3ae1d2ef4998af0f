// Termination and multistart rule of QFactor (Sec. III-A-2 hyperparameters,
// Sec. IV-A parallel multistarts), shared by the host sweep loop and the
// LDS-resident kernel so both take identical decisions.
//
// Readings of the paper's garbled tests (c_i = cost after sweep i, c_0 = cost
// of the initial gates):
//   short plateau: c_{i-1} - c_i <= diff_tol_a + diff_tol_r * c_i
//                  (off when diff_tol_a and diff_tol_r are both 0)
//   long plateau:  i >= L and c_{i-L} - c_i < long_diff_r * c_{i-L},
//                  L = long_diff_count (off when L <= 0)
//   a start that met a plateau test stays marked; the job stops when any
//   active start has c_i < tol, when every start is marked, or at max_iter;
//   no test runs before sweep min_iter; a non-finite cost freezes a start
//   and marks it.
#pragma once

#include <math.h>
#include <stdint.h>

#include "qfactor.h"

namespace qf {

enum : int32_t { kFlagPlateau = 1, kFlagNumeric = 2, kFlagConverged = 4 };
enum : int32_t { kContinue = 0, kStopConverged = 1, kStopPlateau = 2, kStopMaxIter = 3 };

// Per-start test after sweep i.  c_prev = c_{i-1}; c_back = c_{i-L} (ignored
// when i < L).  Returns the new flag word.
__host__ __device__ inline int32_t start_flags_after_sweep(const qf_options& o, double tol, int32_t i,
                                                           int32_t flags, double c_i, double c_prev,
                                                           double c_back) {
  if (!isfinite(c_i)) return flags | kFlagNumeric | kFlagPlateau;
  if (flags & kFlagNumeric) return flags;
  if (i < o.min_iter) return flags;
  if (c_i < tol) flags |= kFlagConverged;
  if (o.diff_tol_a > 0.0 || o.diff_tol_r > 0.0) {
    if (c_prev - c_i <= o.diff_tol_a + o.diff_tol_r * c_i) flags |= kFlagPlateau;
  }
  const int32_t L = o.long_diff_count;
  if (L > 0 && i >= L) {
    if (c_back - c_i < o.long_diff_r * c_back) flags |= kFlagPlateau;
  }
  return flags;
}

// Job-level decision from every start's flags after sweep i.
__host__ __device__ inline int32_t job_decision(const qf_options& o, int32_t i, const int32_t* flags,
                                                int32_t n_starts) {
  if (i >= o.min_iter) {
    bool any_conv = false, all_plat = true;
    for (int32_t s = 0; s < n_starts; ++s) {
      any_conv = any_conv || ((flags[s] & kFlagConverged) && !(flags[s] & kFlagNumeric));
      all_plat = all_plat && (flags[s] & kFlagPlateau);
    }
    if (any_conv) return kStopConverged;
    if (all_plat) return kStopPlateau;
  }
  if (i >= o.max_iter) return kStopMaxIter;
  return kContinue;
}

}  // namespace qf
