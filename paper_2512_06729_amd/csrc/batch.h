// Batched steps shared by xod_batch and the serving loop.
#pragma once

#include <vector>

#include "handles.h"

#define XOD_TRY_B(expr)            \
  do {                             \
    xod_status s_ = (expr);        \
    if (s_ != XOD_OK) return s_;   \
  } while (0)

namespace xod {

// Staging buffers for up to `cap` columns per batched step.
struct BatchRunner {
  int cap = 0;
  ColArgs *d_args = nullptr, *h_args = nullptr;
  UpdArgs *d_upd = nullptr, *h_upd = nullptr;
  RedArgs *d_red = nullptr, *h_red = nullptr;
  double *d_stats = nullptr, *h_stats = nullptr, *d_partial = nullptr;
  double *d_ratio = nullptr, *d_rmax = nullptr, *h_rmax = nullptr;   // mixed refinement
  size_t ratio_cap = 0;
  // one stream per group of equal block size and precision (created on first
  // use, default priority), forked from and joined back to the caller's stream
  static constexpr int kMaxGroups = 16;
  std::vector<hipStream_t> gstream;
  std::vector<hipEvent_t> gevent;
  hipEvent_t fork_ev = nullptr;
  // per caller index, from the last step: refinements, FP64 fallback, final ratio
  std::vector<int> last_iters, last_fallback;
  std::vector<double> last_resid;
  // with time_groups set, each group's device time (ms, events on its
  // stream around its work) of the last step, keyed by (ld, precision)
  bool time_groups = false;
  std::vector<std::pair<std::pair<int, int>, float>> last_group_ms;
  std::vector<hipEvent_t> tev;
  ~BatchRunner();
  xod_status init(int capacity);
  xod_status step(const std::vector<xod_column *> &cols, const double *dts, bool clip,
                  double y_floor, double y_sig, double y_neg, hipStream_t s,
                  std::vector<double> &stats);
};

}  // namespace xod

// A batch handle: its columns and the runner that steps them together.
struct xod_batch {
  std::vector<xod_column *> cols;
  xod::BatchRunner runner;
  hipStream_t stream = nullptr;
  ~xod_batch();
};
