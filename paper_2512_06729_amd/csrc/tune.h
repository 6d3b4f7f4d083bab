// Tile-shape autotuner for the block factorisations: measured settings of
// the factorisation's tile options, kept per (GPU architecture, padded block
// size, precision, factorisation, single column or batch), applied while a
// column of that kind is factored.
#pragma once

#include "handles.h"

namespace xod {

// The tile options the tuner chooses.
struct TuneVals {
  int fused_max_ld, outer, update32, gemm_large, gemm_k, panel_sync, gemm_waves;
};

// While alive, options() on this thread returns the process-wide options
// with the tuned values for this kind of column (if any were measured).
class TunedScope {
 public:
  TunedScope(int ld, xod_precision prec, xod_solver solver, bool batch);
  ~TunedScope();
  TunedScope(const TunedScope &) = delete;
  TunedScope &operator=(const TunedScope &) = delete;

 private:
  Options local_;
  Options *prev_ = nullptr;
  bool on_ = false;
};

}  // namespace xod
