// Internal declarations of libxod: device argument blocks, kernel launch
// helpers and error plumbing.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/xod.h"

namespace xod {

// CGS constants used by the device code.
constexpr double kBoltz = 1.380649e-16;      // erg/K
constexpr double kAmu = 1.66053906660e-24;   // g
constexpr double kPstd = 1.0e6;              // dyn/cm^2 (1 bar)

constexpr int kMaxLd = 1024;   // largest padded block size (one row per thread)
constexpr int kNB = 32;        // Gauss-Jordan panel width
constexpr int kStrip = 16;     // Schur-update column strip (MFMA N)

// Everything a kernel needs to know about one column.  Passed by value for
// single-column launches and as a device array for batched launches.
struct ColArgs {
  int N, S, R, ld;
  double dt;
  // network tables (device)
  const int *rtype, *reac, *prod, *rev, *kooij, *dnu;
  const double *params;
  const int *inc_ptr, *inc_r;
  const double *inc_nu;
  const int *jmap, *jptr, *jc_r;
  const double *jc_nu;
  // grid (device, owned by the column)
  const double *T, *ngas, *tau, *lnpref, *g, *trl, *trd, *tru;
  // operands
  const double *kf_in, *kr_in, *n;
  double *kf, *kr, *w, *f;
  double *B;         // FP64 blocks [N*ld*ld]
  float *Bf;         // FP32 blocks [N*ld*ld] (mixed)
  double *a, *c;     // [N*ld]
  double *rs;        // row scales [N*ld] (mixed)
  int *piv;          // [N*ld] pivot row of each column
  int *rstep;        // [N*ld] pivot step of each row (inverse of piv)
  double *x;         // solve vector [N*S] (in/out)
  double *gs;        // solve scratch [N*ld]
  int *flag;         // [4]: singular layer, singular column, nonfinite, spare
};

// Kernel-side accessors: one column by value, or a device array of columns.
struct OneCol {
  ColArgs a;
  __device__ __forceinline__ const ColArgs &operator()(int) const { return a; }
};
struct ManyCols {
  const ColArgs *p;
  __device__ __forceinline__ const ColArgs &operator()(int c) const { return p[c]; }
};

// Thread-local error message.
void set_error(const std::string &msg);
std::string &last_error();

#define XOD_HIP(call)                                                        \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess) {                                                  \
      ::xod::set_error(std::string("HIP error in ") + #call + ": " +         \
                       hipGetErrorString(e_));                               \
      return XOD_EHIP;                                                       \
    }                                                                        \
  } while (0)

inline int round_up(int v, int m) { return (v + m - 1) / m * m; }

// Process-wide kernel options.
struct Options {
  int gemm_mfma = 1;
  int profile = 0;        // record HIP events around profiled launches
  int profile_every = 1;  // profile layers k with k % profile_every == 0
};
Options &options();

// Event-based launch timing (enabled with the "profile" option).  Kinds:
enum ProfKind { kProfPanel = 0, kProfUpdate, kProfPrologue, kProfSolve, kProfJac,
                kProfRates, kProfRhs, kProfNum };
// Record an event pair around the next launch of `kind` on stream s.
void prof_begin(int kind, hipStream_t s);
void prof_end(int kind, hipStream_t s);
inline bool prof_layer(int k) {
  return options().profile && (k % options().profile_every) == 0;
}

// Launchers (defined in the .hip files).  Each enqueues on `stream` and
// returns hipSuccess or the launch error.
template <class Acc>
hipError_t launch_rates(const Acc &acc, int ncols, int maxN, int maxR, hipStream_t s);
template <class Acc>
hipError_t launch_rhs(const Acc &acc, int ncols, int maxN, int maxR, int maxS, hipStream_t s);
template <class Acc>
hipError_t launch_jacobian(const Acc &acc, int ncols, int maxN, int ld, bool mixed,
                           hipStream_t s);
template <class Acc>
hipError_t launch_factor_fp64(const Acc &acc, int ncols, int maxN, int ld, hipStream_t s);
template <class Acc>
hipError_t launch_solve_fp64(const Acc &acc, int ncols, int maxN, int ld, hipStream_t s);
template <class Acc>
hipError_t launch_factor_mixed(const Acc &acc, int ncols, int maxN, int ld, hipStream_t s);
template <class Acc>
hipError_t launch_residual(const Acc &acc, int ncols, int maxN, int maxS, int maxR,
                           const double *delta, double *dw, hipStream_t s);
template <class Acc>
hipError_t launch_scale(const Acc &acc, int ncols, int maxN, int maxS, hipStream_t s);
template <class Acc>
hipError_t launch_axpy_ratio(const Acc &acc, int ncols, int maxN, double *delta, double *ratio,
                             double *out, hipStream_t s);
template <class Acc>
hipError_t launch_solve_mixed(const Acc &acc, int ncols, int maxN, int ld, hipStream_t s);

// Column set-up arguments (k_setup).
struct SetupArgs {
  int N, S;
  const double *P_bar, *T, *K, *D, *alpha, *mass, *nasa7;
  double t_mid, mbar_amu, g_cgs, sigma_tau;
  double *ngas, *tau, *lnpref, *g, *trl, *trd, *tru, *dz, *dzh, *mix;
};

// State update (n_new = n + delta) and statistics.  Per-block partials,
// kNStat doubles:
//   0 max rel change over y > y_floor     1 min n_new / n_gas
//   2 max control change over y > y_sig   3 clipped amount (sum)
//   4 significant negative (0/1)          5 non-finite (0/1)
constexpr int kNStat = 6;
constexpr int kUpdBlocks = 64;
constexpr int kStatLen = kNStat + 4;   // + the four error flags
struct UpdArgs {
  const double *n, *x, *ngas;
  double *nout;
  double *partial;     // [kUpdBlocks * kNStat]
  int N, S;
  int clip;            // 1: driver semantics (clip negatives)
  double y_floor, y_sig;
};
struct RedArgs {
  const double *partial;
  const int *flag;
  double *out;         // [kStatLen]
};

hipError_t launch_setup(const SetupArgs &a, hipStream_t st);
hipError_t launch_update_state(const UpdArgs *dargs, const RedArgs *dred, int ncols,
                               hipStream_t s);
hipError_t launch_invperm(const int *piv, int *rstep, int N, int ld, hipStream_t s);

}  // namespace xod

