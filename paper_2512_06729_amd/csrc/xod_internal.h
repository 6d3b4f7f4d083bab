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
  const int *jrow, *jptr;           // Jacobian nonzeros by row, their contributions
  const int *jc_ru, *jc_col;        // contribution e: slot jc_ru[e] = 6 r + u, column
  const double *jc_nu;
  const int *rsp;                   // [R*6] distinct species of each reaction
  const int *photo_idx;             // [R] index among the photolysis reactions (-1: none)
  int nph;                          // photolysis reactions
  const double *kph;                // [N*nph] spectral photolysis rates, or null (gray)
  // grid (device, owned by the column)
  const double *T, *ngas, *tau, *lnpref, *g, *trl, *trd, *tru;
  const double *bsrc;               // [S] surface emission / dz_0 into layer 0, or null
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
  double *dx;        // refined increment [N*S] (mixed precision)
  double *x0;        // the unrefined solution of an FP64 refinement [N*S]
  double *dwd;       // [N*R*6] dw_r/dn_x for the distinct species x = rsp[6r+u]
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
  int update32 = 1;       // trailing update in panel-wide strips (0: 16-wide)
  int update32_min = 200; // ... for launches of at least this many (block, strip) pairs
  int outer = 32;         // Gauss-Jordan outer panel width (32: unblocked)
  int outer_nmat = 1;     // ... for launches of at least this many blocks
  double refine_tol = 1e-7;    // mixed refinement: relative size of the last correction
  double refine_atol = 1e-14;  // ... and its floor, relative to the layer's largest increment
  int refine64 = 0;            // FP64 steps: refinements with the FP64 factors (0: none)
  int mixed_sticky = 16;       // mixed steps at or above a step size that fell back: this many
                               // go to FP64 directly before FP32 is tried again (0: never)
  int gemm_large = 1;     // 128 x 128 product tiles for large batches
  int gemm_k = 32;        // K step of the block products staged in LDS (16 or 32)
  int gemm_waves = 16;    // waves per 128-tile work-group of the block products (16 or 8)
  int panel_sync = 2;     // barriers per Gauss-Jordan column (1 or 2)
  int panel_defer = 0;    // 1: panel eliminations of other columns deferred by one column
  int gemm_lib = 0;       // cyclic-reduction block products: 1 = rocBLAS batched GEMM
  int graph = 1;          // replay captured launch sequences (cyclic reduction)
  int fused_max_ld = 64;  // FP64 block Thomas with ld up to this (<= 128, 0: never): one
                          // persistent launch each for a column's factorisation and solve
  int profile = 0;        // record HIP events around profiled launches
  int profile_every = 1;  // profile layers k with k % profile_every == 0
};
Options &options();          // the effective options (a tuned scope's, if one is active)
Options &global_options();   // the process-wide options (xod_set_option)
Options *&options_override();   // this thread's tuned options, or null

// Event-based launch timing (enabled with the "profile" option).  Kinds:
enum ProfKind { kProfPanel = 0, kProfUpdate, kProfPrologue, kProfSolve, kProfJac,
                kProfRates, kProfRhs, kProfGemm, kProfPhoto, kProfNum };
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
hipError_t launch_jacobian(const Acc &acc, int ncols, int maxN, int maxR, int ld, bool mixed,
                           hipStream_t s);
template <class Acc>
hipError_t launch_factor_fp64(const Acc &acc, int ncols, int maxN, int ld, hipStream_t s);
template <class Acc>
hipError_t launch_solve_fp64(const Acc &acc, int ncols, int maxN, int ld, hipStream_t s);
template <class Acc>
hipError_t launch_factor_mixed(const Acc &acc, int ncols, int maxN, int ld, hipStream_t s);
// Refinement (mixed precision), per column of the launch:
//   residual  x = rs * (f - M dx)   (dw: the column's w buffer as scratch;
//             rs null: no row scaling, for FP64 factors)
//   scale     x = rs * f
//   axpy      dx += x, ratio[col * maxN + k] = the componentwise size of x
//             in layer k, max_i |x_i| / (rtol |n_i + dx_i| + atol max|dx_k|)
//             over the components with mixing ratio above 1e-30 (rtol, atol
//             from the options), and out[0] = the maximum over all columns
//             and layers
// A refinement has converged at a size <= 1; refine_next() decides.
enum RefineNext { kRefineMore = 0, kRefineDone, kRefineFallback };
inline RefineNext refine_next(double q, double q_prev, int it, int max_it) {
  if (q <= 1.0) return kRefineDone;
  // stalled (the corrections no longer shrink: the FP64 residual's rounding
  // floor) or out of iterations: accept within ten times the tolerance,
  // otherwise solve again in FP64
  if (q > 0.5 * q_prev || it >= max_it) return q <= 10.0 ? kRefineDone : kRefineFallback;
  return kRefineMore;
}
template <class Acc>
hipError_t launch_residual(const Acc &acc, int ncols, int maxN, int maxS, int maxR,
                           hipStream_t s);
template <class Acc>
hipError_t launch_scale(const Acc &acc, int ncols, int maxN, int maxS, hipStream_t s);
template <class Acc>
hipError_t launch_axpy_ratio(const Acc &acc, int ncols, int maxN, double *ratio, double *out,
                             hipStream_t s);
// The same with explicit rtol, atol and mixing-ratio floor (rtol 1, atol 0:
// the largest relative correction of a component above the floor, a Newton
// iteration's size).
template <class Acc>
hipError_t launch_axpy_size(const Acc &acc, int ncols, int maxN, double *ratio, double *out,
                            double rtol, double atol, double y_floor, hipStream_t s);
template <class Acc>
hipError_t launch_solve_mixed(const Acc &acc, int ncols, int maxN, int ld, hipStream_t s);
// After an FP64 refinement: per layer, x = dx (refined) where the layer's
// correction size ratio[col * maxN + k] is at most `most`, else x = x0 (the
// unrefined solution): a correction that large means the factors' solve is
// too inaccurate for the correction to help.
template <class Acc>
hipError_t launch_keep_refined(const Acc &acc, int ncols, int maxN, int maxS, const double *ratio,
                               double most, hipStream_t s);

// Explicit block systems in mixed precision (caller's FP64 B [N*ld*ld], a, c
// [N*ld]): row scales rs, the scaled FP32 blocks Bf and scaled couplings
// as, cs; and the scaled FP64 residual x = rs * (g - M dx) ([N*S] layout).
hipError_t launch_cast_scale(const double *B, const double *a, const double *c, int N, int ld,
                             float *Bf, double *rs, double *as, double *cs, hipStream_t s);
hipError_t launch_bt_resid(const double *B, const double *a, const double *c, const double *g,
                           const double *dx, const double *rs, int N, int S, int ld, double *x,
                           hipStream_t s);

// One square block inverted in place by Gauss-Jordan elimination: its
// storage, pivot bookkeeping (piv[j] = row chosen for column j, rstep = the
// inverse permutation) and the id reported with a singular pivot.
template <class T>
struct MatRef {
  T *W;
  int *piv, *rstep, *flag;
  int id;
};

// Invert `count` ld x ld blocks listed in dlist (device array).  rstep of
// every listed block must hold INT_MAX on entry.
template <class T>
hipError_t launch_invert_list(const MatRef<T> *dlist, int count, int ld, hipStream_t s);

// Batched dense product on ld x ld row-major blocks:
//   C = (beta ? C : 0) + alpha * (A * B[bg] + A2 * B2[bg2])
// where B[bg] gathers B's rows (row m of the operand is B row bg[m]; bg may
// be null for the identity).  A2 may be null (single product).
template <class T>
struct GemmOp {
  const T *A, *B;
  const int *bg;
  const T *A2, *B2;
  const int *bg2;
  T *C;
  double alpha;
  int beta;
};
// Spectral photolysis rates kph [N*P] (see xod_photolysis_spectral); work of
// photolysis_work_bytes(N, A, L, P) bytes.
size_t photolysis_work_bytes(int N, int A, int L, int P);
hipError_t launch_photolysis(int N, int S, int A, int L, int P, const double *n, const double *dz,
                             const int *absorbers, const double *sig_ext, const double *J0,
                             const double *dlam, const double *sig_ph, double t_f, double mu,
                             void *work, double *kph, hipStream_t s);

template <class T>
hipError_t launch_gemm(const GemmOp<T> *dops, int count, int ld, hipStream_t s);
// dst[r][:] = src[idx[r]][:] for the ld rows of one ld x ld block per op.
template <class T>
struct GatherOp {
  const T *src;
  const int *idx;
  T *dst;
};
template <class T>
hipError_t launch_gather_rows(const GatherOp<T> *dops, int count, int ld, hipStream_t s);

// Batched matrix-vector terms on padded vectors of length ld:
//   y[j] = (b ? b[j] : 0) + sum_t sgn_t * (s_t ? s_t[j] : 1) * v_t[j]
//   v_t[j] = M_t ? sum_m M_t[rm_t ? rm_t[j] : j][m] * x_t[xm_t ? xm_t[m] : m]
//               : x_t[j]                       (diagonal term)
// y may alias b; no x_t may alias y.
template <class T>
struct MvTerm {
  const T *M;
  const int *rm, *xm;
  const double *x, *s;
  double sgn;
};
template <class T>
struct MvOp {
  MvTerm<T> t[2];
  int nterm;
  const double *b;
  double *y;
};
template <class T>
hipError_t launch_mv(const MvOp<T> *dops, int count, int ld, hipStream_t s);

// First level of block cyclic reduction (diagonal couplings a, c): for every
// kept layer k with eliminated neighbours k-1 / k+1 (E = their inverses,
// E[i][j] = W[piv[i]][rstep[j]]):
//   D_k -= a_k E_{k-1} c_{k-1} + c_k E_{k+1} a_{k+1}
//   A_k  = -a_k E_{k-1} a_{k-1}     (if layer k-2 exists)
//   C_k  = -c_k E_{k+1} c_{k+1}     (if layer k+2 exists)
template <class T>
struct CrLevel0Op {
  T *D, *A, *C;                    // A / C null when the new coupling is absent
  const T *Wl, *Wr;                // null when the neighbour is absent
  const int *pl, *ql, *pr, *qr;    // piv / rstep of the neighbours
  const double *ak, *ck, *al, *cl, *ar, *cr;
};
template <class T>
hipError_t launch_cr_level0(const CrLevel0Op<T> *dops, int count, int ld, hipStream_t s);

// rstep <- INT_MAX for n entries, flag[0..3] <- -1.
hipError_t launch_cr_reset(int *rstep, size_t n, int *flag, hipStream_t s);

// Copy between the compact [N*S] layout and the padded [N*ld] layout.
hipError_t launch_pad_copy(const double *src, double *dst, int N, int S, int ld, bool to_padded,
                           hipStream_t s);

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
  double y_neg;        // significant negative: below -y_neg n_gas (0: any)
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
// Lagrangian parcel at layer k: f [S] += the molecular-diffusion gains from
// the profile prof [N*S] (max(trd, 0) at k, trl from k-1, tru from k+1);
// out = min(in, 0) over n doubles (the self-coefficient's loss part).
hipError_t launch_parcel_gain(double *f, const double *prof, const double *trl,
                              const double *trd, const double *tru, int N, int S, int k,
                              hipStream_t s);
hipError_t launch_min0(const double *in, double *out, size_t n, hipStream_t s);
// out = alpha p + beta q over n doubles
hipError_t launch_lincomb(double *out, const double *p, double alpha, const double *q,
                          double beta, size_t n, hipStream_t s);

}  // namespace xod

