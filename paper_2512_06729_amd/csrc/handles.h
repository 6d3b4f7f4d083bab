// Handle layouts shared by the ABI translation units (api.cpp, batch.cpp).
#pragma once

#include <vector>

#include "xod_internal.h"

namespace xod {
template <class T> struct CrPlan;
void cr_destroy(CrPlan<double> *p);
void cr_destroy(CrPlan<float> *p);
}  // namespace xod

using xod::ColArgs;
using xod::RedArgs;
using xod::UpdArgs;

struct xod_network {
  int S = 0, R = 0, E = 0, ld = 0;
  double t_mid = 1000.0;
  std::vector<void *> owned;
  int *rtype = nullptr, *reac = nullptr, *prod = nullptr, *rev = nullptr, *kooij = nullptr,
      *dnu = nullptr;
  double *params = nullptr, *nasa7 = nullptr, *mass = nullptr;
  int *inc_ptr = nullptr, *inc_r = nullptr;
  double *inc_nu = nullptr;
  int *jrow = nullptr, *jc_col = nullptr, *jptr = nullptr, *jc_ru = nullptr, *rsp = nullptr;
  double *jc_nu = nullptr;
  std::vector<double> mass_h;
  int nnz = 0, ncontrib = 0;
  int *photo_idx = nullptr;   // [R]: index among the photolysis reactions, -1 for others
  int nph = 0;                // number of photolysis reactions
  ~xod_network() {
    for (void *p : owned) (void)hipFree(p);
  }
};

struct xod_column {
  const xod_network *net = nullptr;
  int N = 0, S = 0, R = 0, ld = 0;
  xod_precision prec = XOD_FP64;
  hipStream_t stream = nullptr;
  std::vector<void *> owned;
  double *P = nullptr, *T = nullptr, *K = nullptr, *D = nullptr, *alpha = nullptr;
  double *ngas = nullptr, *tau = nullptr, *lnpref = nullptr, *g = nullptr, *trl = nullptr,
         *trd = nullptr, *tru = nullptr, *dz = nullptr, *dzh = nullptr, *mix = nullptr;
  // Spectral photolysis (xod_column_set_photolysis_spectrum): the caller's
  // device tables, the library's rates [N*nph] and scratch.  ph_L = 0: gray.
  int ph_A = 0, ph_L = 0;
  const int *ph_abs = nullptr;
  const double *ph_ext = nullptr, *ph_J0 = nullptr, *ph_dlam = nullptr, *ph_sig = nullptr;
  double ph_tf = 1.0, ph_mu = 1.0;
  double *kph = nullptr;
  void *ph_work = nullptr;
  size_t ph_work_bytes = 0;
  double mix_time = 0.0;
  // Boundary exchange (xod_column_set_boundary): the velocities sit in the
  // transport diagonal trd of the bottom and top layers (rows kept as set up
  // in trd_bot0 / trd_top0), the surface emission in bsrc.
  double T_top = 0.0, mbar_amu = 0.0, g_cgs = 0.0;
  std::vector<double> D_top;               // [S] molecular diffusion of the top layer
  std::vector<double> trd_bot0, trd_top0;  // trd rows 0 and N-1 of the closed column
  double *bsrc = nullptr;
  bool has_bsrc = false;
  bool open_ends = false;   // a boundary exchange with nonzero velocities or emission is set
  // Lagrangian parcel pass (xod_parcel_pass): molecular-diffusion-only
  // transport coefficients [N*S] (trl, trd, tru, the loss part min(trd, 0)),
  // set-up scratch, and the single-layer step buffers; allocated on first use.
  double *pc_trl = nullptr, *pc_trd = nullptr, *pc_tru = nullptr, *pc_loss = nullptr;
  double *pc_setup = nullptr;
  double *pc_p = nullptr, *pc_q = nullptr, *pc_f = nullptr, *pc_x = nullptr, *pc_zero = nullptr;
  double *pc_w = nullptr, *pc_dwd = nullptr, *pc_B = nullptr, *pc_a = nullptr, *pc_c = nullptr;
  double *pc_gs = nullptr, *pc_partial = nullptr, *pc_stats = nullptr;
  int *pc_piv = nullptr, *pc_rstep = nullptr;
  UpdArgs *pc_upd = nullptr;
  RedArgs *pc_red = nullptr;
  double *dwd = nullptr;   // [N*R*6] reaction-rate derivatives of the last Jacobian
  double *n = nullptr, *ntmp = nullptr, *kf = nullptr, *kr = nullptr, *w = nullptr,
         *f = nullptr, *x = nullptr, *gs = nullptr, *resid = nullptr, *dx = nullptr;
  double *B = nullptr;
  float *Bf = nullptr;
  double *a = nullptr, *c = nullptr, *rs = nullptr;
  int *piv = nullptr, *rstep = nullptr, *flag = nullptr;
  double *partial = nullptr, *stats_dev = nullptr, *stats_host = nullptr;
  double *ratio = nullptr, *rmax = nullptr;   // refinement convergence measure
  int max_refine = 10;
  UpdArgs *upd_dev = nullptr, *upd_host = nullptr;   // host side pinned
  RedArgs *red_dev = nullptr, *red_host = nullptr;
  double t = 0.0, dt = 0.0;
  double fact_dt = 0.0;   // dt of the FP64 factorisation held in the blocks (0: none)
  // mixed precision control: smallest step size that fell back to FP64 (0:
  // none) and the steps since taken in FP64 directly
  double mixed_fb_dt = 0.0;
  int mixed_direct = 0;
  double prev_dt = 0.0;   // dt of the step whose starting state ntmp holds (0: none)
  bool in_batch = false;
  // The factorisation xod_btd_factor left in the column's own workspace
  // (cyclic reduction or mixed precision): the caller's FP64 system it came
  // from and how it was factored.  Steps, batches and solver switches drop it.
  struct BtdHeld {
    bool valid = false;
    xod_precision prec = XOD_FP64;
    xod_solver solver = XOD_SOLVER_THOMAS;
    const double *B = nullptr, *a = nullptr, *c = nullptr;
  } btd;
  int btd_iters = 0, btd_fallback = 0;   // refinements / FP64 fallback of the last btd solve
  double btd_size = 0.0;                 // its last componentwise correction size
  xod_solver solver = XOD_SOLVER_THOMAS;
  xod::CrPlan<double> *cr64 = nullptr;   // block cyclic reduction (FP64 column)
  xod::CrPlan<float> *cr32 = nullptr;    // block cyclic reduction (mixed column)
  ~xod_column() {
    xod::cr_destroy(cr64);
    xod::cr_destroy(cr32);
    if (stats_host) (void)hipHostFree(stats_host);
    if (upd_host) (void)hipHostFree(upd_host);
    if (red_host) (void)hipHostFree(red_host);
    for (void *p : owned) (void)hipFree(p);
  }
  ColArgs args() const {
    ColArgs a_{};
    a_.N = N;
    a_.S = S;
    a_.R = R;
    a_.ld = ld;
    a_.dt = dt;
    a_.rtype = net->rtype;
    a_.reac = net->reac;
    a_.prod = net->prod;
    a_.rev = net->rev;
    a_.kooij = net->kooij;
    a_.dnu = net->dnu;
    a_.params = net->params;
    a_.inc_ptr = net->inc_ptr;
    a_.inc_r = net->inc_r;
    a_.inc_nu = net->inc_nu;
    a_.photo_idx = net->photo_idx;
    a_.nph = net->nph;
    a_.kph = ph_L > 0 ? kph : nullptr;
    a_.jrow = net->jrow;
    a_.jc_col = net->jc_col;
    a_.jptr = net->jptr;
    a_.jc_ru = net->jc_ru;
    a_.jc_nu = net->jc_nu;
    a_.rsp = net->rsp;
    a_.dwd = dwd;
    a_.T = T;
    a_.ngas = ngas;
    a_.tau = tau;
    a_.lnpref = lnpref;
    a_.g = g;
    a_.trl = trl;
    a_.trd = trd;
    a_.tru = tru;
    a_.bsrc = has_bsrc ? bsrc : nullptr;
    a_.kf_in = kf;
    a_.kr_in = kr;
    a_.n = n;
    a_.kf = kf;
    a_.kr = kr;
    a_.w = w;
    a_.f = f;
    a_.B = B;
    a_.Bf = Bf;
    a_.a = a;
    a_.c = c;
    a_.rs = rs;
    a_.piv = piv;
    a_.rstep = rstep;
    a_.x = x;
    a_.dx = dx;
    a_.x0 = resid;
    a_.gs = gs;
    a_.flag = flag;
    return a_;
  }
};


namespace xod {
// Enqueue rates + rhs + Jacobian + factor + solve of one column (FP64, or
// mixed with refinement and FP64 fallback); delta ends in col->x.
// hist != null adds hist_coef (n - hist) to the right-hand side (a
// multistep history term) before the factorisation's solve.
xod_status enqueue_solve(xod_column *c, double dt, int *iters, int *fallback, double *resid,
                         const double *hist = nullptr, double hist_coef = 0.0);
// n_new = n + delta into col->ntmp plus statistics (host copy, kStatLen).
xod_status run_update(xod_column *c, bool clip, double y_floor, double y_sig, double *out,
                      double y_neg = 0.0);
// The same, enqueued only: the statistics land in c->stats_host once the
// column's stream has reached them.
xod_status enqueue_update(xod_column *c, bool clip, double y_floor, double y_sig,
                          double y_neg = 0.0);
// Device bytes of the cyclic-reduction workspace of a column.
size_t cr_footprint(const xod_network *net, int N, xod_precision prec);
// Device bytes a column of this network with N layers allocates.
size_t column_footprint(const xod_network *net, int N, xod_precision prec);
}  // namespace xod
