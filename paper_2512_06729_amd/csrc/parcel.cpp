// The Lagrangian parcel scheme of the paper's own model (Section 2, the
// parcel figure; Section 2.1, molecular diffusion as a pseudo-reaction) on
// a column's profile: one global iteration carries an air parcel from the
// bottom layer to the top and back; at each layer it takes the layer's
// temperature and gas density (mixing ratios carried over), stays for the
// layer's eddy mixing time dz^2/K, and evolves by the layer's chemistry
// plus molecular diffusion with the profile's neighbours, after which its
// composition becomes the profile there.
//
// Each visit is a sequence of linearly implicit backward-Euler steps on the
// dense S x S system of one layer (the step matrix kernels run on a
// one-layer view of the column, the block inverted by the Gauss-Jordan
// kernels), under the step control of the steady-state driver inside the
// residence time.  The visits are sequential (each starts from the last one's
// parcel): the work per step is one block, so this path is latency-bound;
// the Eulerian column steps are the throughput path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "handles.h"

using namespace xod;

namespace {

#define PC_TRY(expr)                 \
  do {                               \
    xod_status s_ = (expr);          \
    if (s_ != XOD_OK) return s_;     \
  } while (0)

#define PC_CHECK(cond, msg)          \
  do {                               \
    if (!(cond)) {                   \
      set_error(msg);                \
      return XOD_EINVAL;             \
    }                                \
  } while (0)

template <class T>
xod_status palloc(xod_column *c, T **p, size_t count) {
  XOD_HIP(hipMalloc((void **)p, std::max<size_t>(count, 1) * sizeof(T)));
  c->owned.push_back(*p);
  return XOD_OK;
}

// Buffers and the molecular-diffusion-only transport coefficients (the
// set-up kernel run again with K = 0 into scratch outputs).
xod_status parcel_setup(xod_column *c) {
  if (c->pc_trl) return XOD_OK;
  const int N = c->N, S = c->S, ld = c->ld, R = c->R;
  const size_t NS = (size_t)N * S;
  PC_TRY(palloc(c, &c->pc_trl, NS));
  PC_TRY(palloc(c, &c->pc_trd, NS));
  PC_TRY(palloc(c, &c->pc_tru, NS));
  PC_TRY(palloc(c, &c->pc_loss, NS));
  // scratch outputs of the set-up kernel: K = 0, n_gas, tau, ln P0/kT, G/RT,
  // dz, dzh, mixing time
  PC_TRY(palloc(c, &c->pc_setup, 7 * (size_t)N + NS + 1));
  PC_TRY(palloc(c, &c->pc_p, S));
  PC_TRY(palloc(c, &c->pc_q, S));
  PC_TRY(palloc(c, &c->pc_f, S));
  PC_TRY(palloc(c, &c->pc_x, S));
  PC_TRY(palloc(c, &c->pc_zero, S));
  PC_TRY(palloc(c, &c->pc_w, R));
  PC_TRY(palloc(c, &c->pc_dwd, 6 * (size_t)R));
  PC_TRY(palloc(c, &c->pc_B, (size_t)ld * ld));
  PC_TRY(palloc(c, &c->pc_a, ld));
  PC_TRY(palloc(c, &c->pc_c, ld));
  PC_TRY(palloc(c, &c->pc_gs, ld));
  PC_TRY(palloc(c, &c->pc_partial, (size_t)kUpdBlocks * kNStat));
  PC_TRY(palloc(c, &c->pc_stats, kStatLen));
  PC_TRY(palloc(c, &c->pc_piv, ld));
  PC_TRY(palloc(c, &c->pc_rstep, ld));
  PC_TRY(palloc(c, &c->pc_upd, 1));
  PC_TRY(palloc(c, &c->pc_red, 1));
  XOD_HIP(hipMemsetAsync(c->pc_zero, 0, S * sizeof(double), c->stream));
  double *sc = c->pc_setup;
  double *Kz = sc;
  XOD_HIP(hipMemsetAsync(Kz, 0, N * sizeof(double), c->stream));
  SetupArgs sa{};
  sa.N = N;
  sa.S = S;
  sa.P_bar = c->P;
  sa.T = c->T;
  sa.K = Kz;
  sa.D = c->D;
  sa.alpha = c->alpha;
  sa.mass = c->net->mass;
  sa.nasa7 = c->net->nasa7;
  sa.t_mid = c->net->t_mid;
  sa.mbar_amu = c->mbar_amu;
  sa.g_cgs = c->g_cgs;
  sa.sigma_tau = 0.0;
  sa.ngas = sc + N;
  sa.tau = sc + 2 * (size_t)N;
  sa.lnpref = sc + 3 * (size_t)N;
  sa.dz = sc + 4 * (size_t)N;
  sa.dzh = sc + 5 * (size_t)N;
  sa.mix = sc + 6 * (size_t)N;
  sa.g = sc + 6 * (size_t)N + 1;
  sa.trl = c->pc_trl;
  sa.trd = c->pc_trd;
  sa.tru = c->pc_tru;
  XOD_HIP(launch_setup(sa, c->stream));
  XOD_HIP(launch_min0(c->pc_trd, c->pc_loss, NS, c->stream));
  XOD_HIP(hipStreamSynchronize(c->stream));
  return XOD_OK;
}

// The column's arguments narrowed to layer k for the parcel p: one layer,
// the layer's rate coefficients, the diffusion loss as the self-coefficient,
// no neighbours, the single-block step buffers.
ColArgs layer_view(const xod_column *c, int k, double dt) {
  ColArgs a = c->args();
  const size_t o = (size_t)k * c->S;
  a.N = 1;
  a.dt = dt;
  a.T = c->T + k;
  a.ngas = c->ngas + k;
  a.tau = c->tau + k;
  a.lnpref = c->lnpref + k;
  a.g = c->g + o;
  a.trl = c->pc_zero;
  a.trd = c->pc_loss + o;
  a.tru = c->pc_zero;
  a.bsrc = nullptr;
  a.kf_in = c->kf + (size_t)k * c->R;
  a.kr_in = c->kr + (size_t)k * c->R;
  a.kf = nullptr;
  a.kr = nullptr;
  a.n = c->pc_p;
  a.w = c->pc_w;
  a.f = c->pc_f;
  a.dwd = c->pc_dwd;
  a.B = c->pc_B;
  a.a = c->pc_a;
  a.c = c->pc_c;
  a.piv = c->pc_piv;
  a.rstep = c->pc_rstep;
  a.x = c->pc_x;
  a.gs = c->pc_gs;
  return a;
}

}  // namespace

extern "C" xod_status xod_parcel_pass(xod_column *col, double dt0, double *dt_last,
                                      xod_parcel_stats *st) {
  PC_CHECK(col, "xod_parcel_pass: null column");
  PC_CHECK(!col->in_batch, "xod_parcel_pass: column belongs to a batch");
  PC_CHECK(col->prec == XOD_FP64, "xod_parcel_pass: FP64 columns only");
  PC_CHECK(col->ph_L == 0, "xod_parcel_pass: spectral photolysis is not supported");
  PC_CHECK(!col->open_ends, "xod_parcel_pass: closed columns only");
  PC_CHECK(std::isfinite(dt0) && dt0 > 0, "xod_parcel_pass: dt0 must be > 0");
  const int N = col->N, S = col->S;
  PC_TRY(parcel_setup(col));
  col->fact_dt = 0.0;
  col->prev_dt = 0.0;
  col->btd.valid = false;
  // rate coefficients of every layer (state independent: gray photolysis)
  XOD_HIP(launch_rates(OneCol{col->args()}, 1, N, col->R, col->stream));
  std::vector<double> K(N), dz(N), ngas(N);
  XOD_HIP(hipMemcpyAsync(K.data(), col->K, N * sizeof(double), hipMemcpyDeviceToHost,
                         col->stream));
  XOD_HIP(hipMemcpyAsync(dz.data(), col->dz, N * sizeof(double), hipMemcpyDeviceToHost,
                         col->stream));
  XOD_HIP(hipMemcpyAsync(ngas.data(), col->ngas, N * sizeof(double), hipMemcpyDeviceToHost,
                         col->stream));
  XOD_HIP(hipStreamSynchronize(col->stream));
  for (int k = 0; k < N; ++k)
    PC_CHECK(K[k] > 0.0, "xod_parcel_pass: every layer needs K > 0 (its residence time)");

  const double y_sig = 1e-10, y_floor = 1e-30;
  const int max_consec = 30;
  std::vector<int> seq;
  for (int k = 0; k < N; ++k) seq.push_back(k);
  for (int k = N - 2; k >= 0; --k) seq.push_back(k);
  int64_t steps = 0, rejects = 0;
  double clipped = 0.0, dt = dt0;
  const size_t Sb = (size_t)S * sizeof(double);
  XOD_HIP(hipMemcpyAsync(col->pc_p, col->n + (size_t)seq[0] * S, Sb, hipMemcpyDeviceToDevice,
                         col->stream));
  double stats[kStatLen];
  for (size_t i = 0; i < seq.size(); ++i) {
    const int k = seq[i];
    if (i > 0)
      XOD_HIP(launch_lincomb(col->pc_p, col->pc_p, ngas[k] / ngas[seq[i - 1]], col->pc_p, 0.0,
                             S, col->stream));
    const double t_res = dz[k] * dz[k] / K[k];
    double t = 0.0;
    dt = std::min(dt, t_res);
    int consec = 0;
    while (t < t_res) {
      const double h = std::min(dt, t_res - t);
      ColArgs a = layer_view(col, k, h);
      const OneCol one{a};
      XOD_HIP(launch_rhs(one, 1, 1, col->R, S, col->stream));
      XOD_HIP(launch_parcel_gain(col->pc_f, col->n, col->pc_trl, col->pc_trd, col->pc_tru, N,
                                 S, k, col->stream));
      XOD_HIP(launch_jacobian(one, 1, 1, col->R, col->ld, false, col->stream));
      XOD_HIP(launch_factor_fp64(one, 1, 1, col->ld, col->stream));
      XOD_HIP(hipMemcpyAsync(col->pc_x, col->pc_f, Sb, hipMemcpyDeviceToDevice, col->stream));
      XOD_HIP(launch_solve_fp64(one, 1, 1, col->ld, col->stream));
      // q = p + x with the driver's statistics (clip, significant negatives,
      // control change, non-finite), and the singular flag
      UpdArgs u{};
      u.n = col->pc_p;
      u.x = col->pc_x;
      u.ngas = col->ngas + k;
      u.nout = col->pc_q;
      u.partial = col->pc_partial;
      u.N = 1;
      u.S = S;
      u.clip = 1;
      u.y_floor = y_floor;
      u.y_sig = y_sig;
      RedArgs r{col->pc_partial, col->flag, col->pc_stats};
      XOD_HIP(hipMemcpyAsync(col->pc_upd, &u, sizeof(u), hipMemcpyHostToDevice, col->stream));
      XOD_HIP(hipMemcpyAsync(col->pc_red, &r, sizeof(r), hipMemcpyHostToDevice, col->stream));
      XOD_HIP(launch_update_state(col->pc_upd, col->pc_red, 1, col->stream));
      XOD_HIP(hipMemcpyAsync(stats, col->pc_stats, sizeof(stats), hipMemcpyDeviceToHost,
                             col->stream));
      XOD_HIP(hipStreamSynchronize(col->stream));
      const bool singular = stats[kNStat] >= 0;
      if (singular || stats[5] > 0 || stats[4] > 0) {
        ++rejects;
        if (++consec > max_consec) {
          set_error("xod_parcel_pass: step size collapsed at layer " + std::to_string(k));
          return XOD_ENOTCONVERGED;
        }
        dt = 0.5 * h;
        continue;
      }
      consec = 0;
      clipped += stats[3];
      std::swap(col->pc_p, col->pc_q);
      t += h;
      ++steps;
      const double c = stats[2];
      dt = h * (c < 0.5 ? 2.0 : (c < 0.9 ? 1.2 : 0.7));
    }
    XOD_HIP(hipMemcpyAsync(col->n + (size_t)k * S, col->pc_p, Sb, hipMemcpyDeviceToDevice,
                           col->stream));
  }
  XOD_HIP(hipStreamSynchronize(col->stream));
  if (dt_last) *dt_last = dt;
  if (st) {
    st->steps = steps;
    st->rejects = rejects;
    st->clipped = clipped;
    st->visits = (int32_t)seq.size();
    st->pad_ = 0;
  }
  return XOD_OK;
}
