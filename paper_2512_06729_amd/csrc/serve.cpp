// Continuous-batching request loop for steady-state solves.
//
// Requests (network + profile + initial state + steady-state options) are
// queued on submit.  Each call of xod_serve_step():
//   1. admits queued requests in arrival order while a slot is free and the
//      request's device footprint fits in the HBM budget (state and
//      workspace stay resident on the device until the request retires);
//   2. advances every resident request by one adaptive backward-Euler step
//      with its own dt.  With the cyclic-reduction solver (default) every
//      slot has its own HIP stream and each resident request's step is
//      driven by its own host thread, so the requests' kernels overlap on
//      the device (mixed-precision refinement waits only on its own
//      stream).  With block Thomas, FP64 requests share batched launches on
//      the server stream and mixed ones run one after another;
//   3. applies each request's step control and retires converged or failed
//      requests: the final state is copied to the host, the slot and its
//      memory are freed, and the latency (completion - submission) recorded.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <future>
#include <string>
#include <utility>
#include <map>
#include <memory>
#include <vector>

#include "batch.h"

using namespace xod;

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Req {
  uint64_t id = 0;
  const xod_network *net = nullptr;
  int slot = -1;
  std::vector<double> P, T, K, D, alpha, n0;
  bool hasD = false, hasA = false;
  double mbar = 2.3, g = 2000.0, sigma = 1e-22;
  int N = 0;
  // options
  double tol = 1e-4, yfl = 1e-30, ysig = 1e-10, tend = 1e12, dt0 = 1e-8, yneg = 1e-6;
  int maxs = 5000, maxrej = 30, mixrule = 1;
  // controller state
  double t = 0.0, dt = 0.0, clipped = 0.0, mix = 0.0;
  int64_t steps = 0, rejects = 0;
  int consec = 0;
  int state = 0;   // 0 queued, 1 running, 2 done, 3 failed
  xod_status status = XOD_OK;
  size_t footprint = 0;
  xod_column *col = nullptr;
  double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;
  std::vector<double> n_out;
};

}  // namespace

struct xod_server {
  size_t budget = 0, used = 0;
  int max_slots = 1;
  xod_precision prec = XOD_FP64;
  hipStream_t stream = nullptr;
  uint64_t next_id = 1;
  std::deque<uint64_t> queue;
  std::map<uint64_t, Req> reqs;
  std::vector<uint64_t> active;
  BatchRunner runner;
  int64_t iterations = 0;
  xod_solver solver = XOD_SOLVER_CR;
  std::vector<hipStream_t> slot_stream;   // one per slot (cyclic reduction)
  std::vector<char> slot_busy;
  size_t footprint(const xod_network *net, int N) const {
    return column_footprint(net, N, prec) +
           (solver == XOD_SOLVER_CR ? cr_footprint(net, N, prec) : 0);
  }
  ~xod_server() {
    for (auto &kv : reqs)
      if (kv.second.col) xod_column_destroy(kv.second.col);
    for (hipStream_t st : slot_stream) (void)hipStreamDestroy(st);
  }
};

#define SCHECK(cond, msg)  \
  do {                     \
    if (!(cond)) {         \
      set_error(msg);      \
      return XOD_EINVAL;   \
    }                      \
  } while (0)

extern "C" xod_status xod_serve_create(size_t hbm_budget_bytes, int32_t max_slots,
                                       xod_precision prec, void *stream, xod_server **out) {
  SCHECK(out && max_slots >= 1 && hbm_budget_bytes > 0, "xod_serve_create: bad arguments");
  SCHECK(prec == XOD_FP64 || prec == XOD_MIXED, "xod_serve_create: bad precision");
  std::unique_ptr<xod_server> s(new xod_server());
  s->budget = hbm_budget_bytes;
  s->max_slots = max_slots;
  s->prec = prec;
  s->stream = (hipStream_t)stream;
  XOD_TRY_B(s->runner.init(max_slots));
  s->slot_busy.assign(max_slots, 0);
  for (int i = 0; i < max_slots; ++i) {
    hipStream_t st = nullptr;
    XOD_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    s->slot_stream.push_back(st);
  }
  *out = s.release();
  return XOD_OK;
}

extern "C" xod_status xod_serve_set_solver(xod_server *s, xod_solver solver) {
  SCHECK(s, "xod_serve_set_solver: null server");
  SCHECK(solver == XOD_SOLVER_THOMAS || solver == XOD_SOLVER_CR,
         "xod_serve_set_solver: unknown solver");
  SCHECK(s->reqs.empty(), "xod_serve_set_solver: requests already submitted");
  s->solver = solver;
  return XOD_OK;
}

extern "C" xod_status xod_serve_destroy(xod_server *s) {
  SCHECK(s, "xod_serve_destroy: null server");
  (void)hipStreamSynchronize(s->stream);
  delete s;
  return XOD_OK;
}

extern "C" xod_status xod_serve_footprint(const xod_network *net, int32_t N, xod_precision prec,
                                          size_t *bytes) {
  SCHECK(net && bytes && N >= 1, "xod_serve_footprint: bad arguments");
  *bytes = column_footprint(net, N, prec) + cr_footprint(net, N, prec);
  return XOD_OK;
}

extern "C" xod_status xod_serve_submit(xod_server *s, const xod_network *net,
                                       const xod_profile *p, const double *n0,
                                       const xod_ss_opts *o, uint64_t *req_id) {
  SCHECK(s && net && p && n0 && req_id, "xod_serve_submit: null argument");
  SCHECK(p->N >= 1, "xod_serve_submit: N must be >= 1");
  SCHECK(!o || o->method == 0, "xod_serve_submit: requests are stepped with backward Euler "
                               "(method 0)");
  Req r;
  r.id = s->next_id++;
  r.net = net;
  r.N = p->N;
  const int N = p->N, S = net->S;
  r.P.assign(p->P_bar, p->P_bar + N);
  r.T.assign(p->T_K, p->T_K + N);
  r.K.assign(p->Kzz, p->Kzz + N);
  if (p->Dmol) {
    r.hasD = true;
    r.D.assign(p->Dmol, p->Dmol + (size_t)N * S);
  }
  if (p->alphaT) {
    r.hasA = true;
    r.alpha.assign(p->alphaT, p->alphaT + S);
  }
  r.n0.assign(n0, n0 + (size_t)N * S);
  r.mbar = p->mbar_amu;
  r.g = p->g_cgs;
  r.sigma = p->sigma_tau;
  if (o) {
    if (o->tol_rel > 0) r.tol = o->tol_rel;
    if (o->y_floor > 0) r.yfl = o->y_floor;
    if (o->y_sig > 0) r.ysig = o->y_sig;
    if (o->y_neg > 0) r.yneg = o->y_neg;
    if (o->t_end > 0) r.tend = o->t_end;
    if (o->dt0 > 0) r.dt0 = o->dt0;
    if (o->max_steps > 0) r.maxs = o->max_steps;
    if (o->max_consec_rejects > 0) r.maxrej = o->max_consec_rejects;
    r.mixrule = o->use_mix_rule;
  }
  r.footprint = s->footprint(net, N);
  if (r.footprint > s->budget) {
    set_error("xod_serve_submit: request footprint exceeds the whole HBM budget");
    return XOD_EINVAL;
  }
  r.t_submit = now_s();
  *req_id = r.id;
  s->queue.push_back(r.id);
  s->reqs.emplace(r.id, std::move(r));
  return XOD_OK;
}

static void finish(xod_server *s, Req &r, int state, xod_status st) {
  r.state = state;
  r.status = st;
  r.t_done = now_s();
  r.n_out.assign((size_t)r.N * r.net->S, 0.0);
  if (r.col) {
    (void)xod_column_get_state(r.col, r.n_out.data(), nullptr, nullptr);
    xod_column_destroy(r.col);
    r.col = nullptr;
  }
  if (r.slot >= 0) s->slot_busy[r.slot] = 0;
  r.slot = -1;
  s->used -= r.footprint;
}

extern "C" xod_status xod_serve_step(xod_server *s, int32_t *n_active, int32_t *n_queued) {
  SCHECK(s, "xod_serve_step: null server");
  // 1. admission by slot and HBM footprint, in arrival order
  while (!s->queue.empty() && (int)s->active.size() < s->max_slots) {
    Req &r = s->reqs.at(s->queue.front());
    if (s->used + r.footprint > s->budget) break;
    xod_profile p{};
    p.N = r.N;
    p.P_bar = r.P.data();
    p.T_K = r.T.data();
    p.Kzz = r.K.data();
    p.Dmol = r.hasD ? r.D.data() : nullptr;
    p.alphaT = r.hasA ? r.alpha.data() : nullptr;
    p.mbar_amu = r.mbar;
    p.g_cgs = r.g;
    p.sigma_tau = r.sigma;
    s->queue.pop_front();
    int slot = 0;
    while (s->slot_busy[slot]) ++slot;   // a slot is free: active < max_slots
    const bool cr = s->solver == XOD_SOLVER_CR;
    xod_status st = xod_column_create(r.net, &p, r.n0.data(), s->prec,
                                      cr ? s->slot_stream[slot] : s->stream, &r.col);
    if (st == XOD_OK && cr) st = xod_column_set_solver(r.col, XOD_SOLVER_CR);
    if (st != XOD_OK) {
      if (r.col) xod_column_destroy(r.col);
      r.col = nullptr;
      r.state = 3;
      r.status = st;
      r.t_done = now_s();
      continue;
    }
    s->slot_busy[slot] = 1;
    r.slot = slot;
    s->used += r.footprint;
    double mix = 0.0;
    (void)xod_column_grid(r.col, nullptr, nullptr, nullptr, &mix);
    r.mix = r.mixrule ? mix : 0.0;
    r.dt = r.dt0;
    r.state = 1;
    r.t_admit = now_s();
    s->active.push_back(r.id);
  }
  // 2. one adaptive step of every resident request
  const size_t na = s->active.size();
  std::vector<double> stats;
  if (na > 0) {
    std::vector<xod_column *> cols(na);
    std::vector<double> dts(na);
    for (size_t i = 0; i < na; ++i) {
      Req &r = s->reqs.at(s->active[i]);
      cols[i] = r.col;
      dts[i] = r.dt;
    }
    if (s->prec == XOD_FP64 && s->solver == XOD_SOLVER_THOMAS) {
      // driver semantics: clipping, control statistics; one launch serves
      // every active request, so the y thresholds are the first request's
      const Req &r0 = s->reqs.at(s->active[0]);
      XOD_TRY_B(s->runner.step(cols, dts.data(), true, r0.yfl, r0.ysig, r0.yneg, s->stream,
                               stats));
    } else if (s->solver == XOD_SOLVER_CR) {
      // every request on its own stream, driven by its own host thread (the
      // mixed-precision refinement waits on its stream between iterations),
      // so the requests' kernels overlap on the device
      stats.assign(na * kStatLen, 0.0);
      std::vector<std::future<std::pair<xod_status, std::string>>> tasks;
      for (size_t i = 0; i < na; ++i) {
        Req *r = &s->reqs.at(s->active[i]);
        double *out = &stats[i * kStatLen];
        tasks.push_back(std::async(std::launch::async, [r, out]() {
          int it, fb;
          double res;
          xod_status st = enqueue_solve(r->col, r->dt, &it, &fb, &res);
          if (st == XOD_OK) st = run_update(r->col, true, r->yfl, r->ysig, out, r->yneg);
          return std::make_pair(st, st == XOD_OK ? std::string() : last_error());
        }));
      }
      xod_status first = XOD_OK;
      std::string msg;
      for (auto &t : tasks) {
        auto res = t.get();
        if (res.first != XOD_OK && first == XOD_OK) {
          first = res.first;
          msg = res.second;
        }
      }
      if (first != XOD_OK) {
        set_error(msg);
        return first;
      }
    } else {
      stats.assign(na * kStatLen, 0.0);
      for (size_t i = 0; i < na; ++i) {
        Req &r = s->reqs.at(s->active[i]);
        int it, fb;
        double res;
        XOD_TRY_B(enqueue_solve(r.col, r.dt, &it, &fb, &res));
        XOD_TRY_B(run_update(r.col, true, r.yfl, r.ysig, &stats[i * kStatLen], r.yneg));
      }
    }
  }
  // 3. per-request control, retirement
  std::vector<uint64_t> still;
  for (size_t i = 0; i < na; ++i) {
    Req &r = s->reqs.at(s->active[i]);
    const double *sv = &stats[i * kStatLen];
    const bool singular = sv[kNStat] >= 0;
    if (singular || sv[5] > 0 || sv[4] > 0) {
      ++r.rejects;
      ++r.consec;
      r.dt *= 0.5;
      if (r.consec > r.maxrej) {
        finish(s, r, 3, XOD_ENOTCONVERGED);
        continue;
      }
      still.push_back(r.id);
      continue;
    }
    r.consec = 0;
    r.clipped += sv[3];
    std::swap(r.col->n, r.col->ntmp);
    r.t += r.dt;
    ++r.steps;
    if ((sv[0] < r.tol && r.dt >= r.mix) || r.t >= r.tend) {
      finish(s, r, 2, XOD_OK);
      continue;
    }
    if (r.steps >= r.maxs) {
      finish(s, r, 3, XOD_ENOTCONVERGED);
      continue;
    }
    r.dt *= sv[2] < 0.5 ? 2.0 : (sv[2] < 0.9 ? 1.2 : 0.7);
    still.push_back(r.id);
  }
  s->active.swap(still);
  ++s->iterations;
  if (n_active) *n_active = (int32_t)s->active.size();
  if (n_queued) *n_queued = (int32_t)s->queue.size();
  return XOD_OK;
}

extern "C" xod_status xod_serve_poll(xod_server *s, uint64_t id, int32_t *state, double *n_out,
                                     xod_ss_result *res, double *latency_s) {
  SCHECK(s && state, "xod_serve_poll: null argument");
  auto it = s->reqs.find(id);
  SCHECK(it != s->reqs.end(), "xod_serve_poll: unknown request id");
  Req &r = it->second;
  *state = r.state;
  if (res) {
    res->t = r.t;
    res->dt = r.dt;
    res->clipped = r.clipped;
    res->steps = r.steps;
    res->rejects = r.rejects;
    res->converged = r.state == 2;
  }
  if (latency_s) *latency_s = r.state >= 2 ? r.t_done - r.t_submit : -1.0;
  if (n_out && r.state >= 2 && !r.n_out.empty())
    std::memcpy(n_out, r.n_out.data(), r.n_out.size() * sizeof(double));
  return r.state == 3 ? r.status : XOD_OK;
}

extern "C" xod_status xod_serve_release(xod_server *s, uint64_t id) {
  SCHECK(s, "xod_serve_release: null server");
  auto it = s->reqs.find(id);
  SCHECK(it != s->reqs.end() && it->second.state >= 2, "xod_serve_release: not finished");
  s->reqs.erase(it);
  return XOD_OK;
}

extern "C" xod_status xod_serve_usage(const xod_server *s, size_t *used_bytes, int32_t *active,
                                      int32_t *queued, int64_t *iterations) {
  SCHECK(s, "xod_serve_usage: null server");
  if (used_bytes) *used_bytes = s->used;
  if (active) *active = (int32_t)s->active.size();
  if (queued) *queued = (int32_t)s->queue.size();
  if (iterations) *iterations = s->iterations;
  return XOD_OK;
}
