// Tile-shape autotuner for the block factorisations.  A measured setting is
// kept per (architecture, padded block size, precision, factorisation,
// single column or batch) and applied by TunedScope while such a column is
// factored; the candidates are settings of the existing tile options, so
// every candidate computes the same factorisation up to rounding order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "batch.h"
#include "tune.h"

namespace xod {
xod_status enqueue_solve(xod_column *c, double dt, int *iters, int *fallback, double *resid,
                         const double *hist, double hist_coef);

namespace {

std::mutex &tune_mu() {
  static std::mutex m;
  return m;
}
std::map<std::string, TuneVals> &tune_table() {
  static std::map<std::string, TuneVals> t;
  return t;
}

// The architecture name of the current device, looked up once per device
// (every tuned factorisation asks for it).
std::string arch_name() {
  static std::mutex mu;
  static std::map<int, std::string> names;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return "unknown";
  std::lock_guard<std::mutex> lk(mu);
  auto it = names.find(dev);
  if (it != names.end()) return it->second;
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
  std::string a = p.gcnArchName;
  const size_t colon = a.find(':');
  if (colon != std::string::npos) a = a.substr(0, colon);
  names[dev] = a;
  return a;
}

std::string tune_key(int ld, xod_precision prec, xod_solver solver, bool batch) {
  char buf[96];
  std::snprintf(buf, sizeof buf, "%s/ld%d/%s/%s/%s", arch_name().c_str(), ld,
                prec == XOD_MIXED ? "mixed" : "fp64",
                solver == XOD_SOLVER_CR ? "cr" : "thomas", batch ? "batch" : "column");
  return buf;
}

void apply(const TuneVals &v, Options &o) {
  o.fused_max_ld = v.fused_max_ld;
  o.outer = v.outer;
  o.update32 = v.update32;
  o.gemm_large = v.gemm_large;
  o.gemm_k = v.gemm_k;
  o.panel_sync = v.panel_sync;
  o.gemm_waves = v.gemm_waves;
}

TuneVals current(const Options &o) {
  return TuneVals{o.fused_max_ld, o.outer, o.update32, o.gemm_large, o.gemm_k, o.panel_sync,
                  o.gemm_waves};
}

// Candidates for one kind of column; the first is the process-wide setting.
std::vector<TuneVals> candidates(int ld, xod_precision prec, xod_solver solver) {
  const TuneVals base = current(global_options());
  std::vector<TuneVals> out{base};
  auto add = [&](TuneVals v) {
    for (const TuneVals &w : out)
      if (std::memcmp(&w, &v, sizeof v) == 0) return;
    out.push_back(v);
  };
  if (solver == XOD_SOLVER_CR) {
    for (int large : {1, 0})
      for (int k : {32, 16})
        for (int sync : {2, 1}) {
          TuneVals v = base;
          v.gemm_large = large;
          v.gemm_k = k;
          v.panel_sync = sync;
          add(v);
        }
    for (int sync : {2, 1}) {   // 8-wave 128-tiles (32-wide K only)
      TuneVals v = base;
      v.gemm_large = 1;
      v.gemm_k = 32;
      v.gemm_waves = 8;
      v.panel_sync = sync;
      add(v);
    }
    return out;
  }
  if (prec == XOD_FP64 && ld <= 128) {
    TuneVals v = base;
    v.fused_max_ld = ld;   // the persistent small-block kernels
    add(v);
  }
  for (int outer : {32, 64, 128})
    for (int u32 : {1, 0}) {
      TuneVals v = base;
      v.fused_max_ld = 0;
      v.outer = outer;
      v.update32 = u32;
      add(v);
    }
  return out;
}

void store(const std::string &key, const TuneVals &v) {
  std::lock_guard<std::mutex> lk(tune_mu());
  tune_table()[key] = v;
}

void fill_result(xod_tune_result *r, const std::string &key, const TuneVals &v, int ncand,
                 double best_ms, double default_ms) {
  std::memset(r, 0, sizeof *r);
  std::snprintf(r->key, sizeof r->key, "%s", key.c_str());
  r->candidates = ncand;
  r->best_ms = best_ms;
  r->default_ms = default_ms;
  r->fused_max_ld = v.fused_max_ld;
  r->outer = v.outer;
  r->update32 = v.update32;
  r->gemm_large = v.gemm_large;
  r->gemm_k = v.gemm_k;
  r->panel_sync = v.panel_sync;
  r->gemm_waves = v.gemm_waves;
}

}  // namespace

TunedScope::TunedScope(int ld, xod_precision prec, xod_solver solver, bool batch) {
  TuneVals v;
  {
    std::lock_guard<std::mutex> lk(tune_mu());
    if (tune_table().empty()) return;
    auto it = tune_table().find(tune_key(ld, prec, solver, batch));
    if (it == tune_table().end()) return;
    v = it->second;
  }
  local_ = options();
  apply(v, local_);
  prev_ = options_override();
  options_override() = &local_;
  on_ = true;
}

TunedScope::~TunedScope() {
  if (on_) options_override() = prev_;
}

}  // namespace xod

using namespace xod;

#define TCHECK(cond, msg) \
  do {                    \
    if (!(cond)) {        \
      set_error(msg);     \
      return XOD_EINVAL;  \
    }                     \
  } while (0)

extern "C" xod_status xod_autotune(xod_column *col, double dt, int32_t trials,
                                   xod_tune_result *res) {
  TCHECK(col && res, "xod_autotune: null argument");
  TCHECK(!col->in_batch, "xod_autotune: column belongs to a batch");
  TCHECK(std::isfinite(dt) && dt > 0, "xod_autotune: dt must be > 0");
  TCHECK(trials >= 1 && trials <= 100, "xod_autotune: trials must be in 1..100");
  const std::string key = tune_key(col->ld, col->prec, col->solver, false);
  const std::vector<TuneVals> cand = candidates(col->ld, col->prec, col->solver);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  XOD_HIP(hipEventCreate(&e0));
  XOD_HIP(hipEventCreate(&e1));
  double best = 1e300, def = 0.0;
  TuneVals bestv = cand[0];
  xod_status st = XOD_OK;
  const double fb_dt0 = col->mixed_fb_dt;   // the column's precision history, kept
  const int direct0 = col->mixed_direct;
  for (size_t ci = 0; ci < cand.size() && st == XOD_OK; ++ci) {
    store(key, cand[ci]);
    int it, fb;
    double rr;
    col->mixed_fb_dt = 0.0;   // every candidate starts from FP32 (mixed columns)
    col->mixed_direct = 0;
    st = enqueue_solve(col, dt, &it, &fb, &rr, nullptr, 0.0);   // untimed first use
    if (st != XOD_OK) break;
    if (hipEventRecord(e0, col->stream) != hipSuccess) { st = XOD_EHIP; break; }
    for (int t = 0; t < trials && st == XOD_OK; ++t)
      st = enqueue_solve(col, dt, &it, &fb, &rr, nullptr, 0.0);
    if (st != XOD_OK) break;
    float ms = 0.f;
    if (hipEventRecord(e1, col->stream) != hipSuccess ||
        hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      st = XOD_EHIP;
      break;
    }
    const double avg = ms / trials;
    if (ci == 0) def = avg;
    if (avg < best) {
      best = avg;
      bestv = cand[ci];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  col->mixed_fb_dt = fb_dt0;
  col->mixed_direct = direct0;
  store(key, bestv);
  col->fact_dt = 0.0;   // the tuning steps' factors are not the caller's
  col->btd.valid = false;
  if (st != XOD_OK) return st;
  fill_result(res, key, bestv, (int)cand.size(), best, def);
  return XOD_OK;
}

extern "C" xod_status xod_batch_autotune(xod_batch *b, const double *dts, int32_t trials,
                                         xod_tune_result *res, int32_t max_results,
                                         int32_t *nresults) {
  TCHECK(b && dts && res && nresults && max_results >= 1, "xod_batch_autotune: null argument");
  TCHECK(trials >= 1 && trials <= 20, "xod_batch_autotune: trials must be in 1..20");
  for (size_t i = 0; i < b->cols.size(); ++i)
    TCHECK(std::isfinite(dts[i]) && dts[i] > 0, "xod_batch_autotune: dt must be > 0");
  // the groups of the batch: distinct (ld, precision)
  std::vector<std::pair<int, int>> groups;
  for (xod_column *c : b->cols) {
    const std::pair<int, int> g{c->ld, (int)c->prec};
    bool seen = false;
    for (auto &h : groups) seen = seen || h == g;
    if (!seen) groups.push_back(g);
  }
  TCHECK((int)groups.size() <= max_results, "xod_batch_autotune: too few result slots");
  BatchRunner &r = b->runner;
  r.time_groups = true;
  std::vector<double> stats;
  xod_status st = XOD_OK;
  int nres = 0;
  for (auto &g : groups) {
    const xod_precision prec = (xod_precision)g.second;
    const std::string key = tune_key(g.first, prec, XOD_SOLVER_THOMAS, true);
    const std::vector<TuneVals> cand = candidates(g.first, prec, XOD_SOLVER_THOMAS);
    double best = 1e300, def = 0.0;
    TuneVals bestv = cand[0];
    for (size_t ci = 0; ci < cand.size() && st == XOD_OK; ++ci) {
      store(key, cand[ci]);
      st = r.step(b->cols, dts, false, 1e-30, 1e-10, 0.0, b->stream, stats);   // untimed
      double sum = 0.0;
      for (int t = 0; t < trials && st == XOD_OK; ++t) {
        st = r.step(b->cols, dts, false, 1e-30, 1e-10, 0.0, b->stream, stats);
        for (auto &gm : r.last_group_ms)
          if (gm.first == g) sum += gm.second;
      }
      const double avg = sum / trials;
      if (ci == 0) def = avg;
      if (avg < best) {
        best = avg;
        bestv = cand[ci];
      }
    }
    store(key, bestv);
    if (st != XOD_OK) break;
    fill_result(&res[nres++], key, bestv, (int)cand.size(), best, def);
  }
  r.time_groups = false;
  *nresults = nres;
  return st;
}

extern "C" xod_status xod_autotune_clear(void) {
  std::lock_guard<std::mutex> lk(tune_mu());
  tune_table().clear();
  return XOD_OK;
}
