// Batched backward-Euler steps: columns with the same padded block size share
// every launch (grid dimension over columns); their layer chains advance in
// lock step and shorter columns idle once their chain ends.  Each column
// keeps its own dt, state and statistics.  In FP64 the arithmetic of a column
// does not depend on which other columns share the launch.  Mixed-precision
// columns are refined together: the group iterates until its largest
// correction ratio meets the stopping rule of a single column, so a column
// may receive more refinements than it would alone (each one only brings it
// closer to the FP64 solution); a group that stalls is refactored in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "batch.h"
#include "tune.h"

using namespace xod;

namespace xod {

BatchRunner::~BatchRunner() {
  (void)hipFree(d_args);
  (void)hipFree(d_upd);
  (void)hipFree(d_red);
  (void)hipFree(d_stats);
  (void)hipFree(d_partial);
  for (hipEvent_t e : gevent) (void)hipEventDestroy(e);
  for (hipEvent_t e : tev) (void)hipEventDestroy(e);
  for (hipStream_t st : gstream) (void)hipStreamDestroy(st);
  if (fork_ev) (void)hipEventDestroy(fork_ev);
  (void)hipFree(d_ratio);
  (void)hipFree(d_rmax);
  (void)hipHostFree(h_rmax);
  (void)hipHostFree(h_args);
  (void)hipHostFree(h_upd);
  (void)hipHostFree(h_red);
  (void)hipHostFree(h_stats);
}

xod_status BatchRunner::init(int capacity) {
  cap = capacity;
  const size_t n = (size_t)cap;
  XOD_HIP(hipMalloc((void **)&d_args, n * sizeof(ColArgs)));
  XOD_HIP(hipMalloc((void **)&d_upd, n * sizeof(UpdArgs)));
  XOD_HIP(hipMalloc((void **)&d_red, n * sizeof(RedArgs)));
  XOD_HIP(hipMalloc((void **)&d_stats, n * kStatLen * sizeof(double)));
  XOD_HIP(hipMalloc((void **)&d_partial, n * kUpdBlocks * kNStat * sizeof(double)));
  XOD_HIP(hipHostMalloc((void **)&h_args, n * sizeof(ColArgs), hipHostMallocDefault));
  XOD_HIP(hipHostMalloc((void **)&h_upd, n * sizeof(UpdArgs), hipHostMallocDefault));
  XOD_HIP(hipHostMalloc((void **)&h_red, n * sizeof(RedArgs), hipHostMallocDefault));
  XOD_HIP(hipHostMalloc((void **)&h_stats, n * kStatLen * sizeof(double), hipHostMallocDefault));
  XOD_HIP(hipMalloc((void **)&d_rmax, kMaxGroups * sizeof(double)));
  XOD_HIP(hipHostMalloc((void **)&h_rmax, kMaxGroups * sizeof(double), hipHostMallocDefault));
  XOD_HIP(hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming));
  return XOD_OK;
}

// One FP64 BE step of every column (delta solved, n_new written to ntmp,
// statistics into stats[i*kStatLen..]).  States are not committed here.
xod_status BatchRunner::step(const std::vector<xod_column *> &cols, const double *dts,
                             bool clip, double y_floor, double y_sig, double y_neg,
                             hipStream_t s,
                             std::vector<double> &stats) {
  const int n = (int)cols.size();
  if (n > cap) {
    set_error("batch step: more columns than the runner's capacity");
    return XOD_EINVAL;
  }
  stats.assign((size_t)n * kStatLen, 0.0);
  last_iters.assign(n, 0);
  last_fallback.assign(n, 0);
  last_resid.assign(n, 0.0);
  // Group by padded block size and precision (caller's order inside a
  // group).  Groups are independent: each runs on its own stream, forked
  // from s and joined back before the statistics are read.
  std::map<std::pair<int, int>, std::vector<int>> groups;
  for (int i = 0; i < n; ++i) groups[{cols[i]->ld, (int)cols[i]->prec}].push_back(i);
  struct Group {
    int ld, base, nc, maxN = 0, maxR = 0, maxS = 0;
    bool mixed;
    const std::vector<int> *idx;
    hipStream_t st;
    size_t roff;
    int iters = 0, fallback = 0;
    double ratio = 0.0;
  };
  std::vector<Group> gs;
  int base = 0;
  size_t rneed = 0;
  std::vector<std::pair<int, int>> slots;   // (caller index, staging slot)
  for (auto &kv : groups) {
    Group g{};
    g.ld = kv.first.first;
    g.idx = &kv.second;
    g.base = base;
    g.nc = (int)kv.second.size();
    g.mixed = kv.first.second == (int)XOD_MIXED;
    for (int j = 0; j < g.nc; ++j) {
      xod_column *c = cols[kv.second[j]];
      const int sl = base + j;
      c->dt = dts[kv.second[j]];
      h_args[sl] = c->args();
      if (c->prec == XOD_FP64) h_args[sl].rs = nullptr;   // FP64 refinement: unscaled
      UpdArgs u{};
      u.n = c->n;
      u.x = c->x;
      u.ngas = c->ngas;
      u.nout = c->ntmp;
      u.partial = d_partial + (size_t)sl * kUpdBlocks * kNStat;
      u.N = c->N;
      u.S = c->S;
      u.clip = clip ? 1 : 0;
      u.y_floor = y_floor;
      u.y_sig = y_sig;
      u.y_neg = y_neg;
      h_upd[sl] = u;
      h_red[sl] = RedArgs{u.partial, c->flag, d_stats + (size_t)sl * kStatLen};
      g.maxN = std::max(g.maxN, c->N);
      g.maxR = std::max(g.maxR, c->R);
      g.maxS = std::max(g.maxS, c->S);
      slots.push_back({kv.second[j], sl});
    }
    g.roff = rneed;
    rneed += (size_t)g.nc * g.maxN;
    base += g.nc;
    gs.push_back(g);
  }
  if ((int)gs.size() > kMaxGroups) {
    set_error("batch step: too many distinct block sizes");
    return XOD_EINVAL;
  }
  if (rneed > ratio_cap) {
    (void)hipFree(d_ratio);
    d_ratio = nullptr;
    XOD_HIP(hipMalloc((void **)&d_ratio, rneed * sizeof(double)));
    ratio_cap = rneed;
  }
  while (gstream.size() < gs.size()) {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    XOD_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    XOD_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    gstream.push_back(st);
    gevent.push_back(ev);
  }
  if (time_groups) {
    while (tev.size() < 2 * gs.size()) {
      hipEvent_t ev = nullptr;
      XOD_HIP(hipEventCreate(&ev));
      tev.push_back(ev);
    }
  }
  XOD_HIP(hipEventRecord(fork_ev, s));
  // phase 1: factor and first solve of every group
  for (size_t gi = 0; gi < gs.size(); ++gi) {
    Group &g = gs[gi];
    g.st = gstream[gi];
    const hipStream_t st = g.st;
    XOD_HIP(hipStreamWaitEvent(st, fork_ev, 0));
    if (time_groups) XOD_HIP(hipEventRecord(tev[2 * gi], st));
    const TunedScope tuned(g.ld, g.mixed ? XOD_MIXED : XOD_FP64, XOD_SOLVER_THOMAS, true);
    XOD_HIP(hipMemcpyAsync(d_args + g.base, h_args + g.base, g.nc * sizeof(ColArgs),
                           hipMemcpyHostToDevice, st));
    XOD_HIP(hipMemcpyAsync(d_upd + g.base, h_upd + g.base, g.nc * sizeof(UpdArgs),
                           hipMemcpyHostToDevice, st));
    XOD_HIP(hipMemcpyAsync(d_red + g.base, h_red + g.base, g.nc * sizeof(RedArgs),
                           hipMemcpyHostToDevice, st));
    const ManyCols acc{d_args + g.base};
    XOD_HIP(launch_rates(acc, g.nc, g.maxN, g.maxR, st));
    XOD_HIP(launch_rhs(acc, g.nc, g.maxN, g.maxR, g.maxS, st));
    if (g.mixed) {
      XOD_HIP(launch_jacobian(acc, g.nc, g.maxN, g.maxR, g.ld, true, st));
      XOD_HIP(launch_factor_mixed(acc, g.nc, g.maxN, g.ld, st));
      XOD_HIP(launch_scale(acc, g.nc, g.maxN, g.maxS, st));
      XOD_HIP(launch_solve_mixed(acc, g.nc, g.maxN, g.ld, st));
      for (int j = 0; j < g.nc; ++j) {
        xod_column *c = cols[(*g.idx)[j]];
        XOD_HIP(hipMemcpyAsync(c->dx, c->x, (size_t)c->N * c->S * sizeof(double),
                               hipMemcpyDeviceToDevice, st));
      }
    } else {
      XOD_HIP(launch_jacobian(acc, g.nc, g.maxN, g.maxR, g.ld, false, st));
      XOD_HIP(launch_factor_fp64(acc, g.nc, g.maxN, g.ld, st));
      for (int j = 0; j < g.nc; ++j) {
        xod_column *c = cols[(*g.idx)[j]];
        XOD_HIP(hipMemcpyAsync(c->x, c->f, (size_t)c->N * c->S * sizeof(double),
                               hipMemcpyDeviceToDevice, st));
      }
      XOD_HIP(launch_solve_fp64(acc, g.nc, g.maxN, g.ld, st));
      if (options().refine64 > 0) {
        // the fixed FP64 refinement of a single column's step (the FP64
        // columns' argument copies carry no row scales)
        for (int j = 0; j < g.nc; ++j) {
          xod_column *c = cols[(*g.idx)[j]];
          const size_t bytes = (size_t)c->N * c->S * sizeof(double);
          XOD_HIP(hipMemcpyAsync(c->dx, c->x, bytes, hipMemcpyDeviceToDevice, st));
          XOD_HIP(hipMemcpyAsync(c->resid, c->x, bytes, hipMemcpyDeviceToDevice, st));
        }
        for (int it = 1; it <= options().refine64; ++it) {
          XOD_HIP(launch_residual(acc, g.nc, g.maxN, g.maxS, g.maxR, st));
          XOD_HIP(launch_solve_fp64(acc, g.nc, g.maxN, g.ld, st));
          XOD_HIP(launch_axpy_ratio(acc, g.nc, g.maxN, d_ratio + g.roff, d_rmax + gi, st));
          g.iters = it;
        }
        XOD_HIP(launch_keep_refined(acc, g.nc, g.maxN, g.maxS, d_ratio + g.roff, 1e5, st));
      }
    }
  }
  // phase 2: refinement of mixed groups (each waits on its own stream only)
  for (size_t gi = 0; gi < gs.size(); ++gi) {
    Group &g = gs[gi];
    if (!g.mixed) continue;
    const hipStream_t st = g.st;
    const TunedScope tuned(g.ld, XOD_MIXED, XOD_SOLVER_THOMAS, true);
    const ManyCols acc{d_args + g.base};
    double *ratio = d_ratio + g.roff;
    RefineNext verdict = kRefineFallback;
    double prev = 1e300;
    g.ratio = 1e300;
    for (int it = 1; it <= 10; ++it) {
      XOD_HIP(launch_residual(acc, g.nc, g.maxN, g.maxS, g.maxR, st));
      XOD_HIP(launch_solve_mixed(acc, g.nc, g.maxN, g.ld, st));
      XOD_HIP(launch_axpy_ratio(acc, g.nc, g.maxN, ratio, d_rmax + gi, st));
      XOD_HIP(hipMemcpyAsync(h_rmax + gi, d_rmax + gi, sizeof(double), hipMemcpyDeviceToHost,
                             st));
      XOD_HIP(hipStreamSynchronize(st));
      g.ratio = h_rmax[gi];
      g.iters = it;
      verdict = refine_next(g.ratio, prev, it, 10);
      if (verdict != kRefineMore) break;
      prev = g.ratio;
    }
    const bool ok = verdict == kRefineDone;
    if (ok) {
      for (int j = 0; j < g.nc; ++j) {
        xod_column *c = cols[(*g.idx)[j]];
        XOD_HIP(hipMemcpyAsync(c->x, c->dx, (size_t)c->N * c->S * sizeof(double),
                               hipMemcpyDeviceToDevice, st));
      }
    } else {
      g.fallback = 1;
      XOD_HIP(launch_jacobian(acc, g.nc, g.maxN, g.maxR, g.ld, false, st));
      XOD_HIP(launch_factor_fp64(acc, g.nc, g.maxN, g.ld, st));
      for (int j = 0; j < g.nc; ++j) {
        xod_column *c = cols[(*g.idx)[j]];
        XOD_HIP(hipMemcpyAsync(c->x, c->f, (size_t)c->N * c->S * sizeof(double),
                               hipMemcpyDeviceToDevice, st));
      }
      XOD_HIP(launch_solve_fp64(acc, g.nc, g.maxN, g.ld, st));
    }
  }
  // phase 3: state update and statistics, then join
  for (size_t gi = 0; gi < gs.size(); ++gi) {
    Group &g = gs[gi];
    XOD_HIP(launch_update_state(d_upd + g.base, d_red + g.base, g.nc, g.st));
    if (time_groups) XOD_HIP(hipEventRecord(tev[2 * gi + 1], g.st));
    XOD_HIP(hipEventRecord(gevent[gi], g.st));
    XOD_HIP(hipStreamWaitEvent(s, gevent[gi], 0));
    for (int j = 0; j < g.nc; ++j) {
      const int ci = (*g.idx)[j];
      last_iters[ci] = g.iters;
      last_fallback[ci] = g.fallback;
      last_resid[ci] = g.mixed ? g.ratio : 0.0;
    }
  }
  XOD_HIP(hipMemcpyAsync(h_stats, d_stats, (size_t)n * kStatLen * sizeof(double),
                         hipMemcpyDeviceToHost, s));
  XOD_HIP(hipStreamSynchronize(s));
  last_group_ms.clear();
  if (time_groups)
    for (size_t gi = 0; gi < gs.size(); ++gi) {
      float ms = 0.f;
      XOD_HIP(hipEventElapsedTime(&ms, tev[2 * gi], tev[2 * gi + 1]));
      last_group_ms.push_back({{gs[gi].ld, gs[gi].mixed ? (int)XOD_MIXED : (int)XOD_FP64}, ms});
    }
  for (auto &pr : slots)
    std::memcpy(&stats[(size_t)pr.first * kStatLen], h_stats + (size_t)pr.second * kStatLen,
                kStatLen * sizeof(double));
  return XOD_OK;
}

}  // namespace xod

xod_batch::~xod_batch() {
  for (auto *c : cols) c->in_batch = false;
}

#define BCHECK(cond, msg)  \
  do {                     \
    if (!(cond)) {         \
      set_error(msg);      \
      return XOD_EINVAL;   \
    }                      \
  } while (0)

extern "C" xod_status xod_batch_create(xod_column *const *cols, int32_t ncols, xod_batch **out) {
  BCHECK(cols && out && ncols >= 1, "xod_batch_create: bad arguments");
  *out = nullptr;
  for (int i = 0; i < ncols; ++i) {
    BCHECK(cols[i] != nullptr, "xod_batch_create: null column");
    BCHECK(!cols[i]->in_batch, "xod_batch_create: column already in a batch");
    BCHECK(cols[i]->prec == cols[0]->prec, "xod_batch_create: columns of one precision");
    BCHECK(cols[i]->ph_L == 0, "xod_batch_create: spectral photolysis is not supported in batches");
    for (int j = 0; j < i; ++j) BCHECK(cols[j] != cols[i], "xod_batch_create: duplicate column");
  }
  std::unique_ptr<xod_batch> b(new xod_batch());
  b->cols.assign(cols, cols + ncols);
  b->stream = cols[0]->stream;
  XOD_TRY_B(b->runner.init(ncols));
  // batch steps overwrite each column's blocks and pivots with block-Thomas
  // factors of the batch's dt: no factorisation stays usable by
  // xod_step_frozen, during the batch or after it
  for (auto *c : b->cols) {
    c->in_batch = true;
    c->fact_dt = 0.0;
    c->btd.valid = false;
  }
  *out = b.release();
  return XOD_OK;
}

extern "C" xod_status xod_batch_destroy(xod_batch *b) {
  BCHECK(b, "xod_batch_destroy: null batch");
  (void)hipStreamSynchronize(b->stream);
  delete b;
  return XOD_OK;
}

extern "C" xod_status xod_batch_step(xod_batch *b, const double *dts, xod_step_stats *st) {
  BCHECK(b && dts, "xod_batch_step: null argument");
  for (size_t i = 0; i < b->cols.size(); ++i)
    BCHECK(std::isfinite(dts[i]) && dts[i] > 0, "xod_batch_step: dt must be > 0");
  std::vector<double> stats;
  XOD_TRY_B(b->runner.step(b->cols, dts, false, 1e-30, 1e-10, 0.0, b->stream, stats));
  xod_status ret = XOD_OK;
  for (size_t i = 0; i < b->cols.size(); ++i) {
    xod_column *c = b->cols[i];
    const double *sv = &stats[i * kStatLen];
    if (st) {
      st[i].max_rel_change = sv[0];
      st[i].min_ratio = sv[1];
      st[i].resid_inf = b->runner.last_resid[i];
      st[i].refine_iters = b->runner.last_iters[i];
      st[i].fp64_fallback = b->runner.last_fallback[i];
      st[i].nonfinite = sv[5] > 0 ? 1 : 0;
    }
    if (sv[kNStat] >= 0) {
      set_error("batch column " + std::to_string(i) + ": singular Schur complement at layer " +
                std::to_string((long)sv[kNStat]));
      ret = XOD_ESINGULAR;
      continue;
    }
    if (sv[5] > 0) {
      set_error("batch column " + std::to_string(i) + ": non-finite state");
      if (ret == XOD_OK) ret = XOD_ENONFINITE;
      continue;
    }
    std::swap(c->n, c->ntmp);
    c->t += c->dt;
    c->prev_dt = 0.0;
  }
  return ret;
}
