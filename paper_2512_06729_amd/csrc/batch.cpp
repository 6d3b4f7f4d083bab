// Batched backward-Euler steps: columns with the same padded block size share
// every launch (grid dimension over columns); their layer chains advance in
// lock step and shorter columns idle once their chain ends.  Each column
// keeps its own dt, state and statistics; the arithmetic of a column does not
// depend on which other columns share the launch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "handles.h"

using namespace xod;

struct BatchGroup {
  int ld = 0, maxN = 0, maxR = 0, maxS = 0;
  std::vector<xod_column *> cols;
  ColArgs *d_args = nullptr;
  ColArgs *h_args = nullptr;   // pinned staging
  UpdArgs *d_upd = nullptr;
  UpdArgs *h_upd = nullptr;
  RedArgs *d_red = nullptr;
  RedArgs *h_red = nullptr;
  double *d_stats = nullptr;   // [ncols * kStatLen]
  double *h_stats = nullptr;
  double *d_partial = nullptr; // [ncols * kUpdBlocks * kNStat]
};

struct xod_batch {
  std::vector<xod_column *> cols;
  std::vector<BatchGroup> groups;
  hipStream_t stream = nullptr;
  ~xod_batch() {
    for (auto &g : groups) {
      (void)hipFree(g.d_args);
      (void)hipFree(g.d_upd);
      (void)hipFree(g.d_red);
      (void)hipFree(g.d_stats);
      (void)hipFree(g.d_partial);
      (void)hipHostFree(g.h_args);
      (void)hipHostFree(g.h_upd);
      (void)hipHostFree(g.h_red);
      (void)hipHostFree(g.h_stats);
    }
    for (auto *c : cols) c->in_batch = false;
  }
};

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
    BCHECK(cols[i]->prec == XOD_FP64, "xod_batch_create: batches step FP64 columns");
    for (int j = 0; j < i; ++j) BCHECK(cols[j] != cols[i], "xod_batch_create: duplicate column");
  }
  std::unique_ptr<xod_batch> b(new xod_batch());
  b->cols.assign(cols, cols + ncols);
  b->stream = cols[0]->stream;
  std::map<int, int> by_ld;
  for (auto *c : b->cols) {
    auto it = by_ld.find(c->ld);
    if (it == by_ld.end()) {
      by_ld[c->ld] = (int)b->groups.size();
      b->groups.emplace_back();
      b->groups.back().ld = c->ld;
      it = by_ld.find(c->ld);
    }
    BatchGroup &g = b->groups[it->second];
    g.cols.push_back(c);
    g.maxN = std::max(g.maxN, c->N);
    g.maxR = std::max(g.maxR, c->R);
    g.maxS = std::max(g.maxS, c->S);
  }
  for (auto &g : b->groups) {
    const size_t n = g.cols.size();
    XOD_HIP(hipMalloc((void **)&g.d_args, n * sizeof(ColArgs)));
    XOD_HIP(hipMalloc((void **)&g.d_upd, n * sizeof(UpdArgs)));
    XOD_HIP(hipMalloc((void **)&g.d_red, n * sizeof(RedArgs)));
    XOD_HIP(hipMalloc((void **)&g.d_stats, n * kStatLen * sizeof(double)));
    XOD_HIP(hipMalloc((void **)&g.d_partial, n * kUpdBlocks * kNStat * sizeof(double)));
    XOD_HIP(hipHostMalloc((void **)&g.h_args, n * sizeof(ColArgs), hipHostMallocDefault));
    XOD_HIP(hipHostMalloc((void **)&g.h_upd, n * sizeof(UpdArgs), hipHostMallocDefault));
    XOD_HIP(hipHostMalloc((void **)&g.h_red, n * sizeof(RedArgs), hipHostMallocDefault));
    XOD_HIP(hipHostMalloc((void **)&g.h_stats, n * kStatLen * sizeof(double),
                          hipHostMallocDefault));
  }
  for (auto *c : b->cols) c->in_batch = true;
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
  hipStream_t s = b->stream;
  // Stage per-column arguments (pinned buffers: the copies read them when
  // the stream reaches them, and the step synchronises before returning).
  size_t ci = 0;
  std::map<xod_column *, size_t> index;
  for (size_t i = 0; i < b->cols.size(); ++i) index[b->cols[i]] = i;
  for (auto &g : b->groups) {
    for (size_t j = 0; j < g.cols.size(); ++j) {
      xod_column *c = g.cols[j];
      c->dt = dts[index[c]];
      g.h_args[j] = c->args();
      UpdArgs u{};
      u.n = c->n;
      u.x = c->x;
      u.ngas = c->ngas;
      u.nout = c->ntmp;
      u.partial = g.d_partial + j * kUpdBlocks * kNStat;
      u.N = c->N;
      u.S = c->S;
      u.clip = 0;
      u.y_floor = 1e-30;
      u.y_sig = 1e-10;
      g.h_upd[j] = u;
      g.h_red[j] = RedArgs{u.partial, c->flag, g.d_stats + j * kStatLen};
    }
    const size_t n = g.cols.size();
    XOD_HIP(hipMemcpyAsync(g.d_args, g.h_args, n * sizeof(ColArgs), hipMemcpyHostToDevice, s));
    XOD_HIP(hipMemcpyAsync(g.d_upd, g.h_upd, n * sizeof(UpdArgs), hipMemcpyHostToDevice, s));
    XOD_HIP(hipMemcpyAsync(g.d_red, g.h_red, n * sizeof(RedArgs), hipMemcpyHostToDevice, s));
    ManyCols acc{g.d_args};
    const int nc = (int)n;
    XOD_HIP(launch_rates(acc, nc, g.maxN, g.maxR, s));
    XOD_HIP(launch_rhs(acc, nc, g.maxN, g.maxR, g.maxS, s));
    XOD_HIP(launch_jacobian(acc, nc, g.maxN, g.ld, false, s));
    XOD_HIP(launch_factor_fp64(acc, nc, g.maxN, g.ld, s));
    for (auto *c : g.cols)
      XOD_HIP(hipMemcpyAsync(c->x, c->f, (size_t)c->N * c->S * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
    XOD_HIP(launch_solve_fp64(acc, nc, g.maxN, g.ld, s));
    XOD_HIP(launch_update_state(g.d_upd, g.d_red, nc, s));
    XOD_HIP(hipMemcpyAsync(g.h_stats, g.d_stats, n * kStatLen * sizeof(double),
                           hipMemcpyDeviceToHost, s));
    ci += n;
  }
  XOD_HIP(hipStreamSynchronize(s));
  xod_status ret = XOD_OK;
  for (auto &g : b->groups) {
    for (size_t j = 0; j < g.cols.size(); ++j) {
      xod_column *c = g.cols[j];
      const double *sv = g.h_stats + j * kStatLen;
      const size_t i = index[c];
      if (st) {
        st[i].max_rel_change = sv[0];
        st[i].min_ratio = sv[1];
        st[i].resid_inf = 0.0;
        st[i].refine_iters = 0;
        st[i].fp64_fallback = 0;
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
    }
  }
  (void)ci;
  return ret;
}
