// C ABI of libxod: handles, validation, host-side table construction, the
// backward-Euler step and the steady-state driver.  Every numerical step runs
// in the HIP kernels of k_chem.hip, k_btd.hip, k_mixed.hip and k_step.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "xod_internal.h"

namespace xod {

static thread_local std::string g_err;
void set_error(const std::string &m) { g_err = m; }
std::string &last_error() { return g_err; }
Options &global_options() {
  static Options o;
  return o;
}
Options *&options_override() {
  thread_local Options *p = nullptr;
  return p;
}
Options &options() {
  Options *p = options_override();
  return p ? *p : global_options();
}

}  // namespace xod

using namespace xod;

// ---------------------------------------------------------------------------
// Device buffer helpers.
namespace {

template <class T>
xod_status dalloc(T **p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void **)p, count * sizeof(T));
  if (e != hipSuccess) {
    set_error(std::string("hipMalloc failed: ") + hipGetErrorString(e));
    *p = nullptr;
    return XOD_ENOMEM;
  }
  return XOD_OK;
}

template <class T>
xod_status dupload(T **p, const T *host, size_t count) {
  xod_status s = dalloc(p, count);
  if (s != XOD_OK) return s;
  if (count && host) XOD_HIP(hipMemcpy(*p, host, count * sizeof(T), hipMemcpyHostToDevice));
  return XOD_OK;
}

#define XOD_TRY(expr)                 \
  do {                                \
    xod_status s_ = (expr);           \
    if (s_ != XOD_OK) return s_;      \
  } while (0)

#define XOD_CHECK(cond, msg)          \
  do {                                \
    if (!(cond)) {                    \
      set_error(msg);                 \
      return XOD_EINVAL;              \
    }                                 \
  } while (0)

}  // namespace

#include "handles.h"
#include "cr.h"
#include "tune.h"

namespace {

template <class T>
xod_status nalloc(xod_network *net, T **p, size_t count, const T *host = nullptr) {
  XOD_TRY(host ? dupload(p, host, count) : dalloc(p, count));
  net->owned.push_back(*p);
  return XOD_OK;
}

template <class T>
xod_status calloc_(xod_column *col, T **p, size_t count, const T *host = nullptr) {
  XOD_TRY(host ? dupload(p, host, count) : dalloc(p, count));
  col->owned.push_back(*p);
  return XOD_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
extern "C" xod_status xod_last_error(char *buf, size_t len) {
  if (!buf || len == 0) return XOD_EINVAL;
  const std::string &e = last_error();
  size_t m = std::min(len - 1, e.size());
  std::memcpy(buf, e.data(), m);
  buf[m] = '\0';
  return XOD_OK;
}

extern "C" xod_status xod_set_option(const char *name, int64_t value) {
  XOD_CHECK(name != nullptr, "xod_set_option: null name");
  if (std::strcmp(name, "gemm") == 0) {
    XOD_CHECK(value == 0 || value == 1, "xod_set_option: gemm must be 0 or 1");
    global_options().gemm_mfma = (int)value;
    return XOD_OK;
  }
  if (std::strcmp(name, "gemm_large") == 0) {
    XOD_CHECK(value == 0 || value == 1, "xod_set_option: gemm_large must be 0 or 1");
    global_options().gemm_large = (int)value;
    return XOD_OK;
  }
  if (std::strcmp(name, "gemm_lib") == 0) {
    XOD_CHECK(value == 0 || value == 1, "xod_set_option: gemm_lib must be 0 or 1");
    global_options().gemm_lib = (int)value;
    return XOD_OK;
  }
  if (std::strcmp(name, "panel_sync") == 0) {
    XOD_CHECK(value == 1 || value == 2, "xod_set_option: panel_sync must be 1 or 2");
    global_options().panel_sync = (int)value;
    return XOD_OK;
  }
  if (std::strcmp(name, "panel_defer") == 0) {
    XOD_CHECK(value == 0 || value == 1, "xod_set_option: panel_defer must be 0 or 1");
    global_options().panel_defer = (int)value;
    return XOD_OK;
  }
  if (std::strcmp(name, "mixed_sticky") == 0) {
    XOD_CHECK(value >= 0 && value <= 1000, "xod_set_option: mixed_sticky must be in 0..1000");
    global_options().mixed_sticky = (int)value;
    return XOD_OK;
  }
  if (std::strcmp(name, "gemm_waves") == 0) {
    XOD_CHECK(value == 8 || value == 16, "xod_set_option: gemm_waves must be 8 or 16");
    global_options().gemm_waves = (int)value;
    return XOD_OK;
  }
  if (std::strcmp(name, "gemm_k") == 0) {
    XOD_CHECK(value == 16 || value == 32, "xod_set_option: gemm_k must be 16 or 32");
    global_options().gemm_k = (int)value;
    return XOD_OK;
  }
  if (std::strcmp(name, "refine_tol_exp") == 0) {
    XOD_CHECK(value >= 3 && value <= 15, "xod_set_option: refine_tol_exp must be in 3..15");
    global_options().refine_tol = std::pow(10.0, -(double)value);
    return XOD_OK;
  }
  if (std::strcmp(name, "fused_max_ld") == 0) {
    XOD_CHECK(value == 0 || value == 32 || value == 64 || value == 96 || value == 128,
              "xod_set_option: fused_max_ld must be 0, 32, 64, 96 or 128");
    global_options().fused_max_ld = (int)value;
    return XOD_OK;
  }
  if (std::strcmp(name, "refine64") == 0) {
    XOD_CHECK(value >= 0 && value <= 10, "xod_set_option: refine64 must be in 0..10");
    global_options().refine64 = (int)value;
    return XOD_OK;
  }
  if (std::strcmp(name, "refine_atol_exp") == 0) {
    XOD_CHECK(value >= 8 && value <= 17, "xod_set_option: refine_atol_exp must be in 8..17");
    global_options().refine_atol = std::pow(10.0, -(double)value);
    return XOD_OK;
  }
  if (std::strcmp(name, "outer") == 0) {
    XOD_CHECK(value == 32 || value == 64 || value == 96 || value == 128,
              "xod_set_option: outer must be 32, 64, 96 or 128");
    global_options().outer = (int)value;
    return XOD_OK;
  }
  if (std::strcmp(name, "outer_nmat") == 0) {
    XOD_CHECK(value >= 1 && value <= 1000000, "xod_set_option: outer_nmat must be >= 1");
    global_options().outer_nmat = (int)value;
    return XOD_OK;
  }
  if (std::strcmp(name, "update32_min") == 0) {
    XOD_CHECK(value >= 0 && value <= 1000000, "xod_set_option: update32_min must be in 0..1000000");
    global_options().update32_min = (int)value;
    return XOD_OK;
  }
  if (std::strcmp(name, "update32") == 0) {
    XOD_CHECK(value == 0 || value == 1, "xod_set_option: update32 must be 0 or 1");
    global_options().update32 = (int)value;
    return XOD_OK;
  }
  if (std::strcmp(name, "graph") == 0) {
    XOD_CHECK(value == 0 || value == 1, "xod_set_option: graph must be 0 or 1");
    global_options().graph = (int)value;
    return XOD_OK;
  }
  if (std::strcmp(name, "profile") == 0) {
    XOD_CHECK(value == 0 || value == 1, "xod_set_option: profile must be 0 or 1");
    global_options().profile = (int)value;
    return XOD_OK;
  }
  if (std::strcmp(name, "profile_every") == 0) {
    XOD_CHECK(value >= 1 && value <= 1000000, "xod_set_option: profile_every must be >= 1");
    global_options().profile_every = (int)value;
    return XOD_OK;
  }
  set_error(std::string("xod_set_option: unknown option ") + name);
  return XOD_EINVAL;
}

extern "C" xod_status xod_get_option(const char *name, int64_t *value) {
  XOD_CHECK(name != nullptr && value != nullptr, "xod_get_option: null argument");
  const Options &o = global_options();
  struct Entry { const char *name; int64_t v; };
  const Entry entries[] = {
      {"gemm", o.gemm_mfma},           {"gemm_large", o.gemm_large},
      {"gemm_k", o.gemm_k},            {"outer", o.outer},
      {"gemm_waves", o.gemm_waves},    {"mixed_sticky", o.mixed_sticky},
      {"panel_sync", o.panel_sync},    {"gemm_lib", o.gemm_lib},
      {"panel_defer", o.panel_defer},
      {"outer_nmat", o.outer_nmat},    {"update32", o.update32},
      {"update32_min", o.update32_min},
      {"graph", o.graph},              {"profile", o.profile},
      {"profile_every", o.profile_every},
      {"refine_tol_exp", (int64_t)std::lround(-std::log10(o.refine_tol))},
      {"refine_atol_exp", (int64_t)std::lround(-std::log10(o.refine_atol))},
      {"refine64", o.refine64},        {"fused_max_ld", o.fused_max_ld},
  };
  for (const Entry &e : entries)
    if (std::strcmp(name, e.name) == 0) {
      *value = e.v;
      return XOD_OK;
    }
  set_error(std::string("xod_get_option: unknown option ") + name);
  return XOD_EINVAL;
}

extern "C" xod_status xod_network_create(const xod_network_desc *d, xod_network **out) {
  XOD_CHECK(d && out, "xod_network_create: null argument");
  *out = nullptr;
  XOD_CHECK(d->S >= 1 && d->R >= 0 && d->E >= 0, "xod_network_create: bad sizes");
  XOD_CHECK(d->S <= kMaxLd, "xod_network_create: S > 1024 is not supported");
  const int S = d->S, R = d->R;
  XOD_CHECK(d->mass_amu && d->nasa7, "xod_network_create: null mass/nasa7");
  XOD_CHECK(R == 0 || (d->rtype && d->reac && d->prod && d->reversible && d->tb_kooij &&
                       d->params),
            "xod_network_create: null reaction array");
  for (int y = 0; y < S; ++y)
    XOD_CHECK(std::isfinite(d->mass_amu[y]) && d->mass_amu[y] > 0.0,
              "xod_network_create: species mass must be positive");
  for (int i = 0; i < S * 14; ++i)
    XOD_CHECK(std::isfinite(d->nasa7[i]), "xod_network_create: non-finite NASA-7 coefficient");
  std::vector<int> dnu(R, 0);
  for (int r = 0; r < R; ++r) {
    XOD_CHECK(d->rtype[r] >= 0 && d->rtype[r] <= 2, "xod_network_create: bad reaction type");
    int nre = 0, npr = 0;
    for (int j = 0; j < XOD_MAX_REAC; ++j) {
      const int y = d->reac[r * XOD_MAX_REAC + j];
      XOD_CHECK(y >= -1 && y < S, "xod_network_create: reactant id out of range");
      nre += y >= 0;
    }
    for (int j = 0; j < XOD_MAX_PROD; ++j) {
      const int y = d->prod[r * XOD_MAX_PROD + j];
      XOD_CHECK(y >= -1 && y < S, "xod_network_create: product id out of range");
      npr += y >= 0;
    }
    XOD_CHECK(nre >= 1, "xod_network_create: reaction without reactant");
    for (int j = 0; j < 6; ++j)
      XOD_CHECK(std::isfinite(d->params[r * 6 + j]), "xod_network_create: non-finite parameter");
    dnu[r] = npr - nre;
  }

  std::unique_ptr<xod_network> net(new xod_network());
  net->S = S;
  net->R = R;
  net->E = d->E;
  net->ld = round_up(S, 32);
  net->t_mid = d->t_mid;
  net->mass_h.assign(d->mass_amu, d->mass_amu + S);

  // Net stoichiometry nu[y][r] and the species -> reaction incidence lists.
  std::vector<std::map<int, double>> nu_r(R);
  for (int r = 0; r < R; ++r) {
    for (int j = 0; j < XOD_MAX_PROD; ++j) {
      const int y = d->prod[r * XOD_MAX_PROD + j];
      if (y >= 0) nu_r[r][y] += 1.0;
    }
    for (int j = 0; j < XOD_MAX_REAC; ++j) {
      const int y = d->reac[r * XOD_MAX_REAC + j];
      if (y >= 0) nu_r[r][y] -= 1.0;
    }
  }
  std::vector<std::vector<std::pair<int, double>>> inc(S);
  for (int r = 0; r < R; ++r)
    for (auto &kv : nu_r[r])
      if (kv.second != 0.0) inc[kv.first].push_back({r, kv.second});
  std::vector<int> inc_ptr(S + 1, 0), inc_r;
  std::vector<double> inc_nu;
  for (int y = 0; y < S; ++y) {
    for (auto &e : inc[y]) {
      inc_r.push_back(e.first);
      inc_nu.push_back(e.second);
    }
    inc_ptr[y + 1] = (int)inc_r.size();
  }

  // Jacobian pattern: entry (y, x) collects (r, nu_{y,r}) for every reaction
  // r in which x takes part and y changes.
  // A contribution names the derivative slot 6 r + u of reaction r with
  // respect to its u-th distinct species (rsp lists them, -1 padded).
  std::map<std::pair<int, int>, std::vector<std::pair<int, double>>> ent;
  std::vector<int> rsp((size_t)R * 6, -1);
  for (int r = 0; r < R; ++r) {
    std::vector<int> xs;
    for (int j = 0; j < XOD_MAX_REAC; ++j) {
      const int y = d->reac[r * XOD_MAX_REAC + j];
      if (y >= 0 && std::find(xs.begin(), xs.end(), y) == xs.end()) xs.push_back(y);
    }
    for (int j = 0; j < XOD_MAX_PROD; ++j) {
      const int y = d->prod[r * XOD_MAX_PROD + j];
      if (y >= 0 && std::find(xs.begin(), xs.end(), y) == xs.end()) xs.push_back(y);
    }
    for (size_t u = 0; u < xs.size(); ++u) rsp[(size_t)r * 6 + u] = xs[u];
    for (auto &kv : nu_r[r]) {
      if (kv.second == 0.0) continue;
      for (size_t u = 0; u < xs.size(); ++u)
        ent[{kv.first, xs[u]}].push_back({6 * r + (int)u, kv.second});
    }
  }
  // Nonzero entries in row-major order (the map's order): row y holds
  // entries jrow[y] .. jrow[y+1]-1, entry e sits in column jcol[e] and sums
  // contributions jptr[e] .. jptr[e+1]-1, so row y's contributions are
  // jptr[jrow[y]] .. jptr[jrow[y+1]]-1; jc_col names each one's column.
  std::vector<int> jrow(S + 1, 0), jcol, jptr(1, 0), jc_ru;
  std::vector<double> jc_nu;
  for (auto &kv : ent) {
    jrow[kv.first.first + 1]++;
    jcol.push_back(kv.first.second);
    for (auto &e : kv.second) {
      jc_ru.push_back(e.first);
      jc_nu.push_back(e.second);
    }
    jptr.push_back((int)jc_ru.size());
  }
  for (int y = 0; y < S; ++y) jrow[y + 1] += jrow[y];
  std::vector<int> jc_col(jc_ru.size());   // column of each contribution's entry
  for (size_t e = 0; e + 1 < jptr.size(); ++e)
    for (int q = jptr[e]; q < jptr[e + 1]; ++q) jc_col[q] = jcol[e];
  std::vector<int> photo_idx(R, -1);
  int nph = 0;
  for (int r = 0; r < R; ++r)
    if (d->rtype[r] == XOD_RT_PHOTO) photo_idx[r] = nph++;
  net->nph = nph;
  net->nnz = (int)jptr.size() - 1;
  net->ncontrib = (int)jc_ru.size();

  xod_network *n = net.get();
  XOD_TRY(nalloc(n, &n->rtype, R, d->rtype));
  XOD_TRY(nalloc(n, &n->reac, (size_t)R * XOD_MAX_REAC, d->reac));
  XOD_TRY(nalloc(n, &n->prod, (size_t)R * XOD_MAX_PROD, d->prod));
  XOD_TRY(nalloc(n, &n->rev, R, d->reversible));
  XOD_TRY(nalloc(n, &n->kooij, R, d->tb_kooij));
  XOD_TRY(nalloc(n, &n->dnu, R, dnu.data()));
  XOD_TRY(nalloc(n, &n->params, (size_t)R * 6, d->params));
  XOD_TRY(nalloc(n, &n->nasa7, (size_t)S * 14, d->nasa7));
  XOD_TRY(nalloc(n, &n->mass, S, d->mass_amu));
  XOD_TRY(nalloc(n, &n->inc_ptr, S + 1, inc_ptr.data()));
  XOD_TRY(nalloc(n, &n->inc_r, inc_r.size(), inc_r.data()));
  XOD_TRY(nalloc(n, &n->inc_nu, inc_nu.size(), inc_nu.data()));
  XOD_TRY(nalloc(n, &n->jrow, jrow.size(), jrow.data()));
  XOD_TRY(nalloc(n, &n->jc_col, jc_col.size(), jc_col.data()));
  XOD_TRY(nalloc(n, &n->jptr, jptr.size(), jptr.data()));
  XOD_TRY(nalloc(n, &n->jc_ru, jc_ru.size(), jc_ru.data()));
  XOD_TRY(nalloc(n, &n->rsp, rsp.size(), rsp.data()));
  XOD_TRY(nalloc(n, &n->jc_nu, jc_nu.size(), jc_nu.data()));
  XOD_TRY(nalloc(n, &n->photo_idx, photo_idx.size(), photo_idx.data()));
  *out = net.release();
  return XOD_OK;
}

extern "C" xod_status xod_network_destroy(xod_network *net) {
  XOD_CHECK(net, "xod_network_destroy: null network");
  delete net;
  return XOD_OK;
}

extern "C" xod_status xod_network_sizes(const xod_network *net, int32_t *S, int32_t *R,
                                        int32_t *ld) {
  XOD_CHECK(net, "xod_network_sizes: null network");
  if (S) *S = net->S;
  if (R) *R = net->R;
  if (ld) *ld = net->ld;
  return XOD_OK;
}

extern "C" xod_status xod_column_create(const xod_network *net, const xod_profile *p,
                                        const double *n0, xod_precision prec, void *stream,
                                        xod_column **out) {
  XOD_CHECK(net && p && n0 && out, "xod_column_create: null argument");
  *out = nullptr;
  XOD_CHECK(prec == XOD_FP64 || prec == XOD_MIXED, "xod_column_create: bad precision");
  const int N = p->N, S = net->S;
  XOD_CHECK(N >= 1 && N <= 100000, "xod_column_create: N out of range");
  XOD_CHECK(p->P_bar && p->T_K && p->Kzz, "xod_column_create: null profile array");
  XOD_CHECK(p->mbar_amu > 0 && p->g_cgs > 0 && p->sigma_tau >= 0 &&
                std::isfinite(p->mbar_amu) && std::isfinite(p->g_cgs) &&
                std::isfinite(p->sigma_tau),
            "xod_column_create: bad mbar/g/sigma_tau");
  for (int k = 0; k < N; ++k) {
    XOD_CHECK(std::isfinite(p->P_bar[k]) && p->P_bar[k] > 0, "xod_column_create: P must be > 0");
    XOD_CHECK(std::isfinite(p->T_K[k]) && p->T_K[k] > 0, "xod_column_create: T must be > 0");
    XOD_CHECK(std::isfinite(p->Kzz[k]) && p->Kzz[k] >= 0, "xod_column_create: Kzz must be >= 0");
    if (k > 0)
      XOD_CHECK(p->P_bar[k] < p->P_bar[k - 1], "xod_column_create: P must decrease upward");
  }
  if (p->Dmol)
    for (size_t e = 0; e < (size_t)N * S; ++e)
      XOD_CHECK(std::isfinite(p->Dmol[e]) && p->Dmol[e] >= 0, "xod_column_create: bad Dmol");
  if (p->alphaT)
    for (int y = 0; y < S; ++y)
      XOD_CHECK(std::isfinite(p->alphaT[y]), "xod_column_create: bad alphaT");
  for (size_t e = 0; e < (size_t)N * S; ++e)
    XOD_CHECK(std::isfinite(n0[e]), "xod_column_create: non-finite n0");

  std::unique_ptr<xod_column> col(new xod_column());
  xod_column *c = col.get();
  c->net = net;
  c->N = N;
  c->S = S;
  c->R = net->R;
  c->ld = net->ld;
  c->prec = prec;
  c->stream = (hipStream_t)stream;
  const size_t NS = (size_t)N * S, NR = (size_t)N * net->R, NL = (size_t)N * c->ld;
  const size_t NLL = NL * c->ld;
  XOD_TRY(calloc_(c, &c->P, N, p->P_bar));
  XOD_TRY(calloc_(c, &c->T, N, p->T_K));
  XOD_TRY(calloc_(c, &c->K, N, p->Kzz));
  c->T_top = p->T_K[N - 1];
  c->mbar_amu = p->mbar_amu;
  c->g_cgs = p->g_cgs;
  c->D_top.assign(S, 0.0);
  if (p->Dmol)
    for (int y = 0; y < S; ++y) c->D_top[y] = p->Dmol[(size_t)(N - 1) * S + y];
  if (p->Dmol) XOD_TRY(calloc_(c, &c->D, NS, p->Dmol));
  if (p->alphaT) XOD_TRY(calloc_(c, &c->alpha, (size_t)S, p->alphaT));
  XOD_TRY(calloc_(c, &c->ngas, N));
  XOD_TRY(calloc_(c, &c->tau, N));
  XOD_TRY(calloc_(c, &c->lnpref, N));
  XOD_TRY(calloc_(c, &c->dz, N));
  XOD_TRY(calloc_(c, &c->dzh, N));
  XOD_TRY(calloc_(c, &c->mix, 1));
  XOD_TRY(calloc_(c, &c->g, NS));
  XOD_TRY(calloc_(c, &c->trl, NS));
  XOD_TRY(calloc_(c, &c->trd, NS));
  XOD_TRY(calloc_(c, &c->tru, NS));
  XOD_TRY(calloc_(c, &c->n, NS, n0));
  XOD_TRY(calloc_(c, &c->ntmp, NS));
  XOD_TRY(calloc_(c, &c->f, NS));
  XOD_TRY(calloc_(c, &c->x, NS));
  XOD_TRY(calloc_(c, &c->resid, NS));
  XOD_TRY(calloc_(c, &c->dx, NS));
  XOD_TRY(calloc_(c, &c->kf, NR));
  XOD_TRY(calloc_(c, &c->kr, NR));
  XOD_TRY(calloc_(c, &c->w, NR));
  XOD_TRY(calloc_(c, &c->dwd, 6 * NR));
  XOD_TRY(calloc_(c, &c->gs, NL));
  XOD_TRY(calloc_(c, &c->a, NL));
  XOD_TRY(calloc_(c, &c->c, NL));
  XOD_TRY(calloc_(c, &c->rs, NL));
  XOD_TRY(calloc_(c, &c->piv, NL));
  XOD_TRY(calloc_(c, &c->rstep, NL));
  XOD_TRY(calloc_(c, &c->flag, 4));
  XOD_TRY(calloc_(c, &c->B, NLL));
  if (prec == XOD_MIXED) XOD_TRY(calloc_(c, &c->Bf, NLL));
  XOD_TRY(calloc_(c, &c->ratio, (size_t)N));
  XOD_TRY(calloc_(c, &c->rmax, 1));
  XOD_TRY(calloc_(c, &c->partial, (size_t)kUpdBlocks * kNStat));
  XOD_TRY(calloc_(c, &c->stats_dev, kStatLen));
  XOD_TRY(calloc_(c, &c->upd_dev, 1));
  XOD_TRY(calloc_(c, &c->red_dev, 1));
  XOD_HIP(hipHostMalloc((void **)&c->stats_host, kStatLen * sizeof(double), hipHostMallocDefault));
  XOD_HIP(hipHostMalloc((void **)&c->upd_host, sizeof(UpdArgs), hipHostMallocDefault));
  XOD_HIP(hipHostMalloc((void **)&c->red_host, sizeof(RedArgs), hipHostMallocDefault));

  SetupArgs sa{};
  sa.N = N;
  sa.S = S;
  sa.P_bar = c->P;
  sa.T = c->T;
  sa.K = c->K;
  sa.D = c->D;
  sa.alpha = c->alpha;
  sa.mass = net->mass;
  sa.nasa7 = net->nasa7;
  sa.t_mid = net->t_mid;
  sa.mbar_amu = p->mbar_amu;
  sa.g_cgs = p->g_cgs;
  sa.sigma_tau = p->sigma_tau;
  sa.ngas = c->ngas;
  sa.tau = c->tau;
  sa.lnpref = c->lnpref;
  sa.g = c->g;
  sa.trl = c->trl;
  sa.trd = c->trd;
  sa.tru = c->tru;
  sa.dz = c->dz;
  sa.dzh = c->dzh;
  sa.mix = c->mix;
  XOD_HIP(launch_setup(sa, c->stream));
  XOD_HIP(hipMemcpyAsync(&c->mix_time, c->mix, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  XOD_HIP(hipStreamSynchronize(c->stream));
  *out = col.release();
  return XOD_OK;
}

extern "C" xod_status xod_column_destroy(xod_column *col) {
  XOD_CHECK(col, "xod_column_destroy: null column");
  (void)hipStreamSynchronize(col->stream);
  delete col;
  return XOD_OK;
}

extern "C" xod_status xod_column_get_state(const xod_column *col, double *n, double *t,
                                           double *dt) {
  XOD_CHECK(col && n, "xod_column_get_state: null argument");
  XOD_HIP(hipMemcpyAsync(n, col->n, (size_t)col->N * col->S * sizeof(double),
                         hipMemcpyDeviceToHost, col->stream));
  XOD_HIP(hipStreamSynchronize(col->stream));
  if (t) *t = col->t;
  if (dt) *dt = col->dt;
  return XOD_OK;
}

extern "C" xod_status xod_column_set_state(xod_column *col, const double *n, double t,
                                           double dt) {
  XOD_CHECK(col && n, "xod_column_set_state: null argument");
  for (size_t e = 0; e < (size_t)col->N * col->S; ++e)
    XOD_CHECK(std::isfinite(n[e]), "xod_column_set_state: non-finite state");
  XOD_HIP(hipMemcpyAsync(col->n, n, (size_t)col->N * col->S * sizeof(double),
                         hipMemcpyHostToDevice, col->stream));
  XOD_HIP(hipStreamSynchronize(col->stream));
  col->t = t;
  col->dt = dt;
  col->prev_dt = 0.0;
  col->mixed_fb_dt = 0.0;   // a new state starts a new history of precision choices
  col->mixed_direct = 0;
  return XOD_OK;
}

extern "C" xod_status xod_column_state_ptr(xod_column *col, double **n_dev) {
  XOD_CHECK(col && n_dev, "xod_column_state_ptr: null argument");
  *n_dev = col->n;
  return XOD_OK;
}

extern "C" xod_status xod_column_grid(const xod_column *col, double *ngas, double *tau,
                                      double *dz, double *mix_time) {
  XOD_CHECK(col, "xod_column_grid: null column");
  const size_t bytes = (size_t)col->N * sizeof(double);
  if (ngas) XOD_HIP(hipMemcpyAsync(ngas, col->ngas, bytes, hipMemcpyDeviceToHost, col->stream));
  if (tau) XOD_HIP(hipMemcpyAsync(tau, col->tau, bytes, hipMemcpyDeviceToHost, col->stream));
  if (dz) XOD_HIP(hipMemcpyAsync(dz, col->dz, bytes, hipMemcpyDeviceToHost, col->stream));
  XOD_HIP(hipStreamSynchronize(col->stream));
  if (mix_time) *mix_time = col->mix_time;
  return XOD_OK;
}

// ---------------------------------------------------------------------------
// Hot-path calls on caller-owned device buffers.
namespace xod {
// The column's spectral photolysis rates at its current state, if set.
extern "C" xod_status xod_column_set_boundary(xod_column *col, const xod_boundary *b) {
  XOD_CHECK(col, "xod_column_set_boundary: null column");
  XOD_CHECK(!col->in_batch, "xod_column_set_boundary: column belongs to a batch");
  const int N = col->N, S = col->S;
  std::vector<double> vt(S, 0.0), vd(S, 0.0), phi(S, 0.0);
  if (b) {
    if (b->escape_diff_limited) {
      // V_lim = D (1/H_0 - 1/H_y) with the top layer's D and T, no escape
      // for species heavier than the mean (V_lim < 0)
      const double H0 = kBoltz * col->T_top / (col->mbar_amu * kAmu * col->g_cgs);
      for (int y = 0; y < S; ++y) {
        const int32_t fl = b->escape_diff_limited[y];
        XOD_CHECK(fl == 0 || fl == 1, "xod_column_set_boundary: escape flags must be 0 or 1");
        if (!fl) continue;
        const double Hy = kBoltz * col->T_top / (col->net->mass_h[y] * kAmu * col->g_cgs);
        vt[y] = std::max(col->D_top[y] * (1.0 / H0 - 1.0 / Hy), 0.0);
      }
    }
    for (int y = 0; y < S; ++y) {
      if (b->v_top) {
        XOD_CHECK(std::isfinite(b->v_top[y]) && b->v_top[y] >= 0,
                  "xod_column_set_boundary: v_top must be finite and >= 0");
        vt[y] += b->v_top[y];
      }
      if (b->v_dep) {
        XOD_CHECK(std::isfinite(b->v_dep[y]) && b->v_dep[y] >= 0,
                  "xod_column_set_boundary: v_dep must be finite and >= 0");
        vd[y] = b->v_dep[y];
      }
      if (b->phi_surf) {
        XOD_CHECK(std::isfinite(b->phi_surf[y]), "xod_column_set_boundary: phi_surf not finite");
        phi[y] = b->phi_surf[y];
      }
    }
  }
  const size_t rowb = (size_t)S * sizeof(double);
  double dz[2];
  XOD_HIP(hipMemcpyAsync(&dz[0], col->dz, sizeof(double), hipMemcpyDeviceToHost, col->stream));
  XOD_HIP(hipMemcpyAsync(&dz[1], col->dz + (N - 1), sizeof(double), hipMemcpyDeviceToHost,
                         col->stream));
  if (col->trd_bot0.empty()) {
    col->trd_bot0.resize(S);
    col->trd_top0.resize(S);
    XOD_HIP(hipMemcpyAsync(col->trd_bot0.data(), col->trd, rowb, hipMemcpyDeviceToHost,
                           col->stream));
    XOD_HIP(hipMemcpyAsync(col->trd_top0.data(), col->trd + (size_t)(N - 1) * S, rowb,
                           hipMemcpyDeviceToHost, col->stream));
  }
  XOD_HIP(hipStreamSynchronize(col->stream));
  // a single layer is both the bottom and the top layer
  std::vector<double> bot = col->trd_bot0, top = col->trd_top0;
  std::vector<double> &toprow = N == 1 ? bot : top;
  bool any_src = false;
  std::vector<double> src(S, 0.0);
  for (int y = 0; y < S; ++y) {
    bot[y] -= vd[y] / dz[0];
    toprow[y] -= vt[y] / dz[1];
    src[y] = phi[y] / dz[0];
    any_src = any_src || phi[y] != 0.0;
  }
  XOD_HIP(hipMemcpyAsync(col->trd, bot.data(), rowb, hipMemcpyHostToDevice, col->stream));
  if (N > 1)
    XOD_HIP(hipMemcpyAsync(col->trd + (size_t)(N - 1) * S, top.data(), rowb,
                           hipMemcpyHostToDevice, col->stream));
  if (any_src) {
    if (!col->bsrc) XOD_TRY(calloc_(col, &col->bsrc, (size_t)S));
    XOD_HIP(hipMemcpyAsync(col->bsrc, src.data(), rowb, hipMemcpyHostToDevice, col->stream));
  }
  XOD_HIP(hipStreamSynchronize(col->stream));
  col->has_bsrc = any_src;
  bool any_v = false;
  for (int y = 0; y < S; ++y) any_v = any_v || vt[y] != 0.0 || vd[y] != 0.0;
  col->open_ends = any_src || any_v;
  col->fact_dt = 0.0;     // the step matrix changed
  return XOD_OK;
}

static xod_status enqueue_photolysis(xod_column *c) {
  if (c->ph_L <= 0 || c->net->nph == 0) return XOD_OK;
  XOD_HIP(launch_photolysis(c->N, c->S, c->ph_A, c->ph_L, c->net->nph, c->n, c->dz, c->ph_abs,
                            c->ph_ext, c->ph_J0, c->ph_dlam, c->ph_sig, c->ph_tf, c->ph_mu,
                            c->ph_work, c->kph, c->stream));
  return XOD_OK;
}
}  // namespace xod

extern "C" xod_status xod_column_set_photolysis_spectrum(xod_column *col, int32_t A, int32_t L,
                                                         const int32_t *absorbers,
                                                         const double *sig_ext, const double *J0,
                                                         const double *dlam,
                                                         const double *sig_ph, double t_f,
                                                         double mu) {
  XOD_CHECK(col, "xod_column_set_photolysis_spectrum: null column");
  if (L == 0) {             // back to the gray law
    col->ph_L = 0;
    return XOD_OK;
  }
  XOD_CHECK(L > 0 && A >= 0, "xod_column_set_photolysis_spectrum: need L > 0 and A >= 0");
  XOD_CHECK(mu > 0.0, "xod_column_set_photolysis_spectrum: mu must be positive");
  XOD_CHECK(J0 && dlam && (A == 0 || (absorbers && sig_ext)) && (col->net->nph == 0 || sig_ph),
            "xod_column_set_photolysis_spectrum: null table");
  const int P = col->net->nph;
  if (!col->kph && P > 0) XOD_TRY(calloc_(col, &col->kph, (size_t)col->N * P));
  const size_t need = photolysis_work_bytes(col->N, A, L, P);
  if (need > col->ph_work_bytes) {
    double *w = nullptr;
    XOD_TRY(calloc_(col, &w, (need + sizeof(double) - 1) / sizeof(double)));
    col->ph_work = w;
    col->ph_work_bytes = need;
  }
  col->ph_A = A;
  col->ph_L = L;
  col->ph_abs = absorbers;
  col->ph_ext = sig_ext;
  col->ph_J0 = J0;
  col->ph_dlam = dlam;
  col->ph_sig = sig_ph;
  col->ph_tf = t_f;
  col->ph_mu = mu;
  return XOD_OK;
}

extern "C" xod_status xod_rates(xod_column *col, double *kf, double *kr) {
  XOD_CHECK(col && kf && kr, "xod_rates: null argument");
  XOD_TRY(enqueue_photolysis(col));
  ColArgs a = col->args();
  a.kf = kf;
  a.kr = kr;
  XOD_HIP(launch_rates(OneCol{a}, 1, col->N, col->R, col->stream));
  return XOD_OK;
}

extern "C" xod_status xod_rhs(xod_column *col, const double *kf, const double *kr,
                              const double *n, double *f) {
  XOD_CHECK(col && kf && kr && n && f, "xod_rhs: null argument");
  ColArgs a = col->args();
  a.kf_in = kf;
  a.kr_in = kr;
  a.n = n;
  a.f = f;
  XOD_HIP(launch_rhs(OneCol{a}, 1, col->N, col->R, col->S, col->stream));
  return XOD_OK;
}

extern "C" xod_status xod_jacobian(xod_column *col, const double *kf, const double *kr,
                                   const double *n, double dt, double *B, double *av,
                                   double *cv, int32_t ld) {
  XOD_CHECK(col && kf && kr && n && B && av && cv, "xod_jacobian: null argument");
  XOD_CHECK(ld == col->ld, "xod_jacobian: ld must equal the network's padded size");
  XOD_CHECK(std::isfinite(dt) && dt > 0, "xod_jacobian: dt must be > 0");
  ColArgs a = col->args();
  a.kf_in = kf;
  a.kr_in = kr;
  a.n = n;
  a.dt = dt;
  a.B = B;
  a.a = av;
  a.c = cv;
  XOD_HIP(launch_jacobian(OneCol{a}, 1, col->N, col->R, col->ld, false, col->stream));
  return XOD_OK;
}

static xod_status check_flags(xod_column *col, const double *flags) {
  if (flags[0] >= 0) {
    set_error("singular Schur complement: layer " + std::to_string((long)flags[0]) +
              ", column " + std::to_string((long)flags[1]));
    return XOD_ESINGULAR;
  }
  (void)col;
  return XOD_OK;
}

extern "C" xod_status xod_column_set_solver(xod_column *col, xod_solver solver) {
  XOD_CHECK(col, "xod_column_set_solver: null column");
  XOD_CHECK(solver == XOD_SOLVER_THOMAS || solver == XOD_SOLVER_CR,
            "xod_column_set_solver: unknown solver");
  XOD_CHECK(!col->in_batch, "xod_column_set_solver: column belongs to a batch");
  if (solver == XOD_SOLVER_CR) {
    if (!col->cr64) {   // FP64 columns, and the FP64 fallback of mixed ones
      std::unique_ptr<xod::CrPlan<double>> p(new xod::CrPlan<double>());
      const xod_status st = p->build(col);
      if (st != XOD_OK) return st == XOD_EHIP ? XOD_ENOMEM : st;
      col->cr64 = p.release();
    }
    if (col->prec == XOD_MIXED && !col->cr32) {
      std::unique_ptr<xod::CrPlan<float>> p(new xod::CrPlan<float>());
      const xod_status st = p->build(col);
      if (st != XOD_OK) return st == XOD_EHIP ? XOD_ENOMEM : st;
      col->cr32 = p.release();
    }
  }
  if (col->solver != solver) {
    col->fact_dt = 0.0;
    col->btd.valid = false;
  }
  col->solver = solver;
  return XOD_OK;
}

namespace {

// FP32 blocks (and the single-precision cyclic-reduction plan) of a column
// that was created in FP64, allocated on first use by a mixed explicit factor.
xod_status ensure_fp32_blocks(xod_column *col) {
  if (!col->Bf) {
    float *p = nullptr;
    XOD_TRY(calloc_(col, &p, (size_t)col->N * col->ld * col->ld));
    col->Bf = p;
  }
  if (col->solver == XOD_SOLVER_CR && !col->cr32) {
    std::unique_ptr<xod::CrPlan<float>> p(new xod::CrPlan<float>());
    const xod_status st = p->build(col);
    if (st != XOD_OK) return st == XOD_EHIP ? XOD_ENOMEM : st;
    col->cr32 = p.release();
  }
  return XOD_OK;
}

// FP64 factorisation of the caller's system in the column's own blocks
// (cyclic reduction, or the fallback of a mixed explicit solve).
xod_status factor_own_fp64(xod_column *col, const double *B, const double *av,
                           const double *cv) {
  const TunedScope tuned(col->ld, XOD_FP64, col->solver, false);
  const size_t NL = (size_t)col->N * col->ld;
  XOD_HIP(hipMemcpyAsync(col->B, B, NL * col->ld * sizeof(double), hipMemcpyDeviceToDevice,
                         col->stream));
  XOD_HIP(hipMemcpyAsync(col->a, av, NL * sizeof(double), hipMemcpyDeviceToDevice, col->stream));
  XOD_HIP(hipMemcpyAsync(col->c, cv, NL * sizeof(double), hipMemcpyDeviceToDevice, col->stream));
  if (col->solver == XOD_SOLVER_CR) {
    XOD_TRY(col->cr64->factor(col));
  } else {
    XOD_HIP(launch_factor_fp64(OneCol{col->args()}, 1, col->N, col->ld, col->stream));
  }
  return XOD_OK;
}

xod_status read_singular_flag(xod_column *col) {
  int fl[4];
  XOD_HIP(hipMemcpyAsync(fl, col->flag, sizeof(fl), hipMemcpyDeviceToHost, col->stream));
  XOD_HIP(hipStreamSynchronize(col->stream));
  double fd[2] = {(double)fl[0], (double)fl[1]};
  return check_flags(col, fd);
}

// Solve with the column's own FP64 factors: rhs [N*S] in, solution out.
xod_status solve_own_fp64(xod_column *col, double *rhs) {
  const size_t NSb = (size_t)col->N * col->S * sizeof(double);
  XOD_HIP(hipMemcpyAsync(col->x, rhs, NSb, hipMemcpyDeviceToDevice, col->stream));
  if (col->solver == XOD_SOLVER_CR) {
    XOD_TRY(col->cr64->solve(col));
  } else {
    XOD_HIP(launch_solve_fp64(OneCol{col->args()}, 1, col->N, col->ld, col->stream));
  }
  XOD_HIP(hipMemcpyAsync(rhs, col->x, NSb, hipMemcpyDeviceToDevice, col->stream));
  return XOD_OK;
}

}  // namespace

extern "C" xod_status xod_btd_factor(xod_column *col, double *B, const double *av,
                                     const double *cv, int32_t ld, int32_t *piv,
                                     xod_precision prec) {
  XOD_CHECK(col && B && av && cv, "xod_btd_factor: null argument");
  XOD_CHECK(ld == col->ld, "xod_btd_factor: ld must equal the network's padded size");
  XOD_CHECK(prec == XOD_FP64 || prec == XOD_MIXED, "xod_btd_factor: bad precision");
  XOD_CHECK(!col->in_batch, "xod_btd_factor: column belongs to a batch");
  col->btd.valid = false;
  col->fact_dt = 0.0;     // the column's own blocks no longer hold a step's factors
  if (prec == XOD_FP64 && col->solver == XOD_SOLVER_THOMAS) {
    XOD_CHECK(piv, "xod_btd_factor: null pivot array");
    ColArgs a = col->args();
    a.B = B;
    a.a = const_cast<double *>(av);
    a.c = const_cast<double *>(cv);
    a.piv = piv;
    XOD_HIP(launch_factor_fp64(OneCol{a}, 1, col->N, col->ld, col->stream));
    return read_singular_flag(col);
  }
  if (prec == XOD_FP64) {
    XOD_TRY(factor_own_fp64(col, B, av, cv));
  } else {
    XOD_TRY(ensure_fp32_blocks(col));
    XOD_HIP(launch_cast_scale(B, av, cv, col->N, col->ld, col->Bf, col->rs, col->a, col->c,
                              col->stream));
    if (col->solver == XOD_SOLVER_CR) {
      XOD_TRY(col->cr32->factor(col));
    } else {
      XOD_HIP(launch_factor_mixed(OneCol{col->args()}, 1, col->N, col->ld, col->stream));
    }
  }
  XOD_TRY(read_singular_flag(col));
  col->btd.valid = true;
  col->btd.prec = prec;
  col->btd.solver = col->solver;
  col->btd.B = B;
  col->btd.a = av;
  col->btd.c = cv;
  return XOD_OK;
}

extern "C" xod_status xod_btd_solve(xod_column *col, const double *B, const double *av,
                                    const double *cv, int32_t ld, const int32_t *piv,
                                    double *rhs, int32_t max_refine) {
  XOD_CHECK(col && B && av && cv && rhs, "xod_btd_solve: null argument");
  XOD_CHECK(ld == col->ld, "xod_btd_solve: ld must equal the network's padded size");
  XOD_CHECK(max_refine >= 0 && max_refine <= 100, "xod_btd_solve: max_refine must be in 0..100");
  XOD_CHECK(!col->in_batch, "xod_btd_solve: column belongs to a batch");
  col->btd_iters = 0;
  col->btd_fallback = 0;
  col->btd_size = 0.0;
  const bool held = col->btd.valid && col->btd.B == B && col->btd.a == av &&
                    col->btd.c == cv && col->btd.solver == col->solver;
  if (!held) {
    // block Thomas in FP64 leaves its factors in the caller's arrays
    XOD_CHECK(col->solver == XOD_SOLVER_THOMAS && piv,
              "xod_btd_solve: no factorisation of this system is held by the column "
              "(call xod_btd_factor with the same B, a, c first)");
    XOD_HIP(launch_invperm(piv, col->rstep, col->N, col->ld, col->stream));
    ColArgs a = col->args();
    a.B = const_cast<double *>(B);
    a.a = const_cast<double *>(av);
    a.c = const_cast<double *>(cv);
    a.piv = const_cast<int *>(piv);
    a.x = rhs;
    XOD_HIP(launch_solve_fp64(OneCol{a}, 1, col->N, col->ld, col->stream));
    return XOD_OK;
  }
  if (col->btd.prec == XOD_FP64) return solve_own_fp64(col, rhs);

  // Mixed precision: FP32 solves of the row-scaled system, refined against
  // the caller's FP64 (B, a, c); FP64 refactorisation if refinement fails.
  const bool cr = col->solver == XOD_SOLVER_CR;
  const int N = col->N, S = col->S;
  const size_t NSb = (size_t)N * S * sizeof(double);
  ColArgs a = col->args();
  a.f = rhs;
  a.n = nullptr;          // an explicit system: corrections measured against x itself
  OneCol one{a};
  XOD_HIP(launch_scale(one, 1, N, S, col->stream));                     // x = s g
  if (cr)
    XOD_TRY(col->cr32->solve(col));
  else
    XOD_HIP(launch_solve_mixed(one, 1, N, col->ld, col->stream));
  XOD_HIP(hipMemcpyAsync(col->dx, col->x, NSb, hipMemcpyDeviceToDevice, col->stream));
  RefineNext verdict = max_refine == 0 ? kRefineDone : kRefineFallback;
  double prev = 1e300, size = 0.0;
  for (int it = 1; it <= max_refine; ++it) {
    XOD_HIP(launch_bt_resid(B, av, cv, rhs, col->dx, col->rs, N, S, col->ld, col->x,
                            col->stream));
    if (cr)
      XOD_TRY(col->cr32->solve(col));
    else
      XOD_HIP(launch_solve_mixed(one, 1, N, col->ld, col->stream));
    XOD_HIP(launch_axpy_ratio(one, 1, N, col->ratio, col->rmax, col->stream));
    XOD_HIP(hipMemcpyAsync(col->stats_host, col->rmax, sizeof(double), hipMemcpyDeviceToHost,
                           col->stream));
    XOD_HIP(hipStreamSynchronize(col->stream));
    size = col->stats_host[0];
    col->btd_iters = it;
    verdict = refine_next(size, prev, it, max_refine);
    if (verdict != kRefineMore) break;
    prev = size;
  }
  col->btd_size = size;
  if (verdict == kRefineDone) {
    XOD_HIP(hipMemcpyAsync(rhs, col->dx, NSb, hipMemcpyDeviceToDevice, col->stream));
    XOD_HIP(hipStreamSynchronize(col->stream));
    return XOD_OK;
  }
  // FP64 fallback: the column now holds FP64 factors of the same system
  col->btd_fallback = 1;
  XOD_TRY(factor_own_fp64(col, B, av, cv));
  XOD_TRY(read_singular_flag(col));
  col->btd.prec = XOD_FP64;
  XOD_TRY(solve_own_fp64(col, rhs));
  XOD_HIP(hipStreamSynchronize(col->stream));
  return XOD_OK;
}

extern "C" xod_status xod_btd_solve_info(const xod_column *col, int32_t *refine_iters,
                                         int32_t *fp64_fallback, double *correction) {
  XOD_CHECK(col, "xod_btd_solve_info: null column");
  if (refine_iters) *refine_iters = col->btd_iters;
  if (fp64_fallback) *fp64_fallback = col->btd_fallback;
  if (correction) *correction = col->btd_size;
  return XOD_OK;
}

// ---------------------------------------------------------------------------
// Backward-Euler step on the column's own buffers.
namespace xod {

size_t column_footprint(const xod_network *net, int N, xod_precision prec) {
  const size_t S = net->S, R = net->R, ld = net->ld, n = (size_t)N;
  size_t b = 0;
  b += 8 * (6 * n + 4 * n * S);                 // profile + grid vectors
  b += 8 * (6 * n * S);                         // n, ntmp, f, x, resid, dx
  b += 8 * (9 * n * R);                         // kf, kr, w, rate derivatives
  b += 8 * (4 * n * ld) + 4 * (2 * n * ld);     // gs, a, c, rs, piv, rstep
  b += 8 * n * ld * ld;                         // FP64 blocks
  if (prec == XOD_MIXED) b += 4 * n * ld * ld + 8 * 2 * n * ld;
  b += 64 * 1024;                               // statistics, flags, alignment
  return b;
}

xod_status enqueue_update(xod_column *c, bool clip, double y_floor, double y_sig, double y_neg) {
  UpdArgs &u = *c->upd_host;
  u = UpdArgs{};
  u.n = c->n;
  u.x = c->x;
  u.ngas = c->ngas;
  u.nout = c->ntmp;
  u.partial = c->partial;
  u.N = c->N;
  u.S = c->S;
  u.clip = clip ? 1 : 0;
  u.y_floor = y_floor;
  u.y_sig = y_sig;
  u.y_neg = y_neg;
  *c->red_host = RedArgs{c->partial, c->flag, c->stats_dev};
  XOD_HIP(hipMemcpyAsync(c->upd_dev, c->upd_host, sizeof(UpdArgs), hipMemcpyHostToDevice,
                         c->stream));
  XOD_HIP(hipMemcpyAsync(c->red_dev, c->red_host, sizeof(RedArgs), hipMemcpyHostToDevice,
                         c->stream));
  XOD_HIP(launch_update_state(c->upd_dev, c->red_dev, 1, c->stream));
  XOD_HIP(hipMemcpyAsync(c->stats_host, c->stats_dev, kStatLen * sizeof(double),
                         hipMemcpyDeviceToHost, c->stream));
  return XOD_OK;
}

xod_status run_update(xod_column *c, bool clip, double y_floor, double y_sig, double *out,
                      double y_neg) {
  XOD_TRY(enqueue_update(c, clip, y_floor, y_sig, y_neg));
  XOD_HIP(hipStreamSynchronize(c->stream));
  std::memcpy(out, c->stats_host, kStatLen * sizeof(double));
  return XOD_OK;
}

constexpr double kRefineKeepMost = 1e5;

// Iterative refinement of an FP64 solve with its own factors: the residual
// F - M delta in FP64 from the reaction list and the transport coefficients
// (no row scaling), a solve for the correction, delta += correction, a fixed
// options().refine64 times (no host round trip; batches do the same, so a
// column steps alike alone and in a batch).  The explicit inverses make the
// FP64 solve forward stable only: components far below their layer's
// largest increment carry errors of order cond(M) eps of that increment,
// and one correction brings them to the residual's rounding.  delta in
// c->x on entry and on return.
xod_status refine_fp64(xod_column *c, int *iters) {
  const size_t NSb = (size_t)c->N * c->S * sizeof(double);
  ColArgs a = c->args();
  a.rs = nullptr;
  OneCol one{a};
  const bool cr = c->solver == XOD_SOLVER_CR;
  XOD_HIP(hipMemcpyAsync(c->dx, c->x, NSb, hipMemcpyDeviceToDevice, c->stream));
  XOD_HIP(hipMemcpyAsync(c->resid, c->x, NSb, hipMemcpyDeviceToDevice, c->stream));
  for (int it = 1; it <= options().refine64; ++it) {
    XOD_HIP(launch_residual(one, 1, c->N, c->S, c->R, c->stream));
    if (cr)
      XOD_TRY(c->cr64->solve(c));
    else
      XOD_HIP(launch_solve_fp64(one, 1, c->N, c->ld, c->stream));
    XOD_HIP(launch_axpy_ratio(one, 1, c->N, c->ratio, c->rmax, c->stream));
    *iters = it;
  }
  // layers whose last correction exceeds 1e5 times the tolerance (about 1 %
  // of a density) keep the unrefined solution: there the factors' solve is
  // too inaccurate for a correction to help (nearly singular steps)
  XOD_HIP(launch_keep_refined(one, 1, c->N, c->S, c->ratio, kRefineKeepMost, c->stream));
  return XOD_OK;
}

xod_status enqueue_solve(xod_column *c, double dt, int *iters, int *fallback, double *resid,
                         const double *hist, double hist_coef) {
  const TunedScope tuned(c->ld, c->prec, c->solver, false);
  c->dt = dt;
  ColArgs a = c->args();
  OneCol one{a};
  *iters = 0;
  *fallback = 0;
  *resid = 0.0;
  XOD_TRY(enqueue_photolysis(c));
  XOD_HIP(launch_rates(one, 1, c->N, c->R, c->stream));
  XOD_HIP(launch_rhs(one, 1, c->N, c->R, c->S, c->stream));
  if (hist) {
    const size_t NS = (size_t)c->N * c->S;
    XOD_HIP(launch_lincomb(c->dx, c->n, 1.0, hist, -1.0, NS, c->stream));
    XOD_HIP(launch_lincomb(c->f, c->f, 1.0, c->dx, hist_coef, NS, c->stream));
  }
  const bool cr = c->solver == XOD_SOLVER_CR;
  c->fact_dt = 0.0;
  c->btd.valid = false;   // the column's blocks receive this step's matrix
  if (c->prec == XOD_FP64) {
    XOD_HIP(launch_jacobian(one, 1, c->N, c->R, c->ld, false, c->stream));
    if (cr)
      XOD_TRY(c->cr64->factor(c));
    else
      XOD_HIP(launch_factor_fp64(one, 1, c->N, c->ld, c->stream));
    XOD_HIP(hipMemcpyAsync(c->x, c->f, (size_t)c->N * c->S * sizeof(double),
                           hipMemcpyDeviceToDevice, c->stream));
    if (cr)
      XOD_TRY(c->cr64->solve(c));
    else
      XOD_HIP(launch_solve_fp64(one, 1, c->N, c->ld, c->stream));
    c->fact_dt = dt;
    if (options().refine64 > 0) XOD_TRY(refine_fp64(c, iters));
    return XOD_OK;
  }
  // Mixed precision: row-scaled FP32 Schur complements, FP64 refinement with a
  // matrix-free FP64 residual; FP64 refactorisation if refinement stalls.
  // Precision control: once a step of size dt_f fell back, the next
  // `mixed_sticky` steps of size >= dt_f go to FP64 directly (the FP32
  // factors of the larger, worse-conditioned steps would not converge
  // either), then one tries FP32 again; a step of size >= dt_f that
  // converges in FP32 clears dt_f.
  const size_t NSb = (size_t)c->N * c->S * sizeof(double);
  const int sticky = options().mixed_sticky;
  const bool direct = sticky > 0 && c->mixed_fb_dt > 0.0 && dt >= c->mixed_fb_dt &&
                      c->mixed_direct < sticky;
  if (direct) {
    ++c->mixed_direct;
  } else {
    XOD_HIP(launch_jacobian(one, 1, c->N, c->R, c->ld, true, c->stream));
    if (cr)
      XOD_TRY(c->cr32->factor(c));
    else
      XOD_HIP(launch_factor_mixed(one, 1, c->N, c->ld, c->stream));
    XOD_HIP(launch_scale(one, 1, c->N, c->S, c->stream));
    if (cr)
      XOD_TRY(c->cr32->solve(c));
    else
      XOD_HIP(launch_solve_mixed(one, 1, c->N, c->ld, c->stream));
    XOD_HIP(hipMemcpyAsync(c->dx, c->x, NSb, hipMemcpyDeviceToDevice, c->stream));
    RefineNext verdict = kRefineFallback;
    double prev = 1e300, ratio = 1e300;
    for (int it = 1; it <= c->max_refine; ++it) {
      XOD_HIP(launch_residual(one, 1, c->N, c->S, c->R, c->stream));
      if (cr)
        XOD_TRY(c->cr32->solve(c));
      else
        XOD_HIP(launch_solve_mixed(one, 1, c->N, c->ld, c->stream));
      XOD_HIP(launch_axpy_ratio(one, 1, c->N, c->ratio, c->rmax, c->stream));
      XOD_HIP(hipMemcpyAsync(c->stats_host, c->rmax, sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
      XOD_HIP(hipStreamSynchronize(c->stream));
      ratio = c->stats_host[0];
      *iters = it;
      verdict = refine_next(ratio, prev, it, c->max_refine);
      if (verdict != kRefineMore) break;
      prev = ratio;
    }
    const bool ok = verdict == kRefineDone;
    *resid = ratio;
    if (ok) {
      XOD_HIP(hipMemcpyAsync(c->x, c->dx, NSb, hipMemcpyDeviceToDevice, c->stream));
      if (dt >= c->mixed_fb_dt) c->mixed_fb_dt = 0.0;
      c->mixed_direct = 0;
      return XOD_OK;
    }
    c->mixed_fb_dt = c->mixed_fb_dt > 0.0 ? std::min(c->mixed_fb_dt, dt) : dt;
    c->mixed_direct = 0;
  }
  *fallback = 1;
  XOD_HIP(launch_jacobian(one, 1, c->N, c->R, c->ld, false, c->stream));
  if (cr)
    XOD_TRY(c->cr64->factor(c));
  else
    XOD_HIP(launch_factor_fp64(one, 1, c->N, c->ld, c->stream));
  XOD_HIP(hipMemcpyAsync(c->x, c->f, NSb, hipMemcpyDeviceToDevice, c->stream));
  if (cr)
    XOD_TRY(c->cr64->solve(c));
  else
    XOD_HIP(launch_solve_fp64(one, 1, c->N, c->ld, c->stream));
  if (options().refine64 > 0) {       // as an FP64 column's step
    int it64 = 0;
    XOD_TRY(refine_fp64(c, &it64));
  }
  return XOD_OK;
}

}  // namespace xod

extern "C" xod_status xod_step(xod_column *col, double dt, xod_step_stats *st) {
  XOD_CHECK(col, "xod_step: null column");
  XOD_CHECK(!col->in_batch, "xod_step: column belongs to a batch");
  XOD_CHECK(std::isfinite(dt) && dt > 0, "xod_step: dt must be > 0");
  int iters, fb;
  double res;
  XOD_TRY(enqueue_solve(col, dt, &iters, &fb, &res));
  double s[kStatLen];
  col->prev_dt = 0.0;   // ntmp is about to receive the new state
  XOD_TRY(run_update(col, false, 1e-30, 1e-10, s));
  XOD_TRY(check_flags(col, s + kNStat));
  if (st) {
    st->max_rel_change = s[0];
    st->min_ratio = s[1];
    st->resid_inf = res;
    st->refine_iters = iters;
    st->fp64_fallback = fb;
    st->nonfinite = s[5] > 0 ? 1 : 0;
  }
  if (s[5] > 0) {
    set_error("xod_step: non-finite state after the step");
    return XOD_ENONFINITE;
  }
  std::swap(col->n, col->ntmp);
  col->t += dt;
  col->dt = dt;
  col->prev_dt = dt;
  return XOD_OK;
}

extern "C" xod_status xod_step_frozen(xod_column *col, double dt, xod_step_stats *st) {
  XOD_CHECK(col, "xod_step_frozen: null column");
  XOD_CHECK(!col->in_batch, "xod_step_frozen: column belongs to a batch");
  XOD_CHECK(col->prec == XOD_FP64, "xod_step_frozen: FP64 columns only");
  XOD_CHECK(col->fact_dt > 0 && dt == col->fact_dt,
            "xod_step_frozen: dt must equal that of the held factorisation");
  ColArgs a = col->args();
  OneCol one{a};
  XOD_TRY(enqueue_photolysis(col));
  XOD_HIP(launch_rates(one, 1, col->N, col->R, col->stream));
  XOD_HIP(launch_rhs(one, 1, col->N, col->R, col->S, col->stream));
  XOD_HIP(hipMemcpyAsync(col->x, col->f, (size_t)col->N * col->S * sizeof(double),
                         hipMemcpyDeviceToDevice, col->stream));
  if (col->solver == XOD_SOLVER_CR)
    XOD_TRY(col->cr64->solve(col));
  else
    XOD_HIP(launch_solve_fp64(one, 1, col->N, col->ld, col->stream));
  double s[kStatLen];
  col->prev_dt = 0.0;   // ntmp is about to receive the new state
  XOD_TRY(run_update(col, false, 1e-30, 1e-10, s));
  XOD_TRY(check_flags(col, s + kNStat));
  if (st) {
    st->max_rel_change = s[0];
    st->min_ratio = s[1];
    st->resid_inf = 0.0;
    st->refine_iters = 0;
    st->fp64_fallback = 0;
    st->nonfinite = s[5] > 0 ? 1 : 0;
  }
  if (s[5] > 0) {
    set_error("xod_step_frozen: non-finite state after the step");
    return XOD_ENONFINITE;
  }
  std::swap(col->n, col->ntmp);
  col->t += dt;
  col->prev_dt = dt;
  return XOD_OK;
}

// Two-stage Rosenbrock step ROS2 (Verwer et al. 1999): one factorisation of
// M = I/(g dt) - J(n), g = 1 + 1/sqrt 2, and two solves.  With d_i = g dt k_i,
//   M d1 = F(n),   M d2 = F(n + d1/g) - 2 d1/(g dt),   n_new = n + (3 d1 + d2)/(2g).
// The stage state lives in ntmp (the update writes it only afterwards) and
// d1 in dx (used by the mixed-precision refinement only).
// x = the ROS2 increment (3 d1 + d2)/(2g) of the column's state (FP64).
static xod_status enqueue_ros2(xod_column *col, double dt) {
  const double g = 1.0 + 1.0 / std::sqrt(2.0);
  int iters, fb;
  double res;
  XOD_TRY(enqueue_solve(col, g * dt, &iters, &fb, &res));      // x = d1
  const size_t NS = (size_t)col->N * col->S;
  XOD_HIP(hipMemcpyAsync(col->dx, col->x, NS * sizeof(double), hipMemcpyDeviceToDevice,
                         col->stream));
  col->prev_dt = 0.0;   // the stage state goes to ntmp
  XOD_HIP(launch_lincomb(col->ntmp, col->n, 1.0, col->x, 1.0 / g, NS, col->stream));
  ColArgs a = col->args();
  a.n = col->ntmp;
  XOD_HIP(launch_rhs(OneCol{a}, 1, col->N, col->R, col->S, col->stream));   // f = F(stage)
  XOD_HIP(launch_lincomb(col->x, col->f, 1.0, col->dx, -2.0 / (g * dt), NS, col->stream));
  if (col->solver == XOD_SOLVER_CR)
    XOD_TRY(col->cr64->solve(col));
  else
    XOD_HIP(launch_solve_fp64(OneCol{col->args()}, 1, col->N, col->ld, col->stream));  // x = d2
  XOD_HIP(launch_lincomb(col->x, col->dx, 1.5 / g, col->x, 0.5 / g, NS, col->stream));
  return XOD_OK;
}

extern "C" xod_status xod_step_ros2(xod_column *col, double dt, xod_step_stats *st) {
  XOD_CHECK(col, "xod_step_ros2: null column");
  XOD_CHECK(!col->in_batch, "xod_step_ros2: column belongs to a batch");
  XOD_CHECK(col->prec == XOD_FP64, "xod_step_ros2: FP64 columns only");
  XOD_CHECK(std::isfinite(dt) && dt > 0, "xod_step_ros2: dt must be > 0");
  XOD_TRY(enqueue_ros2(col, dt));
  double s[kStatLen];
  col->prev_dt = 0.0;   // ntmp is about to receive the new state
  XOD_TRY(run_update(col, false, 1e-30, 1e-10, s));
  XOD_TRY(check_flags(col, s + kNStat));
  if (st) {
    st->max_rel_change = s[0];
    st->min_ratio = s[1];
    st->resid_inf = 0.0;
    st->refine_iters = 0;
    st->fp64_fallback = 0;
    st->nonfinite = s[5] > 0 ? 1 : 0;
  }
  if (s[5] > 0) {
    set_error("xod_step_ros2: non-finite state after the step");
    return XOD_ENONFINITE;
  }
  std::swap(col->n, col->ntmp);
  col->t += dt;
  col->dt = dt;
  col->prev_dt = dt;
  return XOD_OK;
}

// Backward Euler solved by modified Newton: the linearised step, then
// iters - 1 corrections with the same factorisation,
//   M delta = F(n + Delta) - Delta/dt,  Delta += delta,  M = I/dt - J(n).
// Delta is kept in dx, the corrected state n + Delta goes to ntmp.
extern "C" xod_status xod_step_newton(xod_column *col, double dt, int32_t iters,
                                      xod_step_stats *st) {
  XOD_CHECK(col, "xod_step_newton: null column");
  XOD_CHECK(!col->in_batch, "xod_step_newton: column belongs to a batch");
  XOD_CHECK(col->prec == XOD_FP64, "xod_step_newton: FP64 columns only");
  XOD_CHECK(std::isfinite(dt) && dt > 0, "xod_step_newton: dt must be > 0");
  XOD_CHECK(iters >= 1 && iters <= 64, "xod_step_newton: iters must be in 1..64");
  int it0, fb;
  double res;
  XOD_TRY(enqueue_solve(col, dt, &it0, &fb, &res));          // x = Delta
  const size_t NS = (size_t)col->N * col->S;
  col->prev_dt = 0.0;   // corrected states go to ntmp
  for (int it = 1; it < iters; ++it) {
    XOD_HIP(hipMemcpyAsync(col->dx, col->x, NS * sizeof(double), hipMemcpyDeviceToDevice,
                           col->stream));
    XOD_HIP(launch_lincomb(col->ntmp, col->n, 1.0, col->dx, 1.0, NS, col->stream));
    ColArgs a = col->args();
    a.n = col->ntmp;
    XOD_HIP(launch_rhs(OneCol{a}, 1, col->N, col->R, col->S, col->stream));
    XOD_HIP(launch_lincomb(col->x, col->f, 1.0, col->dx, -1.0 / dt, NS, col->stream));
    if (col->solver == XOD_SOLVER_CR)
      XOD_TRY(col->cr64->solve(col));
    else
      XOD_HIP(launch_solve_fp64(OneCol{col->args()}, 1, col->N, col->ld, col->stream));
    XOD_HIP(launch_lincomb(col->x, col->dx, 1.0, col->x, 1.0, NS, col->stream));
  }
  double s[kStatLen];
  XOD_TRY(run_update(col, false, 1e-30, 1e-10, s));
  XOD_TRY(check_flags(col, s + kNStat));
  if (st) {
    st->max_rel_change = s[0];
    st->min_ratio = s[1];
    st->resid_inf = 0.0;
    st->refine_iters = iters - 1;
    st->fp64_fallback = 0;
    st->nonfinite = s[5] > 0 ? 1 : 0;
  }
  if (s[5] > 0) {
    set_error("xod_step_newton: non-finite state after the step");
    return XOD_ENONFINITE;
  }
  std::swap(col->n, col->ntmp);
  col->t += dt;
  col->dt = dt;
  col->prev_dt = dt;
  return XOD_OK;
}

// Linearly implicit variable-step BDF2: with w = dt/dt_prev and
// h = (1+w)/(1+2w) dt,
//   (I/h - J(n)) Delta = F(n) + w^2/(1+2w) (n - n_prev) / h,   n <- n + Delta,
// n_prev being the starting state of the previous step, which the state
// swap leaves in ntmp.
extern "C" xod_status xod_step_bdf2(xod_column *col, double dt, xod_step_stats *st) {
  XOD_CHECK(col, "xod_step_bdf2: null column");
  XOD_CHECK(!col->in_batch, "xod_step_bdf2: column belongs to a batch");
  XOD_CHECK(std::isfinite(dt) && dt > 0, "xod_step_bdf2: dt must be > 0");
  XOD_CHECK(col->prev_dt > 0,
            "xod_step_bdf2: the previous step must be a completed step on this column");
  const double w = dt / col->prev_dt;
  const double h = (1.0 + w) / (1.0 + 2.0 * w) * dt;
  int iters, fb;
  double res;
  XOD_TRY(enqueue_solve(col, h, &iters, &fb, &res, col->ntmp, w * w / (1.0 + 2.0 * w) / h));
  double s[kStatLen];
  col->prev_dt = 0.0;   // ntmp is about to receive the new state
  XOD_TRY(run_update(col, false, 1e-30, 1e-10, s));
  XOD_TRY(check_flags(col, s + kNStat));
  if (st) {
    st->max_rel_change = s[0];
    st->min_ratio = s[1];
    st->resid_inf = res;
    st->refine_iters = iters;
    st->fp64_fallback = fb;
    st->nonfinite = s[5] > 0 ? 1 : 0;
  }
  if (s[5] > 0) {
    set_error("xod_step_bdf2: non-finite state after the step");
    return XOD_ENONFINITE;
  }
  std::swap(col->n, col->ntmp);
  col->t += dt;
  col->dt = dt;
  col->prev_dt = dt;
  return XOD_OK;
}

// One backward-Euler step of size dt on the factorisation the column holds
// (of an earlier state and step): modified Newton from Delta = 0,
//   Delta += M_f^-1 (F(n + Delta) - Delta/dt),
// until a correction is at most ntol of every new density with mixing ratio
// above y_sig (ok), or one is not below half the previous, or an iterate is
// not finite, or max_it corrections are spent (not ok).  Delta ends in
// c->x.  Rates are those of the step's start.
static xod_status newton_on_held(xod_column *c, double dt, double ntol, int max_it,
                                 double y_sig, bool *ok, int64_t *iters) {
  const size_t NS = (size_t)c->N * c->S;
  *ok = false;
  c->dt = dt;
  XOD_TRY(enqueue_photolysis(c));
  XOD_HIP(launch_rates(OneCol{c->args()}, 1, c->N, c->R, c->stream));
  XOD_HIP(hipMemsetAsync(c->dx, 0, NS * sizeof(double), c->stream));
  double prev = 1e300;
  for (int it = 1; it <= max_it; ++it) {
    XOD_HIP(launch_lincomb(c->ntmp, c->n, 1.0, c->dx, 1.0, NS, c->stream));   // n + Delta
    ColArgs a = c->args();
    a.n = c->ntmp;
    XOD_HIP(launch_rhs(OneCol{a}, 1, c->N, c->R, c->S, c->stream));          // f = F(n + Delta)
    XOD_HIP(launch_lincomb(c->x, c->f, 1.0, c->dx, -1.0 / dt, NS, c->stream));
    if (c->solver == XOD_SOLVER_CR)
      XOD_TRY(c->cr64->solve(c));
    else
      XOD_HIP(launch_solve_fp64(OneCol{c->args()}, 1, c->N, c->ld, c->stream));
    // Delta += correction; size = max |corr_i| / |n_i + Delta_i| over the
    // components with mixing ratio above y_sig (1e300 if any is not finite)
    XOD_HIP(launch_axpy_size(OneCol{c->args()}, 1, c->N, c->ratio, c->rmax, 1.0, 0.0, y_sig,
                             c->stream));
    XOD_HIP(hipMemcpyAsync(c->stats_host, c->rmax, sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
    XOD_HIP(hipStreamSynchronize(c->stream));
    ++*iters;
    const double size = c->stats_host[0];
    if (size <= ntol) {
      *ok = true;
      break;
    }
    if (!(size <= 0.5 * prev)) break;
    prev = size;
  }
  if (*ok)
    XOD_HIP(hipMemcpyAsync(c->x, c->dx, NS * sizeof(double), hipMemcpyDeviceToDevice,
                           c->stream));
  return XOD_OK;
}

extern "C" xod_status xod_integrate_to_steady_state(xod_column *col, const xod_ss_opts *o,
                                                    xod_ss_result *res) {
  XOD_CHECK(col && res, "xod_integrate_to_steady_state: null argument");
  XOD_CHECK(!col->in_batch, "xod_integrate_to_steady_state: column belongs to a batch");
  double tol = 1e-4, yfl = 1e-30, ysig = 1e-10, tend = 1e12, dt0 = 1e-8, yneg = 1e-6;
  int maxs = 5000, maxrej = 30, mixrule = 1, method = 0;
  if (o) {
    XOD_CHECK(o->method >= 0 && o->method <= 2,
              "xod_integrate_to_steady_state: method must be 0 (backward Euler), 1 (ROS2) "
              "or 2 (backward Euler with kept factorisations)");
    XOD_CHECK(o->method == 0 || col->prec == XOD_FP64,
              "xod_integrate_to_steady_state: methods 1 and 2 need an FP64 column");
    method = o->method;
    if (o->tol_rel > 0) tol = o->tol_rel;
    if (o->y_floor > 0) yfl = o->y_floor;
    if (o->y_sig > 0) ysig = o->y_sig;
    if (o->y_neg > 0) yneg = o->y_neg;
    if (o->t_end > 0) tend = o->t_end;
    if (o->dt0 > 0) dt0 = o->dt0;
    if (o->max_steps > 0) maxs = o->max_steps;
    if (o->max_consec_rejects > 0) maxrej = o->max_consec_rejects;
    mixrule = o->use_mix_rule;
  }
  col->prev_dt = 0.0;   // rejected steps leave their output in ntmp
  const double mix = mixrule ? col->mix_time : 0.0;
  double t = 0.0, dt = dt0, clipped = 0.0;
  int64_t steps = 0, rejects = 0, nnewton = 0;
  int consec = 0;
  int converged = 0, nfact = 0;
  // method 2: the held factorisation's step size and accepted steps
  constexpr double kReuseRatio = 1.3, kNewtonTol = 1e-3;
  constexpr int kMaxNewton = 4, kMaxAge = 20;
  bool held = false;
  double held_dt = 0.0;
  int held_age = 0;
  while (steps < maxs) {
    int iters, fb;
    double rr;
    if (method == 1) {
      XOD_TRY(enqueue_ros2(col, dt));
      ++nfact;
    } else if (method == 2) {
      const double ratio = held ? dt / held_dt : 0.0;
      const bool fresh = !held || !(ratio >= 1.0 / kReuseRatio && ratio <= kReuseRatio) ||
                         held_age >= kMaxAge;
      if (fresh) {
        XOD_TRY(enqueue_solve(col, dt, &iters, &fb, &rr));
        held = true;
        held_dt = dt;
        held_age = 0;
        ++nfact;
      } else {
        bool ok = false;
        XOD_TRY(newton_on_held(col, dt, kNewtonTol, kMaxNewton, ysig, &ok, &nnewton));
        if (!ok) {            // retry this step with a fresh factorisation
          held = false;
          continue;
        }
      }
    } else {
      XOD_TRY(enqueue_solve(col, dt, &iters, &fb, &rr));
      ++nfact;
    }
    double s[kStatLen];
    XOD_TRY(run_update(col, true, yfl, ysig, s, yneg));
    const bool singular = s[kNStat] >= 0;
    if (singular || s[5] > 0 || s[4] > 0) {
      ++rejects;
      ++consec;
      dt *= 0.5;
      if (consec > maxrej) break;
      continue;
    }
    consec = 0;
    clipped += s[3];
    std::swap(col->n, col->ntmp);
    t += dt;
    ++steps;
    ++held_age;
    const double rel = s[0], ctl = s[2];
    if ((rel < tol && dt >= mix) || t >= tend) {
      converged = 1;
      break;
    }
    dt *= ctl < 0.5 ? 2.0 : (ctl < 0.9 ? 1.2 : 0.7);
  }
  col->t = t;
  col->dt = dt;
  col->prev_dt = 0.0;
  res->t = t;
  res->dt = dt;
  res->clipped = clipped;
  res->steps = steps;
  res->rejects = rejects;
  res->converged = converged;
  res->factorizations = nfact;
  res->newton_iters = nnewton;
  if (method == 2) col->fact_dt = held ? held_dt : 0.0;   // of an earlier state
  if (!converged) {
    set_error("steady state not reached (step or rejection limit)");
    return XOD_ENOTCONVERGED;
  }
  return XOD_OK;
}

extern "C" xod_status xod_integrate_fixed_dt(xod_column *col, double dt, int32_t nsteps,
                                             int32_t reuse, xod_reuse_stats *st) {
  XOD_CHECK(col, "xod_integrate_fixed_dt: null column");
  XOD_CHECK(!col->in_batch, "xod_integrate_fixed_dt: column belongs to a batch");
  XOD_CHECK(std::isfinite(dt) && dt > 0, "xod_integrate_fixed_dt: dt must be > 0");
  XOD_CHECK(nsteps >= 0, "xod_integrate_fixed_dt: nsteps must be >= 0");
  XOD_CHECK(reuse == 0 || reuse == 1, "xod_integrate_fixed_dt: reuse must be 0 or 1");
  XOD_CHECK(reuse == 0 || col->prec == XOD_FP64,
            "xod_integrate_fixed_dt: reusing factorisations needs an FP64 column");
  constexpr double kNewtonTol = 1e-3, kYSig = 1e-10;
  constexpr int kMaxNewton = 4, kMaxAge = 20;
  int64_t nfact = 0, ncorr = 0, done = 0;
  bool held = false;
  int age = 0;
  col->prev_dt = 0.0;
  xod_status ret = XOD_OK;
  for (int32_t i = 0; i < nsteps; ++i) {
    bool ok = false;
    if (reuse && held && age < kMaxAge)
      XOD_TRY(newton_on_held(col, dt, kNewtonTol, kMaxNewton, kYSig, &ok, &ncorr));
    if (ok) {
      ++age;
    } else {
      int iters, fb;
      double rr;
      XOD_TRY(enqueue_solve(col, dt, &iters, &fb, &rr));
      held = true;
      age = 1;
      ++nfact;
    }
    double s[kStatLen];
    XOD_TRY(run_update(col, false, 1e-30, kYSig, s));
    XOD_TRY(check_flags(col, s + kNStat));
    if (s[5] > 0) {
      set_error("xod_integrate_fixed_dt: non-finite state at step " + std::to_string(i));
      ret = XOD_ENONFINITE;
      break;
    }
    std::swap(col->n, col->ntmp);
    col->t += dt;
    ++done;
  }
  col->dt = dt;
  col->prev_dt = 0.0;
  col->fact_dt = held ? dt : 0.0;   // of an earlier state when reused
  if (st) {
    st->steps = done;
    st->factorizations = nfact;
    st->newton_iters = ncorr;
  }
  return ret;
}
