// Block cyclic reduction of one column's block-tridiagonal step system.
//
// Level l (h = 2^l) works on the layers that are multiples of h.  Those with
// k/h odd are eliminated: their diagonal blocks are inverted (all of them in
// one batched Gauss-Jordan launch sequence) and folded into their kept
// neighbours k -+ h:
//   D_k <- D_k - A_k E_{k-h} C_{k-h} - C_k E_{k+h} A_{k+h}
//   A_k <- -A_k E_{k-h} A_{k-h},   C_k <- -C_k E_{k+h} C_{k+h}
//   g_k <- g_k - A_k E_{k-h} g_{k-h} - C_k E_{k+h} g_{k+h}
// until one layer, the root, remains: layer 0, or the middle one when the
// last level takes both ends of {0, h, 2h}.  Back substitution runs the
// levels in reverse:
//   x_k = E_k (g_k - A_k x_{k-h} - C_k x_{k+h})  for the eliminated layers.
// The result is the solution of the same block system as block Thomas (both
// are block Gaussian elimination, in different orders); the critical path is
// at most ceil(log2 N) + 1 block inversions instead of N.
//
// Storage besides the blocks themselves: dense A / C blocks for the even
// layers (levels >= 1 have dense couplings), the products T1 = A_k E_{k-h}
// and T2 = C_k E_{k+h} of every level >= 1 (kept for the right-hand-side
// reduction), and a padded solution vector.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <memory>
#include <vector>

#include <rocblas/rocblas.h>

#include "cr.h"
#include "tune.h"

namespace xod {

template <class T>
static T *col_blocks(xod_column *c);
template <>
double *col_blocks<double>(xod_column *c) { return c->B; }
template <>
float *col_blocks<float>(xod_column *c) { return c->Bf; }

template <class T>
template <class U>
xod_status CrPlan<T>::upload(U **dst, const std::vector<U> &v) {
  *dst = nullptr;
  if (v.empty()) return XOD_OK;
  XOD_HIP(hipMalloc((void **)dst, v.size() * sizeof(U)));
  owned.push_back(*dst);
  XOD_HIP(hipMemcpy(*dst, v.data(), v.size() * sizeof(U), hipMemcpyHostToDevice));
  return XOD_OK;
}

template <class T>
CrPlan<T>::~CrPlan() {
  if (blas) (void)rocblas_destroy_handle((rocblas_handle)blas);
  if (gfactor) (void)hipGraphExecDestroy(gfactor);
  if (gsolve) (void)hipGraphExecDestroy(gsolve);
  if (cap) (void)hipStreamDestroy(cap);
  for (void *p : owned) (void)hipFree(p);
}

std::vector<CrLevel> cr_levels(int N) {
  std::vector<CrLevel> out;
  std::vector<int> rem(N);
  for (int k = 0; k < N; ++k) rem[k] = k;
  int h = 1;
  while (rem.size() > 1) {
    CrLevel L;
    L.h = h;
    if (rem.size() == 3 && h > 1) {
      // {0, h, 2h}: both ends go at once (neither couples to the other) and
      // the middle layer is the root, one level sooner than keeping layer 0
      L.elim = {rem[0], rem[2]};
      L.kept = {rem[1]};
    } else {
      for (int k : rem) ((k / h) % 2 ? L.elim : L.kept).push_back(k);
    }
    rem = L.kept;
    out.push_back(L);
    h *= 2;
  }
  return out;
}

int cr_root(int N) {
  const std::vector<CrLevel> lv = cr_levels(N);
  return lv.empty() ? 0 : lv.back().kept[0];
}

size_t cr_extra_blocks(int N) {
  size_t n = 2 * (size_t)((N + 1) / 2);   // A and C of the even layers
  for (const CrLevel &L : cr_levels(N)) {
    if (L.h == 1) continue;
    for (int k : L.kept) n += (k - L.h >= 0) + (k + L.h <= N - 1);
  }
  return n;
}

size_t cr_footprint(const xod_network *net, int N, xod_precision prec) {
  const size_t ld = net->ld, bs = ld * ld;
  const size_t nblk = std::max<size_t>(cr_extra_blocks(N), 1) + (N > 2 ? kGatherBlocks : 0);
  const size_t per = (size_t)N * ld * sizeof(double) + 1024 * (size_t)N + 64 * 1024;
  size_t b = nblk * bs * sizeof(double) + per;                   // FP64 workspace
  if (prec == XOD_MIXED) b += nblk * bs * sizeof(float) + per;   // + FP32 workspace
  return b;
}

template <class T>
xod_status CrPlan<T>::build(xod_column *c) {
  N = c->N;
  ld = c->ld;
  rstep_all = c->rstep;
  flag = c->flag;
  levels = cr_levels(N);
  const size_t bs = (size_t)ld * ld;
  T *blk0 = col_blocks<T>(c);
  auto blk = [&](int k) { return blk0 + (size_t)k * bs; };
  auto pv = [&](int k) { return c->piv + (size_t)k * ld; };
  auto rq = [&](int k) { return c->rstep + (size_t)k * ld; };
  auto av = [&](int k) { return c->a + (size_t)k * ld; };
  auto cv = [&](int k) { return c->c + (size_t)k * ld; };
  auto gsv = [&](int k) { return c->gs + (size_t)k * ld; };

  const size_t nslot = cr_extra_blocks(N);
  XOD_HIP(hipMalloc((void **)&slots, std::max<size_t>(nslot, 1) * bs * sizeof(T)));
  owned.push_back(slots);
  XOD_HIP(hipMalloc((void **)&xs, (size_t)N * ld * sizeof(double)));
  owned.push_back(xs);
  auto aslot = [&](int k) { return slots + (size_t)(k / 2) * 2 * bs; };
  auto cslot = [&](int k) { return slots + ((size_t)(k / 2) * 2 + 1) * bs; };
  size_t next_t = 2 * (size_t)((N + 1) / 2);
  auto xsv = [&](int k) { return xs + (size_t)k * ld; };

  std::vector<MatRef<T>> inv;
  std::vector<CrLevel0Op<T>> l0;
  std::vector<GemmOp<T>> gops;
  std::vector<MvOp<T>> mv;
  const int nlev = (int)levels.size();
  inv_off.assign(nlev + 1, 0);
  inv_cnt.assign(nlev + 1, 0);
  g1_off.assign(nlev, 0);
  g1_cnt.assign(nlev, 0);
  g2_off.assign(nlev, 0);
  g2_cnt.assign(nlev, 0);
  fwd_off.assign(nlev, 0);
  fwd_cnt.assign(nlev, 0);
  bwd1_off.assign(nlev, 0);
  bwd1_cnt.assign(nlev, 0);
  bwd2_off.assign(nlev, 0);
  bwd2_cnt.assign(nlev, 0);
  // T1 / T2 slot of (level, kept layer)
  std::vector<std::vector<T *>> t1(nlev, std::vector<T *>(N, nullptr)),
      t2(nlev, std::vector<T *>(N, nullptr));

  for (int l = 0; l < nlev; ++l) {
    const CrLevel &L = levels[l];
    const int h = L.h;
    inv_off[l] = (int)inv.size();
    for (int k : L.elim) inv.push_back(MatRef<T>{blk(k), pv(k), rq(k), c->flag, k});
    inv_cnt[l] = (int)L.elim.size();
    if (l == 0) {
      for (int k : L.kept) {
        const bool hl = k - 1 >= 0, hr = k + 1 <= N - 1;
        if (!hl && !hr) continue;
        CrLevel0Op<T> o{};
        o.D = blk(k);
        o.A = (k - 2 >= 0) ? aslot(k) : nullptr;
        o.C = (k + 2 <= N - 1) ? cslot(k) : nullptr;
        o.ak = av(k);
        o.ck = cv(k);
        if (hl) {
          o.Wl = blk(k - 1);
          o.pl = pv(k - 1);
          o.ql = rq(k - 1);
          o.al = av(k - 1);
          o.cl = cv(k - 1);
        }
        if (hr) {
          o.Wr = blk(k + 1);
          o.pr = pv(k + 1);
          o.qr = rq(k + 1);
          o.ar = av(k + 1);
          o.cr = cv(k + 1);
        }
        l0.push_back(o);
      }
    } else {
      g1_off[l] = (int)gops.size();
      for (int k : L.kept) {
        if (k - h >= 0) {
          t1[l][k] = slots + next_t++ * bs;
          gops.push_back(GemmOp<T>{aslot(k), blk(k - h), pv(k - h), nullptr, nullptr, nullptr,
                                   t1[l][k], 1.0, 0});
        }
        if (k + h <= N - 1) {
          t2[l][k] = slots + next_t++ * bs;
          gops.push_back(GemmOp<T>{cslot(k), blk(k + h), pv(k + h), nullptr, nullptr, nullptr,
                                   t2[l][k], 1.0, 0});
        }
      }
      g1_cnt[l] = (int)gops.size() - g1_off[l];
      g2_off[l] = (int)gops.size();
      for (int k : L.kept) {
        const int kl = k - h, kr = k + h;
        const bool hl = kl >= 0, hr = kr <= N - 1;
        if (hl && hr)
          gops.push_back(GemmOp<T>{t1[l][k], cslot(kl), pv(kl), t2[l][k], aslot(kr), pv(kr),
                                   blk(k), -1.0, 1});
        else if (hl)
          gops.push_back(GemmOp<T>{t1[l][k], cslot(kl), pv(kl), nullptr, nullptr, nullptr, blk(k),
                                   -1.0, 1});
        else if (hr)
          gops.push_back(GemmOp<T>{t2[l][k], aslot(kr), pv(kr), nullptr, nullptr, nullptr, blk(k),
                                   -1.0, 1});
        if (k - 2 * h >= 0)
          gops.push_back(GemmOp<T>{t1[l][k], aslot(kl), pv(kl), nullptr, nullptr, nullptr,
                                   aslot(k), -1.0, 0});
        if (k + 2 * h <= N - 1)
          gops.push_back(GemmOp<T>{t2[l][k], cslot(kr), pv(kr), nullptr, nullptr, nullptr,
                                   cslot(k), -1.0, 0});
      }
      g2_cnt[l] = (int)gops.size() - g2_off[l];
    }
    // right-hand-side reduction of this level
    fwd_off[l] = (int)mv.size();
    for (int k : L.kept) {
      const int kl = k - h, kr = k + h;
      MvOp<T> o{};
      o.b = gsv(k);
      o.y = gsv(k);
      if (kl >= 0) {
        o.t[o.nterm++] = (l == 0)
            ? MvTerm<T>{blk(kl), pv(kl), pv(kl), gsv(kl), av(k), -1.0}
            : MvTerm<T>{t1[l][k], nullptr, pv(kl), gsv(kl), nullptr, -1.0};
      }
      if (kr <= N - 1) {
        o.t[o.nterm++] = (l == 0)
            ? MvTerm<T>{blk(kr), pv(kr), pv(kr), gsv(kr), cv(k), -1.0}
            : MvTerm<T>{t2[l][k], nullptr, pv(kr), gsv(kr), nullptr, -1.0};
      }
      if (o.nterm) mv.push_back(o);
    }
    fwd_cnt[l] = (int)mv.size() - fwd_off[l];
  }
  // root
  const int root = cr_root(N);
  inv_off[nlev] = (int)inv.size();
  inv.push_back(MatRef<T>{blk(root), pv(root), rq(root), c->flag, root});
  inv_cnt[nlev] = 1;
  root_off = (int)mv.size();
  {
    MvOp<T> o{};
    o.y = xsv(root);
    o.t[o.nterm++] = MvTerm<T>{blk(root), pv(root), pv(root), gsv(root), nullptr, 1.0};
    mv.push_back(o);
  }
  // back substitution, per level
  for (int l = 0; l < nlev; ++l) {
    const CrLevel &L = levels[l];
    const int h = L.h;
    bwd1_off[l] = (int)mv.size();
    for (int k : L.elim) {
      MvOp<T> o{};
      o.b = gsv(k);
      o.y = gsv(k);
      if (k - h >= 0)
        o.t[o.nterm++] = (l == 0)
            ? MvTerm<T>{nullptr, nullptr, nullptr, xsv(k - 1), av(k), -1.0}
            : MvTerm<T>{aslot(k), nullptr, nullptr, xsv(k - h), nullptr, -1.0};
      if (k + h <= N - 1)
        o.t[o.nterm++] = (l == 0)
            ? MvTerm<T>{nullptr, nullptr, nullptr, xsv(k + 1), cv(k), -1.0}
            : MvTerm<T>{cslot(k), nullptr, nullptr, xsv(k + h), nullptr, -1.0};
      mv.push_back(o);
    }
    bwd1_cnt[l] = (int)mv.size() - bwd1_off[l];
    bwd2_off[l] = (int)mv.size();
    for (int k : L.elim) {
      MvOp<T> o{};
      o.y = xsv(k);
      o.t[o.nterm++] = MvTerm<T>{blk(k), pv(k), pv(k), gsv(k), nullptr, 1.0};
      mv.push_back(o);
    }
    bwd2_cnt[l] = (int)mv.size() - bwd2_off[l];
  }
  l0_cnt = (int)l0.size();
  XOD_TRY(upload(&d_inv, inv));
  XOD_TRY(upload(&d_l0, l0));
  XOD_TRY(upload(&d_g, gops));
  XOD_TRY(upload(&d_mv, mv));
  return build_lib(gops);
}

template <class T>
xod_status CrPlan<T>::build_lib(const std::vector<GemmOp<T>> &gops) {
  const int nlev = (int)levels.size();
  pieces_g1.assign(nlev, {});
  pieces_g2.assign(nlev, {});
  if (gops.empty()) return XOD_OK;
  const size_t bs = (size_t)ld * ld;
  XOD_HIP(hipMalloc((void **)&gtemp, (size_t)kGatherBlocks * bs * sizeof(T)));
  owned.push_back(gtemp);
  std::vector<GatherOp<T>> gat;
  std::vector<const T *> pa, pb;
  std::vector<T *> pc;
  struct Term {
    const T *A, *B;
    const int *bg;
    T *C;
    double alpha, beta;
  };
  // One product launch: its first terms grouped by (alpha, beta), then the
  // second terms (accumulated onto the first, beta = 1); cut into pieces of
  // at most kGatherBlocks gathered operands.
  auto split = [&](int off, int cnt, std::vector<BlasPiece> &out) {
    std::vector<Term> first, second;
    for (int i = off; i < off + cnt; ++i) {
      const GemmOp<T> &g = gops[i];
      first.push_back(Term{g.A, g.B, g.bg, g.C, g.alpha, g.beta ? 1.0 : 0.0});
      if (g.A2) second.push_back(Term{g.A2, g.B2, g.bg2, g.C, g.alpha, 1.0});
    }
    std::stable_sort(first.begin(), first.end(), [](const Term &a, const Term &b) {
      return a.alpha != b.alpha ? a.alpha < b.alpha : a.beta < b.beta;
    });
    std::vector<Term> seq = first;
    seq.insert(seq.end(), second.begin(), second.end());
    BlasPiece cur{};
    bool open = false;
    for (const Term &t : seq) {
      if (open && (t.alpha != cur.alpha || t.beta != cur.beta ||
                   (t.bg && cur.gat_cnt == kGatherBlocks))) {
        out.push_back(cur);
        open = false;
      }
      if (!open) {
        cur = BlasPiece{(int)gat.size(), 0, (int)pa.size(), 0, t.alpha, t.beta};
        open = true;
      }
      const T *B = t.B;
      if (t.bg) {
        T *dst = gtemp + (size_t)cur.gat_cnt * bs;
        gat.push_back(GatherOp<T>{t.B, t.bg, dst});
        ++cur.gat_cnt;
        B = dst;
      }
      pa.push_back(t.A);
      pb.push_back(B);
      pc.push_back(t.C);
      ++cur.count;
    }
    if (open) out.push_back(cur);
  };
  for (int l = 1; l < nlev; ++l) {
    split(g1_off[l], g1_cnt[l], pieces_g1[l]);
    split(g2_off[l], g2_cnt[l], pieces_g2[l]);
  }
  XOD_TRY(upload(&d_gat, gat));
  XOD_TRY(upload(&d_pa, pa));
  XOD_TRY(upload(&d_pb, pb));
  XOD_TRY(upload(&d_pc, pc));
  rocblas_handle h = nullptr;
  if (rocblas_create_handle(&h) != rocblas_status_success) {
    set_error("rocblas_create_handle failed");
    return XOD_EHIP;
  }
  blas = h;
  return XOD_OK;
}

// C = alpha A B + beta C on row-major ld x ld blocks: in rocBLAS's
// column-major terms C^T = alpha B^T A^T + beta C^T.
static rocblas_status blas_gemm(rocblas_handle h, int ld, double alpha, const double *const *A,
                                const double *const *B, double beta, double *const *C, int n) {
  return rocblas_dgemm_batched(h, rocblas_operation_none, rocblas_operation_none, ld, ld, ld,
                               &alpha, B, ld, A, ld, &beta, C, ld, n);
}
static rocblas_status blas_gemm(rocblas_handle h, int ld, double alpha, const float *const *A,
                                const float *const *B, double beta, float *const *C, int n) {
  const float a = (float)alpha, b = (float)beta;
  return rocblas_sgemm_batched(h, rocblas_operation_none, rocblas_operation_none, ld, ld, ld, &a,
                               B, ld, A, ld, &b, C, ld, n);
}

template <class T>
xod_status CrPlan<T>::enqueue_gemm_lib(const std::vector<BlasPiece> &pcs, hipStream_t s) {
  rocblas_handle h = (rocblas_handle)blas;
  if (rocblas_set_stream(h, s) != rocblas_status_success) {
    set_error("rocblas_set_stream failed");
    return XOD_EHIP;
  }
  const bool prof = options().profile != 0;
  for (const BlasPiece &p : pcs) {
    XOD_HIP(launch_gather_rows<T>(d_gat + p.gat_off, p.gat_cnt, ld, s));
    if (prof) prof_begin(kProfGemm, s);
    const rocblas_status st = blas_gemm(h, ld, p.alpha, d_pa + p.ptr_off, d_pb + p.ptr_off, p.beta,
                                        d_pc + p.ptr_off, p.count);
    if (prof) prof_end(kProfGemm, s);
    if (st != rocblas_status_success) {
      set_error("rocBLAS batched GEMM failed");
      return XOD_EHIP;
    }
  }
  return XOD_OK;
}

template <class T>
xod_status CrPlan<T>::enqueue_factor(hipStream_t s) {
  XOD_HIP(launch_cr_reset(rstep_all, (size_t)N * ld, flag, s));
  const int nlev = (int)levels.size();
  for (int l = 0; l < nlev; ++l) {
    XOD_HIP(launch_invert_list<T>(d_inv + inv_off[l], inv_cnt[l], ld, s));
    if (l == 0) {
      XOD_HIP(launch_cr_level0<T>(d_l0, l0_cnt, ld, s));
    } else {
      if (options().gemm_lib) {
        XOD_TRY(enqueue_gemm_lib(pieces_g1[l], s));
        XOD_TRY(enqueue_gemm_lib(pieces_g2[l], s));
      } else {
        XOD_HIP(launch_gemm<T>(d_g + g1_off[l], g1_cnt[l], ld, s));
        XOD_HIP(launch_gemm<T>(d_g + g2_off[l], g2_cnt[l], ld, s));
      }
    }
  }
  XOD_HIP(launch_invert_list<T>(d_inv + inv_off[nlev], 1, ld, s));
  return XOD_OK;
}

template <class T>
xod_status CrPlan<T>::enqueue_solve(hipStream_t s, xod_column *c) {
  XOD_HIP(launch_pad_copy(c->x, c->gs, N, c->S, ld, true, s));
  const int nlev = (int)levels.size();
  for (int l = 0; l < nlev; ++l) XOD_HIP(launch_mv<T>(d_mv + fwd_off[l], fwd_cnt[l], ld, s));
  XOD_HIP(launch_mv<T>(d_mv + root_off, 1, ld, s));
  for (int l = nlev - 1; l >= 0; --l) {
    XOD_HIP(launch_mv<T>(d_mv + bwd1_off[l], bwd1_cnt[l], ld, s));
    XOD_HIP(launch_mv<T>(d_mv + bwd2_off[l], bwd2_cnt[l], ld, s));
  }
  XOD_HIP(launch_pad_copy(xs, c->x, N, c->S, ld, false, s));
  return XOD_OK;
}

// Capture the launch sequence once on a private stream (capture needs a
// stream other than the legacy default one), then replay it on the column's
// stream.  The graphs hold kernel nodes only.
template <class T>
xod_status CrPlan<T>::replay(hipGraphExec_t *g, bool factor, xod_column *c) {
  const Options &o = options();
  const std::array<int, 11> key = {o.outer_nmat, o.outer,      o.gemm_k,     o.panel_sync,
                                   o.gemm_lib,   o.gemm_large, o.gemm_mfma,  o.update32,
                                   o.update32_min, o.gemm_waves, o.panel_defer};
  if (!graph_valid || graph_gemm != key) {
    graph_valid = true;
    if (gfactor) XOD_HIP(hipGraphExecDestroy(gfactor));
    if (gsolve) XOD_HIP(hipGraphExecDestroy(gsolve));
    gfactor = gsolve = nullptr;
    graph_gemm = key;
  }
  if (!*g) {
    if (!cap) XOD_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    XOD_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    const xod_status st = factor ? enqueue_factor(cap) : enqueue_solve(cap, c);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(cap, &graph);
    if (st != XOD_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    XOD_HIP(e);
    const hipError_t ei = hipGraphInstantiate(g, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    XOD_HIP(ei);
  }
  XOD_HIP(hipGraphLaunch(*g, c->stream));
  return XOD_OK;
}

template <class T>
xod_status CrPlan<T>::factor(xod_column *c) {
  const TunedScope tuned(c->ld, c->prec, XOD_SOLVER_CR, false);
  if (options().graph && !options().profile) return replay(&gfactor, true, c);
  return enqueue_factor(c->stream);
}

template <class T>
xod_status CrPlan<T>::solve(xod_column *c) {
  const TunedScope tuned(c->ld, c->prec, XOD_SOLVER_CR, false);
  if (options().graph && !options().profile) return replay(&gsolve, false, c);
  return enqueue_solve(c->stream, c);
}

template struct CrPlan<double>;
template struct CrPlan<float>;

void cr_destroy(CrPlan<double> *p) { delete p; }
void cr_destroy(CrPlan<float> *p) { delete p; }

}  // namespace xod
