// Block cyclic reduction plan of one column (host side).
#pragma once

#include <array>
#include <vector>

#include "handles.h"

#ifndef XOD_TRY
#define XOD_TRY(expr)            \
  do {                           \
    xod_status s_ = (expr);      \
    if (s_ != XOD_OK) return s_; \
  } while (0)
#endif

namespace xod {

struct CrLevel {
  int h;                       // layer stride of the level
  std::vector<int> elim, kept; // layers eliminated / kept at this level
};

// Levels of the reduction of N layers (empty for N = 1).
std::vector<CrLevel> cr_levels(int N);
// The layer left after the last level (inverted alone).
int cr_root(int N);
// Dense blocks the reduction needs besides the N diagonal blocks.
size_t cr_extra_blocks(int N);
// Scratch blocks of the library block-product path (gathered operands).
constexpr int kGatherBlocks = 64;

template <class T>
struct CrPlan {
  int N = 0, ld = 0;
  int *rstep_all = nullptr, *flag = nullptr;   // the column's pivot steps and flags
  std::vector<CrLevel> levels;
  std::vector<void *> owned;
  T *slots = nullptr;    // dense A / C blocks of even layers, then T1 / T2 products
  double *xs = nullptr;  // padded solution [N*ld]
  MatRef<T> *d_inv = nullptr;
  CrLevel0Op<T> *d_l0 = nullptr;
  GemmOp<T> *d_g = nullptr;
  MvOp<T> *d_mv = nullptr;
  int l0_cnt = 0, root_off = 0;
  std::vector<int> inv_off, inv_cnt, g1_off, g1_cnt, g2_off, g2_cnt;
  std::vector<int> fwd_off, fwd_cnt, bwd1_off, bwd1_cnt, bwd2_off, bwd2_cnt;

  // Library block products (option gemm_lib): each product launch becomes
  // pieces, each a row gather of its products' gathered operands into the
  // scratch blocks gtemp, then one rocBLAS batched GEMM of products sharing
  // (alpha, beta).
  struct BlasPiece {
    int gat_off, gat_cnt;   // into d_gat
    int ptr_off, count;     // into the device pointer arrays
    double alpha, beta;
  };
  std::vector<std::vector<BlasPiece>> pieces_g1, pieces_g2;   // per level
  GatherOp<T> *d_gat = nullptr;
  const T **d_pa = nullptr, **d_pb = nullptr;
  T **d_pc = nullptr;
  T *gtemp = nullptr;
  void *blas = nullptr;   // rocblas_handle

  // captured launch sequences (kernel nodes only), replayed on the
  // column's stream; built on first use with the options then in force
  hipStream_t cap = nullptr;   // capture stream
  hipGraphExec_t gfactor = nullptr, gsolve = nullptr;
  std::array<int, 11> graph_gemm{};   // the kernel options the graphs were captured with
  bool graph_valid = false;

  ~CrPlan();
  // Device descriptors for the column's buffers (blocks, couplings, pivots).
  xod_status build(xod_column *c);
  // Factor the blocks in place (enqueued on the column's stream).
  xod_status factor(xod_column *c);
  // Solve with the factors: c->x [N*S] in, solution out.
  xod_status solve(xod_column *c);

 private:
  template <class U>
  xod_status upload(U **dst, const std::vector<U> &v);
  xod_status enqueue_factor(hipStream_t s);
  xod_status enqueue_solve(hipStream_t s, xod_column *c);
  xod_status replay(hipGraphExec_t *g, bool factor, xod_column *c);
  xod_status build_lib(const std::vector<GemmOp<T>> &gops);
  xod_status enqueue_gemm_lib(const std::vector<BlasPiece> &pieces, hipStream_t s);
};

}  // namespace xod
