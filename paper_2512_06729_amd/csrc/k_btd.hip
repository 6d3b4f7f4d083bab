// Block Thomas elimination of the block-tridiagonal step system (FP64).
//
// For k = 0..N-1 the Schur complement
//     D'_k = B_k - diag(a_k) D'_{k-1}^{-1} diag(c_{k-1})
// is inverted in place by blocked Gauss-Jordan elimination with implicit
// partial pivoting (rows are never moved; piv[j] records the row chosen for
// column j, rstep[r] the column at which row r became a pivot).  With W the
// in-place result, D'^{-1}[j][i] = W[piv[j]][rstep[i]].
//
// Per layer:
//   k_prologue   D'_k from B_k and the previous layer's inverse (gather)
//   per panel of kNB columns:
//     k_panel    one work-group factors the ld x kNB panel in registers
//                (pivot: largest magnitude among unused rows, compared to
//                42 mantissa bits, lowest row among equals)
//     k_update   Schur update of every other column strip:
//                C <- mask * C + W[:, J] U,  U = W[piv[J], strip]
//                (rows that became pivots in this panel are replaced, the
//                others accumulate), FP64 MFMA 16x16x4 or VALU FMA.
// The solve is a chain of matrix-vector products with the stored inverses.
#include "xod_internal.h"
#include "mfma.h"

#include <algorithm>
#include <climits>
#include <type_traits>

namespace xod {

// Block storage: FP64 blocks (c.B) or FP32 row-scaled blocks (c.Bf).
template <class T> __device__ __forceinline__ T *blocks(const ColArgs &c);
template <> __device__ __forceinline__ double *blocks<double>(const ColArgs &c) { return c.B; }
template <> __device__ __forceinline__ float *blocks<float>(const ColArgs &c) { return c.Bf; }

// ---------------------------------------------------------------------------
template <class Acc>
__global__ void __launch_bounds__(256) k_rstep_init(Acc acc, int maxN) {
  const ColArgs &c = acc(blockIdx.y);
  const size_t total = (size_t)c.N * c.ld;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x)
    c.rstep[e] = INT_MAX;
  if (blockIdx.x == 0 && threadIdx.x < 4) c.flag[threadIdx.x] = -1;
}

// D'_k[i][j] = B_k[i][j] - a_k[i] W_{k-1}[piv_{k-1}[i]][rstep_{k-1}[j]] c_{k-1}[j]
// One work-group per 8 rows of one column; the source rows are contiguous.
template <class Acc, class T>
__global__ void __launch_bounds__(256) k_prologue(Acc acc, int k) {
  const ColArgs &c = acc(blockIdx.y);
  if (k >= c.N || k == 0) return;
  const int ld = c.ld;
  const int *pv = c.piv + (size_t)(k - 1) * ld;
  const int *rq = c.rstep + (size_t)(k - 1) * ld;
  const T *W = blocks<T>(c) + (size_t)(k - 1) * ld * ld;
  T *D = blocks<T>(c) + (size_t)k * ld * ld;
  const double *ak = c.a + (size_t)k * ld;
  const double *cp = c.c + (size_t)(k - 1) * ld;
  const int r0 = blockIdx.x * 8;
  for (int rr = 0; rr < 8; ++rr) {
    const int i = r0 + rr;
    if (i >= ld) break;
    const double ai = ak[i];
    if (ai == 0.0) continue;
    const T *src = W + (size_t)pv[i] * ld;
    T *dst = D + (size_t)i * ld;
    for (int j = threadIdx.x; j < ld; j += blockDim.x) {
      const double cj = cp[j];
      if (cj != 0.0) dst[j] = (T)((double)dst[j] - ai * (double)src[rq[j]] * cj);
    }
  }
}

// ---------------------------------------------------------------------------
// The blocks a Gauss-Jordan launch works on.  Block Thomas: layer k of each
// column in the launch (work-group index b = column).  Lists: entry base + b
// of a device array of MatRef (the layers of one cyclic-reduction level).
template <class Acc, class T>
struct ThomasMats {
  Acc acc;
  __device__ __forceinline__ bool operator()(int b, int k, MatRef<T> &m) const {
    const ColArgs &c = acc(b);
    if (k >= c.N) return false;
    const size_t ld = c.ld;
    m.W = blocks<T>(c) + (size_t)k * ld * ld;
    m.piv = c.piv + (size_t)k * ld;
    m.rstep = c.rstep + (size_t)k * ld;
    m.flag = c.flag;
    m.id = k;
    return true;
  }
};
template <class T>
struct ListMats {
  const MatRef<T> *list;
  __device__ __forceinline__ bool operator()(int b, int base, MatRef<T> &m) const {
    m = list[base + b];
    return true;
  }
};

// ---------------------------------------------------------------------------
// Panel factorisation: Gauss-Jordan on the ld x kNB panel of one block, with
// implicit partial pivoting.
//
// Thread t owns rows R*t .. R*t+R-1 as register vectors (64*ceil(ld/128)
// threads).  Per column:
//   - every unused row forms a key: |x| with its 10 lowest mantissa bits
//     replaced by (1023 - row), so the largest key is the largest magnitude
//     (to 42 mantissa bits) and, among equals, the lowest row; used rows
//     give 0;
//   - a DPP max gives each wave's best key, lane 0 stores it in LDS;
//   - after a barrier every lane reduces the wave keys: the maximum names
//     the pivot row; its owning lane stores the row in LDS (16-byte stores)
//     with the reciprocal of its pivot entry in the pivot column's slot;
//   - after a second barrier every thread reads the row and updates its own.
// (Option panel_sync = 1: every wave publishes its best row before a single
// barrier instead.)  LDS buffers alternate with the column parity.
// Pivot rows are kept unscaled while the panel runs (the elimination update
// is linear in each row, so scaling commutes with it): the pivot row's own
// column is set to 1 and the row is multiplied by its reciprocal pivot when
// the panel is written back.  The loop touches no global memory.
constexpr int kPanelRows = 2;                               // rows per thread
constexpr int kPanelWaves = kMaxLd / (64 * kPanelRows);     // up to 8 waves
constexpr int kGroup = 8;                                   // columns per unrolled group

// cand[w][b]: wave w's candidate row for columns of parity b (one base
// address per wave, so every write of a row folds into the LDS offset field);
// with two barriers per column only cand[0] holds the pivot row.
struct PanelShared {
  alignas(16) double cand[kPanelWaves][2][kNB];
  double key[2][kPanelWaves];
  int piv[kNB];
  int bad;
};

template <int C>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), C, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), C, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double read_lane(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// Maximum over the 64 lanes (quad_perm [1,0,3,2], [2,3,0,1], row_ror:4,
// row_ror:8, then row_bcast:15 / row_bcast:31), read from the last lane.
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_move<0xb1>(v));
  v = fmax(v, dpp_move<0x4e>(v));
  v = fmax(v, dpp_move<0x124>(v));
  v = fmax(v, dpp_move<0x128>(v));
  v = fmax(v, dpp_move<0x142>(v));
  v = fmax(v, dpp_move<0x143>(v));
  return read_lane(v, 63);
}

// Key of a row (see above); mask is all ones for an unused row, 0 for a used
// one.  NaN and Inf map to 1e300: such a pivot is taken, then reported.
__device__ __forceinline__ double pivot_key(double x, int row, unsigned mask) {
  const double a = fmin(fabs(x), 1e300);
  const unsigned lo = ((unsigned)__double2loint(a) & ~1023u) | (unsigned)(1023 - row);
  const unsigned hi = (unsigned)__double2hiint(a);
  return __hiloint2double((int)(hi & mask), (int)(lo & mask));
}
__device__ __forceinline__ int key_row(double k) {
  return 1023 - (__double2loint(k) & 1023);
}

// One Gauss-Jordan column at static position U of the (rotated) rows.
// umask[i]: all ones while row R*t+i is unused.
// The owner lane of row rw (wave-uniform register index rw % R) writes the
// row to slot, with the reciprocal of its column-U entry (NaN if that entry
// is zero or not finite) in place of the entry.
template <int R, int U>
__device__ __forceinline__ void publish_row(const double (&row)[R][kNB], int t, int rw,
                                            double *slot) {
  const int iw = rw % R;
#pragma unroll
  for (int i = 0; i < R; ++i)
    if (i == iw) {
      if (R * t + i == rw) {
        const double pv = row[i][U];
        const double rp = (fabs(pv) > 0.0 && isfinite(pv)) ? 1.0 / pv : __builtin_nan("");
        double2 *dst = reinterpret_cast<double2 *>(slot);
#pragma unroll
        for (int q = 0; q < kNB; q += 2)   // 16-byte stores
          dst[q / 2] = make_double2(q == U ? rp : row[i][q], q + 1 == U ? rp : row[i][q + 1]);
      }
    }
}

// The pivot row of column U reaches every thread one of two ways:
//   kTwo = false: each wave's best row is published before the one barrier
//                 (every wave writes a row, all read the winner's);
//   kTwo = true:  the keys alone go before a first barrier, then the wave
//                 holding the winner publishes it before a second one.
template <int R, int U, bool kTwo>
__device__ __forceinline__ void gj_col(double (&row)[R][kNB], double (&sig)[R],
                                       unsigned (&umask)[R], int (&mystep)[R], PanelShared &sh,
                                       int t, int jcol, int j0) {
  const int lane = t & 63, wid = t >> 6;
  const int buf = jcol & 1;
  double key = 0.0;
#pragma unroll
  for (int i = 0; i < R; ++i) key = fmax(key, pivot_key(row[i][U], R * t + i, umask[i]));
  const double m = wave_max(key);
  if (!kTwo && m > 0.0) publish_row<R, U>(row, t, key_row(m), sh.cand[wid][buf]);   // wave's best
  if (lane == 0) sh.key[buf][wid] = m;
  __syncthreads();
  double K = sh.key[buf][0];
#pragma unroll
  for (int w = 1; w < kPanelWaves; ++w) K = fmax(K, sh.key[buf][w]);
  if (!(K > 0.0)) {                    // no unused row left
    if (t == 0) { sh.piv[jcol] = 0; if (sh.bad < 0) sh.bad = jcol; }
    return;
  }
  const int r = key_row(K);
  if (kTwo) {
    if (r / (64 * R) == wid) publish_row<R, U>(row, t, r, sh.cand[0][buf]);
    __syncthreads();
  }
  const double2 *prow = reinterpret_cast<const double2 *>(sh.cand[kTwo ? 0 : r / (64 * R)][buf]);
  double pr[kNB];
#pragma unroll
  for (int q = 0; q < kNB; q += 2) {     // 16-byte loads
    const double2 v = prow[q / 2];
    pr[q] = v.x;
    pr[q + 1] = v.y;
  }
  double npiv = pr[U];
  if (npiv != npiv) {                  // zero or non-finite pivot
    if (t == 0 && sh.bad < 0) sh.bad = jcol;
    npiv = 1.0;
  }
  sh.piv[jcol] = r;                    // every thread stores the same value
  bool me[R];
  double fm[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    me[i] = R * t + i == r;
    fm[i] = me[i] ? 0.0 : row[i][U] * npiv;
  }
#pragma unroll
  for (int qq = 1; qq < kNB; ++qq) {   // the next column first
    const int q = (U + qq) % kNB;
    const double pq = pr[q];
#pragma unroll
    for (int i = 0; i < R; ++i) row[i][q] = fma(-fm[i], pq, row[i][q]);
  }
#pragma unroll
  for (int i = 0; i < R; ++i) {
    row[i][U] = me[i] ? 1.0 : -fm[i];
    umask[i] = me[i] ? 0u : umask[i];
    sig[i] = me[i] ? npiv : sig[i];
    mystep[i] = me[i] ? j0 + jcol : mystep[i];
  }
}

// The same column step with the elimination of every other panel column
// deferred by one column: pivot U's rank-1 update reaches column U+1 at once
// (the next pivot search needs it) and the remaining columns only after the
// next column's wave key has been published, so those FMAs run while the
// barrier that exchanges the keys is pending.  Each element receives the
// same FMAs in the same order as in gj_col.  dpr / dfm carry the deferred
// pivot row and multipliers; on the group's last column nothing is deferred.
template <int R, int U, bool kTwo>
__device__ __forceinline__ void gj_col_defer(double (&row)[R][kNB], double (&sig)[R],
                                             unsigned (&umask)[R], int (&mystep)[R],
                                             PanelShared &sh, int t, int jcol, int j0,
                                             double (&dpr)[kNB], double (&dfm)[R]) {
  static_assert(kTwo, "deferred eliminations publish the pivot row after the key barrier");
  const int lane = t & 63, wid = t >> 6;
  const int buf = jcol & 1;
  double key = 0.0;
#pragma unroll
  for (int i = 0; i < R; ++i) key = fmax(key, pivot_key(row[i][U], R * t + i, umask[i]));
  const double m = wave_max(key);
  if (lane == 0) sh.key[buf][wid] = m;
  if constexpr (U > 0) {
    // pivot U-1's update of the columns other than U-1 (its own) and U (done)
#pragma unroll
    for (int q = 0; q < kNB; ++q) {
      if (q == U - 1 || q == U) continue;
#pragma unroll
      for (int i = 0; i < R; ++i) row[i][q] = fma(-dfm[i], dpr[q], row[i][q]);
    }
  }
  __syncthreads();
  double K = sh.key[buf][0];
#pragma unroll
  for (int w = 1; w < kPanelWaves; ++w) K = fmax(K, sh.key[buf][w]);
  if (!(K > 0.0)) {                    // no unused row left: nothing to defer
    if (t == 0) { sh.piv[jcol] = 0; if (sh.bad < 0) sh.bad = jcol; }
#pragma unroll
    for (int i = 0; i < R; ++i) dfm[i] = 0.0;
    return;
  }
  const int r = key_row(K);
  if (r / (64 * R) == wid) publish_row<R, U>(row, t, r, sh.cand[0][buf]);
  __syncthreads();
  const double2 *prow = reinterpret_cast<const double2 *>(sh.cand[0][buf]);
#pragma unroll
  for (int q = 0; q < kNB; q += 2) {     // 16-byte loads
    const double2 v = prow[q / 2];
    dpr[q] = v.x;
    dpr[q + 1] = v.y;
  }
  double npiv = dpr[U];
  if (npiv != npiv) {                  // zero or non-finite pivot
    if (t == 0 && sh.bad < 0) sh.bad = jcol;
    npiv = 1.0;
  }
  sh.piv[jcol] = r;                    // every thread stores the same value
  bool me[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    me[i] = R * t + i == r;
    dfm[i] = me[i] ? 0.0 : row[i][U] * npiv;
  }
  if constexpr (U + 1 < kGroup) {
#pragma unroll
    for (int i = 0; i < R; ++i) row[i][U + 1] = fma(-dfm[i], dpr[U + 1], row[i][U + 1]);
  } else {                             // last column of the group: no deferral
#pragma unroll
    for (int q = 0; q < kNB; ++q) {
      if (q == U) continue;
#pragma unroll
      for (int i = 0; i < R; ++i) row[i][q] = fma(-dfm[i], dpr[q], row[i][q]);
    }
  }
#pragma unroll
  for (int i = 0; i < R; ++i) {
    row[i][U] = me[i] ? 1.0 : -dfm[i];
    umask[i] = me[i] ? 0u : umask[i];
    sig[i] = me[i] ? npiv : sig[i];
    mystep[i] = me[i] ? j0 + jcol : mystep[i];
  }
}

template <int R, int U, bool kTwo>
__device__ __forceinline__ void gj_group_defer(double (&row)[R][kNB], double (&sig)[R],
                                               unsigned (&umask)[R], int (&mystep)[R],
                                               PanelShared &sh, int t, int jbase, int j0,
                                               double (&dpr)[kNB], double (&dfm)[R]) {
  gj_col_defer<R, U, kTwo>(row, sig, umask, mystep, sh, t, jbase + U, j0, dpr, dfm);
  if constexpr (U + 1 < kGroup)
    gj_group_defer<R, U + 1, kTwo>(row, sig, umask, mystep, sh, t, jbase, j0, dpr, dfm);
}

template <int R, int U, bool kTwo>
__device__ __forceinline__ void gj_group(double (&row)[R][kNB], double (&sig)[R],
                                         unsigned (&umask)[R], int (&mystep)[R],
                                         PanelShared &sh, int t, int jbase, int j0) {
  gj_col<R, U, kTwo>(row, sig, umask, mystep, sh, t, jbase + U, j0);
  if constexpr (U + 1 < kGroup)
    gj_group<R, U + 1, kTwo>(row, sig, umask, mystep, sh, t, jbase, j0);
}

template <class MA, class T, int R, bool kTwo, bool kDefer = false>
__global__ void __launch_bounds__(64 * kPanelWaves) k_panel(MA ma, int k, int p, int ld) {
  MatRef<T> mat;
  if (!ma(blockIdx.x, k, mat)) return;
  const int t = threadIdx.x;
  const auto W = gmem(mat.W);
  const int j0 = p * kNB;
  __shared__ PanelShared sh;

  double row[R][kNB], sig[R];
  unsigned umask[R];
  int mystep[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int g = R * t + i;
    umask[i] = 0u;
    mystep[i] = INT_MAX;
    sig[i] = 1.0;
    if (g < ld) {
      const auto src = W + (size_t)g * ld + j0;
#pragma unroll
      for (int q = 0; q < kNB; ++q) row[i][q] = (double)src[q];
      mystep[i] = mat.rstep[g];
      umask[i] = mystep[i] < j0 ? 0u : ~0u;
    } else {
#pragma unroll
      for (int q = 0; q < kNB; ++q) row[i][q] = 0.0;
    }
  }
  if (t < 2 * kPanelWaves) sh.key[t / kPanelWaves][t % kPanelWaves] = 0.0;   // absent waves
  if (t == 0) sh.bad = -1;
  __syncthreads();

  // Columns in groups of kGroup at static positions 0..kGroup-1; afterwards
  // every row rotates left by kGroup, so after the last group the rows are
  // back in panel order.
  double dpr[kNB], dfm[R];
#pragma unroll 1
  for (int jb = 0; jb < kNB; jb += kGroup) {
    if constexpr (kDefer)
      gj_group_defer<R, 0, kTwo>(row, sig, umask, mystep, sh, t, jb, j0, dpr, dfm);
    else
      gj_group<R, 0, kTwo>(row, sig, umask, mystep, sh, t, jb, j0);
#pragma unroll
    for (int i = 0; i < R; ++i) {
      double tmp[kGroup];
#pragma unroll
      for (int q = 0; q < kGroup; ++q) tmp[q] = row[i][q];
#pragma unroll
      for (int q = 0; q + kGroup < kNB; ++q) row[i][q] = row[i][q + kGroup];
#pragma unroll
      for (int q = 0; q < kGroup; ++q) row[i][kNB - kGroup + q] = tmp[q];
    }
  }
  __syncthreads();
  if (t < kNB) mat.piv[j0 + t] = sh.piv[t];
  if (t == 0 && sh.bad >= 0 && atomicCAS(mat.flag, -1, mat.id) == -1) mat.flag[1] = j0 + sh.bad;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int g = R * t + i;
    if (g < ld) {
      const auto dst = W + (size_t)g * ld + j0;
#pragma unroll
      for (int q = 0; q < kNB; ++q) dst[q] = (T)(row[i][q] * sig[i]);
      mat.rstep[g] = mystep[i];
    }
  }
}

template <class MA, class T>
void launch_panel(const MA &ma, int nmat, int ld, int k, int p, hipStream_t s) {
  const int threads = 64 * ((ld + 64 * kPanelRows - 1) / (64 * kPanelRows));
  if (options().panel_defer)          // deferred eliminations: two barriers per column
    hipLaunchKernelGGL((k_panel<MA, T, kPanelRows, true, true>), dim3(nmat), dim3(threads), 0, s,
                       ma, k, p, ld);
  else if (options().panel_sync == 2)
    hipLaunchKernelGGL((k_panel<MA, T, kPanelRows, true>), dim3(nmat), dim3(threads), 0, s, ma, k,
                       p, ld);
  else
    hipLaunchKernelGGL((k_panel<MA, T, kPanelRows, false>), dim3(nmat), dim3(threads), 0, s, ma,
                       k, p, ld);
}

// ---------------------------------------------------------------------------
// Schur update of the column strips outside the panel.  One work-group per
// (strip, block); each owns all ld rows of its strip, so reading the pivot
// rows (U) before overwriting them is race-free.
constexpr int kUpdThreads = 1024;   // 16 waves share the row tiles of a strip

// Strips s0 + blockIdx.x are updated, except the panel's own and those in
// [skip0, skip1).  A full launch (s0 = 0) keeps strip s on work-group s, so a
// strip stays on the same XCD for every panel.
template <class MA, class T, bool kMfma, int kMaxTiles = kMaxLd / 16 / (kUpdThreads / 64)>
__global__ void __launch_bounds__(kUpdThreads) k_update(MA ma, int k, int p, int ld, int s0,
                                                        int skip0, int skip1) {
  MatRef<T> mat;
  if (!ma(blockIdx.y, k, mat)) return;
  const int j0 = p * kNB;
  const int s = s0 + blockIdx.x;
  const int c0 = s * kStrip;
  if (c0 >= ld || (c0 >= j0 && c0 < j0 + kNB) || (s >= skip0 && s < skip1)) return;
  const auto W = gmem(mat.W);
  const auto piv = gmem((const int *)mat.piv) + j0;
  const auto rstep = gmem((const int *)mat.rstep);

  __shared__ T sU[kNB][kStrip];               // U = W[piv[J], strip]
  const int t = threadIdx.x;
  const int lane = t & 63, wid = t >> 6;
  const int nwave = blockDim.x >> 6;
  const int ntile = ld / 16;
  if (kMfma) {
    // Prefetch this wave's tiles (A operand, C tile, pivot mask) before U is
    // published, so their latency overlaps the U gather.
    // The pivot mask is applied when the tile is used, so that no load waits
    // for another.  kMaxTiles (tiles per wave) is chosen from ld at launch, so
    // that the prefetched tiles stay in registers.
    T av[kMaxTiles][kNB / 4];
    T cv[kMaxTiles][4];
    int sv[kMaxTiles][4];
#pragma unroll
    for (int u = 0; u < kMaxTiles; ++u) {
      const int tile = wid + nwave * u;
      if (tile < ntile) {
        const int rbase = tile * 16;
        const auto Arow = W + (size_t)(rbase + (lane & 15)) * ld + j0;
#pragma unroll
        for (int kk = 0; kk < kNB / 4; ++kk) av[u][kk] = Arow[4 * kk + (lane >> 4)];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = rbase + mfma_row(T(0), lane, i);
          sv[u][i] = rstep[row];
          cv[u][i] = W[(size_t)row * ld + c0 + (lane & 15)];
        }
      }
    }
    for (int e = t; e < kNB * kStrip; e += blockDim.x) {
      const int q = e / kStrip, col = e % kStrip;
      sU[q][col] = W[(size_t)piv[q] * ld + c0 + col];
    }
    __syncthreads();
    // v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32: lane supplies
    // A[l%16][l/16] and B[l/16][l%16]; output rows per mfma_row().
#pragma unroll
    for (int u = 0; u < kMaxTiles; ++u) {
      const int tile = wid + nwave * u;
      if (tile < ntile) {
        const int rbase = tile * 16;
        typename Vec4<T>::type accv;
#pragma unroll
        for (int i = 0; i < 4; ++i) accv[i] = (sv[u][i] >= j0 && sv[u][i] < j0 + kNB) ? T(0) : cv[u][i];
#pragma unroll
        for (int kk = 0; kk < kNB / 4; ++kk)
          accv = mfma16(av[u][kk], sU[4 * kk + (lane >> 4)][lane & 15], accv);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = rbase + mfma_row(T(0), lane, i);
          W[(size_t)row * ld + c0 + (lane & 15)] = accv[i];
        }
      }
    }
  } else {
    for (int e = t; e < kNB * kStrip; e += blockDim.x) {
      const int q = e / kStrip, col = e % kStrip;
      sU[q][col] = W[(size_t)piv[q] * ld + c0 + col];
    }
    __syncthreads();
    // VALU: thread handles (row = t/16 + multiples of blockDim/16, col = t%16).
    const int col = t & 15;
    for (int row = t >> 4; row < ld; row += blockDim.x >> 4) {
      const int st = rstep[row];
      const T cw = W[(size_t)row * ld + c0 + col];
      T acc = (st >= j0 && st < j0 + kNB) ? T(0) : cw;
      const auto Arow = W + (size_t)row * ld + j0;
#pragma unroll 8
      for (int q = 0; q < kNB; ++q) acc = fma(Arow[q], sU[q][col], acc);
      W[(size_t)row * ld + c0 + col] = acc;
    }
  }
}

// Trailing update in 32-column strips (the panel width): one work-group of
// four waves per (strip, block); each wave walks the 16-row tiles
// wid, wid+4, ... of the strip, loading the next tile's operands before the
// current tile's MFMAs.  The strip's pivot rows U (32 x 32) are read into
// LDS and then into registers before any row of the strip is written.
constexpr int kUpd32Threads = 256;

template <class MA, class T>
__global__ void __launch_bounds__(kUpd32Threads) k_update32(MA ma, int k, int p, int ld, int q0,
                                                            int skip) {
  MatRef<T> mat;
  if (!ma(blockIdx.y, k, mat)) return;
  const int q = q0 + blockIdx.x;
  const int c0 = q * kNB;
  if (q == p || q == skip || c0 >= ld) return;
  const int j0 = p * kNB;
  const auto W = gmem(mat.W);
  const auto piv = gmem((const int *)mat.piv) + j0;
  const auto rstep = gmem((const int *)mat.rstep);
  __shared__ T sU[kNB][kNB + 1];
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  // U: every pivot index first, then every value (two loads deep instead of
  // two per element), with the first tile's operands issued in between.
  constexpr int kUE = kNB * kNB / kUpd32Threads;
  int ur[kUE];
#pragma unroll
  for (int e = 0; e < kUE; ++e) ur[e] = piv[(t + e * kUpd32Threads) / kNB];
  const int ntile = ld / 16;
  // Loads only: the pivot mask is applied when the tile is used, so the
  // next tile's loads stay in flight during the current tile's MFMAs.
  T av[kNB / 4], cv[2][4];
  int sv[4];
  auto load = [&](int tile) {
    const int rbase = tile * 16;
    const auto Arow = W + (size_t)(rbase + (lane & 15)) * ld + j0;
#pragma unroll
    for (int kk = 0; kk < kNB / 4; ++kk) av[kk] = Arow[4 * kk + (lane >> 4)];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = rbase + mfma_row(T(0), lane, i);
      sv[i] = rstep[row];
#pragma unroll
      for (int h = 0; h < 2; ++h) cv[h][i] = W[(size_t)row * ld + c0 + 16 * h + (lane & 15)];
    }
  };
  int tile = wid;
  if (tile < ntile) load(tile);
  T uv[kUE];
#pragma unroll
  for (int e = 0; e < kUE; ++e)
    uv[e] = W[(size_t)ur[e] * ld + c0 + (t + e * kUpd32Threads) % kNB];
#pragma unroll
  for (int e = 0; e < kUE; ++e) {
    const int idx = t + e * kUpd32Threads;
    sU[idx / kNB][idx % kNB] = uv[e];
  }
  __syncthreads();
  // B operand of the two 16-column halves, 8 k-steps each: U[4kk + l/16][16h + l%16]
  T bf[2][kNB / 4];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int kk = 0; kk < kNB / 4; ++kk) bf[h][kk] = sU[4 * kk + (lane >> 4)][16 * h + (lane & 15)];
  __syncthreads();   // every wave holds U before any pivot row of the strip is rewritten
  while (tile < ntile) {
    typename Vec4<T>::type acc[2];
    T a_now[kNB / 4];
#pragma unroll
    for (int kk = 0; kk < kNB / 4; ++kk) a_now[kk] = av[kk];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const bool piv_here = sv[i] >= j0 && sv[i] < j0 + kNB;
#pragma unroll
      for (int h = 0; h < 2; ++h) acc[h][i] = piv_here ? T(0) : cv[h][i];
    }
    const int cur = tile;
    tile += 4;
    if (tile < ntile) load(tile);   // next tile's operands in flight during the MFMAs
#pragma unroll
    for (int kk = 0; kk < kNB / 4; ++kk)
#pragma unroll
      for (int h = 0; h < 2; ++h) acc[h] = mfma16(a_now[kk], bf[h][kk], acc[h]);
    const int rbase = cur * 16;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = rbase + mfma_row(T(0), lane, i);
#pragma unroll
      for (int h = 0; h < 2; ++h) W[(size_t)row * ld + c0 + 16 * h + (lane & 15)] = acc[h][i];
    }
  }
}

// Strips [s0, s0 + nstrip) minus [skip0, skip1) (and the panel's own).
template <class MA, class T>
void launch_update(const MA &ma, int nmat, int ld, int k, int p, hipStream_t s, int s0 = 0,
                   int nstrip = -1, int skip0 = 0, int skip1 = 0) {
  if (nstrip < 0) nstrip = ld / kStrip;
  if (nstrip <= 0) return;
  constexpr int spp = kNB / kStrip;
  // Four-wave 32-column strips when the launch has work-groups enough to
  // fill the chip (many blocks); 16-wave 16-column strips keep more waves
  // per block in flight when only a few blocks are updated.
  const bool many = (size_t)nmat * (ld / kNB) >= (size_t)options().update32_min;
  if (options().gemm_mfma && options().update32 && many && s0 % spp == 0 &&
      nstrip % spp == 0 && skip0 % spp == 0 && skip1 - skip0 <= spp)
    hipLaunchKernelGGL((k_update32<MA, T>), dim3(nstrip / spp, nmat), dim3(kUpd32Threads), 0, s,
                       ma, k, p, ld, s0 / spp, skip1 > skip0 ? skip0 / spp : -1);
  else if (options().gemm_mfma) {
    // tiles per wave: 16-row tiles of the block over the 16 waves
    const int tpw = (ld / 16 + kUpdThreads / 64 - 1) / (kUpdThreads / 64);
    const dim3 grid(nstrip, nmat);
    if (tpw <= 1)
      hipLaunchKernelGGL((k_update<MA, T, true, 1>), grid, dim3(kUpdThreads), 0, s, ma, k, p, ld,
                         s0, skip0, skip1);
    else if (tpw <= 2)
      hipLaunchKernelGGL((k_update<MA, T, true, 2>), grid, dim3(kUpdThreads), 0, s, ma, k, p, ld,
                         s0, skip0, skip1);
    else if (tpw <= 3)
      hipLaunchKernelGGL((k_update<MA, T, true, 3>), grid, dim3(kUpdThreads), 0, s, ma, k, p, ld,
                         s0, skip0, skip1);
    else
      hipLaunchKernelGGL((k_update<MA, T, true>), grid, dim3(kUpdThreads), 0, s, ma, k, p, ld, s0,
                         skip0, skip1);
  }
  else
    hipLaunchKernelGGL((k_update<MA, T, false>), dim3(nstrip, nmat), dim3(kUpdThreads), 0, s,
                       ma, k, p, ld, s0, skip0, skip1);
}

// Outer update: the rank-wo product of an outer panel (wo = 64, 96 or 128
// columns eliminated by its 32-column panels) applied to every 32-column
// strip outside it:  C <- mask * C + W[:, Jo] U,  U = W[piv[Jo], strip],
// mask zeroing the rows pivoted in Jo.  Same strip ownership as k_update32.
template <class MA, class T, int WO>
__global__ void __launch_bounds__(kUpd32Threads) k_update_outer(MA ma, int k, int jo, int ld) {
  MatRef<T> mat;
  if (!ma(blockIdx.y, k, mat)) return;
  const int c0 = blockIdx.x * kNB;
  if (c0 >= ld || (c0 >= jo && c0 < jo + WO)) return;
  const auto W = gmem(mat.W);
  const auto piv = gmem((const int *)mat.piv) + jo;
  const auto rstep = gmem((const int *)mat.rstep);
  __shared__ T sU[WO][kNB + 1];
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  for (int e = t; e < WO * kNB; e += blockDim.x) {
    const int r = e / kNB, col = e % kNB;
    sU[r][col] = W[(size_t)piv[r] * ld + c0 + col];
  }
  __syncthreads();
  const int ntile = ld / 16;
  for (int tile = wid; tile < ntile; tile += 4) {
    const int rbase = tile * 16;
    T av[WO / 4];
    const auto Arow = W + (size_t)(rbase + (lane & 15)) * ld + jo;
#pragma unroll
    for (int kk = 0; kk < WO / 4; ++kk) av[kk] = Arow[4 * kk + (lane >> 4)];
    typename Vec4<T>::type acc[2];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = rbase + mfma_row(T(0), lane, i);
      const int st = rstep[row];
      const bool piv_here = st >= jo && st < jo + WO;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const T cw = W[(size_t)row * ld + c0 + 16 * h + (lane & 15)];
        acc[h][i] = piv_here ? T(0) : cw;
      }
    }
#pragma unroll
    for (int kk = 0; kk < WO / 4; ++kk)
#pragma unroll
      for (int h = 0; h < 2; ++h)
        acc[h] = mfma16(av[kk], sU[4 * kk + (lane >> 4)][16 * h + (lane & 15)], acc[h]);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = rbase + mfma_row(T(0), lane, i);
#pragma unroll
      for (int h = 0; h < 2; ++h) W[(size_t)row * ld + c0 + 16 * h + (lane & 15)] = acc[h][i];
    }
  }
}

// Gauss-Jordan inversion of the blocks of one launch.  Columns are taken in
// outer panels of up to options().outer columns; inside an outer panel each
// 32-column panel is factored and its update applied to the rest of the
// outer panel only, then one rank-(outer width) update covers every other
// column.  With outer = 32 every panel updates the whole block.
template <class MA, class T>
void invert_blocks(const MA &ma, int nmat, int ld, int k, hipStream_t s, bool prof) {
  const int wmax = nmat >= options().outer_nmat ? options().outer : kNB;
  for (int jo = 0; jo < ld; jo += wmax) {
    const int wo = std::min(wmax, ld - jo);
    for (int p = jo / kNB; p < (jo + wo) / kNB; ++p) {
      if (prof) prof_begin(kProfPanel, s);
      launch_panel<MA, T>(ma, nmat, ld, k, p, s);
      if (prof) prof_end(kProfPanel, s);
      if (wo == kNB) {
        if (prof) prof_begin(kProfUpdate, s);
        launch_update<MA, T>(ma, nmat, ld, k, p, s);
        if (prof) prof_end(kProfUpdate, s);
      } else if (wo > kNB) {
        if (prof) prof_begin(kProfUpdate, s);
        launch_update<MA, T>(ma, nmat, ld, k, p, s, jo / kStrip, wo / kStrip);
        if (prof) prof_end(kProfUpdate, s);
      }
    }
    if (wo > kNB && ld > wo) {
      if (prof) prof_begin(kProfUpdate, s);
      const dim3 grid(ld / kNB, nmat);
      if (wo == 64)
        hipLaunchKernelGGL((k_update_outer<MA, T, 64>), grid, dim3(kUpd32Threads), 0, s, ma, k,
                           jo, ld);
      else if (wo == 96)
        hipLaunchKernelGGL((k_update_outer<MA, T, 96>), grid, dim3(kUpd32Threads), 0, s, ma, k,
                           jo, ld);
      else
        hipLaunchKernelGGL((k_update_outer<MA, T, 128>), grid, dim3(kUpd32Threads), 0, s, ma, k,
                           jo, ld);
      if (prof) prof_end(kProfUpdate, s);
    }
  }
}

// ---------------------------------------------------------------------------
// Persistent block Thomas for small blocks (ld up to option fused_max_ld,
// at most kFusedMaxLd): one work-group runs a column's whole layer chain in
// one launch.  It pays where the per-layer launches dominate (ld 32, 64);
// at ld 96 one work-group per column is slower than the panel kernels.
//
// Factorisation.  Thread t owns CW consecutive columns (a part) of row
// t / TPR of the current block in registers.  Per layer k the Schur
// complement
//   D'_k = B_k - diag(a_k) E_{k-1} diag(c_{k-1})
// is formed while B_k is read (E_{k-1} is the registers' previous content),
// then inverted by Gauss-Jordan with implicit partial pivoting, the pivot
// chosen by the panel kernels' key (largest magnitude among unused rows to
// 42 mantissa bits, lowest row among equals).  Columns are eliminated in
// rounds, slot r of every part in round r, and the register tiles rotate by
// one slot per round, so the column being eliminated is always in slot 0
// (static register indices; any column order gives the same inverse).  Per
// column: the candidates' keys reduced per wave and a barrier, the pivot row
// and the column published in LDS and a barrier, every row updated in
// registers.  The result W goes through LDS to natural order,
// E[column pivoted by row r][row pivoting column j] = W[r][j], is written
// back over B_k, and stays in registers for the next layer.  Pivots are
// stored as the identity, so every solve path reads E_k as it would any
// factorisation.
//
// Solve.  One work-group per column: the forward chain
//   y_k = E_k (rhs_k - a_k y_{k-1})          (y_k into gs)
// then the backward chain
//   x_{N-1} = y_{N-1},  x_k = y_k - E_k (c_k x_{k+1}),
// each step a matrix-vector product of the thread's row segment and a
// reduction over the TPR threads of the row.  It reads the stored pivots,
// so it also solves with factors of the panel kernels (the option can
// change between a factorisation and a later solve with it).
constexpr int kFusedMaxLd = 128;

// NT threads per work-group: four waves.  (One wave for blocks up to 64,
// the pivot exchange then staying inside the wave, measured slower: 384
// against 277 us per 12-species step, the wave issuing every step alone.)
template <int LD, int NT>
struct FusedShape {
  static constexpr int R = NT / LD;
  static constexpr int TPR = R >= 8 ? 8 : (R >= 4 ? 4 : (R >= 2 ? 2 : 1));   // threads per row
  static constexpr int CW = LD / TPR;                                     // columns per thread
  static constexpr int THREADS = LD * TPR;
  static constexpr int WAVES = NT / 64;
  static_assert(THREADS <= NT && CW * TPR == LD && WAVES >= 1 && WAVES <= 4, "shape");
};
template <int LD>
constexpr int fused_threads() { return 256; }

// Sum over the TPR consecutive lanes that share a row.
template <int TPR>
__device__ __forceinline__ double row_sum(double z) {
#pragma unroll
  for (int o = 1; o < TPR; o <<= 1) z += __shfl_xor(z, o, 64);
  return z;
}

template <class Acc, int LD, int NT = fused_threads<LD>()>
__global__ void __launch_bounds__(NT) k_btd_fused_factor(Acc acc) {
  using F = FusedShape<LD, NT>;
  constexpr int CW = F::CW, TPR = F::TPR;
  const ColArgs &c = acc(blockIdx.x);
  const int N = c.N, S = c.S;
  const int t = threadIdx.x, lane = t & 63;
  const bool active = t < F::THREADS;
  const int i = active ? t / TPR : 0, h = active ? t % TPR : 0, j0 = h * CW;
  __shared__ double Es[LD][LD];
  __shared__ double rowp[LD], colk[LD];   // rowp in (part, slot) order
  __shared__ double wkey[F::WAVES];
  __shared__ int pvrow[LD];
  if (t < 4) c.flag[t] = -1;
  double A[CW];
#pragma unroll
  for (int q = 0; q < CW; ++q) A[q] = 0.0;
  bool flagged = false;
  // The next layer's block row and couplings are loaded while this layer is
  // eliminated (block k+1 is written only by its own layer).
  double nb[CW], ncp[CW], nai = 0.0;
  auto fetch = [&](int k) {
    if (!active) return;
    const double *Bn = c.B + (size_t)k * LD * LD;
    const double *cp = c.c + (size_t)(k > 0 ? k - 1 : 0) * LD;
    nai = k > 0 ? c.a[(size_t)k * LD + i] : 0.0;
#pragma unroll
    for (int q = 0; q < CW; ++q) {
      nb[q] = Bn[(size_t)i * LD + j0 + q];
      ncp[q] = cp[j0 + q];
    }
  };
  if (N > 0) fetch(0);
  for (int k = 0; k < N; ++k) {
    double *Bk = c.B + (size_t)k * LD * LD;
    if (active) {
#pragma unroll
      for (int q = 0; q < CW; ++q) A[q] = k > 0 ? nb[q] - nai * A[q] * ncp[q] : nb[q];
    }
    if (k + 1 < N) fetch(k + 1);
    if (t < LD) pvrow[t] = t;   // padding columns keep their own row
    bool used = i >= S;         // padding rows are never pivots
    int colof = i;              // the column this row pivots
    int badcol = -1;
    // Columns in rounds: round r takes column h * CW + r of every part h.
    // The tile is rotated left by one slot after each round, so the round's
    // column sits in slot 0 of its part and every register index is static.
    for (int r = 0; r < CW; ++r) {
      for (int hk = 0; hk < TPR; ++hk) {
        const int kcol = hk * CW + r;
        if (kcol >= S) continue;                 // uniform
        const bool own = active && h == hk;      // holds column kcol (slot 0)
        // pivot: the largest key among the unused rows' column entries
        const double key = own ? pivot_key(A[0], i, used ? 0u : ~0u) : 0.0;
        const double m = wave_max(key);
        if (lane == 0) wkey[t >> 6] = m;
        __syncthreads();
        double K = wkey[0];
#pragma unroll
        for (int wv = 1; wv < F::WAVES; ++wv) K = fmax(K, wkey[wv]);
        int p = 1023 - (__double2loint(K) & 1023);
        if (K == 0.0 || p >= S) p = kcol;        // no usable pivot: flagged, stays in bounds
        if (active && i == p) {
#pragma unroll
          for (int q = 0; q < CW; ++q) rowp[j0 + q] = A[q];
        }
        if (own) colk[i] = A[0];
        if (t == 0) pvrow[kcol] = p;
        __syncthreads();
        const double pv = rowp[hk * CW];
        if (!(fabs(pv) > 0.0 && isfinite(pv)) && badcol < 0) badcol = kcol;
        const double rp = 1.0 / pv;
        if (active) {
          if (i == p) {
            A[0] = own ? rp : A[0] * rp;
#pragma unroll
            for (int q = 1; q < CW; ++q) A[q] *= rp;
            used = true;
            colof = kcol;
          } else {
            const double g = colk[i] * rp;
            A[0] = own ? -g : fma(-g, rowp[j0], A[0]);
#pragma unroll
            for (int q = 1; q < CW; ++q) A[q] = fma(-g, rowp[j0 + q], A[q]);
          }
        }
        // no barrier here: the next column rewrites wkey only after every
        // thread passed this column's second barrier (so has read wkey), and
        // rowp / colk only after its first one (so has finished this update)
      }
      const double a0 = A[0];
#pragma unroll
      for (int q = 0; q + 1 < CW; ++q) A[q] = A[q + 1];
      A[CW - 1] = a0;
    }
    // the tile is back in natural column order: E[colof[r]][pvrow[j]] = W[r][j]
    if (active) {
#pragma unroll
      for (int q = 0; q < CW; ++q) Es[colof][pvrow[j0 + q]] = A[q];
    }
    __syncthreads();
    if (active) {
#pragma unroll
      for (int q = 0; q < CW; ++q) {
        A[q] = Es[i][j0 + q];
        Bk[(size_t)i * LD + j0 + q] = A[q];
      }
    }
    if (t < LD) {
      c.piv[(size_t)k * LD + t] = t;
      c.rstep[(size_t)k * LD + t] = t;
    }
    if (t == 0 && badcol >= 0 && !flagged) {
      flagged = true;
      if (atomicCAS(c.flag, -1, k) == -1) c.flag[1] = badcol;
    }
    __syncthreads();
  }
}

template <class Acc, int LD, int NT = fused_threads<LD>()>
__global__ void __launch_bounds__(NT) k_btd_fused_solve(Acc acc) {
  using F = FusedShape<LD, NT>;
  constexpr int CW = F::CW;
  const ColArgs &c = acc(blockIdx.x);
  const int N = c.N, S = c.S;
  const int t = threadIdx.x;
  const bool active = t < F::THREADS;
  const int i = active ? t / F::TPR : 0, j0 = active ? (t % F::TPR) * CW : 0;
  const bool owner = active && j0 == 0;
  __shared__ double v[LD], y[LD];
  if (t < LD) y[t] = 0.0;
  __syncthreads();
  // z_r = sum_m W[r][m] v[piv[m]] for this thread's row r = i and segment,
  // summed over the row's threads; the result belongs to entry rstep[r].
  // (Factors of the persistent kernel have identity pivots; those of the
  // panel kernels are in pivot order.  Out-of-range entries of an
  // incomplete factorisation, which is flagged, read nothing.)
  // Every operand of a layer (the thread's block-row segment and its
  // pivots, the right-hand side or coupling entry, the pivot step of its row)
  // is independent of the solve, so it is loaded one layer ahead; the
  // block-row segment only for blocks up to 64, where registers allow.
  constexpr bool kRowAhead = LD <= 64;
  constexpr int kCW = kRowAhead ? CW : 1;
  struct Ops {
    double w[kCW];
    int pv[kCW];
    double e0, e1;   // forward: x and a entries; backward: the c entry (e1 unused)
    int rs, k;
  };
  auto fetch = [&](int k, bool fwd, Ops &o) {
    o.k = k;
    if constexpr (kRowAhead) {
      const double *W = c.B + (size_t)k * LD * LD + (size_t)i * LD + j0;
      const int *pv = c.piv + (size_t)k * LD + j0;
#pragma unroll
      for (int q = 0; q < CW; ++q) {
        o.w[q] = W[q];
        o.pv[q] = pv[q];
      }
    }
    const int tt = t < S ? t : 0;
    o.rs = c.rstep[(size_t)k * LD + i];
    if (fwd) {
      o.e0 = c.x[(size_t)k * S + tt];
      o.e1 = k > 0 ? c.a[(size_t)k * LD + tt] : 0.0;
    } else {
      o.e0 = c.c[(size_t)k * LD + tt];
      o.e1 = 0.0;
    }
  };
  // z_r = sum_m W[r][m] v[piv[m]] over the row's threads
  auto row_product = [&](const Ops &o) -> double {
    double z = 0.0;
    if constexpr (kRowAhead) {
#pragma unroll
      for (int q = 0; q < CW; ++q) {
        const int m = o.pv[q];
        z = fma(o.w[q], (unsigned)m < (unsigned)S ? v[m] : 0.0, z);
      }
    } else {
      const double *W = c.B + (size_t)o.k * LD * LD + (size_t)i * LD + j0;
      const int *pv = c.piv + (size_t)o.k * LD + j0;
#pragma unroll
      for (int q = 0; q < CW; ++q) {
        const int m = pv[q];
        z = fma(W[q], (unsigned)m < (unsigned)S ? v[m] : 0.0, z);
      }
    }
    return row_sum<F::TPR>(z);
  };
  Ops cur, nxt;
  if (N > 0) fetch(0, true, nxt);
  for (int k = 0; k < N; ++k) {
    cur = nxt;
    if (k + 1 < N) fetch(k + 1, true, nxt);
    else if (N >= 2) fetch(N - 2, false, nxt);   // the backward pass's first layer
    if (t < LD) v[t] = t < S ? cur.e0 - (k > 0 ? cur.e1 * y[t] : 0.0) : 0.0;
    __syncthreads();
    const double z = row_product(cur);
    __syncthreads();
    if (owner) {
      const int j = cur.rs;
      if ((unsigned)j < (unsigned)LD) {
        y[j] = z;
        c.gs[(size_t)k * LD + j] = z;
      }
    }
    __syncthreads();
  }
  // y holds y_{N-1} = x_{N-1}
  if (t < S) c.x[(size_t)(N - 1) * S + t] = y[t];
  for (int k = N - 2; k >= 0; --k) {
    cur = nxt;
    if (k > 0) fetch(k - 1, false, nxt);
    if (t < LD) v[t] = t < S ? cur.e0 * y[t] : 0.0;
    __syncthreads();
    const double z = row_product(cur);
    __syncthreads();
    if (owner) {
      const int j = cur.rs;
      if ((unsigned)j < (unsigned)LD) {
        const double xj = c.gs[(size_t)k * LD + j] - z;
        y[j] = xj;
        if (j < S) c.x[(size_t)k * S + j] = xj;
      }
    }
    __syncthreads();
  }
}

template <class Acc>
hipError_t launch_fused_factor(const Acc &acc, int ncols, int ld, hipStream_t s) {
  switch (ld) {
    case 32: hipLaunchKernelGGL((k_btd_fused_factor<Acc, 32>), dim3(ncols), dim3(fused_threads<32>()), 0, s, acc); break;
    case 64: hipLaunchKernelGGL((k_btd_fused_factor<Acc, 64>), dim3(ncols), dim3(fused_threads<64>()), 0, s, acc); break;
    case 96: hipLaunchKernelGGL((k_btd_fused_factor<Acc, 96>), dim3(ncols), dim3(fused_threads<96>()), 0, s, acc); break;
    case 128: hipLaunchKernelGGL((k_btd_fused_factor<Acc, 128>), dim3(ncols), dim3(fused_threads<128>()), 0, s, acc); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class Acc>
hipError_t launch_fused_solve(const Acc &acc, int ncols, int ld, hipStream_t s) {
  switch (ld) {
    case 32: hipLaunchKernelGGL((k_btd_fused_solve<Acc, 32>), dim3(ncols), dim3(fused_threads<32>()), 0, s, acc); break;
    case 64: hipLaunchKernelGGL((k_btd_fused_solve<Acc, 64>), dim3(ncols), dim3(fused_threads<64>()), 0, s, acc); break;
    case 96: hipLaunchKernelGGL((k_btd_fused_solve<Acc, 96>), dim3(ncols), dim3(fused_threads<96>()), 0, s, acc); break;
    case 128: hipLaunchKernelGGL((k_btd_fused_solve<Acc, 128>), dim3(ncols), dim3(fused_threads<128>()), 0, s, acc); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

inline bool use_fused(int ld) { return ld <= options().fused_max_ld && ld <= kFusedMaxLd; }

template <class Acc, class T>
hipError_t launch_factor(const Acc &acc, int ncols, int maxN, int ld, hipStream_t s) {
  if (maxN <= 0) return hipSuccess;
  if (std::is_same<T, double>::value && use_fused(ld)) {
    if (options().profile) prof_begin(kProfPanel, s);
    const hipError_t e = launch_fused_factor(acc, ncols, ld, s);
    if (options().profile) prof_end(kProfPanel, s);
    return e;
  }
  hipLaunchKernelGGL(k_rstep_init<Acc>, dim3(64, ncols), dim3(256), 0, s, acc, maxN);
  const ThomasMats<Acc, T> ma{acc};
  for (int k = 0; k < maxN; ++k) {
    const bool prof = prof_layer(k);
    if (k > 0) {
      if (prof) prof_begin(kProfPrologue, s);
      hipLaunchKernelGGL((k_prologue<Acc, T>), dim3((ld + 7) / 8, ncols), dim3(256), 0, s, acc, k);
      if (prof) prof_end(kProfPrologue, s);
    }
    invert_blocks<ThomasMats<Acc, T>, T>(ma, ncols, ld, k, s, prof);
  }
  return hipGetLastError();
}

template <class T>
hipError_t launch_invert_list(const MatRef<T> *dlist, int count, int ld, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  invert_blocks<ListMats<T>, T>(ListMats<T>{dlist}, count, ld, 0, s, options().profile != 0);
  return hipGetLastError();
}
template hipError_t launch_invert_list<double>(const MatRef<double> *, int, int, hipStream_t);
template hipError_t launch_invert_list<float>(const MatRef<float> *, int, int, hipStream_t);

template <class Acc>
hipError_t launch_factor_fp64(const Acc &acc, int ncols, int maxN, int ld, hipStream_t s) {
  return launch_factor<Acc, double>(acc, ncols, maxN, ld, s);
}
template <class Acc>
hipError_t launch_factor_mixed(const Acc &acc, int ncols, int maxN, int ld, hipStream_t s) {
  return launch_factor<Acc, float>(acc, ncols, maxN, ld, s);
}

// ---------------------------------------------------------------------------
// Solve.  y = D'^{-1} v:  y[j] = sum_m W[piv[j]][m] v[piv[m]], written as
// z = W v' with v'[m] = v[piv[m]], then y[rstep[r]] = z[r] (rstep = piv^-1).
//
// Forward (k >= 1): g_k = rhs_k - a_k * (D'^{-1}_{k-1} g_{k-1}) into gs.
// Backward:         x_k = D'^{-1}_k (g_k - c_k * x_{k+1}) into x.
// One work-group per 16 rows of W; each wave reduces 4 rows.
template <class Acc, class T, bool kForward>
__global__ void __launch_bounds__(256) k_solve_step(Acc acc, int k) {
  const ColArgs &c = acc(blockIdx.y);
  const int N = c.N, S = c.S, ld = c.ld;
  if (k >= N) return;
  const int kin = kForward ? k - 1 : k;        // layer whose inverse is applied
  if (kForward && k == 0) {
    // g_0 = rhs_0, kept in gs so the backward pass never reads x[0] while
    // other work-groups overwrite it.
    if (blockIdx.x == 0)
      for (int y = threadIdx.x; y < S; y += blockDim.x) c.gs[y] = c.x[y];
    return;
  }
  const T *W = blocks<T>(c) + (size_t)kin * ld * ld;
  const int *pv = c.piv + (size_t)kin * ld;
  const int *rq = c.rstep + (size_t)kin * ld;
  __shared__ double sv[kMaxLd];
  const int t = threadIdx.x;
  // v'[m] = v[piv[m]]
  for (int m = t; m < ld; m += blockDim.x) {
    const int src = pv[m];
    double v = 0.0;
    if (src < S) {
      if (kForward) {
        v = c.gs[(size_t)kin * ld + src];
      } else {
        const double g = c.gs[(size_t)k * ld + src];
        const double nx = (k + 1 < N) ? c.x[(size_t)(k + 1) * S + src] : 0.0;
        v = g - c.c[(size_t)k * ld + src] * nx;
      }
    }
    sv[m] = v;
  }
  __syncthreads();
  const int lane = t & 63, wid = t >> 6;
  for (int rr = 0; rr < 4; ++rr) {
    const int r = blockIdx.x * 16 + wid * 4 + rr;
    if (r >= ld) break;
    const T *row = W + (size_t)r * ld;
    double z = 0.0;
    for (int m = lane; m < ld; m += 64) z = fma((double)row[m], sv[m], z);
    for (int o = 32; o > 0; o >>= 1) z += __shfl_xor(z, o, 64);
    if (lane == 0) {
      const int j = rq[r];
      if (j < S) {
        if (kForward) {
          const size_t o = (size_t)k * S + j;
          c.gs[(size_t)k * ld + j] = c.x[o] - c.a[(size_t)k * ld + j] * z;
        } else {
          c.x[(size_t)k * S + j] = z;
        }
      }
    }
  }
}

template <class Acc, class T>
hipError_t launch_solve(const Acc &acc, int ncols, int maxN, int ld, hipStream_t s) {
  if (maxN <= 0) return hipSuccess;
  if (std::is_same<T, double>::value && use_fused(ld)) {
    if (options().profile) prof_begin(kProfSolve, s);
    const hipError_t e = launch_fused_solve(acc, ncols, ld, s);
    if (options().profile) prof_end(kProfSolve, s);
    return e;
  }
  dim3 grid((ld + 15) / 16, ncols);
  for (int k = 0; k < maxN; ++k) {
    const bool prof = prof_layer(k);
    if (prof) prof_begin(kProfSolve, s);
    hipLaunchKernelGGL((k_solve_step<Acc, T, true>), grid, dim3(256), 0, s, acc, k);
    if (prof) prof_end(kProfSolve, s);
  }
  for (int k = maxN - 1; k >= 0; --k) {
    const bool prof = prof_layer(k);
    if (prof) prof_begin(kProfSolve, s);
    hipLaunchKernelGGL((k_solve_step<Acc, T, false>), grid, dim3(256), 0, s, acc, k);
    if (prof) prof_end(kProfSolve, s);
  }
  return hipGetLastError();
}

template <class Acc>
hipError_t launch_solve_fp64(const Acc &acc, int ncols, int maxN, int ld, hipStream_t s) {
  return launch_solve<Acc, double>(acc, ncols, maxN, ld, s);
}
template <class Acc>
hipError_t launch_solve_mixed(const Acc &acc, int ncols, int maxN, int ld, hipStream_t s) {
  return launch_solve<Acc, float>(acc, ncols, maxN, ld, s);
}

template hipError_t launch_factor_fp64<OneCol>(const OneCol &, int, int, int, hipStream_t);
template hipError_t launch_factor_fp64<ManyCols>(const ManyCols &, int, int, int, hipStream_t);
template hipError_t launch_solve_fp64<OneCol>(const OneCol &, int, int, int, hipStream_t);
template hipError_t launch_solve_fp64<ManyCols>(const ManyCols &, int, int, int, hipStream_t);
template hipError_t launch_factor_mixed<OneCol>(const OneCol &, int, int, int, hipStream_t);
template hipError_t launch_factor_mixed<ManyCols>(const ManyCols &, int, int, int, hipStream_t);
template hipError_t launch_solve_mixed<OneCol>(const OneCol &, int, int, int, hipStream_t);
template hipError_t launch_solve_mixed<ManyCols>(const ManyCols &, int, int, int, hipStream_t);

}  // namespace xod
