// Kernels of block cyclic reduction for the block-tridiagonal step system
//   A_k x_{k-h} + D_k x_k + C_k x_{k+h} = g_k
// (level 0: h = 1, A_k = diag(a_k), C_k = diag(c_k), D_k = B_k).
//
//   k_gemm       batched dense block products on the matrix cores (the
//                Schur terms A_k E C of levels >= 1), FP64 or FP32 MFMA
//   k_cr_level0  the level-0 Schur terms, where the couplings are diagonal
//                and every term is an elementwise product with E
//   k_mv         batched matrix-vector terms of the reduction / substitution
//   k_pad_copy   compact [N*S] <-> padded [N*ld] vectors
//
// Inverses come from the Gauss-Jordan kernels in their permuted form,
// E[i][j] = W[piv[i]][rstep[j]].  A product X E is formed as X (W[piv,:])
// with its columns in pivot-step order; later products with that result
// gather the rows of their right operand by piv instead of permuting back.
#include "xod_internal.h"
#include "mfma.h"

#include <climits>

namespace xod {

// Permutation entries index rows / columns of an ld x ld block; a complete
// inversion leaves every entry in range, the clamp keeps a failed one (flagged
// singular, results discarded) from addressing outside the block.
__device__ __forceinline__ int in_block(int i, int ld) {
  return (int)min((unsigned)i, (unsigned)(ld - 1));
}

// ---------------------------------------------------------------------------
// Block products.  One work-group of NT / 64 waves per BM x BM output tile
// (BM = 64 or 128; NT = 1024, or 512 for 128-tiles with option gemm_waves =
// 8); the waves form a (NT / 256) x 4 grid, each owning a sub-tile of
// TMR x TMC 16 x 16 MFMA accumulators (2 x 2 with 16 waves, 4 x 2 with 8),
// so each LDS fragment feeds TMC or TMR MFMAs.  K is staged through LDS in steps of KB (double-buffered: the next
// step's global loads are issued before the MFMAs of the current one).  Every
// output element accumulates its K terms in increasing order whatever BM and
// KB are.  Rows / columns beyond ld are never touched (ld is a multiple of
// 32).
constexpr int kGemmThreads = 1024;

template <class T, int BM, int KB, int NT = kGemmThreads>
__global__ void __launch_bounds__(NT) k_gemm(const GemmOp<T> *ops, int ld) {
  constexpr int WR = NT / 256;                      // wave rows (4 wave columns)
  constexpr int TMR = BM / (16 * WR);               // MFMA tiles per wave, rows
  constexpr int TMC = BM / 64;                      // MFMA tiles per wave, columns
  constexpr int AL = BM * KB / NT;                  // A elements staged per thread
  constexpr int BL = KB * BM / NT;                  // B elements staged per thread
  static_assert(AL >= 1 && BL >= 1 && TMR >= 1, "tile shape");
  const GemmOp<T> g = ops[blockIdx.z];
  const int tm0 = blockIdx.y * BM, tn0 = blockIdx.x * BM;
  const int t = threadIdx.x, lane = t & 63;
  const int wid = __builtin_amdgcn_readfirstlane(t >> 6);   // wave-uniform
  const int wr = wid >> 2, wc = wid & 3;
  __shared__ T As[2][BM][KB + 1];
  __shared__ T Bs[2][KB][BM + 2];
  __shared__ int sbg[2][kMaxLd];   // the row gathers of B and B2
  typename Vec4<T>::type acc[TMR][TMC];
#pragma unroll
  for (int i = 0; i < TMR; ++i)
#pragma unroll
    for (int j = 0; j < TMC; ++j) acc[i][j] = {0, 0, 0, 0};
  const int nk1 = ld / KB;
  const int nk = g.A2 ? 2 * nk1 : nk1;
  for (int m = threadIdx.x; m < ld; m += blockDim.x) {
    sbg[0][m] = g.bg ? in_block(gmem(g.bg)[m], ld) : m;
    sbg[1][m] = g.bg2 ? in_block(gmem(g.bg2)[m], ld) : m;
  }
  __syncthreads();
  // staging element e of this thread: A (row (t + e*1024) / KB, k % KB),
  // B (k (t + e*1024) / BM, column % BM)
  T ra[AL], rb[BL];
  auto gload = [&](int kt) {
    const bool second = kt >= nk1;
    const auto A = gmem(second ? g.A2 : g.A);
    const auto B = gmem(second ? g.B2 : g.B);
    const int k0 = (second ? kt - nk1 : kt) * KB;
    const int *gb = sbg[second ? 1 : 0];
    // every load unconditional (row / column clamped into the block), so
    // the whole step's loads and gather-index reads issue together; the
    // elements beyond ld become zeros when they are stored to LDS
    int gr[BL];
#pragma unroll
    for (int e = 0; e < BL; ++e) gr[e] = gb[k0 + (t + e * NT) / BM];
#pragma unroll
    for (int e = 0; e < AL; ++e) {
      const int idx = t + e * NT, r = min(tm0 + idx / KB, ld - 1);
      ra[e] = A[(size_t)r * ld + k0 + idx % KB];
    }
#pragma unroll
    for (int e = 0; e < BL; ++e) {
      const int idx = t + e * NT, c = min(tn0 + idx % BM, ld - 1);
      rb[e] = B[(size_t)gr[e] * ld + c];
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int e = 0; e < AL; ++e) {
      const int idx = t + e * NT;
      As[buf][idx / KB][idx % KB] = tm0 + idx / KB < ld ? ra[e] : T(0);
    }
#pragma unroll
    for (int e = 0; e < BL; ++e) {
      const int idx = t + e * NT;
      Bs[buf][idx / BM][idx % BM] = tn0 + idx % BM < ld ? rb[e] : T(0);
    }
  };
  // A wave whose output tiles all lie beyond ld (the last tile row / column
  // of a block whose size is not a multiple of BM) skips its products, one
  // wave-uniform test per K step, and leaves its SIMD to other work-groups.
  // A wave with some tiles inside multiplies all of them (the staged
  // operands beyond ld are zeros, and the stores are masked); with 16 waves
  // each wave's 32 x 32 outputs are wholly inside or outside (ld is a
  // multiple of 32), so only the 8-wave tiles carry such zero products.
  const bool wave_live = tm0 + wr * TMR * 16 < ld && tn0 + wc * TMC * 16 < ld;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) gload(kt + 1);
    if (wave_live) {
#pragma unroll
      for (int kk = 0; kk < KB / 4; ++kk) {
        T av[TMR], bv[TMC];
#pragma unroll
        for (int i = 0; i < TMR; ++i)
          av[i] = As[buf][(wr * TMR + i) * 16 + (lane & 15)][kk * 4 + (lane >> 4)];
#pragma unroll
        for (int j = 0; j < TMC; ++j)
          bv[j] = Bs[buf][kk * 4 + (lane >> 4)][(wc * TMC + j) * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < TMR; ++i)
#pragma unroll
          for (int j = 0; j < TMC; ++j) acc[i][j] = mfma16(av[i], bv[j], acc[i][j]);
      }
    }
    if (kt + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }
  // C is read (when accumulated into) for every output of the wave at once,
  // the addresses clamped into the block, then written where inside it.
  const auto C = gmem(g.C);
  T cold[TMR][TMC][4];
  if (g.beta && wave_live) {
#pragma unroll
    for (int i = 0; i < TMR; ++i)
#pragma unroll
      for (int j = 0; j < TMC; ++j) {
        const int c = min(tn0 + (wc * TMC + j) * 16 + (lane & 15), ld - 1);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = min(tm0 + (wr * TMR + i) * 16 + mfma_row(T(0), lane, q), ld - 1);
          cold[i][j][q] = C[(size_t)r * ld + c];
        }
      }
  }
#pragma unroll
  for (int i = 0; i < TMR; ++i)
#pragma unroll
    for (int j = 0; j < TMC; ++j) {
      const int c = tn0 + (wc * TMC + j) * 16 + (lane & 15);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = tm0 + (wr * TMR + i) * 16 + mfma_row(T(0), lane, q);
        if (r < ld && c < ld) {
          const double v = g.alpha * (double)acc[i][j][q];
          C[(size_t)r * ld + c] = (T)(g.beta ? (double)cold[i][j][q] + v : v);
        }
      }
    }
}

template <class T>
hipError_t launch_gemm(const GemmOp<T> *dops, int count, int ld, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int ntl = (ld + 127) / 128;
  const int nt = (ld + 63) / 64;
  const bool prof = options().profile != 0;
  const bool k32 = options().gemm_k == 32;
  if (prof) prof_begin(kProfGemm, s);
  // large tiles when the batch alone gives every CU two work-groups
  if (options().gemm_large && (size_t)count * ntl * ntl >= 512) {
    if (k32 && options().gemm_waves == 8)
      hipLaunchKernelGGL((k_gemm<T, 128, 32, 512>), dim3(ntl, ntl, count), dim3(512), 0, s, dops,
                         ld);
    else if (k32)
      hipLaunchKernelGGL((k_gemm<T, 128, 32>), dim3(ntl, ntl, count), dim3(kGemmThreads), 0, s,
                         dops, ld);
    else
      hipLaunchKernelGGL((k_gemm<T, 128, 16>), dim3(ntl, ntl, count), dim3(kGemmThreads), 0, s,
                         dops, ld);
  } else {
    if (k32)
      hipLaunchKernelGGL((k_gemm<T, 64, 32>), dim3(nt, nt, count), dim3(kGemmThreads), 0, s, dops,
                         ld);
    else
      hipLaunchKernelGGL((k_gemm<T, 64, 16>), dim3(nt, nt, count), dim3(kGemmThreads), 0, s, dops,
                         ld);
  }
  if (prof) prof_end(kProfGemm, s);
  return hipGetLastError();
}

// Row gathers of block-product operands (for the library GEMM path).  One
// work-group per (row, op).
template <class T>
__global__ void __launch_bounds__(256) k_gather_rows(const GatherOp<T> *ops, int ld) {
  const GatherOp<T> &o = ops[blockIdx.y];
  const int r = blockIdx.x;
  const auto src = gmem(o.src) + (size_t)in_block(gmem(o.idx)[r], ld) * ld;
  const auto dst = gmem(o.dst) + (size_t)r * ld;
  for (int j = threadIdx.x; j < ld; j += blockDim.x) dst[j] = src[j];
}

template <class T>
hipError_t launch_gather_rows(const GatherOp<T> *dops, int count, int ld, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_gather_rows<T>), dim3(ld, count), dim3(256), 0, s, dops, ld);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Level-0 Schur terms.  One work-group of 256 threads per (row r, kept
// layer).
template <class T>
__global__ void __launch_bounds__(256) k_cr_level0(const CrLevel0Op<T> *ops, int ld) {
  const CrLevel0Op<T> &o = ops[blockIdx.y];
  const int r = blockIdx.x;
  const T *wl = o.Wl ? o.Wl + (size_t)in_block(o.pl[r], ld) * ld : nullptr;
  const T *wr = o.Wr ? o.Wr + (size_t)in_block(o.pr[r], ld) * ld : nullptr;
  const double akr = o.ak[r], ckr = o.ck[r];
  T *D = o.D + (size_t)r * ld;
  // A thread's (up to four) entries: every gather index first, then every
  // gathered and row value, then the arithmetic, with no branch around a
  // load (an absent side reads this row of D in place of its index list and
  // inverse row, and discards it), so the chain is two loads deep.
  constexpr int kE = kMaxLd / 256;
  const int t = threadIdx.x;
  const auto ql = gmem(wl ? o.ql : reinterpret_cast<const int *>(D));
  const auto qr = gmem(wr ? o.qr : reinterpret_cast<const int *>(D));
  const auto wlg = gmem(wl ? wl : D), wrg = gmem(wr ? wr : D);
  int il[kE], ir[kE];
#pragma unroll
  for (int e = 0; e < kE; ++e) {
    const int j = min(t + 256 * e, ld - 1);
    il[e] = ql[j];
    ir[e] = qr[j];
  }
  // the op's coupling vectors and outputs, read before any store (a store
  // could otherwise alias them and force every later load to wait)
  const double *cl = o.cl, *al = o.al, *ar = o.ar, *cr = o.cr;
  T *Ao = o.A, *Co = o.C;
  const auto clg = gmem(wl ? cl : o.ak), alg = gmem(wl && Ao ? al : o.ak);
  const auto arg = gmem(wr ? ar : o.ak), crg = gmem(wr && Co ? cr : o.ak);
  double dv[kE], el[kE], er[kE], vcl[kE], val[kE], var[kE], vcr[kE];
#pragma unroll
  for (int e = 0; e < kE; ++e) {
    const int j = min(t + 256 * e, ld - 1);
    dv[e] = (double)gmem(D)[j];
    el[e] = (double)wlg[wl ? in_block(il[e], ld) : j];
    er[e] = (double)wrg[wr ? in_block(ir[e], ld) : j];
    vcl[e] = clg[j];
    val[e] = alg[j];
    var[e] = arg[j];
    vcr[e] = crg[j];
  }
#pragma unroll
  for (int e = 0; e < kE; ++e) {
    const int j = t + 256 * e;
    if (j >= ld) break;
    double d = dv[e];
    if (wl) {
      d -= akr * el[e] * vcl[e];
      if (Ao) Ao[(size_t)r * ld + j] = (T)(-akr * el[e] * val[e]);
    }
    if (wr) {
      d -= ckr * er[e] * var[e];
      if (Co) Co[(size_t)r * ld + j] = (T)(-ckr * er[e] * vcr[e]);
    }
    D[j] = (T)d;
  }
}

template <class T>
hipError_t launch_cr_level0(const CrLevel0Op<T> *dops, int count, int ld, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_cr_level0<T>), dim3(ld, count), dim3(256), 0, s, dops, ld);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Matrix-vector terms.  One work-group of four waves (256 threads) per 8
// output rows of one op; the (gathered) input vectors are staged in LDS.  Each wave reduces
// two rows, with every matrix element it needs loaded before the first is
// used (ld <= kMaxLd: at most 16 per lane, row and term).
constexpr int kMvRows = 2;                 // rows per wave
constexpr int kMvChunks = kMaxLd / 64;     // row elements per lane

template <class T>
__global__ void __launch_bounds__(256) k_mv(const MvOp<T> *__restrict__ ops, int ld) {
  const MvOp<T> &o = ops[blockIdx.y];
  __shared__ double xs[2][kMaxLd];
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const int nterm = o.nterm;
  // The (gathered) input vectors: every gather index first, then every
  // value, then the LDS stores, with no branch around a load, so the chain
  // is two loads deep.  A term without a gather (or absent) reads the op's
  // output vector (ld doubles, always valid) in place of an index list and
  // discards what it read.
  constexpr int kXs = kMaxLd / 256;          // elements per thread and term
  int xi[2][kXs];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const bool gath = q < nterm && o.t[q].xm;
    const auto xm = gmem(gath ? o.t[q].xm : reinterpret_cast<const int *>(o.y));
#pragma unroll
    for (int e = 0; e < kXs; ++e) xi[q][e] = xm[min(t + 256 * e, ld - 1)];
#pragma unroll
    for (int e = 0; e < kXs; ++e) xi[q][e] = gath ? in_block(xi[q][e], ld) : min(t + 256 * e, ld - 1);
  }
  double xv[2][kXs];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const auto x = gmem(q < nterm ? o.t[q].x : o.y);
#pragma unroll
    for (int e = 0; e < kXs; ++e) xv[q][e] = x[xi[q][e]];
  }
#pragma unroll
  for (int q = 0; q < 2; ++q)
    if (q < nterm) {
#pragma unroll
      for (int e = 0; e < kXs; ++e)
        if (t + 256 * e < ld) xs[q][t + 256 * e] = xv[q][e];
    }
  const int j0 = (blockIdx.x * 4 + wid) * kMvRows;
  T mv[kMvRows][2][kMvChunks];
  if constexpr (sizeof(T) == 4) {
    // FP32: every chunk of every (row, term) pair is loaded with its column
    // clamped into the row and no branch, so all 64 loads of a lane are in
    // flight together (branches would each wait for their loads, as the
    // conversion to FP64 moves into them).  A pair that is not present (the
    // same for the whole wave) reads the op's output vector, ld doubles and
    // always valid; the products below skip it and the chunks past ld.
    const T *base[kMvRows][2];
    int src[kMvRows][2];
#pragma unroll
    for (int rr = 0; rr < kMvRows; ++rr)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int j = j0 + rr;
        const MvTerm<T> &tm = o.t[q];
        const bool on = q < nterm && tm.M && j < ld;
        const bool perm = on && tm.rm;
        base[rr][q] = on ? tm.M : reinterpret_cast<const T *>(o.y);
        src[rr][q] = gmem(perm ? tm.rm : reinterpret_cast<const int *>(o.y))[min(j, ld - 1)];
        src[rr][q] = perm ? in_block(src[rr][q], ld) : (on ? j : 0);
      }
#pragma unroll
    for (int rr = 0; rr < kMvRows; ++rr)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const auto row = gmem(base[rr][q]) + (size_t)src[rr][q] * ld;
#pragma unroll
        for (int c = 0; c < kMvChunks; ++c) mv[rr][q][c] = row[min(lane + 64 * c, ld - 1)];
      }
  } else {
    // FP64: one (row, term) pair's 16 loads in flight at a time, which keeps
    // the registers (and so the waves per SIMD) of the FP64 kernel.
#pragma unroll
    for (int rr = 0; rr < kMvRows; ++rr)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int j = j0 + rr;
        const MvTerm<T> &tm = o.t[q];
        const bool on = q < nterm && tm.M && j < ld;
        const auto row =
            gmem(tm.M) + (size_t)(on && tm.rm ? in_block(gmem(tm.rm)[j], ld) : j) * ld;
#pragma unroll
        for (int c = 0; c < kMvChunks; ++c) {
          const int m = lane + 64 * c;
          mv[rr][q][c] = (on && m < ld) ? row[m] : T(0);
        }
      }
  }
  __syncthreads();
#pragma unroll
  for (int rr = 0; rr < kMvRows; ++rr) {
    const int j = j0 + rr;
    if (j >= ld) break;
    double y = o.b ? o.b[j] : 0.0;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (q >= nterm) break;
      const MvTerm<T> &tm = o.t[q];
      double v;
      if (tm.M) {
        double z = 0.0;
#pragma unroll
        for (int c = 0; c < kMvChunks; ++c) {
          const int m = lane + 64 * c;
          if (m < ld) z = fma((double)mv[rr][q][c], xs[q][m], z);
        }
        for (int off = 32; off > 0; off >>= 1) z += __shfl_xor(z, off, 64);
        v = z;
      } else {
        v = xs[q][j];
      }
      y += tm.sgn * (tm.s ? tm.s[j] : 1.0) * v;
    }
    if (lane == 0) o.y[j] = y;
  }
}

template <class T>
hipError_t launch_mv(const MvOp<T> *dops, int count, int ld, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const bool prof = options().profile != 0;
  if (prof) prof_begin(kProfSolve, s);
  const int rows = 4 * kMvRows;
  hipLaunchKernelGGL((k_mv<T>), dim3((ld + rows - 1) / rows, count), dim3(256), 0, s, dops, ld);
  if (prof) prof_end(kProfSolve, s);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
__global__ void k_pad_copy(const double *src, double *dst, int N, int S, int ld, int to_padded) {
  const size_t total = (size_t)N * ld;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const size_t k = e / ld;
    const int y = (int)(e % ld);
    if (to_padded)
      dst[e] = y < S ? src[k * S + y] : 0.0;
    else if (y < S)
      dst[k * S + y] = src[e];
  }
}

hipError_t launch_pad_copy(const double *src, double *dst, int N, int S, int ld, bool to_padded,
                           hipStream_t s) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pad_copy, dim3(64), dim3(256), 0, s, src, dst, N, S, ld,
                     to_padded ? 1 : 0);
  return hipGetLastError();
}

// rstep <- INT_MAX for all N*ld entries, flags <- -1.
__global__ void k_cr_reset(int *rstep, size_t n, int *flag) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    rstep[e] = INT_MAX;
  if (blockIdx.x == 0 && threadIdx.x < 4) flag[threadIdx.x] = -1;
}

hipError_t launch_cr_reset(int *rstep, size_t n, int *flag, hipStream_t s) {
  hipLaunchKernelGGL(k_cr_reset, dim3(64), dim3(256), 0, s, rstep, n, flag);
  return hipGetLastError();
}

template hipError_t launch_gemm<double>(const GemmOp<double> *, int, int, hipStream_t);
template hipError_t launch_gather_rows<double>(const GatherOp<double> *, int, int, hipStream_t);
template hipError_t launch_gather_rows<float>(const GatherOp<float> *, int, int, hipStream_t);
template hipError_t launch_gemm<float>(const GemmOp<float> *, int, int, hipStream_t);
template hipError_t launch_cr_level0<double>(const CrLevel0Op<double> *, int, int, hipStream_t);
template hipError_t launch_cr_level0<float>(const CrLevel0Op<float> *, int, int, hipStream_t);
template hipError_t launch_mv<double>(const MvOp<double> *, int, int, hipStream_t);
template hipError_t launch_mv<float>(const MvOp<float> *, int, int, hipStream_t);

}  // namespace xod
