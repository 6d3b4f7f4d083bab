// State update and step statistics (n_new = n + delta), deterministic
// two-stage reductions (no floating-point atomics).
#include <algorithm>

#include "xod_internal.h"

namespace xod {

__global__ void __launch_bounds__(256) k_update_state(const UpdArgs *args) {
  const UpdArgs u = args[blockIdx.y];
  const size_t total = (size_t)u.N * u.S;
  double mrel = 0.0, mratio = 1e300, mctl = 0.0, clipped = 0.0, negsig = 0.0, nonfin = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(e / u.S);
    const double ng = u.ngas[k];
    const double n0 = u.n[e];
    double v = n0 + u.x[e];
    if (!isfinite(v)) nonfin = 1.0;
    if (u.clip) {
      if (v < 0.0) {
        if (n0 > u.y_sig * ng && v < -u.y_neg * ng) negsig = 1.0;
        clipped += -v;
        v = 0.0;
      }
      if (v > u.y_sig * ng) mctl = fmax(mctl, fabs(v - n0) / fmax(n0, v));
    }
    mratio = fmin(mratio, v / ng);
    if (v > u.y_floor * ng) mrel = fmax(mrel, fabs(v - n0) / v);
    u.nout[e] = v;
  }
  __shared__ double red[kNStat][256];
  const int t = threadIdx.x;
  red[0][t] = mrel; red[1][t] = mratio; red[2][t] = mctl;
  red[3][t] = clipped; red[4][t] = negsig; red[5][t] = nonfin;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) {
      red[0][t] = fmax(red[0][t], red[0][t + o]);
      red[1][t] = fmin(red[1][t], red[1][t + o]);
      red[2][t] = fmax(red[2][t], red[2][t + o]);
      red[3][t] = red[3][t] + red[3][t + o];
      red[4][t] = fmax(red[4][t], red[4][t + o]);
      red[5][t] = fmax(red[5][t], red[5][t + o]);
    }
    __syncthreads();
  }
  if (t < kNStat) u.partial[blockIdx.x * kNStat + t] = red[t][0];
}

// Final reduction, one thread per column, fixed order.  Also copies the
// column's error flags so one transfer brings everything to the host.
__global__ void k_reduce_stats(const RedArgs *args, int ncols) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= ncols) return;
  const RedArgs r = args[col];
  double s[kNStat] = {0.0, 1e300, 0.0, 0.0, 0.0, 0.0};
  for (int b = 0; b < kUpdBlocks; ++b) {
    const double *p = r.partial + b * kNStat;
    s[0] = fmax(s[0], p[0]);
    s[1] = fmin(s[1], p[1]);
    s[2] = fmax(s[2], p[2]);
    s[3] += p[3];
    s[4] = fmax(s[4], p[4]);
    s[5] = fmax(s[5], p[5]);
  }
  for (int q = 0; q < kNStat; ++q) r.out[q] = s[q];
  for (int q = 0; q < 4; ++q) r.out[kNStat + q] = (double)r.flag[q];
}

hipError_t launch_update_state(const UpdArgs *dargs, const RedArgs *dred, int ncols,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_update_state, dim3(kUpdBlocks, ncols), dim3(256), 0, s, dargs);
  hipLaunchKernelGGL(k_reduce_stats, dim3((ncols + 63) / 64), dim3(64), 0, s, dred, ncols);
  return hipGetLastError();
}

// Inverse permutation rstep[piv[j]] = j for every layer (the solve needs it).
__global__ void k_invperm(const int *piv, int *rstep, int N, int ld) {
  const size_t total = (size_t)N * ld;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const size_t k = e / ld;
    const int r = piv[e];
    if (r >= 0 && r < ld) rstep[k * ld + r] = (int)(e - k * ld);
  }
}

hipError_t launch_invperm(const int *piv, int *rstep, int N, int ld, hipStream_t s) {
  hipLaunchKernelGGL(k_invperm, dim3(256), dim3(256), 0, s, piv, rstep, N, ld);
  return hipGetLastError();
}

// out = alpha p + beta q, elementwise over n doubles (the Rosenbrock stage
// state, stage right-hand side and final combination).  out may be p or q.
__global__ void __launch_bounds__(256) k_lincomb(double *out, const double *p, double alpha,
                                                 const double *q, double beta, size_t n) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    out[e] = alpha * p[e] + beta * q[e];
}

hipError_t launch_lincomb(double *out, const double *p, double alpha, const double *q,
                          double beta, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_lincomb, dim3((unsigned)blocks), dim3(256), 0, s, out, p, alpha, q,
                     beta, n);
  return hipGetLastError();
}

// Lagrangian parcel at layer k: the molecular-diffusion gains of its
// right-hand side, f += max(trd_k, 0) prof_k + trl_k prof_{k-1} + tru_k
// prof_{k+1} (the profile's densities as fixed sources), and the loss part
// of the self-coefficient for all layers, loss = min(trd, 0).
__global__ void __launch_bounds__(256) k_parcel_gain(double *f, const double *prof,
                                                     const double *trl, const double *trd,
                                                     const double *tru, int N, int S, int k) {
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  if (y >= S) return;
  const size_t o = (size_t)k * S + y;
  double g = fmax(trd[o], 0.0) * prof[o];
  if (k >= 1) g += trl[o] * prof[o - S];
  if (k + 1 < N) g += tru[o] * prof[o + S];
  f[y] += g;
}

__global__ void __launch_bounds__(256) k_min0(const double *in, double *out, size_t n) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    out[e] = fmin(in[e], 0.0);
}

hipError_t launch_parcel_gain(double *f, const double *prof, const double *trl,
                              const double *trd, const double *tru, int N, int S, int k,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_parcel_gain, dim3((S + 255) / 256), dim3(256), 0, s, f, prof, trl, trd,
                     tru, N, S, k);
  return hipGetLastError();
}

hipError_t launch_min0(const double *in, double *out, size_t n, hipStream_t s) {
  const size_t blocks = std::min<size_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_min0, dim3((unsigned)blocks), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

}  // namespace xod
