// Column set-up, rate coefficients, right-hand side and step-matrix assembly.
//
//   k_setup   grid of one column (Section 2.1 discretisation, Section 2.3.3
//             optical depth, Appendix A Gibbs energies)
//   k_rates   k_f, k_r per (layer, reaction) (Section 2.3.1-2.3.4)
//   k_wrate   reaction rates w = k_f prod n - k_r prod n
//   k_rhs     F = P - L - d(phi)/dz (Eq. continuity, Eq. transportflux)
//   k_jac     dense blocks of M = I/dt - dF/dn plus the diagonal couplings
//
// All arithmetic is FP64.  HBM-bound: one thread per output element, reads
// of per-layer vectors hit L1/L2.
#include "xod_internal.h"
#include "mfma.h"

namespace xod {

// ---------------------------------------------------------------------------
// Column set-up (one work-group; runs once per column).


__device__ __forceinline__ double gibbs_rt(const double *a, double T) {
  // Appendix A: G/RT = a1(1 - ln T) - a2 T/2 - a3 T^2/6 - a4 T^3/12
  //                    - a5 T^4/20 + a6/T - a7
  const double T2 = T * T;
  return a[0] * (1.0 - log(T)) - a[1] * T / 2.0 - a[2] * T2 / 6.0 -
         a[3] * T2 * T / 12.0 - a[4] * T2 * T2 / 20.0 + a[5] / T - a[6];
}

__global__ void __launch_bounds__(256) k_setup(SetupArgs s) {
  const int N = s.N, S = s.S, tid = threadIdx.x;
  const double mbar = s.mbar_amu * kAmu;
  __shared__ double red[256];
  for (int k = tid; k < N; k += blockDim.x) {
    s.ngas[k] = s.P_bar[k] * kPstd / (kBoltz * s.T[k]);
    s.lnpref[k] = log(kPstd / (kBoltz * s.T[k]));
  }
  if (tid == 0) {
    // Hydrostatic heights: z_{k+1} = z_k + k_B T_{k+1/2}/(mbar g) ln(P_k/P_{k+1});
    // layer thickness = mean of the adjacent half-level intervals.
    for (int k = 0; k + 1 < N; ++k) {
      const double Th = 0.5 * (s.T[k] + s.T[k + 1]);
      s.dzh[k] = kBoltz * Th / (mbar * s.g_cgs) * log(s.P_bar[k] / s.P_bar[k + 1]);
    }
    if (N == 1) {
      s.dz[0] = kBoltz * s.T[0] / (mbar * s.g_cgs);
    } else {
      for (int k = 0; k < N; ++k) {
        const double below = k >= 1 ? s.dzh[k - 1] : s.dzh[k];
        const double above = k <= N - 2 ? s.dzh[k] : s.dzh[k - 1];
        s.dz[k] = 0.5 * (below + above);
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    // Optical depth: total-gas column above each layer midpoint.
    double above = 0.0;
    for (int k = N - 1; k >= 0; --k) {
      const double ng = s.P_bar[k] * kPstd / (kBoltz * s.T[k]);
      s.tau[k] = s.sigma_tau * (0.5 * ng * s.dz[k] + above);
      above += ng * s.dz[k];
    }
  }
  __syncthreads();
  double mixloc = 0.0;
  for (int e = tid; e < N * S; e += blockDim.x) {
    const int k = e / S, y = e - k * S;
    const double T = s.T[k];
    const double *a = s.nasa7 + (size_t)y * 14 + (T >= s.t_mid ? 7 : 0);
    s.g[e] = gibbs_rt(a, T);
    // Transport coefficients of f_tr,k = trl n_{k-1} + trd n_k + tru n_{k+1}.
    double p_up = 0.0, q_up = 0.0, p_dn = 0.0, q_dn = 0.0;
    const double Dk = s.D ? s.D[e] : 0.0;
    const double al = s.alpha ? s.alpha[y] : 0.0;
    const double my = s.mass[y] * kAmu;
    if (k + 1 < N) {  // half level k+1/2
      const double Th = 0.5 * (T + s.T[k + 1]);
      const double nh = 0.5 * (s.ngas[k] + s.ngas[k + 1]);
      const double Kh = 0.5 * (s.K[k] + s.K[k + 1]);
      const double Dh = 0.5 * (Dk + (s.D ? s.D[e + S] : 0.0));
      const double dzh = s.dzh[k];
      const double beta = (my - mbar) * s.g_cgs / (kBoltz * Th) +
                          al * (s.T[k + 1] - T) / (Th * dzh);
      const double KD = Kh + Dh;
      p_up = nh * (KD / dzh + 0.5 * Dh * beta) / s.ngas[k + 1];
      q_up = nh * (-KD / dzh + 0.5 * Dh * beta) / s.ngas[k];
      if (KD > 0.0) mixloc = fmax(mixloc, dzh * dzh / KD);
    }
    if (k >= 1) {  // half level k-1/2
      const double Tl = s.T[k - 1];
      const double Th = 0.5 * (Tl + T);
      const double nh = 0.5 * (s.ngas[k - 1] + s.ngas[k]);
      const double Kh = 0.5 * (s.K[k - 1] + s.K[k]);
      const double Dh = 0.5 * ((s.D ? s.D[e - S] : 0.0) + Dk);
      const double dzh = s.dzh[k - 1];
      const double beta = (my - mbar) * s.g_cgs / (kBoltz * Th) +
                          al * (T - Tl) / (Th * dzh);
      const double KD = Kh + Dh;
      p_dn = nh * (KD / dzh + 0.5 * Dh * beta) / s.ngas[k];
      q_dn = nh * (-KD / dzh + 0.5 * Dh * beta) / s.ngas[k - 1];
    }
    const double dz = s.dz[k];
    s.trl[e] = k >= 1 ? -q_dn / dz : 0.0;
    s.trd[e] = (q_up - p_dn) / dz;
    s.tru[e] = k + 1 < N ? p_up / dz : 0.0;
  }
  red[tid] = mixloc;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (tid < o) red[tid] = fmax(red[tid], red[tid + o]);
    __syncthreads();
  }
  if (tid == 0) s.mix[0] = red[0];
}

hipError_t launch_setup(const SetupArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(k_setup, dim3(1), dim3(256), 0, st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Rate coefficients: one thread per (layer, reaction).
template <class Acc>
__global__ void __launch_bounds__(256) k_rates(Acc acc) {
  const ColArgs &c = acc(blockIdx.z);
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (r >= c.R || k >= c.N) return;
  const double T = c.T[k];
  const double lnT = log(T);
  const double *p = c.params + (size_t)r * 6;
  const double lnTb = c.kooij[r] ? lnT - log(300.0) : lnT;
  const int type = c.rtype[r];
  double kf;
  if (type == XOD_RT_BIMOL) {
    kf = exp(p[0] + p[1] * lnTb - p[2] / T);
  } else if (type == XOD_RT_TERMOL) {
    const double k0 = exp(p[0] + p[1] * lnTb - p[2] / T);
    const double ki = exp(p[3] + p[4] * lnTb - p[5] / T);
    const double k0M = k0 * c.ngas[k];
    kf = k0M / (1.0 + k0M / ki);
  } else if (c.kph) {             // spectral rates of this step's starting state
    kf = c.kph[(size_t)k * c.nph + c.photo_idx[r]];
  } else {
    kf = exp(p[0] - c.tau[k]);
  }
  double kr = 0.0;
  if (c.rev[r] && type != XOD_RT_PHOTO) {
    const double *g = c.g + (size_t)k * c.S;
    double dg = 0.0;
    for (int j = 0; j < XOD_MAX_PROD; ++j) {
      const int y = c.prod[r * XOD_MAX_PROD + j];
      if (y >= 0) dg += g[y];
    }
    for (int j = 0; j < XOD_MAX_REAC; ++j) {
      const int y = c.reac[r * XOD_MAX_REAC + j];
      if (y >= 0) dg -= g[y];
    }
    // k_r = k_f / K_c, K_c = exp(-dg) (P0/kT)^dnu
    kr = kf * exp(dg - (double)c.dnu[r] * c.lnpref[k]);
  }
  const size_t o = (size_t)k * c.R + r;
  c.kf[o] = kf;
  c.kr[o] = kr;
}

template <class Acc>
hipError_t launch_rates(const Acc &acc, int ncols, int maxN, int maxR, hipStream_t s) {
  if (maxR <= 0 || maxN <= 0) return hipSuccess;
  dim3 grid((maxR + 255) / 256, maxN, ncols);
  if (options().profile) prof_begin(kProfRates, s);
  hipLaunchKernelGGL(k_rates<Acc>, grid, dim3(256), 0, s, acc);
  if (options().profile) prof_end(kProfRates, s);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Reaction rates and right-hand side.
template <class Acc>
__global__ void __launch_bounds__(256) k_wrate(Acc acc) {
  const ColArgs &c = acc(blockIdx.z);
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (r >= c.R || k >= c.N) return;
  const double *n = c.n + (size_t)k * c.S;
  double fw = 1.0, rv = 1.0;
  for (int j = 0; j < XOD_MAX_REAC; ++j) {
    const int y = c.reac[r * XOD_MAX_REAC + j];
    if (y >= 0) fw *= n[y];
  }
  for (int j = 0; j < XOD_MAX_PROD; ++j) {
    const int y = c.prod[r * XOD_MAX_PROD + j];
    if (y >= 0) rv *= n[y];
  }
  const size_t o = (size_t)k * c.R + r;
  c.w[o] = c.kf_in[o] * fw - c.kr_in[o] * rv;
}

template <class Acc>
__global__ void __launch_bounds__(256) k_rhs(Acc acc) {
  const ColArgs &c = acc(blockIdx.z);
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (y >= c.S || k >= c.N) return;
  const double *w = c.w + (size_t)k * c.R;
  double f = 0.0;
  for (int e = c.inc_ptr[y]; e < c.inc_ptr[y + 1]; ++e) f += c.inc_nu[e] * w[c.inc_r[e]];
  const size_t o = (size_t)k * c.S + y;
  double tr = c.trd[o] * c.n[o];
  if (k >= 1) tr += c.trl[o] * c.n[o - c.S];
  if (k + 1 < c.N) tr += c.tru[o] * c.n[o + c.S];
  if (k == 0 && c.bsrc) tr += c.bsrc[y];
  c.f[o] = f + tr;
}

template <class Acc>
hipError_t launch_rhs(const Acc &acc, int ncols, int maxN, int maxR, int maxS, hipStream_t s) {
  if (maxN <= 0) return hipSuccess;
  if (options().profile) prof_begin(kProfRhs, s);
  if (maxR > 0) {
    dim3 g1((maxR + 255) / 256, maxN, ncols);
    hipLaunchKernelGGL(k_wrate<Acc>, g1, dim3(256), 0, s, acc);
  }
  dim3 g2((maxS + 255) / 256, maxN, ncols);
  hipLaunchKernelGGL(k_rhs<Acc>, g2, dim3(256), 0, s, acc);
  if (options().profile) prof_end(kProfRhs, s);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Step-matrix assembly: one wave per (layer, block row).
//
// dw_r/dn_x = k_f sum_{slots s: reac_s = x} prod_{t != s} n_{reac_t}
//           - k_r sum_{slots s: prod_s = x} prod_{t != s} n_{prod_t}
__device__ __forceinline__ double dwdn(const ColArgs &c, int k, int r, int x) {
  const double *n = c.n + (size_t)k * c.S;
  double df = 0.0, dr = 0.0;
  const int *rc = c.reac + r * XOD_MAX_REAC;
  const int *pc = c.prod + r * XOD_MAX_PROD;
  for (int s = 0; s < XOD_MAX_REAC; ++s) {
    if (rc[s] != x) continue;
    double p = 1.0;
    for (int t = 0; t < XOD_MAX_REAC; ++t)
      if (t != s && rc[t] >= 0) p *= n[rc[t]];
    df += p;
  }
  for (int s = 0; s < XOD_MAX_PROD; ++s) {
    if (pc[s] != x) continue;
    double p = 1.0;
    for (int t = 0; t < XOD_MAX_PROD; ++t)
      if (t != s && pc[t] >= 0) p *= n[pc[t]];
    dr += p;
  }
  const size_t o = (size_t)k * c.R + r;
  return c.kf_in[o] * df - c.kr_in[o] * dr;
}

// dw_r/dn_x for every reaction and each of its distinct species x = rsp[6r+u]
// (zero for unused slots): the Jacobian entries then gather one value per
// contribution.
template <class Acc>
__global__ void __launch_bounds__(256) k_dwd(Acc acc) {
  const ColArgs &c = acc(blockIdx.z);
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (r >= c.R || k >= c.N) return;
  double *out = c.dwd + ((size_t)k * c.R + r) * 6;
#pragma unroll
  for (int u = 0; u < 6; ++u) {
    const int x = c.rsp[r * 6 + u];
    out[u] = x >= 0 ? dwdn(c, k, r, x) : 0.0;
  }
}

constexpr int kJacMaxPer = kMaxLd / 64;

// One wave per (layer, block row): the row is assembled in LDS (zeros, the
// contributions of the row's nonzero entries added in, then the diagonal), then
// read back by columns and stored with full-row coalesced writes (scaled to
// unit max-norm in the mixed path).
template <class Acc, bool kMixed>
__global__ void __launch_bounds__(256) k_jac(Acc acc) {
  const ColArgs &c = acc(blockIdx.z);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = blockIdx.x * 4 + w;
  const int k = blockIdx.y;
  const int ld = c.ld, S = c.S;
  const bool on = k < c.N && i < ld;
  __shared__ double rowbuf[4][kMaxLd];
  double *rb = rowbuf[w];
  if (on) {
    for (int j = lane; j < ld; j += 64) rb[j] = 0.0;
  }
  __syncthreads();
  if (on && i < S) {
    // the row's contributions, spread evenly over the lanes (an entry of a
    // species in many reactions has hundreds), added into LDS
    const auto dk = gmem((const double *)c.dwd) + (size_t)k * c.R * 6;
    const auto jptr = gmem(c.jptr), jrow = gmem(c.jrow);
    const int q1 = jptr[jrow[i + 1]];
#pragma unroll 4
    for (int q = jptr[jrow[i]] + lane; q < q1; q += 64)
      atomicAdd(&rb[gmem(c.jc_col)[q]], -gmem(c.jc_nu)[q] * dk[gmem(c.jc_ru)[q]]);
  }
  __syncthreads();
  if (on && lane == 0)
    rb[i] = i < S ? rb[i] + 1.0 / c.dt - c.trd[(size_t)k * S + i] : 1.0;   // identity padding
  __syncthreads();
  if (!on) return;
  const size_t ro = (size_t)k * ld + i;
  const size_t so = (size_t)k * S + i;
  const double av = i < S ? -c.trl[so] : 0.0;
  const double cv = i < S ? -c.tru[so] : 0.0;
  double vals[kJacMaxPer];
  double amax = fmax(fabs(av), fabs(cv));
#pragma unroll
  for (int q = 0; q < kJacMaxPer; ++q) {
    const int j = lane + 64 * q;
    vals[q] = j < ld ? rb[j] : 0.0;
    amax = fmax(amax, fabs(vals[q]));
  }
  if (kMixed) {
    for (int o = 32; o > 0; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o, 64));
    const double sc = amax > 0.0 ? 1.0 / amax : 1.0;
    const auto Bf = gmem(c.Bf) + ro * ld;
#pragma unroll
    for (int q = 0; q < kJacMaxPer; ++q) {
      const int j = lane + 64 * q;
      if (j < ld) Bf[j] = (float)(sc * vals[q]);
    }
    if (lane == 0) {
      c.rs[ro] = sc;
      c.a[ro] = sc * av;
      c.c[ro] = sc * cv;
    }
  } else {
    const auto B = gmem(c.B) + ro * ld;
#pragma unroll
    for (int q = 0; q < kJacMaxPer; ++q) {
      const int j = lane + 64 * q;
      if (j < ld) B[j] = vals[q];
    }
    if (lane == 0) {
      c.a[ro] = av;
      c.c[ro] = cv;
    }
  }
}

template <class Acc>
hipError_t launch_jacobian(const Acc &acc, int ncols, int maxN, int maxR, int ld, bool mixed,
                           hipStream_t s) {
  if (maxN <= 0) return hipSuccess;
  dim3 grid((ld + 3) / 4, maxN, ncols);
  if (options().profile) prof_begin(kProfJac, s);
  if (maxR > 0)
    hipLaunchKernelGGL(k_dwd<Acc>, dim3((maxR + 255) / 256, maxN, ncols), dim3(256), 0, s, acc);
  if (mixed)
    hipLaunchKernelGGL((k_jac<Acc, true>), grid, dim3(256), 0, s, acc);
  else
    hipLaunchKernelGGL((k_jac<Acc, false>), grid, dim3(256), 0, s, acc);
  if (options().profile) prof_end(kProfJac, s);
  return hipGetLastError();
}

template hipError_t launch_rates<OneCol>(const OneCol &, int, int, int, hipStream_t);
template hipError_t launch_rates<ManyCols>(const ManyCols &, int, int, int, hipStream_t);
template hipError_t launch_rhs<OneCol>(const OneCol &, int, int, int, int, hipStream_t);
template hipError_t launch_rhs<ManyCols>(const ManyCols &, int, int, int, int, hipStream_t);
template hipError_t launch_jacobian<OneCol>(const OneCol &, int, int, int, int, bool,
                                            hipStream_t);
template hipError_t launch_jacobian<ManyCols>(const ManyCols &, int, int, int, int, bool,
                                              hipStream_t);

}  // namespace xod
