// Spectral photolysis rate coefficients (Section 2.3.3: the actinic flux
// with its attenuation by the optical depth, and the rate integral over
// wavelength), FP64:
//   Ncol[k][a] = n[k][sp_a] dz_k / 2 + sum_{j>k} n[j][sp_a] dz_j     (column above)
//   tau[k][b]  = sum_a Ncol[k][a] sig_ext[a][b]                        (GEMM, K = A)
//   E[k][b]    = t_f J0[b] dlam[b] exp(-tau[k][b] / mu)                (epilogue)
//   kph[k][p]  = sum_b E[k][b] sig_ph[p][b]                            (GEMM, K = L)
// The two products run on FP64 MFMA (16x16x4) in 64 x 64 output tiles; a
// product with few output tiles splits K over work-groups, each writing its
// partial tile, and the epilogue sums the parts in order (deterministic).
#include "xod_internal.h"
#include "mfma.h"

#include <algorithm>
#include <mutex>

#define PH_CHECK(cond, msg)      \
  do {                           \
    if (!(cond)) {               \
      ::xod::set_error(msg);     \
      return XOD_EINVAL;         \
    }                            \
  } while (0)

namespace xod {

namespace {

constexpr int kPhTile = 64, kPhK = 32, kPhThreads = 256;

// Column densities above each layer midpoint, one thread per absorber.
__global__ void __launch_bounds__(256) k_ph_column(const double *n, const double *dz,
                                                   const int *absorbers, int N, int S, int A,
                                                   double *ncol) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= A) return;
  const int sp = absorbers[a];
  double above = 0.0;
  for (int k = N - 1; k >= 0; --k) {
    const double c = n[(size_t)k * S + sp] * dz[k];
    ncol[(size_t)k * A + a] = above + 0.5 * c;
    above += c;
  }
}

// Part z of C[M][Nc] = A[M][K] B, with B stored as [K][Nc] (kBT = false) or
// as [Nc][K] (kBT = true); part z sums k in [z*kc, min(K, (z+1)*kc)).
// Four waves in a 2 x 2 grid, each owning a 32 x 32 sub-tile (2 x 2 MFMA
// accumulators); K staged through LDS kPhK at a time, double-buffered: the
// next step's global loads are issued before the current step's MFMAs.
template <bool kBT>
__global__ void __launch_bounds__(kPhThreads) k_ph_gemm(const double *A, const double *B,
                                                        double *part, int M, int Nc, int K,
                                                        int kc) {
  constexpr int kE = kPhTile * kPhK / kPhThreads;   // staged elements per thread and operand
  const int tm0 = blockIdx.y * kPhTile, tn0 = blockIdx.x * kPhTile;
  const int z = blockIdx.z;
  const int kb = z * kc, ke = min(K, kb + kc);
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  __shared__ double As[2][kPhTile][kPhK + 1];
  __shared__ double Bs[2][kPhK][kPhTile + 2];
  double4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (double4_t){0, 0, 0, 0};
  const auto Ag = gmem(A), Bg = gmem(B);
  double ra[kE], rb[kE];
  auto gload = [&](int k0) {
#pragma unroll
    for (int e = 0; e < kE; ++e) {
      const int idx = t + e * kPhThreads;
      const int gr = tm0 + idx / kPhK, gk = k0 + idx % kPhK;
      ra[e] = (gr < M && gk < ke) ? Ag[(size_t)gr * K + gk] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < kE; ++e) {
      const int idx = t + e * kPhThreads;
      // consecutive threads walk K of one column (kBT) or the columns of one k
      const int c = kBT ? idx / kPhK : idx % kPhTile;
      const int kk = kBT ? idx % kPhK : idx / kPhTile;
      const int gc = tn0 + c, gk = k0 + kk;
      double v = 0.0;
      if (gc < Nc && gk < ke) v = kBT ? Bg[(size_t)gc * K + gk] : Bg[(size_t)gk * Nc + gc];
      rb[e] = v;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int e = 0; e < kE; ++e) {
      const int idx = t + e * kPhThreads;
      As[buf][idx / kPhK][idx % kPhK] = ra[e];
      const int c = kBT ? idx / kPhK : idx % kPhTile;
      const int kk = kBT ? idx % kPhK : idx / kPhTile;
      Bs[buf][kk][c] = rb[e];
    }
  };
  const int nsteps = ke > kb ? (ke - kb + kPhK - 1) / kPhK : 0;
  if (nsteps > 0) {
    gload(kb);
    sstore(0);
  }
  __syncthreads();
  for (int st = 0; st < nsteps; ++st) {
    const int buf = st & 1;
    if (st + 1 < nsteps) gload(kb + (st + 1) * kPhK);
#pragma unroll
    for (int q = 0; q < kPhK / 4; ++q) {
      double av[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        av[i] = As[buf][wr * 32 + i * 16 + (lane & 15)][q * 4 + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < 2; ++j)
        bv[j] = Bs[buf][q * 4 + (lane >> 4)][wc * 32 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma16(av[i], bv[j], acc[i][j]);
    }
    if (st + 1 < nsteps) sstore(buf ^ 1);
    __syncthreads();
  }
  const auto P = gmem(part) + (size_t)z * M * Nc;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = tn0 + wc * 32 + j * 16 + (lane & 15);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = tm0 + wr * 32 + i * 16 + mfma_row(0.0, lane, q);
        if (r < M && c < Nc) P[(size_t)r * Nc + c] = acc[i][j][q];
      }
    }
}

// E[k][b] = t_f J0[b] dlam[b] exp(-tau[k][b] / mu), tau the sum of the parts
// (no parts: tau = 0).
__global__ void __launch_bounds__(256) k_ph_flux(const double *part, int nparts, int N, int L,
                                                 const double *J0, const double *dlam,
                                                 double t_f, double mu, double *E) {
  const size_t total = (size_t)N * L;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    double tau = 0.0;
    for (int z = 0; z < nparts; ++z) tau += part[(size_t)z * total + e];
    const int b = (int)(e % L);
    E[e] = t_f * J0[b] * dlam[b] * exp(-tau / mu);
  }
}

// out[e] = sum of the parts, in order.
__global__ void __launch_bounds__(256) k_ph_sum(const double *part, int nparts, size_t total,
                                                double *out) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int z = 0; z < nparts; ++z) s += part[(size_t)z * total + e];
    out[e] = s;
  }
}

// K split so that the launch has about 512 work-groups, parts of at least
// 4 K steps.
int ph_parts(int M, int Nc, int K) {
  const int tiles = ((M + kPhTile - 1) / kPhTile) * ((Nc + kPhTile - 1) / kPhTile);
  const int want = (512 + tiles - 1) / tiles;
  const int most = std::max(1, (K + 4 * kPhK - 1) / (4 * kPhK));
  return std::max(1, std::min(want, most));
}

int ph_chunk(int K, int parts) {
  const int c = (K + parts - 1) / parts;
  return (c + kPhK - 1) / kPhK * kPhK;
}

size_t ph_work_doubles(int N, int A, int L, int P) {
  const int pt = A > 0 ? ph_parts(N, L, A) : 0;
  const int pk = P > 0 ? ph_parts(N, P, L) : 0;
  return (size_t)N * A + (size_t)N * L +
         std::max((size_t)pt * N * L, (size_t)pk * N * P);
}

}  // namespace

size_t photolysis_work_bytes(int N, int A, int L, int P) {
  return ph_work_doubles(N, A, L, P) * sizeof(double);
}

hipError_t launch_photolysis(int N, int S, int A, int L, int P, const double *n, const double *dz,
                             const int *absorbers, const double *sig_ext, const double *J0,
                             const double *dlam, const double *sig_ph, double t_f, double mu,
                             void *work, double *kph, hipStream_t s) {
  double *ncol = (double *)work;
  double *E = ncol + (size_t)N * A;
  double *part = E + (size_t)N * L;
  int pt = 0;
  if (A > 0) {
    hipLaunchKernelGGL(k_ph_column, dim3((A + 255) / 256), dim3(256), 0, s, n, dz, absorbers, N,
                       S, A, ncol);
    pt = ph_parts(N, L, A);
    const dim3 grid((L + kPhTile - 1) / kPhTile, (N + kPhTile - 1) / kPhTile, pt);
    hipLaunchKernelGGL(k_ph_gemm<false>, grid, dim3(kPhThreads), 0, s, ncol, sig_ext, part, N,
                       L, A, ph_chunk(A, pt));
  }
  hipLaunchKernelGGL(k_ph_flux, dim3(1024), dim3(256), 0, s, part, pt, N, L, J0, dlam, t_f, mu,
                     E);
  if (P > 0) {
    const int pk = ph_parts(N, P, L);
    const dim3 grid((P + kPhTile - 1) / kPhTile, (N + kPhTile - 1) / kPhTile, pk);
    if (options().profile) prof_begin(kProfPhoto, s);
    hipLaunchKernelGGL(k_ph_gemm<true>, grid, dim3(kPhThreads), 0, s, E, sig_ph, part, N, P, L,
                       ph_chunk(L, pk));
    if (options().profile) prof_end(kProfPhoto, s);
    hipLaunchKernelGGL(k_ph_sum, dim3(256), dim3(256), 0, s, part, pk, (size_t)N * P, kph);
  }
  return hipGetLastError();
}

}  // namespace xod

using namespace xod;

extern "C" size_t xod_photolysis_workspace(int32_t N, int32_t A, int32_t L, int32_t P) {
  if (N <= 0 || A < 0 || L <= 0 || P < 0) return 0;
  return photolysis_work_bytes(N, A, L, P);
}

extern "C" xod_status xod_photolysis_spectral(int32_t N, int32_t S, int32_t A, int32_t L,
                                              int32_t P, const double *n, const double *dz,
                                              const int32_t *absorbers, const double *sig_ext,
                                              const double *J0, const double *dlam,
                                              const double *sig_ph, double t_f, double mu,
                                              void *work, size_t work_bytes, double *kph,
                                              void *stream) {
  PH_CHECK(N > 0 && S > 0 && A >= 0 && L > 0 && P >= 0,
           "xod_photolysis_spectral: need N, S, L > 0 and A, P >= 0");
  PH_CHECK(mu > 0.0, "xod_photolysis_spectral: mu must be positive");
  PH_CHECK(n && dz && J0 && dlam && work, "xod_photolysis_spectral: null pointer");
  PH_CHECK(A == 0 || (absorbers && sig_ext), "xod_photolysis_spectral: null absorber table");
  PH_CHECK(P == 0 || (sig_ph && kph), "xod_photolysis_spectral: null cross-section table");
  PH_CHECK(work_bytes >= photolysis_work_bytes(N, A, L, P),
           "xod_photolysis_spectral: workspace smaller than xod_photolysis_workspace()");
  XOD_HIP(launch_photolysis(N, S, A, L, P, n, dz, absorbers, sig_ext, J0, dlam, sig_ph, t_f, mu,
                            work, kph, (hipStream_t)stream));
  return XOD_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free variant: the workspace is a fixed device array (one copy
// per device, held until the process ends).  Host code must not pass the
// array's name to a kernel: its device address is looked up once per device
// with hipGetSymbolAddress and kept in scratch_dev.
namespace xod {
namespace {
constexpr size_t kPhScratchBytes = (size_t)64 << 20;
constexpr int kPhMaxDevices = 64;
static __device__ __align__(256) double scratch[kPhScratchBytes / sizeof(double)];
std::mutex scratch_mu;
void *scratch_dev[kPhMaxDevices] = {};

xod_status scratch_address(void **out) {
  int dev = -1;
  XOD_HIP(hipGetDevice(&dev));
  PH_CHECK(dev >= 0 && dev < kPhMaxDevices,
           "xod_photolysis_spectral_noalloc: device index out of range");
  std::lock_guard<std::mutex> g(scratch_mu);
  if (!scratch_dev[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      ::xod::set_error(std::string("xod_photolysis_spectral_noalloc: hipGetSymbolAddress "
                                   "failed: ") + hipGetErrorString(e));
      return XOD_EHIP;
    }
    scratch_dev[dev] = p;
  }
  *out = scratch_dev[dev];
  return XOD_OK;
}
}  // namespace
}  // namespace xod

extern "C" xod_status xod_photolysis_spectral_noalloc(int32_t N, int32_t S, int32_t A,
                                                      int32_t L, int32_t P, const double *n,
                                                      const double *dz, const int32_t *absorbers,
                                                      const double *sig_ext, const double *J0,
                                                      const double *dlam, const double *sig_ph,
                                                      double t_f, double mu, double *kph,
                                                      void *stream) {
  using namespace xod;
  PH_CHECK(N > 0 && S > 0 && A >= 0 && L > 0 && P >= 0,
           "xod_photolysis_spectral_noalloc: need N, S, L > 0 and A, P >= 0");
  PH_CHECK(mu > 0.0, "xod_photolysis_spectral_noalloc: mu must be positive");
  PH_CHECK(n && dz && J0 && dlam, "xod_photolysis_spectral_noalloc: null pointer");
  PH_CHECK(A == 0 || (absorbers && sig_ext),
           "xod_photolysis_spectral_noalloc: null absorber table");
  PH_CHECK(P == 0 || (sig_ph && kph),
           "xod_photolysis_spectral_noalloc: null cross-section table");
  const size_t need = photolysis_work_bytes(N, A, L, P);
  if (need > kPhScratchBytes) {
    ::xod::set_error("xod_photolysis_spectral_noalloc: these sizes need " +
                     std::to_string(need) + " bytes of workspace, more than the fixed " +
                     std::to_string(kPhScratchBytes) + " (use xod_photolysis_spectral)");
    return XOD_EINVAL;
  }
  void *work = nullptr;
  const xod_status st = scratch_address(&work);
  if (st != XOD_OK) return st;
  XOD_HIP(launch_photolysis(N, S, A, L, P, n, dz, absorbers, sig_ext, J0, dlam, sig_ph, t_f, mu,
                            work, kph, (hipStream_t)stream));
  return XOD_OK;
}
