// Mixed-precision solve support: FP64 residuals of the step system computed
// matrix-free from the reaction list and the transport coefficients (no dense
// FP64 copy of the blocks), row scaling of right-hand sides, and the update /
// convergence measure of iterative refinement.
//
//   k_dwrate   dw_r = (dw_r/dn) . delta, the directional derivative of every
//              reaction rate (same product rule as the Jacobian)
//   k_resid    x = s * (F - M delta),  M delta = delta/dt - J_chem delta
//              - (trl delta_{k-1} + trd delta_k + tru delta_{k+1})
//   k_scale    x = s * F
//   k_axpy     delta += x, per-layer componentwise correction size
#include "xod_internal.h"
#include "mfma.h"

namespace xod {

template <class Acc>
__global__ void __launch_bounds__(256) k_dwrate(Acc acc) {
  const ColArgs &c = acc(blockIdx.z);
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (r >= c.R || k >= c.N) return;
  const double *delta = c.dx;
  double *dw = c.w;
  const double *n = c.n + (size_t)k * c.S;
  const double *d = delta + (size_t)k * c.S;
  const int *rc = c.reac + r * XOD_MAX_REAC;
  const int *pc = c.prod + r * XOD_MAX_PROD;
  double df = 0.0, dr = 0.0;
  for (int s = 0; s < XOD_MAX_REAC; ++s) {
    if (rc[s] < 0) continue;
    double p = d[rc[s]];
    for (int t = 0; t < XOD_MAX_REAC; ++t)
      if (t != s && rc[t] >= 0) p *= n[rc[t]];
    df += p;
  }
  for (int s = 0; s < XOD_MAX_PROD; ++s) {
    if (pc[s] < 0) continue;
    double p = d[pc[s]];
    for (int t = 0; t < XOD_MAX_PROD; ++t)
      if (t != s && pc[t] >= 0) p *= n[pc[t]];
    dr += p;
  }
  const size_t o = (size_t)k * c.R + r;
  dw[o] = c.kf_in[o] * df - c.kr_in[o] * dr;
}

template <class Acc>
__global__ void __launch_bounds__(256) k_resid(Acc acc) {
  const ColArgs &c = acc(blockIdx.z);
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (y >= c.S || k >= c.N) return;
  const double *delta = c.dx;
  const double *dw = c.w;
  const double *w = dw + (size_t)k * c.R;
  double jd = 0.0;
  for (int e = c.inc_ptr[y]; e < c.inc_ptr[y + 1]; ++e) jd += c.inc_nu[e] * w[c.inc_r[e]];
  const size_t o = (size_t)k * c.S + y;
  double tr = c.trd[o] * delta[o];
  if (k >= 1) tr += c.trl[o] * delta[o - c.S];
  if (k + 1 < c.N) tr += c.tru[o] * delta[o + c.S];
  const double Md = delta[o] / c.dt - jd - tr;
  const double sc = c.rs ? c.rs[(size_t)k * c.ld + y] : 1.0;   // no scales: FP64 factors
  c.x[o] = sc * (c.f[o] - Md);
}

template <class Acc>
__global__ void __launch_bounds__(256) k_scale(Acc acc) {
  const ColArgs &c = acc(blockIdx.z);
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (y >= c.S || k >= c.N) return;
  const size_t o = (size_t)k * c.S + y;
  c.x[o] = c.rs[(size_t)k * c.ld + y] * c.f[o];
}

// delta += x, then the componentwise size of the correction x in layer k,
//   ratio[k] = max_i |x_i| / (rtol |n_i + delta_i| + atol max_j |delta_j|)
// over the components whose new density n_i + delta_i exceeds y_floor times
// the layer's gas density (0 if there is none).  ratio <= 1 means every
// such component moved by at most rtol of its new value, or by atol of the
// layer's largest increment (the absolute floor below which an FP64 solve
// fixes no component either).
template <class Acc>
__global__ void __launch_bounds__(256) k_axpy(Acc acc, double *ratio, double rtol, double atol,
                                              double y_floor) {
  const ColArgs &c = acc(blockIdx.y);
  const int k = blockIdx.x;
  double *delta = c.dx;
  double *rk = ratio + (size_t)blockIdx.y * gridDim.x + k;
  if (k >= c.N) {
    if (threadIdx.x == 0) *rk = 0.0;
    return;
  }
  __shared__ double red[256];
  double m = 0.0;
  bool bad = false;           // a non-finite correction or sum anywhere in the layer
  for (int y = threadIdx.x; y < c.S; y += blockDim.x) {
    const size_t o = (size_t)k * c.S + y;
    const double d = delta[o] + c.x[o];
    delta[o] = d;
    m = fmax(m, fabs(d));
    bad = bad || !isfinite(d);
  }
  if (bad) m = __builtin_inf();
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  const double floor_abs = atol * red[0];
  const double sig = y_floor * c.ngas[k];
  __syncthreads();
  double q = 0.0;
  for (int y = threadIdx.x; y < c.S; y += blockDim.x) {
    const size_t o = (size_t)k * c.S + y;
    // an explicit system (no state: c.n null) measures the correction
    // against the solution itself, every component
    const double nn = c.n ? fabs(c.n[o] + delta[o]) : fabs(delta[o]);
    if (!c.n || nn > sig) {
      const double den = rtol * nn + floor_abs;
      const double xi = fabs(c.x[o]);
      q = fmax(q, den > 0.0 ? xi / den : (xi > 0.0 ? 1e300 : 0.0));
    }
  }
  red[threadIdx.x] = q;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *rk = (isfinite(red[0]) && isfinite(floor_abs)) ? red[0] : 1e300;
}

// Explicit block systems (xod_btd_factor / xod_btd_solve in mixed precision):
// one wave per block row.
//   k_cast_scale  s_i = 1 / max(|B_k[i][:]|, |a_k[i]|, |c_k[i]|) (1 for a zero
//                 row); Bf = s B in FP32, as = s a, cs = s c
//   k_bt_resid    x = s * (g - M dx) with M the FP64 block-tridiagonal matrix
//                 (B, a, c), dx and g in the compact [N*S] layout
__global__ void __launch_bounds__(256) k_cast_scale(const double *B, const double *a,
                                                    const double *cc, int N, int ld,
                                                    float *Bf, double *rs, double *as,
                                                    double *cs) {
  const int lane = threadIdx.x & 63;
  const size_t row = (size_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= (size_t)N * ld) return;
  const auto Bg = gmem(B) + row * ld;
  double amax = fmax(fabs(a[row]), fabs(cc[row]));
  for (int j = lane; j < ld; j += 64) amax = fmax(amax, fabs(Bg[j]));
  for (int o = 32; o > 0; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o, 64));
  const double sc = amax > 0.0 ? 1.0 / amax : 1.0;
  const auto Bo = gmem(Bf) + row * ld;
  for (int j = lane; j < ld; j += 64) Bo[j] = (float)(sc * Bg[j]);
  if (lane == 0) {
    rs[row] = sc;
    as[row] = sc * a[row];
    cs[row] = sc * cc[row];
  }
}

__global__ void __launch_bounds__(256) k_bt_resid(const double *B, const double *a,
                                                  const double *cc, const double *g,
                                                  const double *dx, const double *rs, int N,
                                                  int S, int ld, double *x) {
  const int lane = threadIdx.x & 63;
  const size_t r = (size_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= (size_t)N * S) return;
  const int k = (int)(r / S), i = (int)(r % S);
  const size_t row = (size_t)k * ld + i;
  const auto Bg = gmem(B) + row * ld;
  const double *d = dx + (size_t)k * S;
  double sum = 0.0;
  for (int j = lane; j < S; j += 64) sum = fma(Bg[j], d[j], sum);
  for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
  if (lane == 0) {
    double md = sum;
    if (k >= 1) md += a[row] * dx[r - S];
    if (k + 1 < N) md += cc[row] * dx[r + S];
    x[r] = rs[row] * (g[r] - md);
  }
}

hipError_t launch_cast_scale(const double *B, const double *a, const double *c, int N, int ld,
                             float *Bf, double *rs, double *as, double *cs, hipStream_t s) {
  const size_t rows = (size_t)N * ld;
  hipLaunchKernelGGL(k_cast_scale, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, B, a, c, N,
                     ld, Bf, rs, as, cs);
  return hipGetLastError();
}

hipError_t launch_bt_resid(const double *B, const double *a, const double *c, const double *g,
                           const double *dx, const double *rs, int N, int S, int ld, double *x,
                           hipStream_t s) {
  const size_t rows = (size_t)N * S;
  hipLaunchKernelGGL(k_bt_resid, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, B, a, c, g,
                     dx, rs, N, S, ld, x);
  return hipGetLastError();
}

__global__ void k_maxreduce(const double *v, int n, double *out) {
  __shared__ double s[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, v[i]);
  s[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = s[0];
}

template <class Acc>
hipError_t launch_residual(const Acc &acc, int ncols, int maxN, int maxS, int maxR,
                           hipStream_t s) {
  if (maxR > 0)
    hipLaunchKernelGGL(k_dwrate<Acc>, dim3((maxR + 255) / 256, maxN, ncols), dim3(256), 0, s,
                       acc);
  hipLaunchKernelGGL(k_resid<Acc>, dim3((maxS + 255) / 256, maxN, ncols), dim3(256), 0, s, acc);
  return hipGetLastError();
}

template <class Acc>
hipError_t launch_scale(const Acc &acc, int ncols, int maxN, int maxS, hipStream_t s) {
  hipLaunchKernelGGL(k_scale<Acc>, dim3((maxS + 255) / 256, maxN, ncols), dim3(256), 0, s, acc);
  return hipGetLastError();
}

template <class Acc>
hipError_t launch_axpy_size(const Acc &acc, int ncols, int maxN, double *ratio, double *out,
                            double rtol, double atol, double y_floor, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy<Acc>, dim3(maxN, ncols), dim3(256), 0, s, acc, ratio, rtol, atol,
                     y_floor);
  hipLaunchKernelGGL(k_maxreduce, dim3(1), dim3(256), 0, s, ratio, maxN * ncols, out);
  return hipGetLastError();
}

template <class Acc>
hipError_t launch_axpy_ratio(const Acc &acc, int ncols, int maxN, double *ratio, double *out,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_axpy<Acc>, dim3(maxN, ncols), dim3(256), 0, s, acc, ratio,
                     options().refine_tol, options().refine_atol, 1e-30);
  hipLaunchKernelGGL(k_maxreduce, dim3(1), dim3(256), 0, s, ratio, maxN * ncols, out);
  return hipGetLastError();
}

template <class Acc>
__global__ void __launch_bounds__(256) k_keep_refined(Acc acc, const double *ratio, int maxN,
                                                      double most) {
  const ColArgs &c = acc(blockIdx.z);
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (y >= c.S || k >= c.N) return;
  const size_t o = (size_t)k * c.S + y;
  const double q = ratio[(size_t)blockIdx.z * maxN + k];
  c.x[o] = q <= most ? c.dx[o] : c.x0[o];
}

template <class Acc>
hipError_t launch_keep_refined(const Acc &acc, int ncols, int maxN, int maxS, const double *ratio,
                               double most, hipStream_t s) {
  hipLaunchKernelGGL(k_keep_refined<Acc>, dim3((maxS + 255) / 256, maxN, ncols), dim3(256), 0, s,
                     acc, ratio, maxN, most);
  return hipGetLastError();
}

template hipError_t launch_residual<OneCol>(const OneCol &, int, int, int, int, hipStream_t);
template hipError_t launch_residual<ManyCols>(const ManyCols &, int, int, int, int, hipStream_t);
template hipError_t launch_keep_refined<OneCol>(const OneCol &, int, int, int, const double *,
                                                double, hipStream_t);
template hipError_t launch_keep_refined<ManyCols>(const ManyCols &, int, int, int,
                                                  const double *, double, hipStream_t);
template hipError_t launch_scale<OneCol>(const OneCol &, int, int, int, hipStream_t);
template hipError_t launch_scale<ManyCols>(const ManyCols &, int, int, int, hipStream_t);
template hipError_t launch_axpy_ratio<OneCol>(const OneCol &, int, int, double *, double *,
                                              hipStream_t);
template hipError_t launch_axpy_size<OneCol>(const OneCol &, int, int, double *, double *, double,
                                             double, double, hipStream_t);
template hipError_t launch_axpy_ratio<ManyCols>(const ManyCols &, int, int, double *, double *,
                                                hipStream_t);

}  // namespace xod
