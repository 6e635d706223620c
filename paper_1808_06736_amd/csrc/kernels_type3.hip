// Type 3 (Sec. 3.3): the per-point and per-target work around the inner
// spreading and type 2 steps, all in FP64.
//
//   minmax   : bounds of up to six coordinate arrays in one launch (per-block
//              partials, then one block per array), for the centres x0, s0
//              and half-widths X, S of eqs. (XS) and (trans)
//   sources  : rescaled source x'' = (x - x0) / gamma (Sec. 3.3 step 1) and the
//              prephase exp(isign i s0.(x - x0)) of eq. (trans)
//   targets  : rescaled target s'' = h gamma (s - s0) (step 2) and one complex
//              factor per target: the correction of step 3 (its quadrature
//              sum from a Chebyshev series built on the host) times the
//              postphase exp(isign i s.x0) of eq. (trans)
//   cmul     : out[t][i] = in[t][i] * fac[i] over the transforms
#include "device_common.hpp"

namespace esn {

constexpr int kT3Block = 256;

__device__ __forceinline__ float2 cmake(float a, float b) { return make_float2(a, b); }
__device__ __forceinline__ double2 cmake(double a, double b) { return make_double2(a, b); }

// Stage 1: per-block (min, max) partials of array blockIdx.y; a NaN or an
// infinity shows as a NaN maximum.
template <typename CT>
__global__ void __launch_bounds__(kT3Block)
minmax_kernel(const MinMaxSets a, double* __restrict__ part, int nb) {
  __shared__ double smin[kT3Block], smax[kT3Block];
  const int arr = blockIdx.y;
  const CT* __restrict__ x = static_cast<const CT*>(a.x[arr]);
  const int64_t n = a.n[arr];
  double lo = INFINITY, hi = -INFINITY;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * kT3Block + threadIdx.x; i < n;
       i += (int64_t)nb * kT3Block) {
    const double v = (double)x[i];
    lo = fmin(lo, v);
    hi = fmax(hi, v);
    bad |= !isfinite(v);
  }
  smin[threadIdx.x] = lo;
  smax[threadIdx.x] = bad ? NAN : hi;
  __syncthreads();
  for (int o = kT3Block / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + o]);
      const double u = smax[threadIdx.x], v = smax[threadIdx.x + o];
      smax[threadIdx.x] = (u != u || v != v) ? NAN : fmax(u, v);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * ((int64_t)arr * nb + blockIdx.x)] = smin[0];
    part[2 * ((int64_t)arr * nb + blockIdx.x) + 1] = smax[0];
  }
}

// Stage 2: one block per array folds its nb partials into out[2 arr], [2 arr + 1].
__global__ void __launch_bounds__(kT3Block)
minmax_fold_kernel(const double* __restrict__ part, int nb, double* __restrict__ out) {
  __shared__ double smin[kT3Block], smax[kT3Block];
  const int arr = blockIdx.x;
  double lo = INFINITY, hi = -INFINITY;
  bool bad = false;
  for (int q = threadIdx.x; q < nb; q += kT3Block) {
    lo = fmin(lo, part[2 * ((int64_t)arr * nb + q)]);
    const double h = part[2 * ((int64_t)arr * nb + q) + 1];
    bad |= (h != h);
    hi = fmax(hi, h);
  }
  smin[threadIdx.x] = lo;
  smax[threadIdx.x] = bad ? NAN : hi;
  __syncthreads();
  for (int o = kT3Block / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + o]);
      const double u = smax[threadIdx.x], v = smax[threadIdx.x + o];
      smax[threadIdx.x] = (u != u || v != v) ? NAN : fmax(u, v);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * arr] = smin[0];
    out[2 * arr + 1] = smax[0];
  }
}

int t3_minmax_blocks(int64_t n) {
  const int64_t b = (n + 8 * kT3Block - 1) / (8 * kT3Block);
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 512));
}

hipError_t launch_minmax(const MinMaxSets& a, int coord_prec, double* part, double* out,
                         hipStream_t s) {
  if (a.count <= 0) return hipSuccess;
  int64_t nmax = 0;
  for (int i = 0; i < a.count; i++) nmax = std::max(nmax, a.n[i]);
  const int nb = t3_minmax_blocks(nmax);
  const dim3 g(nb, a.count);
  if (coord_prec == ESN_SINGLE)
    hipLaunchKernelGGL(minmax_kernel<float>, g, dim3(kT3Block), 0, s, a, part, nb);
  else
    hipLaunchKernelGGL(minmax_kernel<double>, g, dim3(kT3Block), 0, s, a, part, nb);
  hipLaunchKernelGGL(minmax_fold_kernel, dim3(a.count), dim3(kT3Block), 0, s, part, nb, out);
  return hipGetLastError();
}

template <typename CT, typename T>
__global__ void t3_sources_kernel(const T3Args a, const CT* __restrict__ x,
                                  const CT* __restrict__ y, const CT* __restrict__ z,
                                  cplx_t<T>* __restrict__ pre) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n) return;
  const CT* xs[3] = {x, y, z};
  double ph = 0.0;
#pragma unroll
  for (int m = 0; m < 3; m++) {
    if (m >= a.dim) break;
    const double d = (double)xs[m][j] - a.x0[m];
    a.out[m][j] = d * a.inv_gam[m];
    ph += a.s0[m] * d;
  }
  double sn, cs;
  sincos((double)a.isign * ph, &sn, &cs);
  pre[j] = cmake((T)cs, (T)sn);
}

// The step 3 correction sum of dimension m, eqs. (pk1) and (quad):
// g(u) = sum_q wq phi(zq) cos(u zq) at u = alpha gamma (s - s0) = (w/2) s'',
// from its Chebyshev series in u^2 (Clenshaw's recurrence, FP64).
__device__ __forceinline__ double t3_gsum(const double* __restrict__ a, double cscale, double u) {
  const double x = u * u * cscale - 1.0;
  const double x2 = 2.0 * x;
  double b1 = 0.0, b2 = 0.0;
#pragma unroll
  for (int k = kT3Cheb - 1; k >= 1; k--) {
    const double b0 = fma(x2, b1, a[k] - b2);
    b2 = b1;
    b1 = b0;
  }
  return fma(x, b1, a[0] - b2);
}

template <typename CT, typename T>
__global__ void t3_targets_kernel(const T3Args a, const CT* __restrict__ s,
                                  const CT* __restrict__ t, const CT* __restrict__ u,
                                  cplx_t<T>* __restrict__ post) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.n) return;
  const CT* ss[3] = {s, t, u};
  double g = 1.0, ph = 0.0;
#pragma unroll
  for (int m = 0; m < 3; m++) {
    if (m >= a.dim) break;
    const double sk = (double)ss[m][k];
    const double sr = (sk - a.s0[m]) * a.hgam[m];   // s'' = h gamma (s - s0)
    a.out[m][k] = sr;
    g *= (double)a.w * t3_gsum(a.cheb[m], a.cscale[m], 0.5 * a.w * sr);
    ph += sk * a.x0[m];
  }
  const double corr = 1.0 / g;   // the product of 1 / (w g(u)) over the dimensions
  double sn, cs;
  sincos((double)a.isign * ph, &sn, &cs);
  post[k] = cmake((T)(corr * cs), (T)(corr * sn));
}

template <typename T>
__global__ void cmul_kernel(const cplx_t<T>* __restrict__ in,
                            const cplx_t<T>* __restrict__ fac,
                            cplx_t<T>* __restrict__ out, int64_t n, int ntr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const auto g = fac[i];
  for (int t = 0; t < ntr; t++) {
    const auto v = in[(int64_t)t * n + i];
    out[(int64_t)t * n + i] = cmake(v.x * g.x - v.y * g.y, v.x * g.y + v.y * g.x);
  }
}

static unsigned t3_blocks(int64_t n) { return (unsigned)((n + kT3Block - 1) / kT3Block); }

hipError_t launch_t3_sources(const T3Args& a, int coord_prec, int prec, const void* const* x,
                             void* pre, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  const dim3 g(t3_blocks(a.n)), b(kT3Block);
  if (coord_prec == ESN_SINGLE) {
    const float* c[3] = {static_cast<const float*>(x[0]), static_cast<const float*>(x[1]),
                         static_cast<const float*>(x[2])};
    if (prec == ESN_SINGLE)
      hipLaunchKernelGGL((t3_sources_kernel<float, float>), g, b, 0, s, a, c[0], c[1], c[2],
                         static_cast<float2*>(pre));
    else
      hipLaunchKernelGGL((t3_sources_kernel<float, double>), g, b, 0, s, a, c[0], c[1], c[2],
                         static_cast<double2*>(pre));
  } else {
    const double* c[3] = {static_cast<const double*>(x[0]), static_cast<const double*>(x[1]),
                          static_cast<const double*>(x[2])};
    if (prec == ESN_SINGLE)
      hipLaunchKernelGGL((t3_sources_kernel<double, float>), g, b, 0, s, a, c[0], c[1], c[2],
                         static_cast<float2*>(pre));
    else
      hipLaunchKernelGGL((t3_sources_kernel<double, double>), g, b, 0, s, a, c[0], c[1], c[2],
                         static_cast<double2*>(pre));
  }
  return hipGetLastError();
}

hipError_t launch_t3_targets(const T3Args& a, int coord_prec, int prec, const void* const* sx,
                             void* post, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  const dim3 g(t3_blocks(a.n)), b(kT3Block);
  if (coord_prec == ESN_SINGLE) {
    const float* c[3] = {static_cast<const float*>(sx[0]), static_cast<const float*>(sx[1]),
                         static_cast<const float*>(sx[2])};
    if (prec == ESN_SINGLE)
      hipLaunchKernelGGL((t3_targets_kernel<float, float>), g, b, 0, s, a, c[0], c[1], c[2],
                         static_cast<float2*>(post));
    else
      hipLaunchKernelGGL((t3_targets_kernel<float, double>), g, b, 0, s, a, c[0], c[1], c[2],
                         static_cast<double2*>(post));
  } else {
    const double* c[3] = {static_cast<const double*>(sx[0]), static_cast<const double*>(sx[1]),
                          static_cast<const double*>(sx[2])};
    if (prec == ESN_SINGLE)
      hipLaunchKernelGGL((t3_targets_kernel<double, float>), g, b, 0, s, a, c[0], c[1], c[2],
                         static_cast<float2*>(post));
    else
      hipLaunchKernelGGL((t3_targets_kernel<double, double>), g, b, 0, s, a, c[0], c[1], c[2],
                         static_cast<double2*>(post));
  }
  return hipGetLastError();
}

hipError_t launch_cmul(int prec, const void* in, const void* fac, void* out, int64_t n, int ntr,
                       hipStream_t s) {
  if (n <= 0 || ntr <= 0) return hipSuccess;
  const dim3 g(t3_blocks(n)), b(kT3Block);
  if (prec == ESN_SINGLE)
    hipLaunchKernelGGL(cmul_kernel<float>, g, b, 0, s, static_cast<const float2*>(in),
                       static_cast<const float2*>(fac), static_cast<float2*>(out), n, ntr);
  else
    hipLaunchKernelGGL(cmul_kernel<double>, g, b, 0, s, static_cast<const double2*>(in),
                       static_cast<const double2*>(fac), static_cast<double2*>(out), n, ntr);
  return hipGetLastError();
}

}  // namespace esn
