// Kernels of the Toeplitz form of the normal operator A^H W A (A a type 2
// transform, W a diagonal weight): fill a strength vector with ones, scale a
// vector, embed a mode array in the zero-padded doubled grid, and take it back
// out.
#include "device_common.hpp"

namespace esn {

constexpr int kToepBlock = 256;

template <typename T>
__global__ void fill_ones_kernel(cplx_t<T>* __restrict__ c, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kToepBlock + threadIdx.x;
  if (i >= n) return;
  cplx_t<T> v;
  v.x = 1;
  v.y = 0;
  c[i] = v;
}

// Mode index of position i of a dimension of N modes in the given order.
__device__ __forceinline__ int64_t toep_mode(int64_t i, int64_t N, int modeord) {
  if (modeord == 0) return i - N / 2;
  return i < N - N / 2 ? i : i - N;
}

// Grid position of mode k on the doubled grid: k + floor(N/2) in [0, N); the
// convolution only needs one fixed shift for input and output.
template <typename T>
__global__ void toep_pad_kernel(const ToepArgs a, const cplx_t<T>* __restrict__ f,
                                cplx_t<T>* __restrict__ grid) {
  const int64_t g0 = (int64_t)blockIdx.x * kToepBlock + threadIdx.x;
  if (g0 >= a.L[0]) return;
  for (int64_t g2 = blockIdx.z; g2 < a.L[2]; g2 += gridDim.z)
    for (int64_t g1 = blockIdx.y; g1 < a.L[1]; g1 += gridDim.y) {
      cplx_t<T> v;
      v.x = 0;
      v.y = 0;
      if (g0 < a.N[0] && g1 < a.N[1] && g2 < a.N[2]) {
        // position of mode g - floor(N/2) in the caller's array
        int64_t idx = 0;
        const int64_t g[3] = {g0, g1, g2};
        for (int m = 2; m >= 0; m--) {
          const int64_t k = g[m] - a.N[m] / 2;
          const int64_t pos = a.modeord == 0 ? k + a.N[m] / 2 : (k >= 0 ? k : k + a.N[m]);
          idx = idx * a.N[m] + pos;
        }
        v = f[idx];
      }
      grid[g0 + a.L[0] * (g1 + a.L[1] * g2)] = v;
    }
}

template <typename T>
__global__ void toep_extract_kernel(const ToepArgs a, const cplx_t<T>* __restrict__ grid,
                                    cplx_t<T>* __restrict__ f) {
  const int64_t i0 = (int64_t)blockIdx.x * kToepBlock + threadIdx.x;
  if (i0 >= a.N[0]) return;
  for (int64_t i2 = blockIdx.z; i2 < a.N[2]; i2 += gridDim.z)
    for (int64_t i1 = blockIdx.y; i1 < a.N[1]; i1 += gridDim.y) {
      const int64_t i[3] = {i0, i1, i2};
      int64_t gi = 0;
      for (int m = 2; m >= 0; m--) gi = gi * a.L[m] + toep_mode(i[m], a.N[m], a.modeord) + a.N[m] / 2;
      f[i0 + a.N[0] * (i1 + a.N[1] * i2)] = grid[gi];
    }
}

static dim3 toep_grid(int64_t n0, int64_t n1, int64_t n2) {
  return dim3((unsigned)((n0 + kToepBlock - 1) / kToepBlock), (unsigned)std::min<int64_t>(n1, 65535),
              (unsigned)std::min<int64_t>(n2, 65535));
}

hipError_t launch_fill_ones(int prec, void* c, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const dim3 g((unsigned)((n + kToepBlock - 1) / kToepBlock));
  if (prec == ESN_SINGLE)
    hipLaunchKernelGGL(fill_ones_kernel<float>, g, dim3(kToepBlock), 0, s, static_cast<float2*>(c),
                       n);
  else
    hipLaunchKernelGGL(fill_ones_kernel<double>, g, dim3(kToepBlock), 0, s,
                       static_cast<double2*>(c), n);
  return hipGetLastError();
}

template <typename T>
__global__ void scale_kernel(cplx_t<T>* __restrict__ v, int64_t n, T s) {
  const int64_t i = (int64_t)blockIdx.x * kToepBlock + threadIdx.x;
  if (i >= n) return;
  cplx_t<T> x = v[i];
  x.x *= s;
  x.y *= s;
  v[i] = x;
}

hipError_t launch_scale(int prec, void* v, int64_t n, double s, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const dim3 g((unsigned)((n + kToepBlock - 1) / kToepBlock));
  if (prec == ESN_SINGLE)
    hipLaunchKernelGGL(scale_kernel<float>, g, dim3(kToepBlock), 0, st, static_cast<float2*>(v), n,
                       (float)s);
  else
    hipLaunchKernelGGL(scale_kernel<double>, g, dim3(kToepBlock), 0, st, static_cast<double2*>(v),
                       n, s);
  return hipGetLastError();
}

hipError_t launch_toep_pad(const ToepArgs& a, int prec, const void* f, void* grid, hipStream_t s) {
  const dim3 g = toep_grid(a.L[0], a.L[1], a.L[2]);
  if (prec == ESN_SINGLE)
    hipLaunchKernelGGL(toep_pad_kernel<float>, g, dim3(kToepBlock), 0, s, a,
                       static_cast<const float2*>(f), static_cast<float2*>(grid));
  else
    hipLaunchKernelGGL(toep_pad_kernel<double>, g, dim3(kToepBlock), 0, s, a,
                       static_cast<const double2*>(f), static_cast<double2*>(grid));
  return hipGetLastError();
}

hipError_t launch_toep_extract(const ToepArgs& a, int prec, const void* grid, void* f,
                               hipStream_t s) {
  const dim3 g = toep_grid(a.N[0], a.N[1], a.N[2]);
  if (prec == ESN_SINGLE)
    hipLaunchKernelGGL(toep_extract_kernel<float>, g, dim3(kToepBlock), 0, s, a,
                       static_cast<const float2*>(grid), static_cast<float2*>(f));
  else
    hipLaunchKernelGGL(toep_extract_kernel<double>, g, dim3(kToepBlock), 0, s, a,
                       static_cast<const double2*>(grid), static_cast<double2*>(f));
  return hipGetLastError();
}

}  // namespace esn
