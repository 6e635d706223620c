// Correction steps around the FFT.
//
//   fseries : per dimension, the factors p(k) = 1 / (w sum_{j<=p} w_j phi(q_j)
//             cos(alpha k q_j)) for k = 0..floor(N/2), in FP64.  This is
//             p_k = h / psi^(k) = 2 / (w phi^(alpha k)) of eq. (pk1) with
//             phi^ from the Gauss-Legendre rule of eq. (quad) (only the p
//             positive nodes, phi being real and even); alpha = pi w / n
//             (eq. (al)).  In d dims the factor is the product over dims (eq. (pk)).
//   deconv  : type 1 step 3, eq. (pb1): f_k = p_k b^_{k mod n} for k in I
//             (truncation to the N central frequencies of the fine-grid FFT).
//   amplify : type 2 step 1: b^_{k mod n} = p_k f_k for k in I, 0 elsewhere.
#include "device_common.hpp"

namespace esn {

__global__ void fseries_kernel(int w, double beta, const double* __restrict__ nodes,
                               const double* __restrict__ weights, int nq, double alpha,
                               int64_t K, double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  double s = 0.0;
  for (int j = 0; j < nq; j++) {
    const double q = nodes[j];
    const double phi = exp(beta * (sqrt(1.0 - q * q) - 1.0));
    s += weights[j] * phi * cos(alpha * (double)k * q);
  }
  out[k] = 1.0 / ((double)w * s);
}

hipError_t launch_fseries(int w, double beta, const double* d_nodes, const double* d_weights,
                          int nquad, int64_t nf, int64_t N, double* d_out, hipStream_t s) {
  const int64_t K = N / 2 + 1;
  const double alpha = M_PI * (double)w / (double)nf;
  hipLaunchKernelGGL(fseries_kernel, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, s, w,
                     beta, d_nodes, d_weights, nquad, alpha, K, d_out);
  return hipGetLastError();
}

struct CorrArgs {
  int64_t N[3], nf[3];
  int modeord;
  int ntr;
  int64_t gstride, fstride;
  const double* pf[3];
};

// mode index k of output position i in one dimension
__device__ __forceinline__ int64_t mode_of(int64_t i, int64_t N, int modeord) {
  if (modeord == 0) return i - N / 2;
  return i < N - N / 2 ? i : i - N;
}

template <typename T>
__global__ void deconv_kernel(const CorrArgs a, const cplx_t<T>* __restrict__ grid,
                              cplx_t<T>* __restrict__ f) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t Ntot = a.N[0] * a.N[1] * a.N[2];
  if (idx >= Ntot) return;
  const int64_t i0 = idx % a.N[0];
  const int64_t r = idx / a.N[0];
  const int64_t i1 = r % a.N[1];
  const int64_t i2 = r / a.N[1];
  const int64_t k0 = mode_of(i0, a.N[0], a.modeord);
  const int64_t k1 = mode_of(i1, a.N[1], a.modeord);
  const int64_t k2 = mode_of(i2, a.N[2], a.modeord);
  const int64_t g0 = k0 < 0 ? k0 + a.nf[0] : k0;
  const int64_t g1 = k1 < 0 ? k1 + a.nf[1] : k1;
  const int64_t g2 = k2 < 0 ? k2 + a.nf[2] : k2;
  const double p = a.pf[0][k0 < 0 ? -k0 : k0] * a.pf[1][k1 < 0 ? -k1 : k1] *
                   a.pf[2][k2 < 0 ? -k2 : k2];
  const T pt = (T)p;
  const int64_t gi = g0 + a.nf[0] * (g1 + a.nf[1] * g2);
  for (int tr = 0; tr < a.ntr; tr++) {
    cplx_t<T> v = grid[tr * a.gstride + gi];
    v.x *= pt;
    v.y *= pt;
    f[tr * a.fstride + idx] = v;
  }
}

// position of mode index k in the caller's mode array of one dimension
__device__ __forceinline__ int64_t pos_of(int64_t k, int64_t N, int modeord) {
  if (modeord == 0) return k + N / 2;
  return k >= 0 ? k : k + N;
}

// Mode index k of fine-grid position g in one dimension (n cells, N modes), or
// false where g holds no mode.
__device__ __forceinline__ bool mode_at(int64_t g, int64_t N, int64_t n, int64_t* k) {
  if (g < N - N / 2) {  // k = 0 .. ceil(N/2) - 1
    *k = g;
    return true;
  }
  if (g >= n - N / 2) {  // k = -floor(N/2) .. -1
    *k = g - n;
    return true;
  }
  return false;
}

// Threads walk the x positions of a fine-grid row; the launch grid walks the
// rows (y from blockIdx.y, z from blockIdx.z), several per block, so no index
// is divided.  Rows that hold no mode are only cleared, with no loads.
template <typename T>
__global__ void amplify_kernel(const CorrArgs a, cplx_t<T>* __restrict__ grid,
                               const cplx_t<T>* __restrict__ f) {
  cplx_t<T> zero;
  zero.x = 0;
  zero.y = 0;
  for (int64_t g2 = blockIdx.z; g2 < a.nf[2]; g2 += gridDim.z) {
    int64_t k2 = 0;
    const bool in2 = mode_at(g2, a.N[2], a.nf[2], &k2);
    for (int64_t g1 = blockIdx.y; g1 < a.nf[1]; g1 += gridDim.y) {
      int64_t k1 = 0;
      const bool row_in = mode_at(g1, a.N[1], a.nf[1], &k1) && in2;
      const int64_t grow = a.nf[0] * (g1 + a.nf[1] * g2);
      if (!row_in) {
        for (int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g0 < a.nf[0];
             g0 += (int64_t)gridDim.x * blockDim.x)
          for (int tr = 0; tr < a.ntr; tr++) grid[tr * a.gstride + grow + g0] = zero;
        continue;
      }
      const double p12 = a.pf[1][k1 < 0 ? -k1 : k1] * a.pf[2][k2 < 0 ? -k2 : k2];
      const int64_t frow =
          a.N[0] * (pos_of(k1, a.N[1], a.modeord) + a.N[1] * pos_of(k2, a.N[2], a.modeord));
      for (int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g0 < a.nf[0];
           g0 += (int64_t)gridDim.x * blockDim.x) {
        int64_t k0 = 0;
        if (!mode_at(g0, a.N[0], a.nf[0], &k0)) {
          for (int tr = 0; tr < a.ntr; tr++) grid[tr * a.gstride + grow + g0] = zero;
          continue;
        }
        const T pt = (T)(a.pf[0][k0 < 0 ? -k0 : k0] * p12);
        const int64_t fi = frow + pos_of(k0, a.N[0], a.modeord);
        for (int tr = 0; tr < a.ntr; tr++) {
          cplx_t<T> v = f[tr * a.fstride + fi];
          v.x *= pt;
          v.y *= pt;
          grid[tr * a.gstride + grow + g0] = v;
        }
      }
    }
  }
}

// Threads per block of the row kernels: 256, or the row length rounded up to
// whole waves for shorter rows.
static int row_block(int64_t n0) {
  return n0 >= 256 ? 256 : (int)std::max<int64_t>(64, (n0 + 63) / 64 * 64);
}

// Launch grid over rows of n0 cells: about 8 x-steps of a row per block,
// blocks spread over the y rows until about 8192 blocks are in flight.
static dim3 row_grid(int64_t n0, int64_t n1, int64_t n2) {
  const int64_t step = 8 * (int64_t)row_block(n0);
  const int64_t gx = std::min<int64_t>((n0 + step - 1) / step, 65535);
  const int64_t gz = std::min<int64_t>(n2, 65535);
  const int64_t gy = std::min<int64_t>(std::max<int64_t>(n1, 1),
                                       std::max<int64_t>(1, 8192 / (gx * gz)));
  return dim3((unsigned)gx, (unsigned)std::min<int64_t>(gy, 65535), (unsigned)gz);
}

static CorrArgs make_corr(int dim, const int64_t* N, const int64_t* nf, int modeord, int ntr,
                          int64_t gstride, int64_t fstride, const double* const* pf) {
  CorrArgs a;
  for (int m = 0; m < 3; m++) {
    a.N[m] = m < dim ? N[m] : 1;
    a.nf[m] = m < dim ? nf[m] : 1;
    a.pf[m] = pf[m];
  }
  a.modeord = modeord;
  a.ntr = ntr;
  a.gstride = gstride;
  a.fstride = fstride;
  return a;
}

hipError_t launch_deconv(int prec, int dim, const int64_t* N, const int64_t* nf, int modeord,
                         int ntr, const void* grid, int64_t gstride, void* f, int64_t fstride,
                         const double* const* pf, hipStream_t s) {
  CorrArgs a = make_corr(dim, N, nf, modeord, ntr, gstride, fstride, pf);
  const int64_t tot = a.N[0] * a.N[1] * a.N[2];
  const unsigned nb = (unsigned)((tot + 255) / 256);
  if (prec == ESN_SINGLE)
    hipLaunchKernelGGL(deconv_kernel<float>, dim3(nb), dim3(256), 0, s, a,
                       static_cast<const float2*>(grid), static_cast<float2*>(f));
  else
    hipLaunchKernelGGL(deconv_kernel<double>, dim3(nb), dim3(256), 0, s, a,
                       static_cast<const double2*>(grid), static_cast<double2*>(f));
  return hipGetLastError();
}

hipError_t launch_amplify(int prec, int dim, const int64_t* N, const int64_t* nf, int modeord,
                          int ntr, void* grid, int64_t gstride, const void* f, int64_t fstride,
                          const double* const* pf, hipStream_t s) {
  CorrArgs a = make_corr(dim, N, nf, modeord, ntr, gstride, fstride, pf);
  const dim3 g = row_grid(a.nf[0], a.nf[1], a.nf[2]);
  if (prec == ESN_SINGLE)
    hipLaunchKernelGGL(amplify_kernel<float>, g, dim3(row_block(a.nf[0])), 0, s, a,
                       static_cast<float2*>(grid), static_cast<const float2*>(f));
  else
    hipLaunchKernelGGL(amplify_kernel<double>, g, dim3(row_block(a.nf[0])), 0, s, a,
                       static_cast<double2*>(grid), static_cast<const double2*>(f));
  return hipGetLastError();
}

}  // namespace esn
