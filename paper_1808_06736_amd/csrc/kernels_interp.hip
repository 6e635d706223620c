// Interpolation, eq. (interp):  c_j = sum_l b_l psi~(l h - x_j).
//
// interp_lds: one workgroup per subproblem.  The workgroup first copies the
// bin's tile (bin + w cells per dim, periodically wrapped) from the fine grid
// into LDS with consecutive threads reading consecutive cells, then each thread
// takes a point, forms the separable weights (w d kernel evaluations) and sums
// its w^d cells from LDS; the result goes to the point's original index.
//
// interp_gm: one thread per point reading its w^d cells from the fine grid
// through the caches.
#include "device_common.hpp"

namespace esn {

template <int D, int W, typename T>
__global__ void __launch_bounds__(1024)
interp_lds_kernel(const GeomArgs g, const T* __restrict__ grid, cplx_t<T>* __restrict__ c) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx_t<T>* tile = reinterpret_cast<cplx_t<T>*>(smem_raw);
  const int sidx = blockIdx.x;
  const int bin = g.sub_bin[sidx];
  const int start = g.sub_start[sidx];
  const int len = g.sub_len[sidx];
  int bi[3];
  bi[0] = bin % g.nb[0];
  bi[1] = (bin / g.nb[0]) % g.nb[1];
  bi[2] = bin / (g.nb[0] * g.nb[1]);
  const int T0 = g.b[0] + W;
  const int T1 = D >= 2 ? g.b[1] + W : 1;
  const int T2 = D >= 3 ? g.b[2] + W : 1;
  const int tc = T0 * T1 * T2;
  const int ntr = g.ntr;
  const int64_t o0 = (int64_t)bi[0] * g.b[0] - W / 2;
  const int64_t o1 = D >= 2 ? (int64_t)bi[1] * g.b[1] - W / 2 : 0;
  const int64_t o2 = D >= 3 ? (int64_t)bi[2] * g.b[2] - W / 2 : 0;
  const cplx_t<T>* gridc = reinterpret_cast<const cplx_t<T>*>(grid);
  for (int i = threadIdx.x; i < tc; i += blockDim.x) {
    const int i0 = i % T0;
    const int r = i / T0;
    const int i1 = r % T1;
    const int i2 = r / T1;
    const int64_t g0 = wrap_any(o0 + i0, g.n[0]);
    const int64_t g1 = D >= 2 ? wrap_any(o1 + i1, g.n[1]) : 0;
    const int64_t g2 = D >= 3 ? wrap_any(o2 + i2, g.n[2]) : 0;
    const int64_t gi = g0 + g.n[0] * (g1 + g.n[1] * g2);
    for (int tr = 0; tr < ntr; tr++) tile[tr * tc + i] = gridc[tr * g.gstride + gi];
  }
  __syncthreads();

  const T beta = (T)g.beta;
  for (int i = threadIdx.x; i < len; i += blockDim.x) {
    const int64_t j = (int64_t)start + i;
    T ker[D][W];
    int L[3] = {0, 0, 0};
#pragma unroll
    for (int m = 0; m < D; m++) {
      int sh;
      Coord<T> cd = decode_coord<T>(g.pts, g.pts_code, g.fbits[m], j, m, &sh, W);
      L[m] = window_cell(cd.cell, sh, g.n[m]) - bi[m] * g.b[m];
      es_weights_any<W, T>(sh, cd.f, beta, g.ktab, ker[m]);
    }
    const int64_t orig = point_perm(g.pts, g.pts_code, j);
    for (int tr = 0; tr < ntr; tr++) {
      const cplx_t<T>* tl = tile + tr * tc;
      T ar = 0, ai = 0;
      if constexpr (D == 1) {
#pragma unroll
        for (int k0 = 0; k0 < W; k0++) {
          const cplx_t<T> v = tl[L[0] + k0];
          ar += ker[0][k0] * v.x;
          ai += ker[0][k0] * v.y;
        }
      } else if constexpr (D == 2) {
#pragma unroll
        for (int k1 = 0; k1 < W; k1++) {
          const int base = (L[1] + k1) * T0 + L[0];
          T sr = 0, si = 0;
#pragma unroll
          for (int k0 = 0; k0 < W; k0++) {
            const cplx_t<T> v = tl[base + k0];
            sr += ker[0][k0] * v.x;
            si += ker[0][k0] * v.y;
          }
          ar += ker[1][k1] * sr;
          ai += ker[1][k1] * si;
        }
      } else {
        for (int k2 = 0; k2 < W; k2++) {
#pragma unroll
          for (int k1 = 0; k1 < W; k1++) {
            const int base = ((L[2] + k2) * T1 + (L[1] + k1)) * T0 + L[0];
            T sr = 0, si = 0;
#pragma unroll
            for (int k0 = 0; k0 < W; k0++) {
              const cplx_t<T> v = tl[base + k0];
              sr += ker[0][k0] * v.x;
              si += ker[0][k0] * v.y;
            }
            const T w12 = ker[2][k2] * ker[1][k1];
            ar += w12 * sr;
            ai += w12 * si;
          }
        }
      }
      cplx_t<T> out;
      out.x = ar;
      out.y = ai;
      c[tr * g.cstride + orig] = out;
    }
  }
}

template <int D, int W, typename T>
__global__ void __launch_bounds__(256)
interp_gm_kernel(const GeomArgs g, const T* __restrict__ grid, cplx_t<T>* __restrict__ c) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= g.M) return;
  const T beta = (T)g.beta;
  T ker[D][W];
  int64_t l0[3] = {0, 0, 0};
#pragma unroll
  for (int m = 0; m < D; m++) {
    int sh;
    Coord<T> cd = decode_coord<T>(g.pts, g.pts_code, g.fbits[m], j, m, &sh, W);
    l0[m] = (int64_t)cd.cell - W / 2 + sh;
    es_weights_any<W, T>(sh, cd.f, beta, g.ktab, ker[m]);
  }
  int64_t idx0[W];
#pragma unroll
  for (int k = 0; k < W; k++) idx0[k] = wrap_once(l0[0] + k, g.n[0]);
  const int64_t orig = point_perm(g.pts, g.pts_code, j);
  const cplx_t<T>* gridc = reinterpret_cast<const cplx_t<T>*>(grid);
  for (int tr = 0; tr < g.ntr; tr++) {
    const cplx_t<T>* gt = gridc + tr * g.gstride;
    T ar = 0, ai = 0;
    const int K2 = D >= 3 ? W : 1;
    const int K1 = D >= 2 ? W : 1;
    for (int k2 = 0; k2 < K2; k2++) {
      const int64_t r2 = D >= 3 ? wrap_once(l0[2] + k2, g.n[2]) : 0;
      const T w2 = D >= 3 ? ker[D >= 3 ? 2 : 0][k2] : (T)1;
      for (int k1 = 0; k1 < K1; k1++) {
        const int64_t r1 = D >= 2 ? wrap_once(l0[1] + k1, g.n[1]) : 0;
        const T w12 = w2 * (D >= 2 ? ker[D >= 2 ? 1 : 0][k1] : (T)1);
        const int64_t rowbase = g.n[0] * (r1 + g.n[1] * r2);
        T sr = 0, si = 0;
#pragma unroll
        for (int k0 = 0; k0 < W; k0++) {
          const cplx_t<T> v = gt[rowbase + idx0[k0]];
          sr += ker[0][k0] * v.x;
          si += ker[0][k0] * v.y;
        }
        ar += w12 * sr;
        ai += w12 * si;
      }
    }
    cplx_t<T> out;
    out.x = ar;
    out.y = ai;
    c[tr * g.cstride + orig] = out;
  }
}

template <int D, int W, typename T>
static hipError_t interp_dispatch_t(int method, const GeomArgs& g, int nsub, int block,
                                    size_t lds, const void* grid, void* c, hipStream_t s) {
  if (method == 1) {
    if (nsub <= 0) return hipSuccess;
    hipLaunchKernelGGL((interp_lds_kernel<D, W, T>), dim3(nsub), dim3(block), lds, s, g,
                       static_cast<const T*>(grid), static_cast<cplx_t<T>*>(c));
  } else {
    if (g.M <= 0) return hipSuccess;
    const int bs = 256;
    const int64_t nb = (g.M + bs - 1) / bs;
    hipLaunchKernelGGL((interp_gm_kernel<D, W, T>), dim3((unsigned)nb), dim3(bs), 0, s, g,
                       static_cast<const T*>(grid), static_cast<cplx_t<T>*>(c));
  }
  return hipGetLastError();
}

template <int D, typename T>
static hipError_t interp_dispatch_w(int method, int w, const GeomArgs& g, int nsub, int block,
                                    size_t lds, const void* grid, void* c, hipStream_t s) {
  switch (w) {
#define ESN_W(WV) \
  case WV: return interp_dispatch_t<D, WV, T>(method, g, nsub, block, lds, grid, c, s);
    ESN_W(2) ESN_W(3) ESN_W(4) ESN_W(5) ESN_W(6) ESN_W(7) ESN_W(8) ESN_W(9)
    ESN_W(10) ESN_W(11) ESN_W(12) ESN_W(13) ESN_W(14) ESN_W(15) ESN_W(16)
#undef ESN_W
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_interp(int method, int prec, int dim, int w, const GeomArgs& g, int nsub,
                         int block, size_t lds_bytes, const void* grid, void* c,
                         hipStream_t s) {
  if (prec == ESN_SINGLE) {
    if (dim == 1) return interp_dispatch_w<1, float>(method, w, g, nsub, block, lds_bytes, grid, c, s);
    if (dim == 2) return interp_dispatch_w<2, float>(method, w, g, nsub, block, lds_bytes, grid, c, s);
    return interp_dispatch_w<3, float>(method, w, g, nsub, block, lds_bytes, grid, c, s);
  }
  if (dim == 1) return interp_dispatch_w<1, double>(method, w, g, nsub, block, lds_bytes, grid, c, s);
  if (dim == 2) return interp_dispatch_w<2, double>(method, w, g, nsub, block, lds_bytes, grid, c, s);
  return interp_dispatch_w<3, double>(method, w, g, nsub, block, lds_bytes, grid, c, s);
}

}  // namespace esn
