// Spreading, eq. (bl):  b_l = sum_j c_j psi~(l h - x_j)  on the fine grid.
//
// spread_lds: one wave per subproblem (Sec. 5.2).  A subproblem is a run of at
// most maxsub bin-sorted points of one bin.  The wave spreads them into a tile
// in LDS covering the bin plus a halo (bin + w cells per dim, so no index
// wrapping is needed while spreading), then adds the tile to the fine grid
// with periodic wrapping.  Different subproblems may overlap on the fine grid,
// so the add-back uses global atomics; only cells that received a
// contribution are added.
//
// spread_gm: one thread per (sorted or unsorted) point, adding its w^d
// contributions straight into the fine grid with global atomics.
#include "device_common.hpp"

namespace esn {

// Per-point staging of one batch of 64 points, kept in LDS after the tile.
template <int D, int W, typename T>
struct Staging {
  T ker[64][D][W];   // separable kernel values per dim
  int loc[64][D];    // window start inside the tile per dim
};

// One wave (64 lanes) per subproblem.  The wave owns its LDS tile, so no
// atomics are needed inside it: the lanes take the points of the subproblem
// one after another, and for each point every lane updates a different set of
// tile cells (d = 3: lane -> one (x, y) of the w x w footprint and its w cells
// along z; d = 2: lane -> one cell; d = 1: lane -> one cell).  Kernel values are
// computed once per point, a lane per point, in batches of 64.
template <int D, int W, typename T>
__global__ void __launch_bounds__(64)
spread_lds_kernel(const GeomArgs g, const cplx_t<T>* __restrict__ c, T* __restrict__ grid) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
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
  cplx_t<T>* tile = reinterpret_cast<cplx_t<T>*>(smem_raw);
  Staging<D, W, T>* st = reinterpret_cast<Staging<D, W, T>*>(tile + (size_t)tc * ntr);
  // strengths of the batch, [64][ntr], 16-byte aligned; offsets are taken
  // inside the LDS array so the compiler keeps LDS (not flat) accesses
  const size_t stc_off =
      ((size_t)tc * ntr * sizeof(cplx_t<T>) + sizeof(Staging<D, W, T>) + 15) & ~(size_t)15;
  cplx_t<T>* stc = reinterpret_cast<cplx_t<T>*>(smem_raw + stc_off);
  const int lane = threadIdx.x;
  {
    cplx_t<T> z;
    z.x = 0;
    z.y = 0;
    for (int i = lane; i < tc * ntr; i += 64) tile[i] = z;
  }
  const T beta = (T)g.beta;
  for (int b0 = 0; b0 < len; b0 += 64) {
    const int nb = min(64, len - b0);
    __syncthreads();
    if (lane < nb) {
      const int64_t j = (int64_t)start + b0 + lane;
#pragma unroll
      for (int m = 0; m < D; m++) {
        int sh;
        Coord<T> cd = decode_coord<T>(g.pts, g.pts_code, g.fbits[m], j, m, &sh, W);
        st->loc[lane][m] = window_cell(cd.cell, sh, g.n[m]) - bi[m] * g.b[m];
        es_weights_any<W, T>(sh, cd.f, beta, g.ktab, st->ker[lane][m]);
      }
      const int64_t orig = point_perm(g.pts, g.pts_code, j);
      for (int tr = 0; tr < ntr; tr++) stc[lane * ntr + tr] = c[tr * g.cstride + orig];
    }
    __syncthreads();
    for (int q = 0; q < nb; q++) {
      if constexpr (D == 1) {
        if (lane < W) {
          const int idx = st->loc[q][0] + lane;
          const T k0 = st->ker[q][0][lane];
          for (int tr = 0; tr < ntr; tr++) {
            const cplx_t<T> cv = stc[q * ntr + tr];
            cplx_t<T> v = tile[tr * tc + idx];
            v.x += k0 * cv.x;
            v.y += k0 * cv.y;
            tile[tr * tc + idx] = v;
          }
        }
      } else if constexpr (D == 2) {
        for (int xy = lane; xy < W * W; xy += 64) {
          const int lx = xy % W, ly = xy / W;
          const int idx = (st->loc[q][1] + ly) * T0 + st->loc[q][0] + lx;
          const T kxy = st->ker[q][0][lx] * st->ker[q][1][ly];
          for (int tr = 0; tr < ntr; tr++) {
            const cplx_t<T> cv = stc[q * ntr + tr];
            cplx_t<T> v = tile[tr * tc + idx];
            v.x += kxy * cv.x;
            v.y += kxy * cv.y;
            tile[tr * tc + idx] = v;
          }
        }
      } else {
        T kz[W];
#pragma unroll
        for (int k = 0; k < W; k++) kz[k] = st->ker[q][2][k];
        const int plane = T0 * T1;
        for (int xy = lane; xy < W * W; xy += 64) {
          const int lx = xy % W, ly = xy / W;
          const int base = (st->loc[q][2] * T1 + st->loc[q][1] + ly) * T0 + st->loc[q][0] + lx;
          const T kxy = st->ker[q][0][lx] * st->ker[q][1][ly];
          for (int tr = 0; tr < ntr; tr++) {
            const cplx_t<T> cv = stc[q * ntr + tr];
            const T cr = kxy * cv.x, ci = kxy * cv.y;
            cplx_t<T>* tl = tile + tr * tc + base;
            cplx_t<T> v[W];
#pragma unroll
            for (int k = 0; k < W; k++) v[k] = tl[k * plane];
#pragma unroll
            for (int k = 0; k < W; k++) {
              v[k].x += kz[k] * cr;
              v[k].y += kz[k] * ci;
            }
#pragma unroll
            for (int k = 0; k < W; k++) tl[k * plane] = v[k];
          }
        }
      }
    }
  }
  __syncthreads();

  // add the tile back into the periodic fine grid (consecutive lanes take
  // consecutive cells along x)
  const int64_t o0 = (int64_t)bi[0] * g.b[0] - W / 2;
  const int64_t o1 = D >= 2 ? (int64_t)bi[1] * g.b[1] - W / 2 : 0;
  const int64_t o2 = D >= 3 ? (int64_t)bi[2] * g.b[2] - W / 2 : 0;
  for (int i = lane; i < tc; i += 64) {
    const int i0 = i % T0;
    const int r = i / T0;
    const int i1 = r % T1;
    const int i2 = r / T1;
    const int64_t g0 = wrap_any(o0 + i0, g.n[0]);
    const int64_t g1 = D >= 2 ? wrap_any(o1 + i1, g.n[1]) : 0;
    const int64_t g2 = D >= 3 ? wrap_any(o2 + i2, g.n[2]) : 0;
    const int64_t gi = g0 + g.n[0] * (g1 + g.n[1] * g2);
    for (int tr = 0; tr < ntr; tr++) {
      const cplx_t<T> v = tile[tr * tc + i];
      if (v.x != (T)0 || v.y != (T)0) {
        T* dst = grid + 2 * (tr * g.gstride + gi);
        atomicAdd(dst, v.x);
        atomicAdd(dst + 1, v.y);
      }
    }
  }
}

template <int D, int W, typename T>
__global__ void __launch_bounds__(256)
spread_gm_kernel(const GeomArgs g, const cplx_t<T>* __restrict__ c, T* __restrict__ grid) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= g.M) return;
  const T beta = (T)g.beta;
  T ker[D][W];
  int64_t l0[3] = {0, 0, 0};
#pragma unroll
  for (int m = 0; m < D; m++) {
    int sh;
    Coord<T> cd = decode_coord<T>(g.pts, g.pts_code, g.fbits[m], j, m, &sh, W);
    l0[m] = (int64_t)cd.cell - W / 2 + sh;   // in [-W/2, n)
    es_weights_any<W, T>(sh, cd.f, beta, g.ktab, ker[m]);
  }
  int64_t idx0[W];
#pragma unroll
  for (int k = 0; k < W; k++) idx0[k] = wrap_once(l0[0] + k, g.n[0]);
  const int64_t orig = point_perm(g.pts, g.pts_code, j);
  for (int tr = 0; tr < g.ntr; tr++) {
    const cplx_t<T> cv = c[tr * g.cstride + orig];
    T* gt = grid + 2 * tr * g.gstride;
    const int K2 = D >= 3 ? W : 1;
    const int K1 = D >= 2 ? W : 1;
    for (int k2 = 0; k2 < K2; k2++) {
      const int64_t r2 = D >= 3 ? wrap_once(l0[2] + k2, g.n[2]) : 0;
      const T w2 = D >= 3 ? ker[D >= 3 ? 2 : 0][k2] : (T)1;
      for (int k1 = 0; k1 < K1; k1++) {
        const int64_t r1 = D >= 2 ? wrap_once(l0[1] + k1, g.n[1]) : 0;
        const T w12 = w2 * (D >= 2 ? ker[D >= 2 ? 1 : 0][k1] : (T)1);
        const T cr = w12 * cv.x, ci = w12 * cv.y;
        const int64_t rowbase = g.n[0] * (r1 + g.n[1] * r2);
#pragma unroll
        for (int k0 = 0; k0 < W; k0++) {
          T* dst = gt + 2 * (rowbase + idx0[k0]);
          atomicAdd(dst, ker[0][k0] * cr);
          atomicAdd(dst + 1, ker[0][k0] * ci);
        }
      }
    }
  }
}

size_t tile_lds_bytes(int prec, int dim, int w, const int* b, int ntr, bool staging) {
  size_t cells = (size_t)(b[0] + w);
  if (dim >= 2) cells *= (size_t)(b[1] + w);
  if (dim >= 3) cells *= (size_t)(b[2] + w);
  size_t el = prec == ESN_DOUBLE ? sizeof(double) : sizeof(float);
  size_t bytes = cells * 2 * el * (size_t)ntr;
  // spreading also stages a batch of 64 points: kernel values, window starts
  // and strengths (the latter 16-byte aligned)
  if (staging)
    bytes += 64 * ((size_t)dim * w * el + (size_t)dim * sizeof(int)) + 16 + 64 * 2 * el * ntr;
  return bytes;
}

template <int D, int W, typename T>
static hipError_t spread_dispatch_t(int method, const GeomArgs& g, int nsub, int block,
                                    size_t lds, const void* c, void* grid, hipStream_t s) {
  if (method == 1) {
    if (nsub <= 0) return hipSuccess;
    hipLaunchKernelGGL((spread_lds_kernel<D, W, T>), dim3(nsub), dim3(64), lds, s, g,
                       static_cast<const cplx_t<T>*>(c), static_cast<T*>(grid));
  } else {
    if (g.M <= 0) return hipSuccess;
    const int bs = 256;
    const int64_t nb = (g.M + bs - 1) / bs;
    hipLaunchKernelGGL((spread_gm_kernel<D, W, T>), dim3((unsigned)nb), dim3(bs), 0, s, g,
                       static_cast<const cplx_t<T>*>(c), static_cast<T*>(grid));
  }
  return hipGetLastError();
}

template <int D, typename T>
static hipError_t spread_dispatch_w(int method, int w, const GeomArgs& g, int nsub, int block,
                                    size_t lds, const void* c, void* grid, hipStream_t s) {
  switch (w) {
#define ESN_W(WV) \
  case WV: return spread_dispatch_t<D, WV, T>(method, g, nsub, block, lds, c, grid, s);
    ESN_W(2) ESN_W(3) ESN_W(4) ESN_W(5) ESN_W(6) ESN_W(7) ESN_W(8) ESN_W(9)
    ESN_W(10) ESN_W(11) ESN_W(12) ESN_W(13) ESN_W(14) ESN_W(15) ESN_W(16)
#undef ESN_W
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_spread(int method, int prec, int dim, int w, const GeomArgs& g, int nsub,
                         int block, size_t lds_bytes, const void* c, void* grid,
                         hipStream_t s) {
  if (prec == ESN_SINGLE) {
    if (dim == 1) return spread_dispatch_w<1, float>(method, w, g, nsub, block, lds_bytes, c, grid, s);
    if (dim == 2) return spread_dispatch_w<2, float>(method, w, g, nsub, block, lds_bytes, c, grid, s);
    return spread_dispatch_w<3, float>(method, w, g, nsub, block, lds_bytes, c, grid, s);
  }
  if (dim == 1) return spread_dispatch_w<1, double>(method, w, g, nsub, block, lds_bytes, c, grid, s);
  if (dim == 2) return spread_dispatch_w<2, double>(method, w, g, nsub, block, lds_bytes, c, grid, s);
  return spread_dispatch_w<3, double>(method, w, g, nsub, block, lds_bytes, c, grid, s);
}

}  // namespace esn
