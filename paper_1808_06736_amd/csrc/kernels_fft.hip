// Column FFTs of the fine grid (Sec. 3.1 step 2 and Sec. 3.2 step 2): the y
// and z passes of a 3D transform, applied only to the x columns that hold
// modes.  A 3D DFT is three passes of 1D DFTs, one per dimension; the y and z
// passes act on each x column by itself, so they may skip the others.
//
// A block takes 32 neighbouring x columns of one plane (a z plane for the y
// pass, a y row for the z pass) and runs their 32 length-L DFTs, unnormalised,
// with exponent sign sgn: out[r] = sum_j in[j] exp(sgn 2 pi i j r / L).
// * Reads and writes move 32 consecutive complex values (256 bytes) per grid
//   row, so every access is coalesced whatever the stride between the DFT's
//   points.
// * Self-sorting (Stockham) radix-4 stages with a final radix-2 stage when
//   log2 L is odd.  The first stage reads the grid, the last writes it; the
//   stages in between exchange through one LDS array of L x 32 values (each
//   thread holds all inputs of its butterflies before the barrier that
//   precedes the writes).
// * Twiddle factors exp(2 pi i e / L) come from a table computed in FP64 on the
//   host, staged in LDS.
#include "device_common.hpp"

namespace esn {

constexpr int kColW = kColWidth;                 // columns per block
constexpr int kColThreads = 256;
constexpr int kColGroups = kColThreads / kColW;  // butterfly groups per column

__device__ __forceinline__ float2 cmulf(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Radix-4 butterfly in place: v[r] = sum_m v[m] (sgn i)^(m r).
__device__ __forceinline__ void bfly4(float2* v, float sgn) {
  const float2 t0 = make_float2(v[0].x + v[2].x, v[0].y + v[2].y);
  const float2 t1 = make_float2(v[0].x - v[2].x, v[0].y - v[2].y);
  const float2 t2 = make_float2(v[1].x + v[3].x, v[1].y + v[3].y);
  const float2 d = make_float2(v[1].x - v[3].x, v[1].y - v[3].y);
  const float2 t3 = make_float2(-sgn * d.y, sgn * d.x);   // d (sgn i)
  v[0] = make_float2(t0.x + t2.x, t0.y + t2.y);
  v[2] = make_float2(t0.x - t2.x, t0.y - t2.y);
  v[1] = make_float2(t1.x + t3.x, t1.y + t3.y);
  v[3] = make_float2(t1.x - t3.x, t1.y - t3.y);
}

// Grid access of a thread: point idx = g + u of its column, with u uniform
// over the block.  The address is a uniform base (kept in scalar registers)
// plus the thread's 32-bit byte offset (c + g es) * 8, so a pass needs one
// address register per thread however many loads are in flight.
struct ColPtr {
  char* base;       // the plane's first column of the block
  int64_t es8;      // bytes between consecutive points of a DFT
  uint32_t loff;    // (c + g es) * 8
  __device__ __forceinline__ float2& at(int u) const {
    return *reinterpret_cast<float2*>(base + (int64_t)u * es8 + loff);
  }
};

// Stages from sub-transform length LS on.  A radix-4 stage combines, for
// j = q LS + k (k < LS), the points q LS + k + m L/4 (m = 0..3), twiddled by
// w^(k m L / (4 LS)), into q 4 LS + k + r LS (r = 0..3); w = exp(sgn 2 pi i / L).
// Thread (c, g) takes j = g + 8 b; for LS >= 8, k = g + (8 b mod LS) and
// q = 8 b / LS, so the grid points of the first and last stages are g plus a
// uniform part.
template <int L, int LS>
__device__ __forceinline__ void col_stages(float2* __restrict__ s, const float2* __restrict__ tw,
                                           float sgn, const ColPtr& gp, int c, int g) {
  if constexpr (4 * LS <= L) {
    constexpr bool first = LS == 1;
    constexpr bool last = 4 * LS == L;
    static_assert(!last || LS >= kColGroups, "last radix-4 stage from LS >= 8");
    constexpr int B = L / 4 / kColGroups;   // butterflies per thread
    float2 v[B][4];
#pragma unroll
    for (int b = 0; b < B; b++) {
      const int j = g + kColGroups * b, k = j % LS, q = j / LS;
#pragma unroll
      for (int m = 0; m < 4; m++) {
        if constexpr (first)
          v[b][m] = gp.at(kColGroups * b + m * (L / 4));
        else
          v[b][m] = s[(q * LS + k + m * (L / 4)) * kColW + c];
      }
      if constexpr (!first) {
#pragma unroll
        for (int m = 1; m < 4; m++) v[b][m] = cmulf(v[b][m], tw[k * m * (L / (4 * LS))]);
      }
      bfly4(v[b], sgn);
    }
    if constexpr (!first) __syncthreads();   // every read of s is done
#pragma unroll
    for (int b = 0; b < B; b++) {
      const int j = g + kColGroups * b, k = j % LS, q = j / LS;
#pragma unroll
      for (int r = 0; r < 4; r++) {
        if constexpr (last)
          gp.at((kColGroups * b / LS) * 4 * LS + (kColGroups * b) % LS + r * LS) = v[b][r];
        else
          s[(q * 4 * LS + k + r * LS) * kColW + c] = v[b][r];
      }
    }
    if constexpr (!last) {
      __syncthreads();
      col_stages<L, 4 * LS>(s, tw, sgn, gp, c, g);
    }
  } else {
    // radix 2, LS = L / 2: points k and k + L/2, twiddle w^k
    static_assert(2 * LS == L, "stage lengths");
    constexpr int B = L / 2 / kColGroups;
#pragma unroll
    for (int b = 0; b < B; b++) {
      const int k = g + kColGroups * b;
      const float2 a0 = s[k * kColW + c];
      const float2 a1 = cmulf(s[(k + L / 2) * kColW + c], tw[k]);
      gp.at(kColGroups * b) = make_float2(a0.x + a1.x, a0.y + a1.y);
      gp.at(kColGroups * b + LS) = make_float2(a0.x - a1.x, a0.y - a1.y);
    }
  }
}

template <int L>
__global__ __launch_bounds__(kColThreads) void fft_cols_kernel(float2* __restrict__ data,
                                                               const ColFFTArgs a,
                                                               const double2* __restrict__ twd) {
  static_assert(L >= 32 && (L & (L - 1)) == 0, "power-of-two lengths from 32");
  __shared__ float2 s[L * kColW];
  __shared__ float2 tw[L];
  const int c = threadIdx.x % kColW, g = threadIdx.x / kColW;
  const float sgn = (float)a.sign;
  for (int i = threadIdx.x; i < L; i += kColThreads)
    tw[i] = make_float2((float)twd[i].x, (float)(a.sign * twd[i].y));
  const int chunk = (int)blockIdx.x < a.chunks_a ? (int)blockIdx.x
                                                  : a.chunk_b0 + ((int)blockIdx.x - a.chunks_a);
  float2* gt = data + (int64_t)blockIdx.z * a.tstride + (int64_t)chunk * kColW;
  ColPtr gp;
  gp.es8 = a.estride * (int64_t)sizeof(float2);
  gp.loff = (uint32_t)((c + (int64_t)g * a.estride) * (int64_t)sizeof(float2));
  for (int64_t pl = blockIdx.y; pl < a.nplanes; pl += gridDim.y) {
    if (pl != (int64_t)blockIdx.y) __syncthreads();   // the last plane's reads of s are done
    gp.base = reinterpret_cast<char*>(gt + pl * a.pstride);
    col_stages<L, 1>(s, tw, sgn, gp, c, g);
  }
}

hipError_t launch_fft_cols(float2* data, int L, const ColFFTArgs& a, const double2* tw,
                           int nchunks, int ntr, hipStream_t s) {
  const dim3 grid((unsigned)nchunks, (unsigned)std::min<int64_t>(a.nplanes, 65535),
                  (unsigned)ntr);
  const dim3 block(kColThreads);
  switch (L) {
    case 32: hipLaunchKernelGGL(fft_cols_kernel<32>, grid, block, 0, s, data, a, tw); break;
    case 64: hipLaunchKernelGGL(fft_cols_kernel<64>, grid, block, 0, s, data, a, tw); break;
    case 128: hipLaunchKernelGGL(fft_cols_kernel<128>, grid, block, 0, s, data, a, tw); break;
    case 256: hipLaunchKernelGGL(fft_cols_kernel<256>, grid, block, 0, s, data, a, tw); break;
    case 512: hipLaunchKernelGGL(fft_cols_kernel<512>, grid, block, 0, s, data, a, tw); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace esn
