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
// * Self-sorting (Stockham) mixed-radix stages: radix 4 while it divides, one
//   radix 2 for an odd power of two, then radix 3 and radix 5 (lengths
//   L = 2^a 3^b 5^c with a >= 5, up to 512).  The first stage reads the grid,
//   the last writes it; the stages in between exchange through one LDS array
//   of L x 32 values (each thread holds all inputs of its butterflies before
//   the barrier that precedes the writes).
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

__device__ __forceinline__ float2 caddf(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csubf(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// a (sgn i)
__device__ __forceinline__ float2 crotf(float2 a, float sgn) {
  return make_float2(-sgn * a.y, sgn * a.x);
}

// Radix-R butterflies in place: v[r] = sum_m v[m] exp(sgn 2 pi i m r / R).
__device__ __forceinline__ void bfly2(float2* v) {
  const float2 a = v[0];
  v[0] = caddf(a, v[1]);
  v[1] = csubf(a, v[1]);
}

__device__ __forceinline__ void bfly3(float2* v, float sgn) {
  constexpr float kS3 = 0.86602540378443864676f;   // sin(2 pi / 3)
  const float2 t1 = caddf(v[1], v[2]);
  const float2 t2 = make_float2(v[0].x - 0.5f * t1.x, v[0].y - 0.5f * t1.y);
  const float2 d = csubf(v[1], v[2]);
  const float2 t3 = crotf(make_float2(kS3 * d.x, kS3 * d.y), sgn);
  v[0] = caddf(v[0], t1);
  v[1] = caddf(t2, t3);
  v[2] = csubf(t2, t3);
}

__device__ __forceinline__ void bfly5(float2* v, float sgn) {
  constexpr float c1 = 0.30901699437494742410f;    // cos(2 pi / 5)
  constexpr float c2 = -0.80901699437494742410f;   // cos(4 pi / 5)
  constexpr float s1 = 0.95105651629515357212f;    // sin(2 pi / 5)
  constexpr float s2 = 0.58778525229247312917f;    // sin(4 pi / 5)
  const float2 t1 = caddf(v[1], v[4]), t2 = caddf(v[2], v[3]);
  const float2 t3 = csubf(v[1], v[4]), t4 = csubf(v[2], v[3]);
  const float2 b1 = make_float2(v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y);
  const float2 b2 = make_float2(v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y);
  const float2 d1 = crotf(make_float2(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y), sgn);
  const float2 d2 = crotf(make_float2(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y), sgn);
  v[0] = caddf(v[0], caddf(t1, t2));
  v[1] = caddf(b1, d1);
  v[4] = csubf(b1, d1);
  v[2] = caddf(b2, d2);
  v[3] = csubf(b2, d2);
}

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

// Stages from sub-transform length LS on, radices R, Rest... .  A radix-R
// stage combines, for j = q LS + k (k < LS), the points q LS + k + m L/R
// (m < R), twiddled by w^(k m L / (R LS)), into q R LS + k + r LS (r < R);
// w = exp(sgn 2 pi i / L).  Thread (c, g) takes j = g + 8 b; where LS is a
// multiple of 8, k = g + (8 b mod LS) and q = 8 b / LS, so the grid points of
// the first and the last stage are g plus a uniform part.
template <int L, int LS, int R, int... Rest>
__device__ __forceinline__ void col_stages(float2* __restrict__ s, const float2* __restrict__ tw,
                                           float sgn, const ColPtr& gp, int c, int g) {
  constexpr bool first = LS == 1;
  constexpr bool last = sizeof...(Rest) == 0;
  static_assert((L / R) % kColGroups == 0, "butterflies split evenly over the groups");
  static_assert(!last || (LS % kColGroups == 0 && LS * R == L), "last stage");
  constexpr int B = L / R / kColGroups;   // butterflies per thread
  float2 v[B][R];
#pragma unroll
  for (int b = 0; b < B; b++) {
    const int j = g + kColGroups * b, k = j % LS, q = j / LS;
#pragma unroll
    for (int m = 0; m < R; m++) {
      if constexpr (first)
        v[b][m] = gp.at(kColGroups * b + m * (L / R));
      else
        v[b][m] = s[(q * LS + k + m * (L / R)) * kColW + c];
    }
    if constexpr (!first) {
#pragma unroll
      for (int m = 1; m < R; m++) v[b][m] = cmulf(v[b][m], tw[k * m * (L / (R * LS))]);
    }
    if constexpr (R == 2) bfly2(v[b]);
    else if constexpr (R == 3) bfly3(v[b], sgn);
    else if constexpr (R == 4) bfly4(v[b], sgn);
    else bfly5(v[b], sgn);
  }
  if constexpr (!first) __syncthreads();   // every read of s is done
#pragma unroll
  for (int b = 0; b < B; b++) {
    const int j = g + kColGroups * b, k = j % LS, q = j / LS;
#pragma unroll
    for (int r = 0; r < R; r++) {
      if constexpr (last)
        gp.at((kColGroups * b / LS) * R * LS + (kColGroups * b) % LS + r * LS) = v[b][r];
      else
        s[(q * R * LS + k + r * LS) * kColW + c] = v[b][r];
    }
  }
  if constexpr (!last) {
    __syncthreads();
    col_stages<L, LS * R, Rest...>(s, tw, sgn, gp, c, g);
  }
}

template <int L, int... Rs>
__global__ __launch_bounds__(kColThreads) void fft_cols_kernel(float2* __restrict__ data,
                                                               const ColFFTArgs a,
                                                               const double2* __restrict__ twd) {
  static_assert(L >= 32 && L <= 512, "lengths 32 .. 512");
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
  for (int64_t i = blockIdx.y; i < a.nplanes; i += gridDim.y) {
    if (i != (int64_t)blockIdx.y) __syncthreads();   // the last plane's reads of s are done
    const int64_t pl = i < a.planes_a ? i : a.plane_b0 + (i - a.planes_a);
    gp.base = reinterpret_cast<char*>(gt + pl * a.pstride);
    col_stages<L, 1, Rs...>(s, tw, sgn, gp, c, g);
  }
}

bool fft_cols_supported(int64_t L) {
  switch (L) {
    case 32: case 64: case 96: case 128: case 160: case 192:
    case 256: case 288: case 320: case 384: case 480: case 512: return true;
    default: return false;
  }
}

#define ESN_COLS(LEN, ...)                                                                     \
  case LEN:                                                                                    \
    hipLaunchKernelGGL((fft_cols_kernel<LEN, __VA_ARGS__>), grid, block, 0, s, data, a, tw); \
    break;

hipError_t launch_fft_cols(float2* data, int L, const ColFFTArgs& a, const double2* tw,
                           int nchunks, int ntr, hipStream_t s) {
  const dim3 grid((unsigned)nchunks, (unsigned)std::min<int64_t>(a.nplanes, 65535),
                  (unsigned)ntr);
  const dim3 block(kColThreads);
  // radix 4 while it divides, one radix 2 for an odd power of two, then 3s and 5s
  switch (L) {
    ESN_COLS(32, 4, 4, 2)
    ESN_COLS(64, 4, 4, 4)
    ESN_COLS(96, 4, 4, 2, 3)
    ESN_COLS(128, 4, 4, 4, 2)
    ESN_COLS(160, 4, 4, 2, 5)
    ESN_COLS(192, 4, 4, 4, 3)
    ESN_COLS(256, 4, 4, 4, 4)
    ESN_COLS(288, 4, 4, 2, 3, 3)
    ESN_COLS(320, 4, 4, 4, 5)
    ESN_COLS(384, 4, 4, 4, 2, 3)
    ESN_COLS(480, 4, 4, 2, 3, 5)
    ESN_COLS(512, 4, 4, 4, 4, 2)
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#undef ESN_COLS

}  // namespace esn
