// Column FFTs of the fine grid (Sec. 3.1 step 2 and Sec. 3.2 step 2): the y
// and z passes of a 3D transform, applied only to the x columns that hold
// modes.  A 3D DFT is three passes of 1D DFTs, one per dimension; the y and z
// passes act on each x column by itself, so they may skip the others.
//
// A block takes W = 16 or 32 neighbouring x columns of one plane (a z plane
// for the y pass, a y row for the z pass) and runs their W length-L DFTs,
// unnormalised, with exponent sign sgn: out[r] = sum_j in[j] exp(sgn 2 pi i j
// r / L).
// * Reads and writes move W consecutive complex values (128 or 256 bytes) per
//   grid row, so every access is coalesced whatever the stride between the
//   DFT's points.  W = 16 (half the LDS, twice the blocks per CU) where every
//   stage splits over 16 threads per column.
// * Self-sorting (Stockham) mixed-radix stages: radix 4 while it divides, one
//   radix 2 for an odd power of two, then radix 3 and radix 5 (lengths
//   L = 2^a 3^b 5^c with a >= 5, up to 512).  The first stage reads the grid,
//   the last writes it; the stages in between exchange through one LDS array
//   of L x W values (each thread holds all inputs of its butterflies before
//   the barrier that precedes the writes).
// * Twiddle factors exp(2 pi i e / L) come from a table computed in FP64 on the
//   host, staged in LDS.
// * The z pass may take the correction of Sec. 3.1 step 3 / Sec. 3.2 step 1
//   itself: type 1 writes f_k = p_k b^_k (eq. (pb1)) into the mode array, type
//   2 reads p_k f_k from it (zero at the fine-grid points that hold no mode).
#include "device_common.hpp"

namespace esn {

constexpr int kColThreads = 256;

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

// What the first stage reads and the last stage writes (in / out modes):
//   kColPlain  the grid;
//   kColMasked the grid, but only the kept points j < keep_lo or
//              j >= L - keep_hi (the others read as zero, or are not stored);
//   kColModes  (z pass) the mode array with the correction factors: type 2
//              reads p_k f_k at the kept points (zero elsewhere, eq. (pb1)
//              read backwards), type 1 writes f_k = p_k b^_k (eq. (pb1)).
constexpr int kColPlain = 0, kColMasked = 1, kColModes = 2;

// Thread's view of the mode array for one column (x = chunk 32 + c, y = the
// plane) of the z pass.  The z points' offsets in the mode array and their
// factors p_kz come from a per-block LDS table (zoff < 0: no mode).
struct ColIO {
  ColPtr gp;
  int64_t keep_lo, keep_hi;
  // modes
  float2* f;                // this transform's mode array
  int fxy;                  // position of (kx, ky) in it
  double pxy;               // p_kx p_ky (0 where (x, y) holds no mode)
  const int* zoff;          // [L] N1 N2 .. position of kz, or -1
  const double* zfac;       // [L] p_kz
  // the correction p_k = p_kx p_ky p_kz, formed in FP64 and rounded once (as
  // the separate deconvolution and amplification kernels do)
  __device__ __forceinline__ float factor(int j) const { return (float)(pxy * zfac[j]); }
  bool col_ok;              // (x, y) holds modes
  __device__ __forceinline__ bool kept(int j, int L) const {
    return j < keep_lo || j >= L - keep_hi;
  }
  template <int IN, int L>
  __device__ __forceinline__ float2 load(int g, int u) const {
    if constexpr (IN == kColPlain) return gp.at(u);
    const int j = g + u;
    if constexpr (IN == kColMasked) return kept(j, L) ? gp.at(u) : make_float2(0.f, 0.f);
    const int zo = zoff[j];
    if (!col_ok || zo < 0) return make_float2(0.f, 0.f);
    const float p = factor(j);
    const float2 v = f[fxy + zo];
    return make_float2(v.x * p, v.y * p);
  }
  template <int OUT, int L>
  __device__ __forceinline__ void store(int g, int u, float2 v) const {
    if constexpr (OUT == kColPlain) {
      gp.at(u) = v;
      return;
    }
    const int j = g + u;
    if constexpr (OUT == kColMasked) {
      if (kept(j, L)) gp.at(u) = v;
      return;
    }
    const int zo = zoff[j];
    if (!col_ok || zo < 0) return;
    const float p = factor(j);
    f[fxy + zo] = make_float2(v.x * p, v.y * p);
  }
};

// Stages from sub-transform length LS on, radices R, Rest... .  A radix-R
// stage combines, for j = q LS + k (k < LS), the points q LS + k + m L/R
// (m < R), twiddled by w^(k m L / (R LS)), into q R LS + k + r LS (r < R);
// w = exp(sgn 2 pi i / L).  A block of W columns has G = 256 / W threads per
// column; thread (c, g) takes j = g + G b.  Where LS is a multiple of G,
// k = g + (G b mod LS) and q = G b / LS, so the grid points of the first and
// the last stage are g plus a uniform part.
template <int L, int W, int IN, int OUT, int LS, int R, int... Rest>
__device__ __forceinline__ void col_stages(float2* __restrict__ s, const float2* __restrict__ tw,
                                           float sgn, const ColIO& io, int c, int g) {
  constexpr int G = kColThreads / W;
  constexpr bool first = LS == 1;
  constexpr bool last = sizeof...(Rest) == 0;
  static_assert((L / R) % G == 0, "butterflies split evenly over the groups");
  static_assert(!last || (LS % G == 0 && LS * R == L), "last stage");
  constexpr int B = L / R / G;   // butterflies per thread
  float2 v[B][R];
#pragma unroll
  for (int b = 0; b < B; b++) {
    const int j = g + G * b, k = j % LS, q = j / LS;
#pragma unroll
    for (int m = 0; m < R; m++) {
      if constexpr (first)
        v[b][m] = io.load<IN, L>(g, G * b + m * (L / R));
      else
        v[b][m] = s[(q * LS + k + m * (L / R)) * W + c];
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
    const int j = g + G * b, k = j % LS, q = j / LS;
#pragma unroll
    for (int r = 0; r < R; r++) {
      if constexpr (last)
        io.store<OUT, L>(g, (G * b / LS) * R * LS + (G * b) % LS + r * LS,
                         v[b][r]);
      else
        s[(q * R * LS + k + r * LS) * W + c] = v[b][r];
    }
  }
  if constexpr (!last) {
    __syncthreads();
    col_stages<L, W, IN, OUT, LS * R, Rest...>(s, tw, sgn, io, c, g);
  }
}

template <int L, int W, int IN, int OUT, int... Rs>
__global__ __launch_bounds__(kColThreads) void fft_cols_kernel(float2* __restrict__ data,
                                                               const ColFFTArgs a,
                                                               const double2* __restrict__ twd,
                                                               const ColModes cm) {
  static_assert(L >= 32 && L <= 512, "lengths 32 .. 512");
  __shared__ float2 s[L * W];
  __shared__ float2 tw[L];
  const int c = threadIdx.x % W, g = threadIdx.x / W;
  const float sgn = (float)a.sign;
  for (int i = threadIdx.x; i < L; i += kColThreads)
    tw[i] = make_float2((float)twd[i].x, (float)(a.sign * twd[i].y));
  const int chunk = (int)blockIdx.x < a.chunks_a ? (int)blockIdx.x
                                                  : a.chunk_b0 + ((int)blockIdx.x - a.chunks_a);
  float2* gt = data + (int64_t)blockIdx.z * a.tstride + (int64_t)chunk * W;
  ColIO io;
  io.gp.es8 = a.estride * (int64_t)sizeof(float2);
  io.gp.loff = (uint32_t)((c + (int64_t)g * a.estride) * (int64_t)sizeof(float2));
  io.keep_lo = a.keep_lo;
  io.keep_hi = a.keep_hi;
  io.f = nullptr;
  io.fxy = 0;
  io.pxy = 0.0;
  io.zoff = nullptr;
  io.zfac = nullptr;
  io.col_ok = false;
  int64_t kx = 0;
  bool x_ok = false;
  constexpr bool modes = IN == kColModes || OUT == kColModes;
  __shared__ int zoff[modes ? L : 1];
  __shared__ double zfac[modes ? L : 1];
  if constexpr (modes) {
    const int64_t x = (int64_t)chunk * W + c;
    const int64_t N0 = cm.N[0], N2 = cm.N[2];
    x_ok = x < N0 - N0 / 2 || x >= cm.n0 - N0 / 2;
    kx = x < N0 - N0 / 2 ? x : x - cm.n0;
    io.f = cm.f + (int64_t)blockIdx.z * cm.fstride;
    // z point j holds mode kz = j (j < ceil(N3/2)) or j - L (j >= L - floor(N3/2))
    for (int j = threadIdx.x; j < L; j += kColThreads) {
      const bool ok = j < N2 - N2 / 2 || j >= L - N2 / 2;
      const int64_t k = j < N2 - N2 / 2 ? j : (int64_t)j - L;
      const int64_t pos = cm.modeord == 0 ? k + N2 / 2 : (k >= 0 ? k : k + N2);
      zoff[j] = ok ? (int)(pos * cm.N[0] * cm.N[1]) : -1;
      zfac[j] = ok ? cm.pf[2][k < 0 ? -k : k] : 0.0;
    }
    io.zoff = zoff;
    io.zfac = zfac;
    __syncthreads();
  }
  for (int64_t i = blockIdx.y; i < a.nplanes; i += gridDim.y) {
    if (i != (int64_t)blockIdx.y) __syncthreads();   // the last plane's reads of s are done
    const int64_t pl = i < a.planes_a ? i : a.plane_b0 + (i - a.planes_a);
    io.gp.base = reinterpret_cast<char*>(gt + pl * a.pstride);
    if constexpr (modes) {
      // the plane is a y row that holds modes (the z pass runs on those only)
      const int64_t N0 = cm.N[0], N1 = cm.N[1];
      const int64_t ky = pl < N1 - N1 / 2 ? pl : pl - cm.n1;
      const bool y_ok = pl < N1 - N1 / 2 || pl >= cm.n1 - N1 / 2;
      io.col_ok = x_ok && y_ok;
      const int64_t px = cm.modeord == 0 ? kx + N0 / 2 : (kx >= 0 ? kx : kx + N0);
      const int64_t py = cm.modeord == 0 ? ky + N1 / 2 : (ky >= 0 ? ky : ky + N1);
      io.fxy = (int)(px + N0 * py);
      io.pxy = io.col_ok ? cm.pf[0][kx < 0 ? -kx : kx] * cm.pf[1][ky < 0 ? -ky : ky] : 0.0;
    }
    col_stages<L, W, IN, OUT, 1, Rs...>(s, tw, sgn, io, c, g);
  }
}

// Zero the x columns x0 .. x1 - 1 (even, x1 > x0) of every row: the columns
// that no column pass writes but the x pass reads.
__global__ void zero_cols_kernel(float2* __restrict__ data, int64_t n0, int64_t rows, int64_t x0,
                                 int64_t x1, int64_t tstride) {
  float4* base = reinterpret_cast<float4*>(data + (int64_t)blockIdx.z * tstride);
  const int64_t npair = (x1 - x0) / 2;
  for (int64_t r = blockIdx.y; r < rows; r += gridDim.y)
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npair;
         i += (int64_t)gridDim.x * blockDim.x)
      base[(r * n0 + x0) / 2 + i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

hipError_t launch_zero_cols(float2* data, int64_t n0, int64_t rows, int64_t x0, int64_t x1,
                            int ntr, int64_t tstride, hipStream_t s) {
  if (x1 <= x0) return hipSuccess;
  const int64_t npair = (x1 - x0) / 2;
  const int bs = npair >= 256 ? 256 : 64 * (int)((npair + 63) / 64);
  const int64_t gx = std::min<int64_t>((npair + bs - 1) / bs, 65535);
  const int64_t gy = std::min<int64_t>(rows, std::max<int64_t>(1, 16384 / gx));
  hipLaunchKernelGGL(zero_cols_kernel, dim3((unsigned)gx, (unsigned)std::min<int64_t>(gy, 65535),
                                           (unsigned)ntr),
                     dim3(bs), 0, s, data, n0, rows, x0, x1, tstride);
  return hipGetLastError();
}

bool fft_cols_supported(int64_t L) {
  switch (L) {
    case 32: case 64: case 96: case 128: case 160: case 192:
    case 256: case 288: case 320: case 384: case 480: case 512: return true;
    default: return false;
  }
}

// Blocks of 16 columns (128-byte rows; half the LDS of 32, so twice the
// blocks per CU) where every stage splits over 16 threads per column, i.e.
// L a multiple of 64; 32 columns otherwise.  a, nchunks: in blocks of 32.
template <int IN, int OUT>
static hipError_t launch_cols_io(float2* data, int L, const ColFFTArgs& a, const double2* tw,
                                 const ColModes& cm, int nchunks, int ntr, hipStream_t s) {
  const dim3 block(kColThreads);
  const int narrow = L % 64 == 0 ? 2 : 1;   // blocks per 32 columns
  ColFFTArgs b = a;
  b.chunks_a *= narrow;
  b.chunk_b0 *= narrow;
  const dim3 grid((unsigned)(nchunks * narrow), (unsigned)std::min<int64_t>(a.nplanes, 65535),
                  (unsigned)ntr);
#define ESN_COLS(LEN, WID, ...)                                                              \
  case LEN:                                                                                  \
    hipLaunchKernelGGL((fft_cols_kernel<LEN, WID, IN, OUT, __VA_ARGS__>), grid, block, 0, s, \
                       data, b, tw, cm);                                                     \
    break;
  // radix 4 while it divides, one radix 2 for an odd power of two, then 3s and 5s
  switch (L) {
    ESN_COLS(32, 32, 4, 4, 2)
    ESN_COLS(64, 16, 4, 4, 4)
    ESN_COLS(96, 32, 4, 4, 2, 3)
    ESN_COLS(128, 16, 4, 4, 4, 2)
    ESN_COLS(160, 32, 4, 4, 2, 5)
    ESN_COLS(192, 16, 4, 4, 4, 3)
    ESN_COLS(256, 16, 4, 4, 4, 4)
    ESN_COLS(288, 32, 4, 4, 2, 3, 3)
    ESN_COLS(320, 16, 4, 4, 4, 5)
    ESN_COLS(384, 16, 4, 4, 4, 2, 3)
    ESN_COLS(480, 32, 4, 4, 2, 3, 5)
    ESN_COLS(512, 16, 4, 4, 4, 4, 2)
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fft_cols(float2* data, int L, const ColFFTArgs& a, const double2* tw,
                           int nchunks, int ntr, int in_mode, int out_mode, const ColModes& cm,
                           hipStream_t s) {
  if (in_mode == kColPlain && out_mode == kColPlain)
    return launch_cols_io<kColPlain, kColPlain>(data, L, a, tw, cm, nchunks, ntr, s);
  if (in_mode == kColModes && out_mode == kColPlain)
    return launch_cols_io<kColModes, kColPlain>(data, L, a, tw, cm, nchunks, ntr, s);
  if (in_mode == kColMasked && out_mode == kColPlain)
    return launch_cols_io<kColMasked, kColPlain>(data, L, a, tw, cm, nchunks, ntr, s);
  if (in_mode == kColPlain && out_mode == kColMasked)
    return launch_cols_io<kColPlain, kColMasked>(data, L, a, tw, cm, nchunks, ntr, s);
  if (in_mode == kColPlain && out_mode == kColModes)
    return launch_cols_io<kColPlain, kColModes>(data, L, a, tw, cm, nchunks, ntr, s);
  return hipErrorInvalidValue;
}

#undef ESN_COLS

}  // namespace esn
