// Spreading and interpolation in 2D on the matrix cores (single and double
// precision, w <= 13), four waves per subproblem (a run of at most maxsub
// bin-sorted points of one bin, Sec. 5.2).
//
// Points are binned by window cell (the cell floor(w/2) after the first cell
// of the point's window) and, inside a bin, sorted by B x B blocks of window
// cells (B = 8 for w <= 9, else 4).  A point in window cell l has its w window
// cells at l - floor(w/2) .. l - floor(w/2) + w - 1, so the points of one
// block put all their weights in the 16 cells from B (l / B) - floor(w/2) in
// each dimension: at slots (l mod B) .. (l mod B) + w - 1 of a 16 x 16
// footprint.  Spreading the points
// of a block, eq. (bl), is then a dense contraction over the points,
//
//     G[x, y] += sum_p  kx_p(x)  *  ky_p(y) c_p,
//
// of a 16 x P matrix of x weights with a P x 16 matrix of y weights times the
// strength (real and imaginary parts separately), which the wave runs with the
// 16 x 16 x 4 matrix instructions (4 points per instruction, two instructions
// for the two parts).  When a wave moves on to the next block, its 16 x 16
// result is added into its LDS tile of the bin (bin + 16 - B cells per dim);
// the tiles go to the fine grid once at the end (global atomics on the
// touched cells only).
//
// Interpolation, eq. (interp), runs the contraction the other way: for the
// points of one block, U[y, p] = sum_x G[x, y] kx_p(x) (the grid tile as the
// first operand, 16 points per instruction group), then c_p = sum_y ky_p(y)
// U[y, p] in registers and across the lane groups, with the bin's grid tile
// copied into LDS first.
//
// Layouts of the 16 x 16 x 4 instructions (A 16 x 4, B 4 x 16, D 16 x 16): lane
// i supplies A[i mod 16][i / 16] and B[i / 16][i mod 16] and holds four
// elements of column i mod 16 of D: rows 4 (i / 16) + j (single precision) or
// rows i / 16 + 4 j (double precision), j = 0 .. 3.
#include "device_common.hpp"

namespace esn {

template <typename T> struct Mfma16;
template <> struct Mfma16<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  __device__ static __forceinline__ v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // row of D element j held by lane group kq = lane / 16
  __device__ static __forceinline__ int row(int kq, int j) { return 4 * kq + j; }
};
template <> struct Mfma16<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __device__ static __forceinline__ v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ int row(int kq, int j) { return kq + 4 * j; }
};

// Staged points per batch: 64, then points that the last steps of a run may
// read past the batch (weights of a point beyond a run only meet masked or
// unstored operands; they stay finite).
constexpr int kStage2d = 80;

// Block size of a width: blocks of B window cells keep every window inside the
// 16 slots from the block's first cell (B - 1 + w <= 16).
__host__ __device__ constexpr int block2d(int w) { return w <= 9 ? 8 : 4; }

// Tile of a bin of b0 x b1 window cells: footprints start at B (l / B) for
// window cells l of the bin and are 16 wide, so bin + 16 - B cells per dim.
__host__ __device__ inline int tile2d_dim(int b, int bs) { return b + 16 - bs; }

// LDS layouts.  The local data share has 32 banks; a wave's 32-bit reads take
// as many cycles as the most distinct words asked of one bank (two when the 64
// lanes spread evenly), 64-bit reads the same over 32 banks of 8 bytes, and
// 32-bit writes go 16 lanes at a time.  Every layout below keeps each access
// of the kernels at that minimum:
//  * tiles are planar (real and imaginary parts in separate planes) with a row
//    pitch of 4 mod 32 elements, so the 16 x 4 lanes of a matrix operand or
//    result (column r16 one row apart, k group kq one or four elements apart)
//    fall on distinct banks;
//  * spreading stages the weights point-major (16 slots per point) with the
//    slot index XORed by a function of the point, so that staging (one point
//    per lane, same slot) and the operand reads (16 slots of 4 points) are
//    both spread over all banks;
//  * interpolation stages them slot-major with pitches of 16 mod 32 (x) and
//    16 or 4 mod 32 (y, single precision: four consecutive slots per k group).
__host__ __device__ inline int tile2d_pitch(int tx) { return tx + ((4 - tx) & 31); }
template <typename T>
__device__ __forceinline__ int stage_swz(int p) { return sizeof(T) == 4 ? (p >> 1) & 15 : p & 15; }
constexpr int kPitchX2d = 80;
template <typename T> __host__ __device__ constexpr int pitch_y2d() { return sizeof(T) == 4 ? 84 : 80; }

size_t mfma2d_lds_bytes(int prec, int w, const int* b, int ntr, bool spread) {
  const size_t cs = prec == ESN_DOUBLE ? 16 : 8, rs = prec == ESN_DOUBLE ? 8 : 4;
  const int bs = block2d(w);
  const size_t plane = (size_t)tile2d_pitch(tile2d_dim(b[0], bs)) * tile2d_dim(b[1], bs);
  // spreading keeps two copies of the tiles, interpolation one
  const size_t tile = (spread ? 2 : 1) * 2 * plane * rs * ntr;
  const size_t stage = spread ? 2 * kStage2d * 16 * rs
                              : 16 * (kPitchX2d + (prec == ESN_DOUBLE ? 80 : 84)) * rs;
  // strengths or results [64], run keys, footprint offsets and original indices [64]
  return tile + stage + 64 * cs + 3 * 64 * sizeof(int) + 16;
}

// The 16 staged weights of one point along one dimension: w kernel values from
// the window cell's offset in its block, zeros elsewhere.  Returns the window
// cell relative to the bin origin o.
template <int W, typename T>
__device__ __forceinline__ int weights16(const GeomArgs& g, int64_t i, int m, int o, T (&r)[16]) {
  constexpr int BS = block2d(W);
  int sh;
  const Coord<T> cd = decode_coord<T>(g.pts, g.pts_code, g.fbits[m], i, m, &sh, W);
  T k[W];
  es_weights_any<W, T>(sh, cd.f, (T)g.beta, g.ktab, k);
  const int l = window_cell(cd.cell, sh, g.n[m]) - o;
  const int off = l & (BS - 1);
#pragma unroll
  for (int s = 0; s < 16; s++) r[s] = s < W ? k[s] : (T)0;
  // shift by off, one bit at a time (selects, no indexed registers)
#pragma unroll
  for (int b = 1; b < BS; b <<= 1) {
    const bool sft = (off & b) != 0;
#pragma unroll
    for (int s = 15; s >= 0; s--) r[s] = sft ? (s >= b ? r[s - b] : (T)0) : r[s];
  }
  return l;
}

// Bin of subproblem sidx and its origin (window cells).
__device__ __forceinline__ void bin_origin2d(const GeomArgs& g, int bin, int* o0, int* o1) {
  const int bi0 = bin % g.nb[0], bi1 = bin / g.nb[0];
  *o0 = bi0 * g.b[0];
  *o1 = bi1 * g.b[1];
}

// Window cell of sorted point i along dimension m relative to the bin origin o.
template <int W, typename T>
__device__ __forceinline__ int rel_cell2d(const GeomArgs& g, int64_t i, int m, int o) {
  int sh;
  const Coord<T> cd = decode_coord<T>(g.pts, g.pts_code, g.fbits[m], i, m, &sh, W);
  return window_cell(cd.cell, sh, g.n[m]) - o;
}

// Adds a 16 x 16 result (this lane's four elements of column r16) into a tile
// plane at the block's footprint.  Single precision: the four rows are
// consecutive cells, one 16-byte access.
__device__ __forceinline__ void add_block(float* dst, int kq, Mfma16<float>::v4 acc) {
  auto* d = reinterpret_cast<Mfma16<float>::v4*>(dst + 4 * kq);
  *d += acc;
}
__device__ __forceinline__ void add_block(double* dst, int kq, Mfma16<double>::v4 acc) {
#pragma unroll
  for (int j = 0; j < 4; j++) dst[kq + 4 * j] += acc[j];
}

// Four waves per subproblem share the staged weights.  Wave v takes the real
// (v even) or imaginary (v odd) part and the even (v < 2) or odd steps of
// every run; the two step halves add into two copies of the tile, so no two
// waves write the same LDS value.  Per batch of 64 points wave 0 stages the x
// weights and the run data, wave 1 the y weights, wave 2 the first
// transform's strengths.  Transforms 0 .. g.ntr - 1 share the staged weights,
// each with its own tiles.
template <int W, typename T>
__global__ void __launch_bounds__(256)
spread2d_mfma_kernel(const GeomArgs g, const cplx_t<T>* __restrict__ c, T* __restrict__ grid) {
  using M = Mfma16<T>;
  using v4 = typename M::v4;
  constexpr int H = W / 2;
  constexpr int BS = block2d(W);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int TX = tile2d_dim(g.b[0], BS), TY = tile2d_dim(g.b[1], BS);
  const int TP = tile2d_pitch(TX);
  const int plane = TP * TY;
  const int ntr = g.ntr;
  T* tile = reinterpret_cast<T*>(smem_raw);                             // [2][ntr][2][TY][TP]
  T* sx = tile + (size_t)4 * plane * ntr;                               // [kStage2d][16]
  T* sy = sx + kStage2d * 16;                                           // [kStage2d][16]
  cplx_t<T>* sc = reinterpret_cast<cplx_t<T>*>(sy + kStage2d * 16);     // [64]
  int* srun = reinterpret_cast<int*>(sc + 64);                          // [64] block id
  int* sorg = srun + 64;                                                // [64] footprint offset
  int* sperm = sorg + 64;                                               // [64] original index

  const int sidx = blockIdx.x;
  const int bin = g.sub_bin[sidx];
  const int p0 = g.sub_start[sidx];
  const int p1 = p0 + g.sub_len[sidx];
  int ox, oy;
  bin_origin2d(g, bin, &ox, &oy);
  const int tid = threadIdx.x;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int part = wv & 1, half = wv >> 1;
  for (int i = tid; i < 4 * plane * ntr; i += 256) tile[i] = (T)0;
  for (int i = tid; i < 2 * kStage2d * 16; i += 256) sx[i] = (T)0;
  const int r16 = lane & 15;   // A row / B column / D column
  const int kq = lane >> 4;    // k group (the step's point) / D row group
  // this wave's plane: copy `half`, part `part`
  T* mine = tile + (size_t)(half * 2 * ntr + part) * plane;

  for (int base = p0; base < p1; base += 64) {
    const int nbatch = min(64, p1 - base);
    __syncthreads();
    if (lane < nbatch) {
      const int64_t i = base + lane;
      if (wv < 2) {
        T r[16];
        const int l = weights16<W, T>(g, i, wv, wv == 0 ? ox : oy, r);
        T* row = (wv == 0 ? sx : sy) + lane * 16;
        const int sw = stage_swz<T>(lane);
#pragma unroll
        for (int s = 0; s < 16; s++) row[s ^ sw] = r[s];
        if (wv == 0) {
          const int ly = rel_cell2d<W, T>(g, i, 1, oy);
          srun[lane] = (l / BS) + (g.b[0] / BS) * (ly / BS);
          sorg[lane] = (ly & ~(BS - 1)) * TP + (l & ~(BS - 1));
          sperm[lane] = (int)point_perm(g.pts, g.pts_code, i);
        }
      } else if (wv == 2) {
        sc[lane] = c[point_perm(g.pts, g.pts_code, i)];
      }
    }
    __syncthreads();
    const bool starts = lane < nbatch && (lane == 0 || srun[lane] != srun[lane - 1]);
    const uint64_t runs0 = __ballot(starts);
    for (int tr = 0; tr < ntr; tr++) {
      if (tr > 0) {
        __syncthreads();
        if (tid < nbatch) sc[tid] = c[(int64_t)tr * g.cstride + sperm[tid]];
        __syncthreads();
      }
      T* tl = mine + (size_t)2 * tr * plane;
      uint64_t runs = runs0;
      while (runs) {
        const int q0 = __ffsll((unsigned long long)runs) - 1;
        runs &= runs - 1;
        const int q1 = runs ? __ffsll((unsigned long long)runs) - 1 : nbatch;
        // steps q0 + 4 half, q0 + 4 half + 8, ..., alternately into two
        // accumulators so that consecutive matrix products do not wait
        v4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
        for (int q = q0 + 4 * half; q < q1; q += 16) {
          {
            const int p = q + kq;               // this lane's point (< kStage2d: q <= 63)
            const int o = p * 16 + (r16 ^ stage_swz<T>(p));
            const cplx_t<T> cv = sc[min(p, 63)];
            acc0 = M::mma(sx[o], p < q1 ? sy[o] * (part ? cv.y : cv.x) : (T)0, acc0);
          }
          if (q + 8 < q1) {
            const int p = q + 8 + kq;
            const int o = p * 16 + (r16 ^ stage_swz<T>(p));
            const cplx_t<T> cv = sc[min(p, 63)];
            acc1 = M::mma(sx[o], p < q1 ? sy[o] * (part ? cv.y : cv.x) : (T)0, acc1);
          }
        }
        acc0 += acc1;
        // add the block's 16 x 16 result into the plane: column r16 is y slot
        const int org = __builtin_amdgcn_readfirstlane(sorg[q0]);
        add_block(tl + org + r16 * TP, kq, acc0);
      }
    }
  }
  __syncthreads();

  // add the tiles (both step halves) to the periodic fine grid (touched cells only)
  const int gx0 = ox - H, gy0 = oy - H;
  for (int i = tid; i < TX * TY; i += 256) {
    const int ix = i % TX, iy = i / TX;
    const int64_t gx = wrap_any(gx0 + ix, g.n[0]);
    const int64_t gy = wrap_any(gy0 + iy, g.n[1]);
    const int64_t gi = gx + g.n[0] * gy;
    const int li = iy * TP + ix;
    for (int tr = 0; tr < ntr; tr++) {
      const T* t0 = tile + (size_t)2 * tr * plane + li;
      const T* t1 = t0 + (size_t)2 * ntr * plane;
      const T vx = t0[0] + t1[0], vy = t0[plane] + t1[plane];
      if (vx != (T)0 || vy != (T)0) {
        T* d = grid + 2 * ((int64_t)tr * g.gstride + gi);
        atomicAdd(d, vx);
        atomicAdd(d + 1, vy);
      }
    }
  }
}

// Four waves per subproblem share the grid tiles and the staged weights.
// Wave v takes the real (v even) or imaginary (v odd) part and the even
// (v < 2) or odd 16-point groups of every run.  Per batch wave 0 stages the x
// weights and the run data, wave 1 the y weights.
template <int W, typename T>
__global__ void __launch_bounds__(256)
interp2d_mfma_kernel(const GeomArgs g, const cplx_t<T>* __restrict__ grid,
                     cplx_t<T>* __restrict__ c) {
  using M = Mfma16<T>;
  using v4 = typename M::v4;
  constexpr int H = W / 2;
  constexpr int BS = block2d(W);
  constexpr int PX = kPitchX2d, PY = pitch_y2d<T>();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int TX = tile2d_dim(g.b[0], BS), TY = tile2d_dim(g.b[1], BS);
  const int TP = tile2d_pitch(TX);
  const int plane = TP * TY;
  const int ntr = g.ntr;
  T* tile = reinterpret_cast<T*>(smem_raw);                             // [ntr][2][TY][TP]
  T* sx = tile + (size_t)2 * plane * ntr;                               // [16][PX]
  T* sy = sx + 16 * PX;                                                 // [16][PY]
  cplx_t<T>* sout = reinterpret_cast<cplx_t<T>*>(sy + 16 * PY);         // [64]
  int* srun = reinterpret_cast<int*>(sout + 64);
  int* sorg = srun + 64;
  int* sperm = sorg + 64;

  const int sidx = blockIdx.x;
  const int bin = g.sub_bin[sidx];
  const int p0 = g.sub_start[sidx];
  const int p1 = p0 + g.sub_len[sidx];
  int ox, oy;
  bin_origin2d(g, bin, &ox, &oy);
  const int tid = threadIdx.x;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int part = wv & 1, half = wv >> 1;
  for (int i = tid; i < 16 * (PX + PY); i += 256) sx[i] = (T)0;
  {
    // the bin's tiles from the periodic fine grid
    const int gx0 = ox - H, gy0 = oy - H;
    for (int i = tid; i < TX * TY; i += 256) {
      const int ix = i % TX, iy = i / TX;
      const int64_t gi = wrap_any(gx0 + ix, g.n[0]) + g.n[0] * wrap_any(gy0 + iy, g.n[1]);
      const int li = iy * TP + ix;
      for (int tr = 0; tr < ntr; tr++) {
        const cplx_t<T> v = grid[(int64_t)tr * g.gstride + gi];
        tile[(size_t)2 * tr * plane + li] = v.x;
        tile[(size_t)(2 * tr + 1) * plane + li] = v.y;
      }
    }
  }
  const int r16 = lane & 15;   // A row (y slot) / B column (point) / D column
  const int kq = lane >> 4;    // k group (x slot within a 4-slot step) / D row group
  T* sout_part = reinterpret_cast<T*>(sout) + part;

  for (int base = p0; base < p1; base += 64) {
    const int nbatch = min(64, p1 - base);
    __syncthreads();
    if (lane < nbatch && wv < 2) {
      const int64_t i = base + lane;
      T r[16];
      const int l = weights16<W, T>(g, i, wv, wv == 0 ? ox : oy, r);
      T* col = (wv == 0 ? sx : sy) + lane;
      const int pitch = wv == 0 ? PX : PY;
#pragma unroll
      for (int s = 0; s < 16; s++) col[s * pitch] = r[s];
      if (wv == 0) {
        const int ly = rel_cell2d<W, T>(g, i, 1, oy);
        srun[lane] = (l / BS) + (g.b[0] / BS) * (ly / BS);
        sorg[lane] = (ly & ~(BS - 1)) * TP + (l & ~(BS - 1));
        sperm[lane] = (int)point_perm(g.pts, g.pts_code, i);
      }
    }
    __syncthreads();
    const bool starts = lane < nbatch && (lane == 0 || srun[lane] != srun[lane - 1]);
    const uint64_t runs0 = __ballot(starts);
    for (int tr = 0; tr < ntr; tr++) {
      const T* tl = tile + (size_t)(2 * tr + part) * plane;
      uint64_t runs = runs0;
      while (runs) {
        const int q0 = __ffsll((unsigned long long)runs) - 1;
        runs &= runs - 1;
        const int q1 = runs ? __ffsll((unsigned long long)runs) - 1 : nbatch;
        if (q0 + 16 * half >= q1) continue;
        const int org = __builtin_amdgcn_readfirstlane(sorg[q0]);
        // grid operand of the block: A[y][x] = G[x, y], x slot 4 s + kq, y slot r16
        T gp[4];
#pragma unroll
        for (int s = 0; s < 4; s++) gp[s] = tl[org + r16 * TP + 4 * s + kq];
        for (int q = q0 + 16 * half; q < q1; q += 32) {
          const int p = q + r16;                // this lane's point (< kStage2d)
          v4 u = {0, 0, 0, 0};
#pragma unroll
          for (int s = 0; s < 4; s++) u = M::mma(gp[s], sx[(4 * s + kq) * PX + p], u);
          // c_p = sum_y ky_p(y) U[y, p]: this lane's four y slots, then the
          // four lane groups
          T v = (T)0;
#pragma unroll
          for (int j = 0; j < 4; j++) v += sy[M::row(kq, j) * PY + p] * u[j];
          v += __shfl_xor(v, 16);
          v += __shfl_xor(v, 32);
          if (kq == 0 && p < q1) sout_part[2 * p] = v;
        }
      }
      __syncthreads();
      if (tid < nbatch) c[(int64_t)tr * g.cstride + sperm[tid]] = sout[tid];
      __syncthreads();
    }
  }
}

template <int W, typename T>
static hipError_t spread2d_w(const GeomArgs& g, int nsub, const void* c, void* grid,
                             hipStream_t s) {
  if (nsub <= 0) return hipSuccess;
  const int prec = sizeof(T) == 8 ? ESN_DOUBLE : ESN_SINGLE;
  hipLaunchKernelGGL((spread2d_mfma_kernel<W, T>), dim3(nsub), dim3(256),
                     mfma2d_lds_bytes(prec, W, g.b, g.ntr, true), s, g,
                     static_cast<const cplx_t<T>*>(c), static_cast<T*>(grid));
  return hipGetLastError();
}

template <int W, typename T>
static hipError_t interp2d_w(const GeomArgs& g, int nsub, const void* grid, void* c,
                             hipStream_t s) {
  if (nsub <= 0) return hipSuccess;
  const int prec = sizeof(T) == 8 ? ESN_DOUBLE : ESN_SINGLE;
  hipLaunchKernelGGL((interp2d_mfma_kernel<W, T>), dim3(nsub), dim3(256),
                     mfma2d_lds_bytes(prec, W, g.b, g.ntr, false), s, g,
                     static_cast<const cplx_t<T>*>(grid), static_cast<cplx_t<T>*>(c));
  return hipGetLastError();
}

template <typename T>
static hipError_t spread2d_t(int w, const GeomArgs& g, int nsub, const void* c, void* grid,
                             hipStream_t s) {
  switch (w) {
    case 2: return spread2d_w<2, T>(g, nsub, c, grid, s);
    case 3: return spread2d_w<3, T>(g, nsub, c, grid, s);
    case 4: return spread2d_w<4, T>(g, nsub, c, grid, s);
    case 5: return spread2d_w<5, T>(g, nsub, c, grid, s);
    case 6: return spread2d_w<6, T>(g, nsub, c, grid, s);
    case 7: return spread2d_w<7, T>(g, nsub, c, grid, s);
    case 8: return spread2d_w<8, T>(g, nsub, c, grid, s);
    case 9: return spread2d_w<9, T>(g, nsub, c, grid, s);
    case 10: return spread2d_w<10, T>(g, nsub, c, grid, s);
    case 11: return spread2d_w<11, T>(g, nsub, c, grid, s);
    case 12: return spread2d_w<12, T>(g, nsub, c, grid, s);
    case 13: return spread2d_w<13, T>(g, nsub, c, grid, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
static hipError_t interp2d_t(int w, const GeomArgs& g, int nsub, const void* grid, void* c,
                             hipStream_t s) {
  switch (w) {
    case 2: return interp2d_w<2, T>(g, nsub, grid, c, s);
    case 3: return interp2d_w<3, T>(g, nsub, grid, c, s);
    case 4: return interp2d_w<4, T>(g, nsub, grid, c, s);
    case 5: return interp2d_w<5, T>(g, nsub, grid, c, s);
    case 6: return interp2d_w<6, T>(g, nsub, grid, c, s);
    case 7: return interp2d_w<7, T>(g, nsub, grid, c, s);
    case 8: return interp2d_w<8, T>(g, nsub, grid, c, s);
    case 9: return interp2d_w<9, T>(g, nsub, grid, c, s);
    case 10: return interp2d_w<10, T>(g, nsub, grid, c, s);
    case 11: return interp2d_w<11, T>(g, nsub, grid, c, s);
    case 12: return interp2d_w<12, T>(g, nsub, grid, c, s);
    case 13: return interp2d_w<13, T>(g, nsub, grid, c, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_spread_mfma2d(int prec, int w, const GeomArgs& g, int nsub, const void* c,
                                void* grid, hipStream_t s) {
  return prec == ESN_DOUBLE ? spread2d_t<double>(w, g, nsub, c, grid, s)
                            : spread2d_t<float>(w, g, nsub, c, grid, s);
}

hipError_t launch_interp_mfma2d(int prec, int w, const GeomArgs& g, int nsub, const void* grid,
                                void* c, hipStream_t s) {
  return prec == ESN_DOUBLE ? interp2d_t<double>(w, g, nsub, grid, c, s)
                            : interp2d_t<float>(w, g, nsub, grid, c, s);
}

}  // namespace esn
