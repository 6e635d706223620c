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

// Staged points per batch in spreading: 64, then one row that staging never
// writes (zero), which masked lanes read.
constexpr int kStage2d = 65;

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
//    pitch of 4 (single) or 2 (double precision) mod 32 elements, so the
//    16 x 4 lanes of a matrix operand or result (column r16 one row apart,
//    k group kq one or four elements apart) fall on distinct banks;
//  * spreading stages the weights point-major (16 slots per point) with the
//    slot index XORed by bits of the point index (p / 2 mod 8 single, p / 2
//    mod 16 double precision: 64-bit writes go 32 lanes at a time), so that
//    staging (one point per lane, same slot) and the operand reads (16 slots
//    of 4 points) are both spread over all banks;
//  * interpolation stages them slot-major with pitches of 16 mod 32 (x) and
//    16 or 4 mod 32 (y, single precision: four consecutive slots per k group).
__host__ __device__ inline int tile2d_pitch(int tx, int prec) {
  return tx + (((prec == ESN_DOUBLE ? 2 : 4) - tx) & 31);
}
template <typename T>
__device__ __forceinline__ int stage_swz(int p) { return sizeof(T) == 4 ? (p >> 1) & 7 : (p >> 1) & 15; }
// Offset of slot r16 of staged point p (the swizzle repeats every 32 points).
template <typename T>
__device__ __forceinline__ int stage_off(int p, int r16) { return p * 16 + (r16 ^ stage_swz<T>(p)); }
constexpr int kPitchX2d = 80;
template <typename T> __host__ __device__ constexpr int pitch_y2d() { return sizeof(T) == 4 ? 84 : 80; }

size_t mfma2d_lds_bytes(int prec, int w, const int* b, int ntr, bool spread) {
  const size_t cs = prec == ESN_DOUBLE ? 16 : 8, rs = prec == ESN_DOUBLE ? 8 : 4;
  const int bs = block2d(w);
  const size_t plane = (size_t)tile2d_pitch(tile2d_dim(b[0], bs), prec) * tile2d_dim(b[1], bs);
  // real and imaginary planes per transform; spreading keeps two copies
  const size_t tile = (spread ? 2 : 1) * 2 * plane * rs * ntr;
  // spreading: x weights and the y weights times the strength's real and
  // imaginary parts [kStage2d][16] each (with several transforms also the
  // plain y weights), run keys and footprint offsets [64];
  // interpolation: x and y weights slot-major, results [64], run keys,
  // footprint offsets and original indices [64]
  if (spread)
    return tile + (ntr > 1 ? 4 : 3) * kStage2d * 16 * rs + 2 * 64 * sizeof(int) + 16;
  return tile + 16 * (kPitchX2d + (prec == ESN_DOUBLE ? 80 : 84)) * rs + 64 * cs +
         3 * 64 * sizeof(int) + 16;
}

// A sorted point's record (coordinates and original index), loaded ahead of
// its batch: fixed point a = (x, y, z, index); FP64 a = (x, y), b = (z, index).
typedef uint32_t u32x4_2d __attribute__((ext_vector_type(4)));
struct Rec2d {
  u32x4_2d a, b;
};
__device__ __forceinline__ Rec2d load_rec2d(const GeomArgs& g, int64_t i) {
  Rec2d r;
  if (g.pts_code == kPtsFixed32) {
    r.a = *reinterpret_cast<const u32x4_2d*>(g.pts + i * 16);
    r.b = r.a;
  } else {
    r.a = *reinterpret_cast<const u32x4_2d*>(g.pts + i * 32);
    r.b = *reinterpret_cast<const u32x4_2d*>(g.pts + i * 32 + 16);
  }
  return r;
}
template <int W, typename T>
__device__ __forceinline__ Coord<T> rec_coord(const GeomArgs& g, const Rec2d& r, int m, int* sh) {
  if (g.pts_code == kPtsFixed32) return decode_fixed<T>(r.a[m], g.fbits[m], sh, W);
  const uint64_t bits = ((uint64_t)r.a[2 * m + 1] << 32) | r.a[2 * m];
  return decode_f64<T>(__longlong_as_double((long long)bits), sh, W);
}
__device__ __forceinline__ int64_t rec_perm(const GeomArgs& g, const Rec2d& r) {
  return g.pts_code == kPtsFixed32 ? (int32_t)r.a[3] : (int32_t)r.b[2];
}

// Window cell of record r along dimension m relative to the bin origin o.
template <int W, typename T>
__device__ __forceinline__ int rec_cell2d(const GeomArgs& g, const Rec2d& r, int m, int o) {
  int sh;
  const Coord<T> cd = rec_coord<W, T>(g, r, m, &sh);
  return window_cell(cd.cell, sh, g.n[m]) - o;
}

// The 16 staged weights of a point along dimension m: w kernel values from
// the window cell's offset in its block, zeros elsewhere.  Returns the window
// cell relative to the bin origin o.
template <int W, typename T>
__device__ __forceinline__ int weights16(const GeomArgs& g, const Rec2d& rec, int m, int o,
                                         T (&r)[16]) {
  constexpr int BS = block2d(W);
  int sh;
  const Coord<T> cd = rec_coord<W, T>(g, rec, m, &sh);
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

// Periodic wrap of a tile index v in [-w/2, n + bin + 16): one correction
// each way in 32-bit arithmetic, the general remainder only on grids smaller
// than a tile.
__device__ __forceinline__ int wrap_tile(int v, int n) {
  v = v < 0 ? v + n : v;
  v = v >= n ? v - n : v;
  if (v < 0 || v >= n) v = (int)wrap_any(v, n);
  return v;
}

// Bin of subproblem sidx and its origin (window cells).
__device__ __forceinline__ void bin_origin2d(const GeomArgs& g, int bin, int* o0, int* o1) {
  const int bi0 = bin % g.nb[0], bi1 = bin / g.nb[0];
  *o0 = bi0 * g.b[0];
  *o1 = bi1 * g.b[1];
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

// Sum of v over the four 16-lane rows of the wave (lanes l, l ^ 16, l ^ 32,
// l ^ 48), in every lane: the row swaps of the lane-permute unit, no LDS.
__device__ __forceinline__ float rows_sum(float v) {
  const auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false,
                                                  false);
  v = __uint_as_float(a[0]) + __uint_as_float(a[1]);
  const auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false,
                                                  false);
  return __uint_as_float(b[0]) + __uint_as_float(b[1]);
}
__device__ __forceinline__ double rows_sum(double v) {
  // the same permutation on both halves of each value
  uint32_t lo = (uint32_t)__double_as_longlong(v), hi = (uint32_t)(__double_as_longlong(v) >> 32);
  const auto l1 = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto h1 = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  v = __longlong_as_double(((int64_t)h1[0] << 32) | l1[0]) +
      __longlong_as_double(((int64_t)h1[1] << 32) | l1[1]);
  lo = (uint32_t)__double_as_longlong(v);
  hi = (uint32_t)(__double_as_longlong(v) >> 32);
  const auto l2 = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto h2 = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return __longlong_as_double(((int64_t)h2[0] << 32) | l2[0]) +
         __longlong_as_double(((int64_t)h2[1] << 32) | l2[1]);
}

// Four waves per subproblem share the staged weights.  Wave v takes the real
// (v even) or imaginary (v odd) part and the even (v < 2) or odd steps of
// every run; the two step halves add into two copies of the tile, so no two
// waves write the same LDS value (LDS atomics measured far slower).  Per batch of 64 points wave 0 stages the x weights, wave 1 the y
// weights times the strength (real and imaginary part rows), wave 2 the run
// data; each loads the next batch's point records while the batch is
// contracted, wave 1 also the next strengths.  Transforms 0 .. g.ntr - 1
// share the x weights and the runs, wave 1 restaging the y rows with each
// transform's strengths from a staged copy of the plain y weights; each
// transform has its own tiles.
template <int W, typename T>
__global__ void __launch_bounds__(256)
spread2d_mfma_kernel(const GeomArgs g, const cplx_t<T>* __restrict__ c, T* __restrict__ grid) {
  using M = Mfma16<T>;
  using v4 = typename M::v4;
  constexpr int H = W / 2;
  constexpr int BS = block2d(W);
  constexpr int RS = kStage2d * 16;   // one staged array
  constexpr int kZero = 64 * 16;      // offset of the zero row
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int TX = tile2d_dim(g.b[0], BS), TY = tile2d_dim(g.b[1], BS);
  const int TP = tile2d_pitch(TX, sizeof(T) == 8 ? ESN_DOUBLE : ESN_SINGLE);
  const int plane = TP * TY;
  const int ntr = g.ntr;
  T* tile = reinterpret_cast<T*>(smem_raw);                             // [2][ntr][2][TY][TP]
  T* sx = tile + (size_t)4 * plane * ntr;                               // [kStage2d][16]
  T* syc = sx + RS;                                                     // [2][kStage2d][16]
  T* sky = syc + 2 * RS;                                                // [kStage2d][16] if ntr > 1
  int* srun = reinterpret_cast<int*>(sky + (ntr > 1 ? RS : 0));         // [64] block id
  int* sorg = srun + 64;                                                // [64] footprint offset

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
  for (int i = tid; i < 3 * RS; i += 256) sx[i] = (T)0;
  const int r16 = lane & 15;   // A row / B column / D column
  const int kq = lane >> 4;    // k group (the step's point) / D row group
  const T* syp = syc + part * RS;
  Rec2d cur;                   // waves 0 - 2: this batch's record of this lane
  Rec2d nxt;                   // and the next batch's
  cplx_t<T> cnext;             // wave 1: the next batch's strength
  if (wv < 3 && lane < min(64, p1 - p0)) {
    nxt = load_rec2d(g, p0 + lane);
    if (wv == 1) cnext = c[rec_perm(g, nxt)];
  }

  for (int base = p0; base < p1; base += 64) {
    const int nbatch = min(64, p1 - base);
    const int nnext = min(64, p1 - base - 64);
    __syncthreads();
    if (wv < 3 && lane < nbatch) {
      cur = nxt;
      const int sw = stage_swz<T>(lane);
      if (wv == 0) {
        T r[16];
        weights16<W, T>(g, cur, 0, ox, r);
        T* row = sx + lane * 16;
#pragma unroll
        for (int s = 0; s < 16; s++) row[s ^ sw] = r[s];
      } else if (wv == 1) {
        T ry[16];
        weights16<W, T>(g, cur, 1, oy, ry);
        T* row = syc + lane * 16;
#pragma unroll
        for (int s = 0; s < 16; s++) {
          row[s ^ sw] = ry[s] * cnext.x;
          row[RS + (s ^ sw)] = ry[s] * cnext.y;
        }
        if (ntr > 1) {
#pragma unroll
          for (int s = 0; s < 16; s++) row[2 * RS + (s ^ sw)] = ry[s];
        }
      } else {
        const int lx = rec_cell2d<W, T>(g, cur, 0, ox);
        const int ly = rec_cell2d<W, T>(g, cur, 1, oy);
        srun[lane] = (lx / BS) + (g.b[0] / BS) * (ly / BS);
        sorg[lane] = (ly & ~(BS - 1)) * TP + (lx & ~(BS - 1));
      }
    }
    if (wv < 3 && lane < nnext) nxt = load_rec2d(g, base + 64 + lane);
    __syncthreads();
    const bool starts = lane < nbatch && (lane == 0 || srun[lane] != srun[lane - 1]);
    const uint64_t runs0 = __ballot(starts);
    for (int tr = 0; tr < ntr; tr++) {
      if (tr > 0) {
        __syncthreads();
        if (wv == 1 && lane < nbatch) {
          const cplx_t<T> cv = c[(int64_t)tr * g.cstride + rec_perm(g, cur)];
          T* row = syc + lane * 16;
#pragma unroll
          for (int s = 0; s < 16; s++) {
            const T ky = row[2 * RS + s];
            row[s] = ky * cv.x;
            row[RS + s] = ky * cv.y;
          }
        }
        __syncthreads();
      }
      // this wave's plane: copy `half`, transform tr, part `part`
      T* tl = tile + (size_t)((half * ntr + tr) * 2 + part) * plane;
      uint64_t runs = runs0;
      while (runs) {
        const int q0 = __ffsll((unsigned long long)runs) - 1;
        runs &= runs - 1;
        const int q1 = runs ? __ffsll((unsigned long long)runs) - 1 : nbatch;
        // this wave's steps q0 + 4 half + 8 k, k even into acc0 and odd into
        // acc1; a step's lane reads slot r16 of point q + kq, at offsets o[k mod
        // 4] that grow by 512 every fourth step (the swizzle repeats every 32
        // points).  Points past the run read the zero row instead (a select of
        // the offset, no branch).  The first two steps run unconditionally, so
        // both accumulators start from a matrix product.
        int q = q0 + 4 * half;
        const int pk = q + kq;
        int o0 = stage_off<T>(pk, r16), o1 = stage_off<T>(pk + 8, r16);
        int o2 = stage_off<T>(pk + 16, r16), o3 = stage_off<T>(pk + 24, r16);
        const v4 zero = {0, 0, 0, 0};
        int xa = q + kq < q1 ? o0 : kZero, xb = q + 8 + kq < q1 ? o1 : kZero;
        v4 acc0 = M::mma(sx[xa], syp[xa], zero);
        v4 acc1 = M::mma(sx[xb], syp[xb], zero);
        for (q += 16; q < q1; q += 16) {
          xa = q + kq < q1 ? o2 : kZero;
          xb = q + 8 + kq < q1 ? o3 : kZero;
          acc0 = M::mma(sx[xa], syp[xa], acc0);
          acc1 = M::mma(sx[xb], syp[xb], acc1);
          o0 += 512;
          o1 += 512;
          q += 16;
          if (q >= q1) break;
          xa = q + kq < q1 ? o0 : kZero;
          xb = q + 8 + kq < q1 ? o1 : kZero;
          acc0 = M::mma(sx[xa], syp[xa], acc0);
          acc1 = M::mma(sx[xb], syp[xb], acc1);
          o2 += 512;
          o3 += 512;
        }
        // add the block's 16 x 16 result into the plane: column r16 is y slot
        const int org = __builtin_amdgcn_readfirstlane(sorg[q0]);
        add_block(tl + org + r16 * TP, kq, acc0 + acc1);
      }
    }
    // the next batch's strengths (its records were loaded before the barrier)
    if (wv == 1 && lane < nnext) cnext = c[rec_perm(g, nxt)];
  }
  __syncthreads();

  // add the tiles (both step halves) to the periodic fine grid (touched cells only)
  const int gx0 = ox - H, gy0 = oy - H;
  for (int i = tid; i < TX * TY; i += 256) {
    const int ix = i % TX, iy = i / TX;
    const int nx = (int)g.n[0], ny = (int)g.n[1];
    const int64_t gi = wrap_tile(gx0 + ix, nx) + (int64_t)nx * wrap_tile(gy0 + iy, ny);
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
// (v < 2) or odd 16-point groups of every run, two groups at a time where the
// run has them.  Per batch wave 0 stages the x weights, wave 1 the y weights,
// wave 2 the run data; each loads the next batch's point records while the
// batch is contracted.
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
  const int TP = tile2d_pitch(TX, sizeof(T) == 8 ? ESN_DOUBLE : ESN_SINGLE);
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
  Rec2d nxt;                   // waves 0 - 2: the next batch's record of this lane
  if (wv < 3 && lane < min(64, p1 - p0)) nxt = load_rec2d(g, p0 + lane);
  for (int i = tid; i < 16 * (PX + PY); i += 256) sx[i] = (T)0;
  {
    // the bin's tiles from the periodic fine grid
    const int gx0 = ox - H, gy0 = oy - H;
    for (int i = tid; i < TX * TY; i += 256) {
      const int ix = i % TX, iy = i / TX;
      const int nx = (int)g.n[0], ny = (int)g.n[1];
      const int64_t gi = wrap_tile(gx0 + ix, nx) + (int64_t)nx * wrap_tile(gy0 + iy, ny);
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
    const int nnext = min(64, p1 - base - 64);
    __syncthreads();
    if (wv < 3 && lane < nbatch) {
      const Rec2d cur = nxt;
      if (wv < 2) {
        T r[16];
        weights16<W, T>(g, cur, wv, wv == 0 ? ox : oy, r);
        T* col = (wv == 0 ? sx : sy) + lane;
        const int pitch = wv == 0 ? PX : PY;
#pragma unroll
        for (int s = 0; s < 16; s++) col[s * pitch] = r[s];
      } else {
        const int lx = rec_cell2d<W, T>(g, cur, 0, ox);
        const int ly = rec_cell2d<W, T>(g, cur, 1, oy);
        srun[lane] = (lx / BS) + (g.b[0] / BS) * (ly / BS);
        sorg[lane] = (ly & ~(BS - 1)) * TP + (lx & ~(BS - 1));
        sperm[lane] = (int)rec_perm(g, cur);
      }
    }
    if (wv < 3 && lane < nnext) nxt = load_rec2d(g, base + 64 + lane);
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
        int q = q0 + 16 * half;
        // two groups (q and q + 32) at a time
        for (; q + 32 < q1; q += 64) {
          const int pa = q + r16, pb = pa + 32;   // < PX
          v4 ua = {0, 0, 0, 0}, ub = {0, 0, 0, 0};
#pragma unroll
          for (int s = 0; s < 4; s++) {
            ua = M::mma(gp[s], sx[(4 * s + kq) * PX + pa], ua);
            ub = M::mma(gp[s], sx[(4 * s + kq) * PX + pb], ub);
          }
          // c_p = sum_y ky_p(y) U[y, p]: this lane's four y slots, then the
          // four lane rows
          T va = (T)0, vb = (T)0;
#pragma unroll
          for (int j = 0; j < 4; j++) {
            va += sy[M::row(kq, j) * PY + pa] * ua[j];
            vb += sy[M::row(kq, j) * PY + pb] * ub[j];
          }
          va = rows_sum(va);
          vb = rows_sum(vb);
          if (kq == 0) {
            if (pa < q1) sout_part[2 * pa] = va;
            if (pb < q1) sout_part[2 * pb] = vb;
          }
        }
        if (q < q1) {
          const int pa = q + r16;
          v4 ua = {0, 0, 0, 0};
#pragma unroll
          for (int s = 0; s < 4; s++) ua = M::mma(gp[s], sx[(4 * s + kq) * PX + pa], ua);
          T va = (T)0;
#pragma unroll
          for (int j = 0; j < 4; j++) va += sy[M::row(kq, j) * PY + pa] * ua[j];
          va = rows_sum(va);
          if (kq == 0 && pa < q1) sout_part[2 * pa] = va;
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
