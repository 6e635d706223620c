// Spreading and interpolation on the matrix cores (3D, single precision,
// w <= 7), one wave per subproblem (a run of at most maxsub bin-sorted points
// of one bin, Sec. 5.2).
//
// Points are binned by window cell (the cell floor(w/2) after the first cell
// of the point's window), so a point in window cell l has its w window cells
// at l - floor(w/2) .. l - floor(w/2) + w - 1.  Two neighbouring window cells
// 2j, 2j + 1 then have all their windows inside the 8 cells from
// 2j - floor(w/2): a point of cell 2j + (l & 1) puts its weights at slots
// (l & 1) .. (l & 1) + w - 1 of that 8-wide footprint.  Within a bin the
// points are sorted by 2 x 2 block of (x, y) columns and then by z cell, so
// every such block is a run of sorted points sharing one 8 x 8 footprint.
// Spreading the points of a column block, eq. (bl), is then a dense
// contraction over the points,
//
//     B[(z, x), (y, re/im)] = sum_p  kz_p(z) kx_p(x)  *  ky_p(y) c_p,
//
// of a 64 x P matrix of z-x weights with a P x 16 matrix of y weight times
// strength.  The wave runs it with v_mfma_f32_16x16x4_f32: the 64 rows are
// four 16-row tiles (two z planes x 8 x cells each), each instruction takes 4
// points.  The 8 planes form a ring (tile-relative plane r -> slot r mod 8):
// once the wave moves on to a later pair of z cells of the block, the planes
// below it receive nothing more, so they are added into the wave's LDS tile
// of the bin (bin + 6 cells per dim) and their slots reused; a plane lives in
// half the lanes of one row tile, so this costs 4 read-modify-writes on those
// lanes.  The wave owns the tile, so these adds are plain read-modify-writes;
// the tile goes to the fine grid once at the end (global atomics on the
// touched cells only).
//
// Interpolation, eq. (interp), runs the same contraction the other way: for
// the points of one 2 x 2 x 2 block of window cells, T[z, p] = sum_(x,y)
// B[z, (x, y)] kx_p(x) ky_p(y) on the matrix cores (8 planes (re, im) x 64
// footprint cells x 16 points), then c_p = sum_z kz_p(z) T[z, p] in registers
// and across the four lane groups that hold a point's planes, with the bin's
// grid tile (bin + 6 cells per dim) copied into LDS first.
#include "device_common.hpp"

namespace esn {

typedef float v4f __attribute__((ext_vector_type(4)));

// ES kernel values of one point at its w window cells (as es_weights_f32),
// using the hardware square root and base-2 exponential: bl = beta log2(e),
// ker[k] = 2^(bl (sqrt(1 - z^2) - 1)).  Only the two edge cells need the
// clamp of 1 - z^2 at zero: with the offset off = sh - floor(w/2) - f in
// (sh - floor(w/2) - 1, sh - floor(w/2)], sh in {0, 1}, the cells k = 1 ..
// w - 2 have |off + k| <= floor((w - 1) / 2) < w / 2, so |z| <= 1 - 1/w.
template <int W>
__device__ __forceinline__ void es_weights_hw(int sh, float f, float bl, float* ker) {
  const float off = (float)(sh - W / 2) - f;
  const float s = 2.0f / (float)W;
#pragma unroll
  for (int k = 0; k < W; k++) {
    const float z = (off + (float)k) * s;
    float a = fmaf(-z, z, 1.0f);
    if (k == 0 || k == W - 1) a = fmaxf(a, 0.0f);
    ker[k] = __builtin_amdgcn_exp2f(fmaf(bl, __builtin_amdgcn_sqrtf(a), -bl));
  }
}

// The w kernel values placed at slots sh .. sh + w - 1 of an 8-slot vector
// (sh in {0, 1}), zeros elsewhere; built with selects so it stays in registers.
template <int W>
__device__ __forceinline__ void slots8(const float* k, int sh, float* v) {
#pragma unroll
  for (int s = 0; s < 8; s++) {
    const float a = s < W ? k[s] : 0.f;          // sh = 0
    const float b = (s >= 1 && s - 1 < W) ? k[s - 1] : 0.f;   // sh = 1
    v[s] = sh ? b : a;
  }
}

// Rotate an 8-vector left by r (0..7): out[(s + r) & 7] = in[s], in three
// conditional stages so it stays in registers.
__device__ __forceinline__ void rotate8(float* v, int r) {
  float t[8];
  if (r & 1) {
#pragma unroll
    for (int s = 0; s < 8; s++) t[(s + 1) & 7] = v[s];
#pragma unroll
    for (int s = 0; s < 8; s++) v[s] = t[s];
  }
  if (r & 2) {
#pragma unroll
    for (int s = 0; s < 8; s++) t[(s + 2) & 7] = v[s];
#pragma unroll
    for (int s = 0; s < 8; s++) v[s] = t[s];
  }
  if (r & 4) {
#pragma unroll
    for (int s = 0; s < 8; s++) t[(s + 4) & 7] = v[s];
#pragma unroll
    for (int s = 0; s < 8; s++) v[s] = t[s];
  }
}

__device__ __forceinline__ void store8(float* dst, const float* v) {
  reinterpret_cast<float4*>(dst)[0] = make_float4(v[0], v[1], v[2], v[3]);
  reinterpret_cast<float4*>(dst)[1] = make_float4(v[4], v[5], v[6], v[7]);
}

// Periodic wrap of an index that lies within a few periods of [0, n).
__device__ __forceinline__ int wrap2(int g, int n) {
  while (g < 0) g += n;
  while (g >= n) g -= n;
  return g;
}

// Hides a register value from the optimizer (no instruction is emitted), so
// that loads indexed by it, issued a loop step ahead, are not merged back into
// the next step.
__device__ __forceinline__ void opaque(int& v) { asm volatile("" : "+v"(v)); }

// Keeps the memory accesses before it ahead of the code after it (a compiler
// barrier only: no instruction, no wait).
__device__ __forceinline__ void keep_order() { asm volatile("" ::: "memory"); }

// Wait states before a VALU instruction may read the result of a matrix
// instruction.  The MAI dependency rules of the CDNA3 / CDNA4 instruction set
// require, between an XDL instruction writing VGPRs and a VALU read or write
// of those VGPRs, as many independent instructions or wait states as the XDL
// instruction's passes plus 3.  v_mfma_f32_16x16x4_f32 takes 8 passes (32
// cycles: SQ_VALU_MFMA_BUSY_CYCLES counts 32 per instruction on gfx950), so
// 11.  The waits are issued explicitly, tied to the accumulators: after the
// asm statement below the compiler sees the registers as written by it, not
// by the matrix instruction, and adds no waits of its own, so the statement
// itself must cover the whole requirement.  (Without explicit waits a stress
// run found rare results read before the products had landed.)
constexpr int kMfma16x16x4f32Passes = 8;
constexpr int kXdlToValuWaits = kMfma16x16x4f32Passes + 3;
// s_nop n waits n + 1 states, n <= 15
template <int N>
__device__ __forceinline__ void xdl_waits(v4f& a) {
  static_assert(N >= 1 && N <= 16, "one s_nop covers 1 .. 16 wait states");
  asm volatile("s_nop %1" : "+a"(a) : "i"(N - 1));
}
template <int N>
__device__ __forceinline__ void xdl_waits(v4f& a, v4f& b) {
  static_assert(N >= 1 && N <= 16, "one s_nop covers 1 .. 16 wait states");
  asm volatile("s_nop %2" : "+a"(a), "+a"(b) : "i"(N - 1));
}

// Floats per z plane of a bin tile of T0 x T1 complex cells: 2 T0 T1 padded
// to 8 mod 32, so that the 8 planes a wave touches at once start in distinct
// LDS banks.
__host__ __device__ inline int plane_floats(int T0, int T1) {
  return ((2 * T0 * T1 + 23) / 32) * 32 + 8;
}

// Rows of staged points in the spreading kernel: 64 per batch, then zero rows
// so that the steps, which read 16 points ahead, may reach row 64 + 15
// without a bound check.
constexpr int kSpreadStage = 80;

// Rows of staged z weights in the interpolation kernel: a step reads the
// weights of 16 points from a start of at most 64 (one batch), so reads reach
// row 79; rows past the batch only feed output columns that are not stored.
constexpr int kInterpRows = 80;

// Floats of the interpolation kernel's staging area: the staged weights, or,
// while the bin's grid tile is read, a table of two ints per tile row.
__host__ __device__ inline int interp_stage_floats(int T1, int T2) {
  const int w = (2 * 64 + kInterpRows) * 8;
  return 2 * T1 * T2 > w ? 2 * T1 * T2 : w;
}

// LDS layouts.  Both start with the bin tile (bin + 6 cells per dim, planes of
// plane_floats) and end with the wrapped grid offsets of the tile's z planes
// (int64), per-point ints and the offsets of the tile's x and y lines.
// Spreading stages [80][8] x and z weights and [80][16] B operands;
// interpolation [64][8] x and y weights and [80][8] z weights (an area that
// first holds the table of tile rows, sized for both) and a float2 result per
// point.
static inline size_t mfma_tail_bytes(const int* b, int nint) {
  const size_t T0 = b[0] + 6, T1 = b[1] + 6, T2 = b[2] + 6;
  return T2 * sizeof(int64_t) + (size_t)nint * 64 * sizeof(int) + (T0 + T1) * sizeof(int);
}

static inline size_t mfma_tile_bytes(const int* b) {
  const size_t T0 = b[0] + 6, T1 = b[1] + 6, T2 = b[2] + 6;
  return T2 * plane_floats((int)T0, (int)T1) * sizeof(float);
}

size_t mfma_spread_lds_bytes(int w, const int* b) {
  (void)w;   // 8-wide footprints for every w
  return mfma_tile_bytes(b) + (size_t)kSpreadStage * (8 + 8 + 16) * sizeof(float) +
         mfma_tail_bytes(b, 2);
}

size_t mfma_interp_lds_bytes(const int* b) {
  return mfma_tile_bytes(b) + (size_t)interp_stage_floats(b[1] + 6, b[2] + 6) * sizeof(float) +
         64 * sizeof(float2) + mfma_tail_bytes(b, 2);
}

// Fill the wrapped grid offsets of the tile lines whose origin is (ox, oy, oz):
// gx[i] = wrap(ox + i), gy[i] = n0 wrap(oy + i), gz[i] = n0 n1 wrap(oz + i).
__device__ __forceinline__ void tile_offsets(int tid, int nthr, int T0, int T1, int T2, int ox,
                                             int oy, int oz, int n0, int n1, int n2, int* gx,
                                             int* gy, int64_t* gz) {
  for (int i = tid; i < T0; i += nthr) gx[i] = wrap2(ox + i, n0);
  for (int i = tid; i < T1; i += nthr) gy[i] = n0 * wrap2(oy + i, n1);
  for (int i = tid; i < T2; i += nthr) gz[i] = (int64_t)n0 * n1 * wrap2(oz + i, n2);
}

// Walks the cells tid, tid + nthr, ... of a T0 x T1 x T2 tile (x fastest),
// keeping (ix, iy, iz) without divisions in the loop.
struct TileWalk {
  int ix, iy, iz, dx, dq, T0, T1;
  // float offset of the cell in a tile with planes of ps floats
  __device__ __forceinline__ int ofs(int ps) const { return iz * ps + 2 * (iy * T0 + ix); }
  __device__ __forceinline__ TileWalk(int tid, int nthr, int T0_, int T1_) : T0(T0_), T1(T1_) {
    ix = tid % T0;
    const int r = tid / T0;
    iy = r % T1;
    iz = r / T1;
    dx = nthr % T0;
    dq = nthr / T0;
  }
  __device__ __forceinline__ void next() {
    ix += dx;
    iy += dq;
    if (ix >= T0) {
      ix -= T0;
      iy++;
    }
    while (iy >= T1) {
      iy -= T1;
      iz++;
    }
  }
};

// Kernel values k[0 .. w-1] of one fixed-point coordinate q (fbits fraction
// bits) at its window cells, and its window cell relative to the bin origin o
// (in [0, b)); the window shift is decided on the exact fraction bits, as
// everywhere else.
template <int W>
__device__ __forceinline__ int window_weights(uint32_t q, int fbits, int n, int o, float bl,
                                              const float* ktab, float* k) {
  const uint32_t fr = q & ((1u << fbits) - 1u);
  const int sh = window_shift_fixed(fr, fbits, W);
  if (ktab) es_weights_poly<W, float>(sh, ldexpf((float)fr, -fbits), ktab, k);
  else es_weights_hw<W>(sh, ldexpf((float)fr, -fbits), bl, k);
  return window_cell((int)(q >> fbits), sh, n) - o;
}

// Window cell of a fixed-point coordinate relative to the bin origin o.
template <int W>
__device__ __forceinline__ int rel_window_cell(uint32_t q, int fbits, int n, int o) {
  return window_cell((int)(q >> fbits), window_shift_fixed(q & ((1u << fbits) - 1u), fbits, W),
                     n) - o;
}

// Two waves per subproblem share the bin tile and the staged weights.  Wave
// wv accumulates row tiles 2 wv and 2 wv + 1, i.e. ring slots 4 wv .. 4 wv + 3;
// a tile plane always lives in the same ring slot (plane r -> slot r mod 8),
// so the two waves never add into the same plane.  In each batch wave 0
// computes the x and y weights and wave 1 the z weights, strengths and cells.
template <int W>
__global__ void __launch_bounds__(128)
spread_mfma_kernel(const GeomArgs g, const float2* __restrict__ c, float* __restrict__ grid) {
  static_assert(W >= 2 && W <= 7, "matrix-core spreading needs w <= 7");
  constexpr int H = W / 2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int b0 = g.b[0], b1 = g.b[1], b2 = g.b[2];
  // 8-wide footprints from even window cells of the bin (even bin sizes)
  const int T0 = b0 + 6, T1 = b1 + 6, T2 = b2 + 6;
  const int tc = T0 * T1 * T2;
  const int ps = plane_floats(T0, T1);               // floats per tile plane
  constexpr int NS = kSpreadStage;
  float* otf = reinterpret_cast<float*>(smem_raw);               // [T2][ps]: [T1][T0][2]
  float* skx = otf + T2 * ps;                                     // [NS][8] x slots
  float* skz = skx + NS * 8;                                      // [NS][8] z ring, pairs split
  float* sb = skz + NS * 8;                                       // [NS][16] B operand
  int64_t* gz = reinterpret_cast<int64_t*>(sb + NS * 16);         // [T2]
  int* scol = reinterpret_cast<int*>(gz + T2);                    // [64] column in the bin
  int* szr = scol + 64;                                           // [64] z cell in the bin
  int* gx = szr + 64;                                             // [T0]
  int* gy = gx + T0;                                              // [T1]

  const int sidx = blockIdx.x;
  const int bin = g.sub_bin[sidx];
  const int p0 = g.sub_start[sidx];
  const int p1 = p0 + g.sub_len[sidx];
  const int bi0 = bin % g.nb[0], bi1 = (bin / g.nb[0]) % g.nb[1], bi2 = bin / (g.nb[0] * g.nb[1]);
  const int bx0 = bi0 * b0, by0 = bi1 * b1, bz0 = bi2 * b2;
  const int tid = threadIdx.x;
  // the wave index, known to the compiler as the same across the wave, so that
  // ballots and run bounds derived from it stay in scalar registers
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const float bl = (float)(g.beta * 1.4426950408889634);   // beta log2(e)
  const float* ktab = static_cast<const float*>(g.ktab);    // kernel table or null
  const int n0 = (int)g.n[0], n1 = (int)g.n[1], n2 = (int)g.n[2];

  {
    // the tile and the staging (whose padding points stay zero)
    float4* o4 = reinterpret_cast<float4*>(otf);
    const int n4 = (T2 * ps + NS * 32) / 4;
    for (int i = tid; i < n4; i += 128) o4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  tile_offsets(tid, 128, T0, T1, T2, bx0 - H, by0 - H, bz0 - H, n0, n1, n2, gx, gy, gz);

  // lane roles in the accumulators: row tile t holds ring slots 2t + hz, x
  // cells x0 .. x0 + 3 (one per accumulator element), y cell yl, re/im reim
  const int yl = (lane & 15) >> 1;
  const int reim = lane & 1;
  const int hz = lane >> 5;
  const int x0 = 4 * ((lane >> 4) & 1);
  // LDS float offsets of this lane's operands for point 0 of a step: x weight
  // (row l & 7), its 2 ring weights (rows of tiles 2 wv, 2 wv + 1), B column
  const int kg = lane >> 4;   // the step's point this lane feeds
  const int ox = kg * 8 + (lane & 7);
  const int oz = kg * 8 + 4 * ((lane >> 3) & 1) + 2 * wv;
  const int ob = kg * 16 + (lane & 15);
  v4f acc[2];
  acc[0] = acc[1] = v4f{0.f, 0.f, 0.f, 0.f};
  int cur = -1;        // current column (lx + b0 ly), -1: none
  int colbase = 0;     // this lane's float offset in a tile plane for the current column
  int pend = 0;        // the ring holds tile planes pend .. pend + 7

  // add this wave's ring slots in mask fm (block-uniform) into the bin tile and clear them
  auto flush = [&](unsigned fm) {
    // the wait states before the products are read (a flush is rare: the
    // largest single s_nop, 16 states, above the 11 required)
    static_assert(16 >= kXdlToValuWaits, "flush waits below the MAI rule");
    xdl_waits<16>(acc[0], acc[1]);
#pragma unroll
    for (int u = 0; u < 2; u++) {
      const int t = 2 * wv + u;
      if (fm & (3u << (2 * t))) {
        const int s = 2 * t + hz;
        if ((fm >> s) & 1u) {
          float* d = otf + (pend + ((s - pend) & 7)) * ps + colbase;
#pragma unroll
          for (int i = 0; i < 4; i++) d[2 * i] += acc[u][i];
          acc[u] = v4f{0.f, 0.f, 0.f, 0.f};
        }
      }
    }
  };

  // point records flow through registers one batch ahead of the matrix work
  // (both waves read them; the strengths, gathered one batch ahead, are used
  // by wave 1).  The loads are unconditional, at indices clamped into the
  // subproblem, so that the waits for them can be placed where the values are used.
  const uint4* rec = reinterpret_cast<const uint4*>(g.pts);
  const int plast = p1 - 1;
  uint4 r0 = rec[min(p0 + lane, plast)];
  uint4 r1 = rec[min(p0 + 64 + lane, plast)];
  float2 cc0 = c[(int)r0.w];
  for (int base = p0; base < p1; base += 64) {
    const int nbatch = min(64, p1 - base);
    const uint4 r2 = rec[min(base + 128 + lane, plast)];
    const float2 cc1 = c[(int)r1.w];
    __syncthreads();
    {
      float k[W], v[8];
      if (wv == 0) {
        // x weights by footprint slot, z weights by ring slot
        const int lx = window_weights<W>(r0.x, g.fbits[0], n0, bx0, bl, ktab, k);
        slots8<W>(k, lx & 1, v);
        store8(skx + lane * 8, v);
        const int zr = window_weights<W>(r0.z, g.fbits[2], n2, bz0, bl, ktab, k);
        slots8<W>(k, 0, v);    // planes zr .. zr + 7 of the tile
        rotate8(v, zr & 7);    // -> ring slots
        float vz[8];
#pragma unroll
        for (int i = 0; i < 4; i++) {
          vz[i] = v[2 * i];
          vz[4 + i] = v[2 * i + 1];
        }
        store8(skz + lane * 8, vz);
      } else {
        // B operand: y weight times strength, column 2 y + (re, im)
        const int ly = window_weights<W>(r0.y, g.fbits[1], n1, by0, bl, ktab, k);
        slots8<W>(k, ly & 1, v);
        float4* b4 = reinterpret_cast<float4*>(sb + lane * 16);
#pragma unroll
        for (int i = 0; i < 4; i++)
          b4[i] = make_float4(v[2 * i] * cc0.x, v[2 * i] * cc0.y, v[2 * i + 1] * cc0.x,
                              v[2 * i + 1] * cc0.y);
        const int lx = rel_window_cell<W>(r0.x, g.fbits[0], n0, bx0);
        scol[lane] = (lx >> 1) + b0 * (ly >> 1);
        szr[lane] = rel_window_cell<W>(r0.z, g.fbits[2], n2, bz0);
      }
    }
    r0 = r1;
    r1 = r2;
    cc0 = cc1;
    __syncthreads();
    // runs of points with the same column block and pair of z cells
    const bool starts = lane < nbatch && (lane == 0 || (szr[lane] >> 1) != (szr[lane - 1] >> 1) ||
                                          scol[lane] != scol[lane - 1]);
    uint64_t runs = __ballot(starts);
    while (runs) {
      const int q0 = __ffsll((unsigned long long)runs) - 1;
      runs &= runs - 1;
      const int q1 = runs ? __ffsll((unsigned long long)runs) - 1 : nbatch;
      const int col = scol[q0];
      const int zr = szr[q0] & ~1;   // the run's planes: zr .. zr + 7
      if (col != cur) {
        if (cur >= 0) flush(0xffu);
        cur = col;
        const int clx = col % b0, cly = col / b0;
        colbase = ((2 * cly + yl) * T0 + 2 * clx + x0) * 2 + reim;
        pend = zr;
      } else if (zr > pend) {
        // planes pend .. zr - 1 receive nothing more
        const int nfl = zr - pend;
        unsigned fm = 0xffu;
        if (nfl < 8) {
          const unsigned m = ((1u << nfl) - 1u) << (pend & 7);
          fm = (m | (m >> 8)) & 0xffu;
        }
        flush(fm);
        pend = zr;
      }
      // Four 4-point steps per iteration.  The operands of step i are read
      // from LDS into its registers 16 points ahead, right after the step has
      // used them, so three other steps' work covers the read latency
      // (scheduling barriers keep the reads where they are written, and the
      // first reads are issued in the loop's order so that each step waits
      // only for its own).  Full iterations need no mask; the last 1 .. 15
      // points of a run take masked steps.  Reads may run past the run (other
      // runs' points, or the zero rows at the end of the staging; the
      // furthest is row q1 - 1 + 16 <= 79, and every row read is finite).
      const float* px = skx + ox;   // + 8 q: x weight of this lane's row
      const float* pz = skz + oz;   // + 8 q: its two ring-slot weights
      const float* pb = sb + ob;    // + 16 q: its B column
      float ax[4], bv[4];
      float2 kz[4];
#pragma unroll
      for (int i = 0; i < 4; i++) {
        ax[i] = px[8 * q0 + 32 * i];
        kz[i] = *reinterpret_cast<const float2*>(pz + 8 * q0 + 32 * i);
        bv[i] = pb[16 * q0 + 64 * i];
        __builtin_amdgcn_sched_barrier(0);
      }
      int q = q0;
      for (; q + 16 <= q1; q += 16) {
#pragma unroll
        for (int i = 0; i < 4; i++) {
          acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(ax[i] * kz[i].x, bv[i], acc[0], 0, 0, 0);
          acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(ax[i] * kz[i].y, bv[i], acc[1], 0, 0, 0);
          const int qa = q + 16;
          ax[i] = px[8 * qa + 32 * i];
          kz[i] = *reinterpret_cast<const float2*>(pz + 8 * qa + 32 * i);
          bv[i] = pb[16 * qa + 64 * i];
          __builtin_amdgcn_sched_barrier(0);
        }
      }
#pragma unroll
      for (int i = 0; i < 4; i++) {
        if (q + 4 * i < q1) {
          const float b = kg < q1 - q - 4 * i ? bv[i] : 0.f;
          acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(ax[i] * kz[i].x, b, acc[0], 0, 0, 0);
          acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(ax[i] * kz[i].y, b, acc[1], 0, 0, 0);
        }
      }
    }
  }
  if (cur >= 0) flush(0xffu);
  __syncthreads();

  // add the bin tile to the periodic fine grid (touched cells only)
  TileWalk tw(tid, 128, T0, T1);
  for (int i = tid; i < tc; i += 128, tw.next()) {
    const float2 v = *reinterpret_cast<const float2*>(otf + tw.ofs(ps));
    if (v.x != 0.f || v.y != 0.f) {
      float* dst = grid + 2 * (gz[tw.iz] + gy[tw.iy] + gx[tw.ix]);
      atomicAdd(dst, v.x);
      atomicAdd(dst + 1, v.y);
    }
  }
}

// Two waves per subproblem share the grid tile and the staged weights: in
// each batch wave 0 computes the x and y weights and wave 1 the z weights and
// each point's footprint origin in the tile; the waves then share the runs
// (points of one 2 x 2 x 2 block of window cells): alternate 16-point steps of
// longer runs, and one-step runs in turn.
//
// Matrix layout of a step (16 points q .. q + 15 of a run):
//   A[m][k] = G[x, y, z(m), re/im(m)]   grid tile, m = lane & 15, k = lane >> 4,
//             x = 4 (s & 1) + k, y = s >> 1 for instruction s = 0 .. 15;
//             row m holds plane z(m) = (m >> 2) + 4 ((m >> 1) & 1), part m & 1
//   B[k][n] = kx_p(x) ky_p(y)          point p = q + n
// so the output row 4 kq + i of lane (kq, n) is plane kq + 4 (i >> 1), part
// i & 1 of point q + n, and the z weights a lane needs sit at the same slots
// kq and kq + 4 as its x weights.  Rows past a run (other points, or stale
// rows) only reach output columns that are not stored.
template <int W>
__global__ void __launch_bounds__(128)
interp_mfma_kernel(const GeomArgs g, const float2* __restrict__ grid, float2* __restrict__ c) {
  static_assert(W >= 2 && W <= 7, "matrix-core interpolation needs w <= 7");
  constexpr int H = W / 2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int b0 = g.b[0], b1 = g.b[1], b2 = g.b[2];
  // 8-wide footprints from even window cells of the bin (even bin sizes)
  const int T0 = b0 + 6, T1 = b1 + 6, T2 = b2 + 6;
  const int ps = plane_floats(T0, T1);               // floats per tile plane
  float* gtf = reinterpret_cast<float*>(smem_raw);                 // [T2][ps]: [T1][T0][2]
  float* skx = gtf + T2 * ps;                                      // [64][8] x slots
  float* sky = skx + 64 * 8;                                       // [64][8] y slots
  float* skz = sky + 64 * 8;                                       // [80][8] z slots
  // [64] results, after the staging area (the weights, or the row table)
  float2* sout = reinterpret_cast<float2*>(skx + interp_stage_floats(T1, T2));
  int64_t* gz = reinterpret_cast<int64_t*>(sout + 64);             // [T2]
  int* sorg = reinterpret_cast<int*>(gz + T2);                     // [64] footprint origin
  int* sperm = sorg + 64;                                          // [64]
  int* gx = sperm + 64;                                            // [T0]
  int* gy = gx + T0;                                               // [T1]

  const int sidx = blockIdx.x;
  const int bin = g.sub_bin[sidx];
  const int p0 = g.sub_start[sidx];
  const int p1 = p0 + g.sub_len[sidx];
  const int bi0 = bin % g.nb[0], bi1 = (bin / g.nb[0]) % g.nb[1], bi2 = bin / (g.nb[0] * g.nb[1]);
  const int bx0 = bi0 * b0, by0 = bi1 * b1, bz0 = bi2 * b2;
  const int tid = threadIdx.x;
  // the wave index, known to the compiler as the same across the wave, so that
  // ballots and run bounds derived from it stay in scalar registers
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const float bl = (float)(g.beta * 1.4426950408889634);   // beta log2(e)
  const float* ktab = static_cast<const float*>(g.ktab);    // kernel table or null
  const int n0 = (int)g.n[0], n1 = (int)g.n[1], n2 = (int)g.n[2];

  // (record loads are unconditional, at indices clamped into the subproblem,
  // so that the waits for them can be placed where the values are used)
  const uint4* rec = reinterpret_cast<const uint4*>(g.pts);
  const int plast = p1 - 1;
  uint4 r0 = rec[min(p0 + lane, plast)];
  tile_offsets(tid, 128, T0, T1, T2, bx0 - H, by0 - H, bz0 - H, n0, n1, n2, gx, gy, gz);
  __syncthreads();
  {
    // the bin's grid tile, by tile rows (y, z): lanes 16 j .. 16 j + 15 of the
    // block read x cells x0 .. x0 + 15 of rows j, j + 8, ..., four rows in
    // flight per thread.  Each row's grid offset (fine grids hold under 2^31
    // cells) and float offset in the tile come from a table built in the
    // staging area, which the first batch overwrites only after a barrier.
    const int nrow = T1 * T2;
    int* rowg = reinterpret_cast<int*>(skx);   // [nrow] gz[z] + gy[y]
    int* rowt = rowg + nrow;                    // [nrow] z ps + 2 y T0
    for (int r = tid; r < nrow; r += 128) {
      const int iy = r % T1, iz = r / T1;
      rowg[r] = (int)(gz[iz] + gy[iy]);
      rowt[r] = iz * ps + 2 * iy * T0;
    }
    __syncthreads();
    constexpr int U = 4;
    const int lx = tid & 15;
    for (int x0 = 0; x0 < T0; x0 += 16) {
      const int ix = x0 + lx;
      const int gxi = gx[min(ix, T0 - 1)];
      for (int rb = tid >> 4; rb < nrow; rb += 8 * U) {
        float2 v[U];
        // (rows past the last are read at the last row and not stored)
#pragma unroll
        for (int u = 0; u < U; u++) v[u] = grid[rowg[min(rb + 8 * u, nrow - 1)] + gxi];
#pragma unroll
        for (int u = 0; u < U; u++)
          if (ix < T0 && rb + 8 * u < nrow)
            *reinterpret_cast<float2*>(gtf + rowt[rb + 8 * u] + 2 * ix) = v[u];
      }
    }
  }

  const int n = lane & 15;         // MFMA row of A / column of B and of the output
  const int kq = lane >> 4;        // MFMA k lane group
  // this lane's float offset in the tile for instruction 0 (x = kq, y = 0)
  const int lane_g = ((n >> 2) + 4 * ((n >> 1) & 1)) * ps + 2 * kq + (n & 1);
  for (int base = p0; base < p1; base += 64) {
    const int nbatch = min(64, p1 - base);
    const uint4 r1 = rec[min(base + 64 + lane, plast)];
    __syncthreads();
    {
      float v[8];
      if (wv == 0) {
        float k[W];
        const int lx = window_weights<W>(r0.x, g.fbits[0], n0, bx0, bl, ktab, k);
        slots8<W>(k, lx & 1, v);
        store8(skx + lane * 8, v);
        const int ly = window_weights<W>(r0.y, g.fbits[1], n1, by0, bl, ktab, k);
        slots8<W>(k, ly & 1, v);
        store8(sky + lane * 8, v);
      } else {
        float k[W];
        const int lz = window_weights<W>(r0.z, g.fbits[2], n2, bz0, bl, ktab, k);
        slots8<W>(k, lz & 1, v);
        store8(skz + lane * 8, v);
        // footprint origin of the point's 2 x 2 x 2 block of window cells:
        // tile cell (lx & ~1, ly & ~1, lz & ~1), since the tile starts H cells
        // before the bin
        const int lx = rel_window_cell<W>(r0.x, g.fbits[0], n0, bx0);
        const int ly = rel_window_cell<W>(r0.y, g.fbits[1], n1, by0);
        sorg[lane] = (lz & ~1) * ps + 2 * ((ly & ~1) * T0 + (lx & ~1));
        sperm[lane] = (int)r0.w;
      }
    }
    r0 = r1;
    __syncthreads();
    const bool starts = lane < nbatch && (lane == 0 || sorg[lane] != sorg[lane - 1]);
    uint64_t runs = __ballot(starts);
    // Runs of more than one 16-point step are taken by both waves in
    // alternate steps (a batch is often a single run); one-step runs go to the
    // waves in turn.
    int nshort = 0;
    while (runs) {
      const int q0 = __ffsll((unsigned long long)runs) - 1;
      runs &= runs - 1;
      const int q1 = runs ? __ffsll((unsigned long long)runs) - 1 : nbatch;
      const bool one_step = q1 - q0 <= 16;
      if (one_step && (nshort++ & 1) != wv) continue;
      const int qstride = one_step ? 16 : 32;
      const int org = __builtin_amdgcn_readfirstlane(sorg[q0]);
      // grid operand of the run: one address per footprint row y, the x halves
      // at +8 floats
      float gop[16];
      {
        const float* gl = gtf + org + lane_g;
#pragma unroll
        for (int y = 0; y < 8; y++) {
          const float* r = gl + 2 * y * T0;
          gop[2 * y] = r[0];
          gop[2 * y + 1] = r[8];
        }
      }
      // weights of a step's points, read one step ahead (from a start of at
      // most 64, inside the staged rows)
      const float* wx = skx + n * 8 + kq;   // + 8 q: x slots kq, kq + 4; z at + 1024
      const float* wy = sky + n * 8;        // + 8 q: y slots 0 .. 7
      const int qs = one_step ? q0 : q0 + 16 * wv;   // this wave's first step
      const int qf = min(qs, 64);
      float kxa_n = wx[8 * qf], kxb_n = wx[8 * qf + 4];
      float4 kya_n = *reinterpret_cast<const float4*>(wy + 8 * qf);
      float4 kyb_n = *reinterpret_cast<const float4*>(wy + 8 * qf + 4);
      float kz0_n = wx[8 * qf + 1024], kz4_n = wx[8 * qf + 1028];
      // A step's z-weighted sums are formed right after its products; their
      // cross-lane reduction and store run in the next step, behind its
      // matrix work.
      float rep = 0.f, imp = 0.f;
      int qp = qs - qstride;   // the pending step (none before the first)
      auto finish = [&](float re, float im, int qb) {
        // the lower half of the wave sums re over lane groups (0, 2) and
        // (1, 3), the upper half im: one swap of re's upper 32 lanes with
        // im's lower 32 (v_permlane32_swap) leaves lane l < 32 with re(l) and
        // re(l + 32), lane l >= 32 with im(l - 32) and im(l)
        const auto h = __builtin_amdgcn_permlane32_swap(__float_as_uint(re), __float_as_uint(im),
                                                        false, false);
        const float u = __uint_as_float(h[0]) + __uint_as_float(h[1]);
        // every row of 16 lanes then adds its neighbour row (odd rows swapped
        // with even rows, v_permlane16_swap)
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(u), __float_as_uint(u),
                                                        false, false);
        const float v = __uint_as_float(r[0]) + __uint_as_float(r[1]);
        const int pt = qb + n;
        // row 0 stores re, row 2 im
        if ((kq & 1) == 0 && pt >= q0 && pt < q1)
          reinterpret_cast<float*>(sout)[2 * pt + (kq >> 1)] = v;
      };
      for (int q = qs; q < q1; q += qstride) {
        // the step's B operands are formed before the next step's weights are
        // read into the same registers
        const float ky[8] = {kya_n.x, kya_n.y, kya_n.z, kya_n.w, kyb_n.x, kyb_n.y, kyb_n.z, kyb_n.w};
        float bop[16];
#pragma unroll
        for (int s = 0; s < 16; s++) bop[s] = ((s & 1) ? kxb_n : kxa_n) * ky[s >> 1];
        const float kz0 = kz0_n, kz4 = kz4_n;
        // (scheduling barriers keep the products, the next step's reads and
        // the matrix work in this order, so the reads have the whole step)
        __builtin_amdgcn_sched_barrier(0);
        {
          int qn = min(q + qstride, 64);
          opaque(qn);
          kxa_n = wx[8 * qn];
          kxb_n = wx[8 * qn + 4];
          kya_n = *reinterpret_cast<const float4*>(wy + 8 * qn);
          kyb_n = *reinterpret_cast<const float4*>(wy + 8 * qn + 4);
          kz0_n = wx[8 * qn + 1024];
          kz4_n = wx[8 * qn + 1028];
          keep_order();
        }
        __builtin_amdgcn_sched_barrier(0);
        v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 16; s++)
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(gop[s], bop[s], acc, 0, 0, 0);
        finish(rep, imp, qp);
        // the wait states before the results are read
        xdl_waits<kXdlToValuWaits>(acc);
        // output rows 4 kq + i: plane kq + 4 (i >> 1), part i & 1
        rep = fmaf(kz4, acc[2], kz0 * acc[0]);
        imp = fmaf(kz4, acc[3], kz0 * acc[1]);
        qp = q;
      }
      finish(rep, imp, qp);
    }
    __syncthreads();
    if (tid < nbatch) c[sperm[tid]] = sout[tid];
  }
}

template <int W>
static hipError_t spread_mfma_w(const GeomArgs& g, int nsub, const void* c, void* grid,
                                hipStream_t s) {
  if (nsub <= 0) return hipSuccess;
  hipLaunchKernelGGL((spread_mfma_kernel<W>), dim3(nsub), dim3(128), mfma_spread_lds_bytes(W, g.b),
                     s, g, static_cast<const float2*>(c), static_cast<float*>(grid));
  return hipGetLastError();
}

template <int W>
static hipError_t interp_mfma_w(const GeomArgs& g, int nsub, const void* grid, void* c,
                                hipStream_t s) {
  if (nsub <= 0) return hipSuccess;
  hipLaunchKernelGGL((interp_mfma_kernel<W>), dim3(nsub), dim3(128), mfma_interp_lds_bytes(g.b), s,
                     g, static_cast<const float2*>(grid), static_cast<float2*>(c));
  return hipGetLastError();
}

hipError_t launch_spread_mfma(int w, const GeomArgs& g, int nsub, const void* c, void* grid,
                              hipStream_t s) {
  switch (w) {
    case 2: return spread_mfma_w<2>(g, nsub, c, grid, s);
    case 3: return spread_mfma_w<3>(g, nsub, c, grid, s);
    case 4: return spread_mfma_w<4>(g, nsub, c, grid, s);
    case 5: return spread_mfma_w<5>(g, nsub, c, grid, s);
    case 6: return spread_mfma_w<6>(g, nsub, c, grid, s);
    case 7: return spread_mfma_w<7>(g, nsub, c, grid, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_interp_mfma(int w, const GeomArgs& g, int nsub, const void* grid, void* c,
                              hipStream_t s) {
  switch (w) {
    case 2: return interp_mfma_w<2>(g, nsub, grid, c, s);
    case 3: return interp_mfma_w<3>(g, nsub, grid, c, s);
    case 4: return interp_mfma_w<4>(g, nsub, grid, c, s);
    case 5: return interp_mfma_w<5>(g, nsub, grid, c, s);
    case 6: return interp_mfma_w<6>(g, nsub, grid, c, s);
    case 7: return interp_mfma_w<7>(g, nsub, grid, c, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace esn
