// Spreading and interpolation on the matrix cores (3D, single precision,
// w <= 7), one wave per subproblem (a run of at most maxsub bin-sorted points
// of one bin, Sec. 4.2).
//
// Within a bin the points are sorted by column (x, y cell) and then by z cell.
// For the points of one column every window lies in the (w+1) x (w+1)
// footprint x in [x_c - floor(w/2), x_c - floor(w/2) + w] (same for y), so
// spreading them, eq. (bl), is
//
//     B[(x, y), z] = sum_p  kx_p(x) ky_p(y)  *  c_p kz_p(z),
//
// a dense contraction over the points of a 64 x P matrix of separable x-y
// weights with a P x (z planes) matrix of strength times z weight.  The wave
// runs it with v_mfma_f32_16x16x4_f32: the 64 footprint rows are four 16-row
// tiles, the 16 columns are 8 z planes x (re, im), each instruction takes 4
// points.  The 8 planes form a ring (plane z -> slot z mod 8): once the wave
// moves past cell z_c no later point of the column reaches plane
// z_c - floor(w/2) - 1, which is then added into the wave's LDS tile of the
// bin (bin + w cells per dim) and its slot reused.  The wave owns the tile, so
// these adds are plain read-modify-writes; the tile goes to the fine grid once
// at the end (global atomics on the touched cells only).
//
// Interpolation, eq. (interp), runs the same contraction the other way: for
// the points of one cell, T[p, z] = sum_(x,y) kx_p(x) ky_p(y) B[(x, y), z] on
// the matrix cores (16 points x 64 footprint cells x 8 planes (re, im)), then
// c_p = sum_z kz_p(z) T[p, z] by lane shuffles, with the bin's grid tile
// (bin + 7 cells per dim) copied into LDS first with coalesced reads.
#include "device_common.hpp"

namespace esn {

typedef float v4f __attribute__((ext_vector_type(4)));

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


// Tile of tc complex cells, padded to a 16-byte boundary so that the staging
// arrays after it are aligned for 16-byte LDS accesses.
__host__ __device__ inline size_t tile_bytes16(size_t tc) { return (tc * sizeof(float2) + 15) & ~(size_t)15; }

size_t mfma_spread_lds_bytes(int w, const int* b) {
  const size_t tile = tile_bytes16((size_t)(b[0] + w) * (b[1] + w) * (b[2] + w));
  return tile + 3 * 64 * 8 * sizeof(float) + 64 * sizeof(float2) + 2 * 64 * sizeof(int);
}

size_t mfma_interp_lds_bytes(const int* b) {
  const size_t tile = tile_bytes16((size_t)(b[0] + 7) * (b[1] + 7) * (b[2] + 7));
  return tile + 3 * 64 * 8 * sizeof(float) + 3 * 64 * sizeof(int);
}

// Kernel values of one point for the matrix-core kernels: x and y weights by
// footprint slot (8 slots; y de-interleaved as {0, 2, 4, 6, 1, 3, 5, 7} when
// ydeint), z weights either by ring slot (ring) or relative to the cell.
template <int W>
__device__ __forceinline__ void point_weights(uint32_t qx, uint32_t qy, uint32_t qz,
                                              const GeomArgs& g, float beta, bool ring,
                                              bool ydeint, float* vx, float* vy, float* vz,
                                              int* cell) {
  constexpr int H = W / 2;
  const uint32_t q[3] = {qx, qy, qz};
  float k[3][W];
  int sh[3];
#pragma unroll
  for (int m = 0; m < 3; m++) {
    const uint32_t fr = q[m] & ((1u << g.fbits[m]) - 1u);
    // window shift decided on the exact fraction bits (see decode_coord)
    sh[m] = (W & 1) ? (fr > (1u << (g.fbits[m] - 1))) : (fr != 0u);
    cell[m] = (int)(q[m] >> g.fbits[m]);
    es_weights_f32<W>(sh[m], ldexpf((float)fr, -g.fbits[m]), beta, k[m]);
  }
  slots8<W>(k[0], sh[0], vx);
  float t[8];
  slots8<W>(k[1], sh[1], t);
  if (ydeint) {
#pragma unroll
    for (int i = 0; i < 4; i++) {
      vy[i] = t[2 * i];
      vy[4 + i] = t[2 * i + 1];
    }
  } else {
#pragma unroll
    for (int i = 0; i < 8; i++) vy[i] = t[i];
  }
  if (ring) {
    slots8<W>(k[2], 0, vz);
    rotate8(vz, (cell[2] - H + sh[2]) & 7);
  } else {
    slots8<W>(k[2], sh[2], vz);
  }
}

template <int W>
__global__ void __launch_bounds__(64)
spread_mfma_kernel(const GeomArgs g, const float2* __restrict__ c, float* __restrict__ grid) {
  static_assert(W >= 2 && W <= 7, "matrix-core spreading needs w <= 7");
  constexpr int H = W / 2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int b0 = g.b[0], b1 = g.b[1], b2 = g.b[2];
  const int T0 = b0 + W, T1 = b1 + W, T2 = b2 + W;
  const int tc = T0 * T1 * T2;
  float* otf = reinterpret_cast<float*>(smem_raw);               // [T2][T1][T0][2]
  float* skx = reinterpret_cast<float*>(smem_raw + tile_bytes16(tc));   // [64][8] x slots
  float* sky = skx + 64 * 8;                                      // [64][8] y slots, de-interleaved
  float* skz = sky + 64 * 8;                                      // [64][8] z ring slots
  float2* sc = reinterpret_cast<float2*>(skz + 64 * 8);           // [64]
  int* scol = reinterpret_cast<int*>(sc + 64);                    // [64] column in the bin
  int* szc = scol + 64;                                           // [64] z cell

  const int sidx = blockIdx.x;
  const int bin = g.sub_bin[sidx];
  const int p0 = g.sub_start[sidx];
  const int p1 = p0 + g.sub_len[sidx];
  const int bi0 = bin % g.nb[0], bi1 = (bin / g.nb[0]) % g.nb[1], bi2 = bin / (g.nb[0] * g.nb[1]);
  const int bx0 = bi0 * b0, by0 = bi1 * b1, bz0 = bi2 * b2;
  const int lane = threadIdx.x;
  const float beta = (float)g.beta;

  for (int i = lane; i < tc * 2; i += 64) otf[i] = 0.f;
  v4f acc[4];
#pragma unroll
  for (int t = 0; t < 4; t++) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
  const int myslot = (lane & 15) >> 1;   // ring slot of this lane's accumulator column
  const int reim = lane & 1;
  int cur = -1;                          // current column (lx + b0 ly), -1: none
  int clx = 0, cly = 0;
  int pend = bz0 - H;                    // the ring holds planes pend .. pend + 7

  // add plane P of the current column's ring into the bin tile
  auto flush = [&](int P) {
    const int rel = P - (bz0 - H);
    const bool mine = myslot == (P & 7);
    if (mine && rel >= 0 && rel < T2) {
#pragma unroll
      for (int t = 0; t < 4; t++) {
#pragma unroll
        for (int i = 0; i < 4; i++) {
          const int row = 16 * t + 4 * (lane >> 4) + i;   // footprint (x, y) = (row & 7, row >> 3)
          const int x = clx + (row & 7), y = cly + (row >> 3);
          if (x < T0 && y < T1) {
            float* d = otf + ((rel * T1 + y) * T0 + x) * 2 + reim;
            *d += acc[t][i];
          }
        }
      }
    }
    if (mine) {
#pragma unroll
      for (int t = 0; t < 4; t++) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
    }
  };

  // point records flow through registers one batch ahead of the matrix work:
  // while batch b runs on the matrix cores, the records of batch b+2 and the
  // strengths of batch b+1 (gathered through the permutation) are in flight
  const uint4* rec = reinterpret_cast<const uint4*>(g.pts);
  uint4 r0 = make_uint4(0, 0, 0, 0), r1 = make_uint4(0, 0, 0, 0);
  float2 cc0 = make_float2(0.f, 0.f);
  if (p0 + lane < p1) {
    r0 = rec[p0 + lane];
    cc0 = c[(int)r0.w];
  }
  if (p0 + 64 + lane < p1) r1 = rec[p0 + 64 + lane];
  for (int base = p0; base < p1; base += 64) {
    const int nbatch = min(64, p1 - base);
    float2 cc1 = make_float2(0.f, 0.f);
    uint4 r2 = make_uint4(0, 0, 0, 0);
    if (base + 64 + lane < p1) cc1 = c[(int)r1.w];
    if (base + 128 + lane < p1) r2 = rec[base + 128 + lane];
    __syncthreads();
    if (lane < nbatch) {
      float vx[8], vy[8], vz[8];
      int cell[3];
      point_weights<W>(r0.x, r0.y, r0.z, g, beta, true, true, vx, vy, vz, cell);
      store8(skx + lane * 8, vx);
      store8(sky + lane * 8, vy);
      store8(skz + lane * 8, vz);
      sc[lane] = cc0;
      scol[lane] = (cell[0] - bx0) + b0 * (cell[1] - by0);
      szc[lane] = cell[2];
    }
    r0 = r1;
    r1 = r2;
    cc0 = cc1;
    __syncthreads();
    // runs of points with the same column and z cell
    const bool starts = lane < nbatch &&
                        (lane == 0 || szc[lane] != szc[lane - 1] || scol[lane] != scol[lane - 1]);
    uint64_t runs = __ballot(starts);
    while (runs) {
      const int q0 = __ffsll((unsigned long long)runs) - 1;
      runs &= runs - 1;
      const int q1 = runs ? __ffsll((unsigned long long)runs) - 1 : nbatch;
      const int col = scol[q0];
      const int zc = szc[q0];
      if (col != cur) {
        if (cur >= 0)
          for (int f = 0; f < 8; f++) flush(pend + f);
        cur = col;
        clx = col % b0;
        cly = col / b0;
        pend = bz0 - H;
      }
      int nfl = zc - H - pend;           // planes below zc - H receive nothing more
      if (nfl > 0) {
        if (nfl > 8) nfl = 8;
        for (int f = 0; f < nfl; f++) flush(pend + f);
        pend = zc - H;
      }
      for (int q = q0; q < q1; q += 4) {
        const int qq = q + (lane >> 4);
        const float valid = qq < q1 ? 1.f : 0.f;
        const int qs = qq < q1 ? qq : q0;
        const float ax = skx[qs * 8 + (lane & 7)];
        const float4 ky4 = *reinterpret_cast<const float4*>(sky + qs * 8 + ((lane >> 3) & 1) * 4);
        const float2 cv = sc[qs];
        const float bv = (reim ? cv.y : cv.x) * (skz[qs * 8 + myslot] * valid);
        acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(ax * ky4.x, bv, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(ax * ky4.y, bv, acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(ax * ky4.z, bv, acc[2], 0, 0, 0);
        acc[3] = __builtin_amdgcn_mfma_f32_16x16x4f32(ax * ky4.w, bv, acc[3], 0, 0, 0);
      }
    }
  }
  if (cur >= 0)
    for (int f = 0; f < 8; f++) flush(pend + f);
  __syncthreads();

  // add the bin tile to the periodic fine grid (touched cells only)
  const int n0 = (int)g.n[0], n1 = (int)g.n[1], n2 = (int)g.n[2];
  const int ox = bx0 - H, oy = by0 - H, oz = bz0 - H;
  for (int i = lane; i < tc; i += 64) {
    const float vr = otf[2 * i], vi = otf[2 * i + 1];
    if (vr != 0.f || vi != 0.f) {
      const int ix = i % T0;
      const int r = i / T0;
      const int gx = wrap2(ox + ix, n0);
      const int gy = wrap2(oy + r % T1, n1);
      const int gz = wrap2(oz + r / T1, n2);
      float* dst = grid + 2 * ((int64_t)gx + (int64_t)n0 * ((int64_t)gy + (int64_t)n1 * gz));
      atomicAdd(dst, vr);
      atomicAdd(dst + 1, vi);
    }
  }
}

template <int W>
__global__ void __launch_bounds__(64)
interp_mfma_kernel(const GeomArgs g, const float2* __restrict__ grid, float2* __restrict__ c) {
  static_assert(W >= 2 && W <= 7, "matrix-core interpolation needs w <= 7");
  constexpr int H = W / 2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int b0 = g.b[0], b1 = g.b[1], b2 = g.b[2];
  const int T0 = b0 + 7, T1 = b1 + 7, T2 = b2 + 7;   // 8-wide footprints for every w
  const int tc = T0 * T1 * T2;
  float2* gt = reinterpret_cast<float2*>(smem_raw);               // [T2][T1][T0]
  const float* gtf = reinterpret_cast<const float*>(gt);
  float* skx = reinterpret_cast<float*>(smem_raw + tile_bytes16(tc));   // [64][8] x slots
  float* sky = skx + 64 * 8;                                       // [64][8] y slots
  float* skz = sky + 64 * 8;                                       // [64][8] z rel. to the cell
  int* scol = reinterpret_cast<int*>(skz + 64 * 8);                // [64]
  int* szc = scol + 64;                                            // [64]
  int* sperm = szc + 64;                                           // [64]

  const int sidx = blockIdx.x;
  const int bin = g.sub_bin[sidx];
  const int p0 = g.sub_start[sidx];
  const int p1 = p0 + g.sub_len[sidx];
  const int bi0 = bin % g.nb[0], bi1 = (bin / g.nb[0]) % g.nb[1], bi2 = bin / (g.nb[0] * g.nb[1]);
  const int bx0 = bi0 * b0, by0 = bi1 * b1, bz0 = bi2 * b2;
  const int lane = threadIdx.x;
  const float beta = (float)g.beta;
  const int n0 = (int)g.n[0], n1 = (int)g.n[1], n2 = (int)g.n[2];
  const int ox = bx0 - H, oy = by0 - H, oz = bz0 - H;

  const uint4* rec = reinterpret_cast<const uint4*>(g.pts);
  uint4 r0 = make_uint4(0, 0, 0, 0);
  if (p0 + lane < p1) r0 = rec[p0 + lane];
  for (int i = lane; i < tc; i += 64) {
    const int ix = i % T0;
    const int r = i / T0;
    const int gx = wrap2(ox + ix, n0);
    const int gy = wrap2(oy + r % T1, n1);
    const int gz = wrap2(oz + r / T1, n2);
    gt[i] = grid[(int64_t)gx + (int64_t)n0 * ((int64_t)gy + (int64_t)n1 * gz)];
  }

  const int n = lane & 15;         // MFMA column: plane n >> 1, (re, im) = n & 1
  const int kq = lane >> 4;        // MFMA k lane group
  for (int base = p0; base < p1; base += 64) {
    const int nbatch = min(64, p1 - base);
    uint4 r1 = make_uint4(0, 0, 0, 0);
    if (base + 64 + lane < p1) r1 = rec[base + 64 + lane];
    __syncthreads();
    if (lane < nbatch) {
      float vx[8], vy[8], vz[8];
      int cell[3];
      point_weights<W>(r0.x, r0.y, r0.z, g, beta, false, false, vx, vy, vz, cell);
      store8(skx + lane * 8, vx);
      store8(sky + lane * 8, vy);
      store8(skz + lane * 8, vz);
      scol[lane] = (cell[0] - bx0) + b0 * (cell[1] - by0);
      szc[lane] = cell[2];
      sperm[lane] = (int)r0.w;
    }
    r0 = r1;
    __syncthreads();
    const bool starts = lane < nbatch &&
                        (lane == 0 || szc[lane] != szc[lane - 1] || scol[lane] != scol[lane - 1]);
    uint64_t runs = __ballot(starts);
    while (runs) {
      const int q0 = __ffsll((unsigned long long)runs) - 1;
      runs &= runs - 1;
      const int q1 = runs ? __ffsll((unsigned long long)runs) - 1 : nbatch;
      const int col = scol[q0];
      const int lx = col % b0, ly = col / b0;
      const int zrel = szc[q0] - bz0;      // first window plane of the cell, in the tile
      // B operand of the run: footprint cell (x, y) = (4 (s & 1) + kq, s >> 1), plane n >> 1
      float bop[16];
#pragma unroll
      for (int s = 0; s < 16; s++) {
        const int x = lx + 4 * (s & 1) + kq, y = ly + (s >> 1);
        bop[s] = gtf[(((zrel + (n >> 1)) * T1 + y) * T0 + x) * 2 + (n & 1)];
      }
      for (int q = q0; q < q1; q += 16) {
        const int qq = q + n;                   // this lane's point (MFMA row)
        const float valid = qq < q1 ? 1.f : 0.f;
        const int qs = qq < q1 ? qq : q0;
        const float kxa = skx[qs * 8 + kq] * valid;
        const float kxb = skx[qs * 8 + 4 + kq] * valid;
        const float4 kya = *reinterpret_cast<const float4*>(sky + qs * 8);
        const float4 kyb = *reinterpret_cast<const float4*>(sky + qs * 8 + 4);
        const float ky[8] = {kya.x, kya.y, kya.z, kya.w, kyb.x, kyb.y, kyb.z, kyb.w};
        v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 16; s++) {
          const float a = ((s & 1) ? kxb : kxa) * ky[s >> 1];
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bop[s], acc, 0, 0, 0);
        }
        // acc[i] = T[point q + 4 kq + i][column n]: weight by kz and sum the columns
#pragma unroll
        for (int i = 0; i < 4; i++) {
          const int pt = q + 4 * kq + i;
          const bool pv = pt < q1;
          const int ps = pv ? pt : q0;         // keeps the LDS index in range
          float v = pv ? acc[i] * skz[ps * 8 + (n >> 1)] : 0.f;
          v += __shfl_xor(v, 2);
          v += __shfl_xor(v, 4);
          v += __shfl_xor(v, 8);
          const float vim = __shfl_down(v, 1);
          if (pv && n == 0) c[sperm[ps]] = make_float2(v, vim);
        }
      }
    }
  }
}

template <int W>
static hipError_t spread_mfma_w(const GeomArgs& g, int nsub, const void* c, void* grid,
                                hipStream_t s) {
  if (nsub <= 0) return hipSuccess;
  hipLaunchKernelGGL((spread_mfma_kernel<W>), dim3(nsub), dim3(64), mfma_spread_lds_bytes(W, g.b),
                     s, g, static_cast<const float2*>(c), static_cast<float*>(grid));
  return hipGetLastError();
}

template <int W>
static hipError_t interp_mfma_w(const GeomArgs& g, int nsub, const void* grid, void* c,
                                hipStream_t s) {
  if (nsub <= 0) return hipSuccess;
  hipLaunchKernelGGL((interp_mfma_kernel<W>), dim3(nsub), dim3(64), mfma_interp_lds_bytes(g.b), s,
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
