// Spreading of dense 3D columns with matrix-core (MFMA) accumulation.
//
// A column is the run of fine-grid cells (x_c, y_c, z) of one bin.  Every point
// of the column has its window inside the (w+1) x (w+1) footprint
// x in [x_c - floor(w/2), x_c - floor(w/2) + w] (same for y), so the column's
// contribution to the fine grid, eq. (bl), restricted to one z plane, is
//
//     B[(x, y), z] = sum_p  kx_p(x) ky_p(y)  *  c_p kz_p(z)
//
// a product of a 64 x P matrix (separable x-y weights of the P points) and a
// P x (z values) matrix (strength times z weight): a dense contraction over the
// points.  One wave runs it on the matrix cores with v_mfma_f32_16x16x4_f32:
// the 64 footprint rows are four 16-row tiles, the 16 columns are 8 z planes x
// (re, im), and each instruction takes 4 points.  The 8 z planes form a ring
// (plane z -> slot z mod 8): points are sorted by z cell, and once the wave
// moves past cell z_c no later point can reach plane z_c - floor(w/2) - 1, so
// that plane is written out to an LDS tile of the column and its ring slot is
// reused.  The column's LDS tile is added to the fine grid at the end (global
// atomics, consecutive lanes on consecutive x).  Requires w <= 7 (w + 1 <= 8
// planes per cell) and single precision.
#include "device_common.hpp"

namespace esn {

typedef float v4f __attribute__((ext_vector_type(4)));

size_t dense_lds_bytes(int w, const int* b) {
  const size_t np = (size_t)b[2] + w;                // planes of the column tile
  return np * 64 * sizeof(float2)                    // column tile
         + 3 * 64 * 8 * sizeof(float)                // x, y, z weights of 64 points
         + 64 * sizeof(float2) + 64 * sizeof(int);   // strengths, z cells
}

template <int W>
__global__ void __launch_bounds__(64)
spread_dense_kernel(const GeomArgs g, const DenseArgs d, const float2* __restrict__ c,
                    float* __restrict__ grid) {
  static_assert(W >= 2 && W <= 7, "dense spreading needs w <= 7");
  constexpr int H = W / 2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int b0 = g.b[0], b1 = g.b[1], b2 = g.b[2];
  const int NP = b2 + W;
  float* otf = reinterpret_cast<float*>(smem_raw);              // [NP][8][8][2]
  float* skx = otf + (size_t)NP * 128;                           // [64][8] by x slot
  float* sky = skx + 64 * 8;                                     // [64][8] y slots {0,2,4,6,1,3,5,7}
  float* skz = sky + 64 * 8;                                     // [64][8] z ring slots
  float2* sc = reinterpret_cast<float2*>(skz + 64 * 8);          // [64]
  int* szc = reinterpret_cast<int*>(sc + 64);                    // [64]

  const int u = blockIdx.x;
  const int col = d.unit_col[u];
  const int p0 = d.unit_p0[u], p1 = d.unit_p1[u];
  const int cpc = b0 * b1;
  const int bin = col / cpc;
  const int rr = col - bin * cpc;
  const int lx = rr % b0, ly = rr / b0;
  const int bi0 = bin % g.nb[0], bi1 = (bin / g.nb[0]) % g.nb[1], bi2 = bin / (g.nb[0] * g.nb[1]);
  const int X0 = bi0 * b0 + lx - H;      // footprint origin in x, y
  const int Y0 = bi1 * b1 + ly - H;
  const int Zlo = bi2 * b2 - H;          // lowest plane the column reaches
  const int lane = threadIdx.x;
  const float beta = (float)g.beta;

  for (int i = lane; i < NP * 128; i += 64) otf[i] = 0.f;
  v4f acc[4];
#pragma unroll
  for (int t = 0; t < 4; t++) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};

  // lanes holding ring slot s are those with ((lane & 15) >> 1) == s
  const int myslot = (lane & 15) >> 1;
  const int reim = lane & 1;
  int pend = Zlo;   // the ring holds planes pend .. pend + 7

  auto flush = [&](int P) {
    const int rel = P - Zlo;
    const bool mine = myslot == (P & 7);
    if (mine && rel < NP) {
#pragma unroll
      for (int t = 0; t < 4; t++) {
#pragma unroll
        for (int i = 0; i < 4; i++) {
          const int row = 16 * t + 4 * (lane >> 4) + i;   // (x, y) = (row & 7, row >> 3)
          otf[(rel * 64 + row) * 2 + reim] = acc[t][i];
        }
      }
    }
    if (mine) {
#pragma unroll
      for (int t = 0; t < 4; t++) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
    }
  };

  for (int base = p0; base < p1; base += 64) {
    const int nbatch = min(64, p1 - base);
    __syncthreads();
    if (lane < nbatch) {
      const int64_t j = (int64_t)base + lane;
      int shx, shy, shz;
      const Coord<float> cx = decode_coord<float>(g.t[0], g.pts_code, g.fbits[0], j, &shx, W);
      const Coord<float> cy = decode_coord<float>(g.t[1], g.pts_code, g.fbits[1], j, &shy, W);
      const Coord<float> cz = decode_coord<float>(g.t[2], g.pts_code, g.fbits[2], j, &shz, W);
      float kx[W], ky[W], kz[W];
      es_weights_f32<W>(shx, cx.f, beta, kx);
      es_weights_f32<W>(shy, cy.f, beta, ky);
      es_weights_f32<W>(shz, cz.f, beta, kz);
      float* px = skx + lane * 8;
      float* py = sky + lane * 8;
      float* pz = skz + lane * 8;
#pragma unroll
      for (int s = 0; s < 8; s++) {
        px[s] = 0.f;
        py[s] = 0.f;
        pz[s] = 0.f;
      }
      const int z0 = cz.cell - H + shz;
#pragma unroll
      for (int k = 0; k < W; k++) {
        px[shx + k] = kx[k];
        const int fy = shy + k;
        py[(fy & 1) * 4 + (fy >> 1)] = ky[k];
        pz[(z0 + k) & 7] = kz[k];
      }
      sc[lane] = c[g.perm[j]];
      szc[lane] = cz.cell;
    }
    __syncthreads();
    // runs of points with the same z cell (points are sorted by z within the column)
    const bool starts = lane < nbatch && (lane == 0 || szc[lane] != szc[lane - 1]);
    uint64_t runs = __ballot(starts);
    while (runs) {
      const int q0 = __ffsll((unsigned long long)runs) - 1;
      runs &= runs - 1;
      const int q1 = runs ? __ffsll((unsigned long long)runs) - 1 : nbatch;
      const int zc = szc[q0];
      // planes below zc - H receive nothing more: write them out
      const int upto = zc - H;       // first plane still open
      int nfl = upto - pend;
      if (nfl > 0) {
        if (nfl > 8) nfl = 8;
        for (int f = 0; f < nfl; f++) flush(pend + f);
        pend = upto;
      }
      for (int q = q0; q < q1; q += 4) {
        const int qq = q + (lane >> 4);
        const bool valid = qq < q1;
        const int qs = valid ? qq : q0;
        const float ax = skx[qs * 8 + (lane & 7)];
        const float4 ky4 = *reinterpret_cast<const float4*>(sky + qs * 8 + ((lane >> 3) & 1) * 4);
        const float2 cv = sc[qs];
        const float kzv = skz[qs * 8 + myslot];
        const float bv = valid ? (reim ? cv.y : cv.x) * kzv : 0.f;
        acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(ax * ky4.x, bv, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(ax * ky4.y, bv, acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(ax * ky4.z, bv, acc[2], 0, 0, 0);
        acc[3] = __builtin_amdgcn_mfma_f32_16x16x4f32(ax * ky4.w, bv, acc[3], 0, 0, 0);
      }
    }
  }
  for (int f = 0; f < 8; f++) flush(pend + f);
  __syncthreads();

  // add the column tile to the periodic fine grid
  const int n0 = (int)g.n[0], n1 = (int)g.n[1], n2 = (int)g.n[2];
  for (int i = lane; i < NP * 64; i += 64) {
    const float vr = otf[2 * i], vi = otf[2 * i + 1];
    if (vr != 0.f || vi != 0.f) {
      int gx = (X0 + (i & 7)) % n0;
      int gy = (Y0 + ((i >> 3) & 7)) % n1;
      int gz = (Zlo + (i >> 6)) % n2;
      gx += gx < 0 ? n0 : 0;
      gy += gy < 0 ? n1 : 0;
      gz += gz < 0 ? n2 : 0;
      float* dst = grid + 2 * ((int64_t)gx + (int64_t)n0 * ((int64_t)gy + (int64_t)n1 * gz));
      atomicAdd(dst, vr);
      atomicAdd(dst + 1, vi);
    }
  }
}

template <int W>
static hipError_t dense_launch_w(const GeomArgs& g, const DenseArgs& d, int nunits,
                                 const void* c, void* grid, hipStream_t s) {
  if (nunits <= 0) return hipSuccess;
  const size_t lds = dense_lds_bytes(W, g.b);
  hipLaunchKernelGGL((spread_dense_kernel<W>), dim3(nunits), dim3(64), lds, s, g, d,
                     static_cast<const float2*>(c), static_cast<float*>(grid));
  return hipGetLastError();
}

hipError_t launch_spread_dense(int w, const GeomArgs& g, const DenseArgs& d, int nunits,
                               const void* c, void* grid, hipStream_t s) {
  switch (w) {
    case 2: return dense_launch_w<2>(g, d, nunits, c, grid, s);
    case 3: return dense_launch_w<3>(g, d, nunits, c, grid, s);
    case 4: return dense_launch_w<4>(g, d, nunits, c, grid, s);
    case 5: return dense_launch_w<5>(g, d, nunits, c, grid, s);
    case 6: return dense_launch_w<6>(g, d, nunits, c, grid, s);
    case 7: return dense_launch_w<7>(g, d, nunits, c, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace esn
