// Bin sort of the nonuniform points (Sec. 5.1) and the work lists for
// spreading (Sec. 5.2).
//
// The paper counts the points per bin, turns the counts into the bins'
// breakpoints and writes each point into its bin.  Here the count goes down
// to fine-grid cells: every point gets the key of its window cell (the cell
// floor(w/2) after its window start), cells numbered bin-major, so that every
// bin (and, in 3D, every column or 2 x 2 column block of a bin) is a run of
// keys, and the points are ordered by key.
//
// Large point sets: a least-significant-digit radix sort of the point records
// by key, with digits of at most 8 bits (three passes for the 24-bit keys of
// the 3D benchmark grids, four above 24 bits):
//   rsort_keys  : once, in input order: fold each coordinate into [0, 2pi),
//                 rescale it to t = x n / 2pi in FP64, check it, build the
//                 point's record and its key, and count the first pass's
//                 digit per tile;
// then per pass, over tiles of consecutive points:
//   rsort_count : each tile's count of every digit of the pass (passes after
//                 the first);
//   scan        : exclusive scan of the counts in digit-major order = where
//                 each tile's points of each digit start;
//   rsort_pass  : every point, record and key, to its place: a tile is moved
//                 in chunks, each chunk's points ranked stably by digit (each
//                 wave its own 64-point steps, lanes of one digit found by
//                 ballots of the digit's bits), put in digit order in LDS and
//                 written out from there, so that a digit's points leave as
//                 one contiguous run;
// and at the end
//   ends        : where the sorted keys move on to another bin gives that
//                 bin's end; the bins' starts follow by a running maximum.
// The sort is stable: points of one cell keep their input order.
//
// Small point sets: a counting sort over the cells (a radix sort's fixed
// cost dominates there):
//   bin_count : key as above, and count the point into its cell; the count
//               before the increment is the point's slot within the cell.
//   scan      : exclusive prefix sums of the counts = first position of a cell.
//   scatter   : place point j at start[cell] + slot, storing its record.
//   starts    : a bin starts where its first cell starts.
// Both then split each bin's points into runs of at most maxsub (subproblems),
// by tiles of bins: counts per tile, then offsets from the tiles before.
#include <algorithm>
#include <cstring>
#include <type_traits>

#include "device_common.hpp"

namespace esn {

constexpr double kThreePi = 9.42477796076937971539;   // 3 pi

// Fold x into [0, 2pi) and rescale to t = x n / 2pi in [0, n), in FP64:
// t = x (n / 2pi) (scale = n / 2pi) less whole periods n (inv_n = 1 / n).
__device__ __forceinline__ double fold_rescale(double x, double scale, double dn, double inv_n) {
  double t = x * scale;
  t -= dn * floor(t * inv_n);        // a rounding slip here is fixed below
  t = t < 0.0 ? t + dn : t;
  t = t >= dn ? t - dn : t;
  return (t >= 0.0 && t < dn) ? t : 0.0;
}

// Fixed-point form t 2^fbits of t in [0, n) (pow2f = 2^fbits): n 2^fbits <=
// 2^32, so the rounded value (ties to even) is an exact integer below 2^32
// once a round-up to the period is wrapped.
__device__ __forceinline__ uint32_t encode_fixed(double t, double span, double pow2f) {
  double v = rint(t * pow2f);
  if (v >= span) v -= span;
  return (uint32_t)v;
}

// Encode t for storage; returns the window cell (c + sh wrapped into [0, n),
// see window_cell) of the stored value.
__device__ __forceinline__ int encode_t(double t, int64_t n, int code, int fbits, double span,
                                        double pow2f, int w, uint32_t* q_out, double* t_out) {
  if (code == kPtsFixed32) {
    const uint32_t q = encode_fixed(t, span, pow2f);
    *q_out = q;
    return window_cell((int)(q >> fbits), window_shift_fixed(q & ((1u << fbits) - 1u), fbits, w),
                       n);
  }
  *t_out = t;
  const double c = floor(t);
  return window_cell((int)c, window_shift_f64(t - c, w), n);
}

template <typename CTy>
__device__ __forceinline__ double load_coord(const void* p, int64_t j) {
  return (double)static_cast<const CTy*>(p)[j];
}

// Key of the window cells cell[0 .. dim-1] of a point.  In 3D the cells of a
// bin are ordered by z within each (x, y) column; with a.blocked the columns
// come in 2 x 2 blocks and a block's four columns are merged in z order (cell
// (lx, ly, lz) at 4 (lz + b2 (block)) + 2 (ly & 1) + (lx & 1)), so that each
// block's points with z cells 2j, 2j + 1 are one run.  In 2D with a.blocked2d
// = B the cells come in B x B blocks (block-major), so each block is one run.
__device__ __forceinline__ int key_of_cells(const SortArgs& a, const int* cell) {
  int bx, by, bz;
  if (a.bpow2) {           // bin sizes 2^bshift: shifts instead of divisions
    bx = cell[0] >> a.bshift[0];
    by = cell[1] >> a.bshift[1];
    bz = cell[2] >> a.bshift[2];
  } else {
    bx = cell[0] / a.b[0];
    by = cell[1] / a.b[1];
    bz = cell[2] / a.b[2];
  }
  const int lx = cell[0] - bx * a.b[0], ly = cell[1] - by * a.b[1], lz = cell[2] - bz * a.b[2];
  const int bin = bx + a.nb[0] * (by + a.nb[1] * bz);
  const int cpb = a.b[0] * a.b[1] * a.b[2];
  int local;
  if (a.dim == 3) {
    if (a.blocked)
      local = (lx & 1) + 2 * (ly & 1) +
              4 * (lz + a.b[2] * ((lx >> 1) + (a.b[0] >> 1) * (ly >> 1)));
    else
      local = lz + a.b[2] * (lx + a.b[0] * ly);
  } else if (a.blocked2d) {
    const int B = a.blocked2d, sB = B == 8 ? 3 : 2;
    local = (lx & (B - 1)) + B * (ly & (B - 1)) +
            B * B * ((lx >> sB) + (a.b[0] >> sB) * (ly >> sB));
  } else {
    local = lx + a.b[0] * ly;
  }
  return bin * cpb + local;
}

// Cell key of a point with coordinates xs[0 .. dim-1] (see SortArgs); also
// returns the encoded coordinates.  Cells are window cells.
__device__ __forceinline__ int point_key_of(const SortArgs& a, const double* xs, int* flag,
                                            uint32_t* q, double* t) {
  int cell[3] = {0, 0, 0};
#pragma unroll
  for (int m = 0; m < 3; m++) {
    if (m >= a.dim) break;
    const double x = xs[m];
    if (!isfinite(x)) *flag |= 1;
    else if (a.chkbnds && fabs(x) > kThreePi) *flag |= 2;
    const double tt = isfinite(x) ? fold_rescale(x, a.scale[m], (double)a.n[m], a.inv_n[m]) : 0.0;
    cell[m] = encode_t(tt, a.n[m], a.pts_code, a.fbits[m], a.span[m], a.pow2f[m], a.w, &q[m],
                       &t[m]);
  }
  return key_of_cells(a, cell);
}

// Cell key of point j, loading its coordinates.
template <typename CTy>
__device__ __forceinline__ int point_key(const SortArgs& a, int64_t j, int* flag, uint32_t* q,
                                         double* t) {
  double xs[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int m = 0; m < 3; m++)
    if (m < a.dim) xs[m] = load_coord<CTy>(a.x[m], j);
  return point_key_of(a, xs, flag, q, t);
}

// Store sorted point pos: coordinates (unused dims 0) and original index j,
// as one 16-byte or two 16-byte vector stores.
__device__ __forceinline__ void write_record(const SortArgs& a, int64_t pos, const uint32_t* q,
                                             const double* t, int64_t j) {
  if (a.pts_code == kPtsFixed32) {
    uint4 r;
    r.x = q[0];
    r.y = a.dim >= 2 ? q[1] : 0u;
    r.z = a.dim >= 3 ? q[2] : 0u;
    r.w = (uint32_t)j;
    reinterpret_cast<uint4*>(a.pts)[pos] = r;
  } else {
    double2* d = reinterpret_cast<double2*>(a.pts + pos * 32);
    d[0] = make_double2(t[0], a.dim >= 2 ? t[1] : 0.0);
    double2 hi;
    hi.x = a.dim >= 3 ? t[2] : 0.0;
    hi.y = __longlong_as_double((long long)(uint32_t)j);   // perm in the low 32 bits
    d[1] = hi;
  }
}

template <typename CTy>
__global__ void bin_count_kernel(const SortArgs a) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.M) return;
  int flag = 0;
  uint32_t q[3];
  double t[3];
  const int key = point_key<CTy>(a, j, &flag, q, t);
  if (flag) atomicOr(a.flags, flag);
  a.key[j] = (uint32_t)key;
  a.slot[j] = atomicAdd(&a.count[key], 1);
}

template <typename CTy>
__global__ void scatter_kernel(const SortArgs a) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.M) return;
  int flag = 0;
  uint32_t q[3];
  double t[3];
  point_key<CTy>(a, j, &flag, q, t);
  const int64_t pos = (int64_t)a.sstart[a.key[j]] + a.slot[j];
  write_record(a, pos, q, t, j);
}

__global__ void bin_starts_kernel(const int32_t* __restrict__ sstart, int64_t cpb, int64_t nbins,
                                  int32_t* __restrict__ bstart) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b <= nbins) bstart[b] = sstart[b * cpb];
}

// endpos[b] = one past the last sorted position of bin b = key / cpb, for every
// bin that holds points (empty bins keep the caller's zeros).  Four keys per
// thread; the key after them decides whether the last one ends its bin.
__global__ void bin_ends_kernel(const uint32_t* __restrict__ skey, int64_t M, uint32_t cpb,
                                int32_t* __restrict__ endpos) {
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (i0 >= M) return;
  uint32_t b[5];
  if (i0 + 4 < M) {
    const uint4 v = *reinterpret_cast<const uint4*>(skey + i0);   // i0 is a multiple of 4
    b[0] = v.x / cpb; b[1] = v.y / cpb; b[2] = v.z / cpb; b[3] = v.w / cpb;
    b[4] = skey[i0 + 4] / cpb;
  } else {
#pragma unroll
    for (int u = 0; u < 5; u++) b[u] = i0 + u < M ? skey[i0 + u] / cpb : 0xffffffffu;
  }
#pragma unroll
  for (int u = 0; u < 4; u++)
    if (i0 + u < M && b[u + 1] != b[u]) endpos[b[u]] = (int32_t)(i0 + u + 1);
}

template <typename CTy>
__global__ void encode_unsorted_kernel(const SortArgs a) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.M) return;
  int flag = 0;
  uint32_t q[3];
  double t[3];
  point_key<CTy>(a, j, &flag, q, t);
  if (flag) atomicOr(a.flags, flag);
  write_record(a, j, q, t, j);
}

static unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t launch_bin_count(const SortArgs& a, hipStream_t s) {
  if (a.M <= 0) return hipSuccess;
  if (a.coord_prec == ESN_SINGLE)
    hipLaunchKernelGGL(bin_count_kernel<float>, dim3(nblocks(a.M, 256)), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(bin_count_kernel<double>, dim3(nblocks(a.M, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_scatter(const SortArgs& a, hipStream_t s) {
  if (a.M <= 0) return hipSuccess;
  if (a.coord_prec == ESN_SINGLE)
    hipLaunchKernelGGL(scatter_kernel<float>, dim3(nblocks(a.M, 256)), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(scatter_kernel<double>, dim3(nblocks(a.M, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_bin_starts(const int32_t* sstart, int64_t cpb, int64_t nbins, int32_t* bstart,
                             hipStream_t s) {
  hipLaunchKernelGGL(bin_starts_kernel, dim3(nblocks(nbins + 1, 256)), dim3(256), 0, s, sstart,
                     cpb, nbins, bstart);
  return hipGetLastError();
}

hipError_t launch_bin_ends(const uint32_t* skey, int64_t M, int cpb, int32_t* endpos,
                           hipStream_t s) {
  if (M <= 0) return hipSuccess;
  hipLaunchKernelGGL(bin_ends_kernel, dim3(nblocks((M + 3) / 4, 256)), dim3(256), 0, s, skey, M,
                     (uint32_t)cpb, endpos);
  return hipGetLastError();
}

hipError_t launch_encode_unsorted(const SortArgs& a, hipStream_t s) {
  if (a.M <= 0) return hipSuccess;
  if (a.coord_prec == ESN_SINGLE)
    hipLaunchKernelGGL(encode_unsorted_kernel<float>, dim3(nblocks(a.M, 256)), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(encode_unsorted_kernel<double>, dim3(nblocks(a.M, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ---- radix sort of the point records (large point sets) ----
//
// Each pass splits the points into ntiles tiles of consecutive points (tile t:
// points [t tp, (t + 1) tp)), counts the pass's digit per tile, scans the
// counts in digit-major order (the scan of count[d][t] is where tile t's
// points of digit d go) and then moves every point, record and key, to its
// place.  A tile is moved in chunks: the chunk's points are ranked stably by
// digit, put in digit order in LDS and written out from there, so that the
// points of one digit leave as one contiguous run.  Tiles are handed to blocks
// so that a run of consecutive tiles runs on one XCD (consecutive blocks go to
// different XCDs): the count matrix's columns of neighbouring tiles share
// cache lines there.
constexpr int kRsWaves = 8;                       // waves per block
constexpr int kRsThreads = 64 * kRsWaves;
constexpr int kRsXcds = 8;                        // tiles come in multiples of this
constexpr int kRsMaxR = 1 << kRsMaxDigitBits;     // digits per pass at most

// Points per lane and chunk of a pass: 6 with 16-byte records, 3 with
// 32-byte ones (a chunk of records and keys is staged in LDS).
template <int RB> struct RsItems { static constexpr int value = RB == 16 ? 6 : 3; };

// Tile of block b: block b takes tile (b mod 8) ntiles / 8 + b / 8 (ntiles a
// multiple of 8).
__device__ __forceinline__ int rs_tile(int b, int ntiles) {
  return (b % kRsXcds) * (ntiles / kRsXcds) + b / kRsXcds;
}

template <int RB> struct alignas(16) RecT { uint4 v[RB / 16]; };

// Block barrier that orders LDS accesses only: global loads and stores in
// flight (the next chunk's records, the last chunk's stores) stay in flight.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Key of a stored record: its window cells from the stored coordinates, decided
// on the same bits as when the record was built.
template <int RB>
__device__ __forceinline__ uint32_t record_key(const SortArgs& a, const RecT<RB>& r) {
  int cell[3] = {0, 0, 0};
#pragma unroll
  for (int m = 0; m < 3; m++) {
    if (m >= a.dim) break;
    if constexpr (RB == 16) {
      const uint32_t q = m == 0 ? r.v[0].x : (m == 1 ? r.v[0].y : r.v[0].z);
      const int fb = a.fbits[m];
      cell[m] = window_cell((int)(q >> fb), window_shift_fixed(q & ((1u << fb) - 1u), fb, a.w),
                            a.n[m]);
    } else {
      uint32_t lo, hi;
      if (m == 0) { lo = r.v[0].x; hi = r.v[0].y; }
      else if (m == 1) { lo = r.v[0].z; hi = r.v[0].w; }
      else { lo = r.v[1].x; hi = r.v[1].y; }
      const double t = __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
      const double c = floor(t);
      cell[m] = window_cell((int)c, window_shift_f64(t - c, a.w), a.n[m]);
    }
  }
  return (uint32_t)key_of_cells(a, cell);
}

// Lanes of the wave whose digit equals this lane's (among the valid lanes),
// from one ballot per digit bit.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, int dbits, uint64_t valid) {
  uint64_t m = valid;
#pragma unroll
  for (int b = 0; b < kRsMaxDigitBits; b++) {
    if (b >= dbits) break;
    const uint64_t bb = __builtin_amdgcn_ballot_w64((d >> b) & 1u);
    const uint64_t flip = 0ull - (uint64_t)((d >> b) & 1u);   // all ones when the bit is set
    m &= ~(bb ^ flip);
  }
  return m;
}

// Number of lanes below this one in mask m.
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// First pass, part 1: the record and key of every point in input order (FP64
// fold, rescale and encoding of the caller's coordinates, with their checks)
// and each tile's count of the first digit, count[d][t] (digit-major).  Four
// consecutive points per thread.
template <int RB, typename CTy>
__global__ void __launch_bounds__(kRsThreads)
rsort_keys_kernel(const SortArgs a, RsortArgs r, unsigned char* __restrict__ recs,
                  uint32_t* __restrict__ keys) {
  __shared__ uint32_t hist[kRsMaxR];
  const int R = 1 << r.dbits;
  const int tile = rs_tile(blockIdx.x, r.ntiles);
  for (int i = threadIdx.x; i < R; i += kRsThreads) hist[i] = 0u;
  __syncthreads();
  const int64_t j0 = (int64_t)tile * r.tp;
  const int64_t j1 = min(j0 + r.tp, a.M);
  constexpr int64_t STEP = (int64_t)kRsThreads * 4;
  int flag = 0;
  // coordinates of four consecutive points, the next step's loaded while
  // this step's are folded
  auto load4 = [&](int64_t jt, double (&xs)[4][3]) {
#pragma unroll
    for (int u = 0; u < 4; u++)
#pragma unroll
      for (int m = 0; m < 3; m++) xs[u][m] = 0.0;
    if (jt >= j1) return;
    if (r.vec4 && jt + 4 <= j1) {
#pragma unroll
      for (int m = 0; m < 3; m++) {
        if (m >= a.dim) break;
        const CTy* src = static_cast<const CTy*>(a.x[m]) + jt;
        if constexpr (sizeof(CTy) == 4) {
          const float4 v = *reinterpret_cast<const float4*>(src);
          xs[0][m] = v.x; xs[1][m] = v.y; xs[2][m] = v.z; xs[3][m] = v.w;
        } else {
          const double2 v0 = reinterpret_cast<const double2*>(src)[0];
          const double2 v1 = reinterpret_cast<const double2*>(src)[1];
          xs[0][m] = v0.x; xs[1][m] = v0.y; xs[2][m] = v1.x; xs[3][m] = v1.y;
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < 4; u++)
#pragma unroll
        for (int m = 0; m < 3; m++)
          if (m < a.dim && jt + u < j1) xs[u][m] = load_coord<CTy>(a.x[m], jt + u);
    }
  };
  double nxt[4][3];
  load4(j0 + 4 * (int64_t)threadIdx.x, nxt);   // tp is a multiple of 4
  for (int64_t base = j0; base < j1; base += STEP) {
    const int64_t jt = base + 4 * (int64_t)threadIdx.x;
    double xs[4][3];
#pragma unroll
    for (int u = 0; u < 4; u++)
#pragma unroll
      for (int m = 0; m < 3; m++) xs[u][m] = nxt[u][m];
    if (base + STEP < j1) load4(jt + STEP, nxt);
    if (jt >= j1) continue;
    uint32_t k4[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const int64_t j = jt + u;
      if (j >= j1) break;
      uint32_t q[3] = {0u, 0u, 0u};
      double t[3] = {0.0, 0.0, 0.0};
      const uint32_t key = (uint32_t)point_key_of(a, xs[u], &flag, q, t);
      k4[u] = key;
      uint4* dst = reinterpret_cast<uint4*>(recs + j * RB);
      if constexpr (RB == 16) {
        dst[0] = make_uint4(q[0], a.dim >= 2 ? q[1] : 0u, a.dim >= 3 ? q[2] : 0u, (uint32_t)j);
      } else {
        const unsigned long long u0 = __double_as_longlong(t[0]);
        const unsigned long long u1 = __double_as_longlong(a.dim >= 2 ? t[1] : 0.0);
        const unsigned long long u2 = __double_as_longlong(a.dim >= 3 ? t[2] : 0.0);
        dst[0] = make_uint4((uint32_t)u0, (uint32_t)(u0 >> 32), (uint32_t)u1, (uint32_t)(u1 >> 32));
        dst[1] = make_uint4((uint32_t)u2, (uint32_t)(u2 >> 32), (uint32_t)j, 0u);
      }
      atomicAdd(&hist[key & (uint32_t)(R - 1)], 1u);
    }
    if (jt + 4 <= j1) {
      *reinterpret_cast<uint4*>(keys + jt) = make_uint4(k4[0], k4[1], k4[2], k4[3]);
    } else {
      for (int u = 0; u < 4 && jt + u < j1; u++) keys[jt + u] = k4[u];
    }
  }
  __syncthreads();
  for (int d = threadIdx.x; d < R; d += kRsThreads) r.count[(size_t)d * r.ntiles + tile] = hist[d];
  if (flag) atomicOr(a.flags, flag);
}

// Later passes, part 1: each tile's count of the pass's digit, from the keys
// in the previous pass's order (four per thread per load).
__global__ void __launch_bounds__(kRsThreads)
rsort_count_kernel(const int64_t M, RsortArgs r, int pass, const uint32_t* __restrict__ keys) {
  __shared__ uint32_t hist[kRsMaxR];
  const int R = 1 << r.dbits;
  const int shift = pass * r.dbits;
  const int tile = rs_tile(blockIdx.x, r.ntiles);
  for (int i = threadIdx.x; i < R; i += kRsThreads) hist[i] = 0u;
  __syncthreads();
  const int64_t j0 = (int64_t)tile * r.tp;
  const int64_t j1 = min(j0 + r.tp, M);
  constexpr int U = 4;                     // loads of 4 keys in flight per thread
  for (int64_t base = j0; base < j1; base += (int64_t)kRsThreads * 4 * U) {
    uint4 v[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int64_t jt = base + ((int64_t)u * kRsThreads + threadIdx.x) * 4;   // multiple of 4
      if (jt + 4 <= j1) {
        v[u] = *reinterpret_cast<const uint4*>(keys + jt);
      } else {
        v[u] = make_uint4(jt < j1 ? keys[jt] : 0u, jt + 1 < j1 ? keys[jt + 1] : 0u,
                          jt + 2 < j1 ? keys[jt + 2] : 0u, 0u);
      }
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int64_t jt = base + ((int64_t)u * kRsThreads + threadIdx.x) * 4;
      const uint32_t w[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
      for (int k = 0; k < 4; k++)
        if (jt + k < j1) atomicAdd(&hist[(w[k] >> shift) & (uint32_t)(R - 1)], 1u);
    }
  }
  __syncthreads();
  for (int d = threadIdx.x; d < R; d += kRsThreads) r.count[(size_t)d * r.ntiles + tile] = hist[d];
}

// Four 32-bit words as a native vector (kept in registers).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// The lane's CH points of a chunk: records (V 16-byte parts each) and keys.
template <int V, int CH>
__device__ __forceinline__ void load_chunk(u32x4 (&rec)[CH * V], uint32_t (&key)[CH],
                                           const unsigned char* __restrict__ in,
                                           const uint32_t* __restrict__ ikey, int64_t t0,
                                           int64_t j1) {
#pragma unroll
  for (int c = 0; c < CH; c++) {
    const int64_t j = t0 + (int64_t)c * 64;
    if (j < j1) {
      const u32x4* src = reinterpret_cast<const u32x4*>(in) + j * V;
#pragma unroll
      for (int u = 0; u < V; u++) rec[c * V + u] = src[u];
      key[c] = ikey[j];
    }
  }
}

// One digit pass over tile rs_tile(blockIdx.x), in chunks of kRsThreads x CH
// points (records with their keys): rank stably by digit, place in digit order
// in LDS, write out from there to the scanned start of the digit in this
// tile.  Ranks: every wave takes its own 64-point steps in order; the lanes of
// one digit in a step (found by ballots of the digit's bits) are counted
// into the wave's LDS table by their lowest lane, whose atomic add returns the
// count before them, passed on to the others.  The next chunk is loaded while
// a chunk is ranked and written.
template <int RB>
__global__ void __launch_bounds__(kRsThreads)
rsort_pass_kernel(const SortArgs a, RsortArgs r, int pass, const unsigned char* __restrict__ in,
                  const uint32_t* __restrict__ ikey, unsigned char* __restrict__ out,
                  uint32_t* __restrict__ okey) {
  constexpr int CH = RsItems<RB>::value;
  constexpr int T = kRsThreads * CH;
  constexpr int V = RB / 16;                    // uint4 per record
  __shared__ u32x4 stage[T * V];                // the chunk's records in digit order
  __shared__ uint32_t skey[T];                  // and their keys
  __shared__ uint32_t whist[kRsWaves][kRsMaxR]; // per wave: points per digit, then offsets
  __shared__ uint32_t gbase[kRsMaxR];           // where the tile's next points of a digit go
  __shared__ uint32_t cstart[kRsMaxR];          // first chunk position of a digit
  __shared__ uint32_t wsum[kRsWaves];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int R = 1 << r.dbits;
  const int shift = pass * r.dbits;
  const int tile = rs_tile(blockIdx.x, r.ntiles);
  const int64_t j0 = (int64_t)tile * r.tp;
  const int64_t j1 = min(j0 + r.tp, a.M);
  // thread d < R owns digit d
  if (tid < R) gbase[tid] = (uint32_t)r.offset[(size_t)tid * r.ntiles + tile];
  const int64_t lofs = (int64_t)wave * CH * 64 + lane;   // the lane's first point of a chunk
  u32x4 nrec[CH * V];
  uint32_t nkey[CH];
  load_chunk<V, CH>(nrec, nkey, in, ikey, j0 + lofs, j1);

  for (int64_t cbase = j0; cbase < j1; cbase += T) {
    const int nchunk = (int)min((int64_t)T, j1 - cbase);
    const int64_t t0 = cbase + lofs;
    u32x4 rec[CH * V];
    uint32_t key[CH];
#pragma unroll
    for (int c = 0; c < CH; c++) {
#pragma unroll
      for (int u = 0; u < V; u++) rec[c * V + u] = nrec[c * V + u];
      key[c] = nkey[c];
    }
    if (cbase + T < j1) load_chunk<V, CH>(nrec, nkey, in, ikey, t0 + T, j1);
    for (int i = tid; i < kRsWaves * R; i += kRsThreads) (&whist[0][0])[(i / R) * kRsMaxR + (i % R)] = 0u;
    lds_barrier();
    // stable ranks within the wave's points: the steps' adds go out back to
    // back (LDS atomics of one wave apply in order), then the counts before
    // each group come back from its lowest lane
    uint32_t d[CH], below[CH], first[CH], base[CH];
#pragma unroll
    for (int c = 0; c < CH; c++) {
      const bool valid = t0 + (int64_t)c * 64 < j1;
      d[c] = (key[c] >> shift) & (uint32_t)(R - 1);
      const uint64_t m = match_digit(d[c], r.dbits, __builtin_amdgcn_ballot_w64(valid));
      below[c] = lanes_below(m);
      first[c] = valid ? (uint32_t)__builtin_ctzll(m) : (uint32_t)lane;
      base[c] = 0u;
      if (valid && below[c] == 0u) base[c] = atomicAdd(&whist[wave][d[c]], (uint32_t)__popcll(m));
    }
#pragma unroll
    for (int c = 0; c < CH; c++) base[c] = __shfl(base[c], (int)first[c]) + below[c];
    lds_barrier();
    // digit tid: offsets of the waves, the chunk's count, its first position
    uint32_t total = 0u;
    if (tid < R) {
#pragma unroll
      for (int wv = 0; wv < kRsWaves; wv++) {
        const uint32_t h = whist[wv][tid];
        whist[wv][tid] = total;
        total += h;
      }
    }
    uint32_t v = total;                 // inclusive scan over the digits
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t o = __shfl_up(v, off);
      if (lane >= off) v += o;
    }
    if (lane == 63) wsum[wave] = v;
    lds_barrier();
    uint32_t woff = 0u;
    for (int wv = 0; wv < wave; wv++) woff += wsum[wv];
    if (tid < R) cstart[tid] = woff + v - total;
    lds_barrier();
#pragma unroll
    for (int c = 0; c < CH; c++) {
      if (t0 + (int64_t)c * 64 >= j1) continue;
      const uint32_t p = cstart[d[c]] + whist[wave][d[c]] + base[c];
#pragma unroll
      for (int u = 0; u < V; u++) stage[p * V + u] = rec[c * V + u];
      skey[p] = key[c];
    }
    lds_barrier();
    // out in digit order: a digit's points go to consecutive places
#pragma unroll
    for (int c = 0; c < CH; c++) {
      const int i = tid + c * kRsThreads;
      if (i >= nchunk) continue;
      u32x4 x[V];
#pragma unroll
      for (int u = 0; u < V; u++) x[u] = stage[i * V + u];
      const uint32_t k = skey[i];
      const uint32_t dd = (k >> shift) & (uint32_t)(R - 1);
      const int64_t pos = (int64_t)gbase[dd] + (i - (int)cstart[dd]);
      if (pos < 0 || pos >= a.M) continue;     // (never in a working sort)
      u32x4* dst = reinterpret_cast<u32x4*>(out + pos * RB);
#pragma unroll
      for (int u = 0; u < V; u++) dst[u] = x[u];
      okey[pos] = k;
    }
    lds_barrier();
    if (tid < R) gbase[tid] += total;
  }
}

// Key of every stored record (debug view of the sort).
template <int RB>
__global__ void record_keys_kernel(const SortArgs a, const unsigned char* __restrict__ pts,
                                   uint32_t* __restrict__ key, int32_t* __restrict__ perm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.M) return;
  RecT<RB> r;
  const uint4* src = reinterpret_cast<const uint4*>(pts + i * RB);
#pragma unroll
  for (int u = 0; u < RB / 16; u++) r.v[u] = src[u];
  key[i] = record_key<RB>(a, r);
  perm[i] = RB == 16 ? (int32_t)r.v[0].w : (int32_t)r.v[1].z;
}

hipError_t launch_record_keys(const SortArgs& a, const unsigned char* pts, uint32_t* key,
                              int32_t* perm, hipStream_t s) {
  if (a.M <= 0) return hipSuccess;
  if (pts_record_bytes(a.pts_code) == 16)
    hipLaunchKernelGGL(record_keys_kernel<16>, dim3(nblocks(a.M, 256)), dim3(256), 0, s, a, pts,
                       key, perm);
  else
    hipLaunchKernelGGL(record_keys_kernel<32>, dim3(nblocks(a.M, 256)), dim3(256), 0, s, a, pts,
                       key, perm);
  return hipGetLastError();
}

int radix_digits(int key_bits, int* dbits) {
  const int kb = key_bits < 1 ? 1 : key_bits;
  const int passes = (kb + kRsMaxDigitBits - 1) / kRsMaxDigitBits;
  *dbits = (kb + passes - 1) / passes;
  return passes;
}

// Tiles of a sort of M points: at most two per CU of the chip (256 CUs), a
// multiple of kRsXcds, each a multiple of 64 points.
static void radix_tiles(int64_t M, int rec_bytes, int* ntiles, int64_t* tp) {
  const int64_t chunk = (int64_t)kRsThreads * (rec_bytes == 16 ? RsItems<16>::value
                                                                : RsItems<32>::value);
  int64_t nt = std::min<int64_t>((M + chunk - 1) / chunk, 512);
  nt = std::max<int64_t>(kRsXcds, (nt + kRsXcds - 1) / kRsXcds * kRsXcds);
  int64_t per = (M + nt - 1) / nt;
  per = std::max<int64_t>(64, (per + 63) / 64 * 64);
  *ntiles = (int)nt;
  *tp = per;
}

// Scratch layout: count and offset matrices (2^dbits x ntiles int32 each),
// scan partials, one record buffer (the records in input order, or between
// passes) and two key buffers (M each); the sorted keys end in one of them.
struct RadixLayout {
  int passes, dbits, ntiles;
  int64_t tp;
  size_t count_off, offset_off, scan_off, rec_off, key_off[2], total;
};

static RadixLayout radix_layout(int64_t M, int key_bits, int rec_bytes) {
  RadixLayout L;
  L.passes = radix_digits(key_bits, &L.dbits);
  radix_tiles(M, rec_bytes, &L.ntiles, &L.tp);
  const size_t nmat = ((size_t)1 << L.dbits) * (size_t)L.ntiles;
  auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
  size_t off = 0;
  L.count_off = off;
  off = up(off + 4 * nmat);
  L.offset_off = off;
  off = up(off + 4 * nmat);
  L.scan_off = off;
  off = up(off + 4 * (size_t)(scan_tmp_elems((int64_t)nmat) + 1));
  L.rec_off = off;
  off = up(off + (size_t)rec_bytes * (size_t)M);
  for (int k = 0; k < 2; k++) {
    L.key_off[k] = off;
    off = up(off + 4 * (size_t)M);
  }
  L.total = off;
  return L;
}

size_t radix_scratch_bytes(int64_t M, int key_bits, int rec_bytes) {
  return radix_layout(M, key_bits, rec_bytes).total;
}

hipError_t radix_sort_points(const SortArgs& a, int key_bits, unsigned char* out_rec,
                             void* scratch, size_t scratch_bytes, uint32_t** sorted_keys,
                             hipStream_t s) {
  const int rb = pts_record_bytes(a.pts_code);
  const RadixLayout L = radix_layout(a.M, key_bits, rb);
  if (scratch_bytes < L.total || L.passes > kRsMaxPasses || a.M >= ((int64_t)1 << 31))
    return hipErrorInvalidValue;
  unsigned char* base = static_cast<unsigned char*>(scratch);
  RsortArgs r;
  r.passes = L.passes;
  r.dbits = L.dbits;
  r.ntiles = L.ntiles;
  r.tp = L.tp;
  r.count = reinterpret_cast<int32_t*>(base + L.count_off);
  r.offset = reinterpret_cast<int32_t*>(base + L.offset_off);
  int32_t* scan_tmp = reinterpret_cast<int32_t*>(base + L.scan_off);
  unsigned char* tmp_rec = base + L.rec_off;
  uint32_t* keys[2] = {reinterpret_cast<uint32_t*>(base + L.key_off[0]),
                       reinterpret_cast<uint32_t*>(base + L.key_off[1])};
  // pass p reads keys[p & 1] and writes keys[(p + 1) & 1]
  *sorted_keys = keys[L.passes & 1];
  if (a.M <= 0) return hipSuccess;
  // 4-point vector loads need every coordinate array aligned to 4 values
  const uintptr_t al = a.coord_prec == ESN_SINGLE ? 16 : 32;
  r.vec4 = 1;
  for (int m = 0; m < a.dim; m++)
    if (reinterpret_cast<uintptr_t>(a.x[m]) % al) r.vec4 = 0;
  const int64_t nmat = ((int64_t)1 << L.dbits) * L.ntiles;
  const dim3 grid((unsigned)L.ntiles), block(kRsThreads);
  // the records in input order go where the first pass does not write; the
  // passes alternate between the two record buffers and end in out_rec
  unsigned char* recs0 = (L.passes % 2 == 0) ? out_rec : tmp_rec;
  hipError_t e;
  if (rb == 16) {
    if (a.coord_prec == ESN_SINGLE)
      hipLaunchKernelGGL((rsort_keys_kernel<16, float>), grid, block, 0, s, a, r, recs0, keys[0]);
    else
      hipLaunchKernelGGL((rsort_keys_kernel<16, double>), grid, block, 0, s, a, r, recs0, keys[0]);
  } else {
    if (a.coord_prec == ESN_SINGLE)
      hipLaunchKernelGGL((rsort_keys_kernel<32, float>), grid, block, 0, s, a, r, recs0, keys[0]);
    else
      hipLaunchKernelGGL((rsort_keys_kernel<32, double>), grid, block, 0, s, a, r, recs0, keys[0]);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const unsigned char* in = recs0;
  for (int p = 0; p < L.passes; p++) {
    if (p > 0) {
      hipLaunchKernelGGL(rsort_count_kernel, grid, block, 0, s, a.M, r, p,
                         (const uint32_t*)keys[p & 1]);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if ((e = exclusive_scan_i32(r.count, r.offset, nmat, scan_tmp, s)) != hipSuccess) return e;
    unsigned char* dst = (in == out_rec) ? tmp_rec : out_rec;
    if (rb == 16)
      hipLaunchKernelGGL((rsort_pass_kernel<16>), grid, block, 0, s, a, r, p, in,
                         (const uint32_t*)keys[p & 1], dst, keys[(p + 1) & 1]);
    else
      hipLaunchKernelGGL((rsort_pass_kernel<32>), grid, block, 0, s, a, r, p, in,
                         (const uint32_t*)keys[p & 1], dst, keys[(p + 1) & 1]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    in = dst;
  }
  return in == out_rec ? hipSuccess : hipErrorInvalidValue;
}

// ---- exclusive scan of int32 (three phases, recursive over block sums) ----
constexpr int kScanBS = 256;           // threads per block
constexpr int kScanIPT = 4;            // items per thread
constexpr int kScanTile = kScanBS * kScanIPT;

// Inclusive scan of one value per thread across the block; returns the
// thread's inclusive prefix, *total gets the block sum.
__device__ __forceinline__ int32_t block_inclusive_scan(int32_t v, int32_t* sh, int32_t* total) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < kScanBS; off <<= 1) {
    int32_t add = tid >= off ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += add;
    __syncthreads();
  }
  int32_t r = sh[tid];
  *total = sh[kScanBS - 1];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(kScanBS)
scan_sums_kernel(const int32_t* __restrict__ in, int64_t n, int32_t* __restrict__ sums) {
  __shared__ int32_t sh[kScanBS];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanIPT;
  int32_t s = 0;
  for (int i = 0; i < kScanIPT; i++)
    if (base + i < n) s += in[base + i];
  int32_t total;
  block_inclusive_scan(s, sh, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanBS)
scan_apply_kernel(const int32_t* __restrict__ in, int32_t* __restrict__ out, int64_t n,
                  const int32_t* __restrict__ offsets) {
  __shared__ int32_t sh[kScanBS];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanIPT;
  int32_t v[kScanIPT];
  int32_t s = 0;
  for (int i = 0; i < kScanIPT; i++) {
    v[i] = (base + i < n) ? in[base + i] : 0;
    s += v[i];
  }
  int32_t total;
  int32_t incl = block_inclusive_scan(s, sh, &total);
  int32_t run = incl - s + (offsets ? offsets[blockIdx.x] : 0);
  for (int i = 0; i < kScanIPT; i++) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
}

int64_t scan_tmp_elems(int64_t n) {
  int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb <= 1) return 0;
  return 2 * nb + scan_tmp_elems(nb);
}

hipError_t exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* tmp,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 1) {
    hipLaunchKernelGGL(scan_apply_kernel, dim3(1), dim3(kScanBS), 0, s, in, out, n,
                       (const int32_t*)nullptr);
    return hipGetLastError();
  }
  int32_t* sums = tmp;
  int32_t* offs = tmp + nb;
  hipLaunchKernelGGL(scan_sums_kernel, dim3((unsigned)nb), dim3(kScanBS), 0, s, in, n, sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = exclusive_scan_i32(sums, offs, nb, tmp + 2 * nb, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nb), dim3(kScanBS), 0, s, in, out, n,
                     (const int32_t*)offs);
  return hipGetLastError();
}

// ---- bins and subproblems by tiles of kBinTile bins (one block each) ----
constexpr int kBinBS = 256;
constexpr int kBinIPT = 8;
constexpr int kBinTile = kBinBS * kBinIPT;

int64_t bin_tiles(int64_t nbins) { return (nbins + kBinTile - 1) / kBinTile; }

struct OpMax {
  __device__ static int32_t id() { return 0; }
  __device__ static int32_t op(int32_t a, int32_t b) { return max(a, b); }
};
struct OpSum {
  __device__ static int32_t id() { return 0; }
  __device__ static int32_t op(int32_t a, int32_t b) { return a + b; }
};

// Exclusive scan of one value per thread over the block (kBinBS threads);
// *total gets the whole block's reduction.
template <typename Op>
__device__ int32_t block_exclusive(int32_t v, int32_t* sh, int32_t* total) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < kBinBS; off <<= 1) {
    const int32_t o = tid >= off ? sh[tid - off] : Op::id();
    __syncthreads();
    sh[tid] = Op::op(sh[tid], o);
    __syncthreads();
  }
  const int32_t incl = sh[tid];
  *total = sh[kBinBS - 1];
  const int32_t excl = tid > 0 ? sh[tid - 1] : Op::id();
  __syncthreads();
  return excl;
}

// Reduction of v[0 .. n-1] by the whole block (every thread gets the result).
template <typename Op>
__device__ int32_t block_reduce_prefix(const int32_t* __restrict__ v, int64_t n, int32_t* sh) {
  int32_t r = Op::id();
  for (int64_t i = threadIdx.x; i < n; i += kBinBS) r = Op::op(r, v[i]);
  int32_t total;
  block_exclusive<Op>(r, sh, &total);
  return total;
}

// Pass 1 (radix sort): the largest bin end in each tile.
__global__ void __launch_bounds__(kBinBS)
bin_tile_max_kernel(const int32_t* __restrict__ endpos, int64_t nbins, int32_t* __restrict__ tmax) {
  __shared__ int32_t sh[kBinBS];
  const int64_t b0 = (int64_t)blockIdx.x * kBinTile + (int64_t)threadIdx.x * kBinIPT;
  int32_t m = 0;
  for (int u = 0; u < kBinIPT; u++)
    if (b0 + u < nbins) m = max(m, endpos[b0 + u]);
  int32_t total;
  block_exclusive<OpMax>(m, sh, &total);
  if (threadIdx.x == 0) tmax[blockIdx.x] = total;
}

// Pass 2: bin starts and subproblem counts per tile.  From the bin ends (radix
// sort) a bin's points follow those of every earlier bin, so its start is the
// largest end before it; from the bin starts (counting sort) the count is the
// difference of consecutive starts.
__global__ void __launch_bounds__(kBinBS)
bin_tile_count_kernel(const int32_t* __restrict__ endpos, int32_t* __restrict__ bstart,
                      int64_t nbins, int64_t M, int maxsub, const int32_t* __restrict__ tmax,
                      int32_t* __restrict__ nsub, int32_t* __restrict__ tsub,
                      int32_t* __restrict__ tnonempty) {
  __shared__ int32_t sh[kBinBS];
  const int64_t b0 = (int64_t)blockIdx.x * kBinTile + (int64_t)threadIdx.x * kBinIPT;
  int32_t cnt[kBinIPT];
  if (endpos) {
    const int32_t carry = block_reduce_prefix<OpMax>(tmax, blockIdx.x, sh);
    int32_t e[kBinIPT], m = 0;
    for (int u = 0; u < kBinIPT; u++) {
      e[u] = b0 + u < nbins ? endpos[b0 + u] : 0;
      m = max(m, e[u]);
    }
    int32_t total;
    int32_t run = max(carry, block_exclusive<OpMax>(m, sh, &total));
    for (int u = 0; u < kBinIPT; u++) {
      if (b0 + u < nbins) bstart[b0 + u] = run;
      cnt[u] = e[u] > 0 ? e[u] - run : 0;
      run = max(run, e[u]);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) bstart[nbins] = (int32_t)M;
  } else {
    for (int u = 0; u < kBinIPT; u++)
      cnt[u] = b0 + u < nbins ? bstart[b0 + u + 1] - bstart[b0 + u] : 0;
  }
  int32_t ns = 0, ne = 0;
  for (int u = 0; u < kBinIPT; u++) {
    const int32_t k = (cnt[u] + maxsub - 1) / maxsub;
    if (b0 + u < nbins) nsub[b0 + u] = k;
    ns += k;
    ne += cnt[u] > 0;
  }
  int32_t t1, t2;
  block_exclusive<OpSum>(ns, sh, &t1);
  block_exclusive<OpSum>(ne, sh, &t2);
  if (threadIdx.x == 0) {
    tsub[blockIdx.x] = t1;
    tnonempty[blockIdx.x] = t2;
  }
}

// Pass 3: each bin's subproblems {bin, first sorted position, length} at the
// number of subproblems of the bins before it.  The last tile writes the
// totals: totals[0] = subproblems, totals[1] = bins with points.
__global__ void __launch_bounds__(kBinBS)
bin_tile_fill_kernel(const int32_t* __restrict__ bstart, const int32_t* __restrict__ nsub,
                     int64_t nbins, int maxsub, const int32_t* __restrict__ tsub,
                     const int32_t* __restrict__ tnonempty, int32_t* __restrict__ sub_bin,
                     int32_t* __restrict__ sub_start, int32_t* __restrict__ sub_len,
                     int32_t* __restrict__ totals) {
  __shared__ int32_t sh[kBinBS];
  const int64_t b0 = (int64_t)blockIdx.x * kBinTile + (int64_t)threadIdx.x * kBinIPT;
  const int32_t carry = block_reduce_prefix<OpSum>(tsub, blockIdx.x, sh);
  int32_t k[kBinIPT], m = 0;
  for (int u = 0; u < kBinIPT; u++) {
    k[u] = b0 + u < nbins ? nsub[b0 + u] : 0;
    m += k[u];
  }
  int32_t total;
  int32_t o = carry + block_exclusive<OpSum>(m, sh, &total);
  for (int u = 0; u < kBinIPT; u++) {
    if (k[u] > 0) {
      const int32_t st = bstart[b0 + u];
      const int32_t cnt = bstart[b0 + u + 1] - st;
      for (int j = 0; j < k[u]; j++) {
        sub_bin[o + j] = (int32_t)(b0 + u);
        sub_start[o + j] = st + j * maxsub;
        sub_len[o + j] = min(maxsub, cnt - j * maxsub);
      }
    }
    o += k[u];
  }
  if (blockIdx.x == gridDim.x - 1) {
    const int32_t ne = block_reduce_prefix<OpSum>(tnonempty, gridDim.x, sh);
    if (threadIdx.x == 0) {
      totals[0] = carry + total;
      totals[1] = ne;
    }
  }
}

hipError_t launch_bin_subproblems(const int32_t* endpos, int32_t* bstart, int64_t nbins,
                                  int64_t M, int maxsub, int32_t* nsub, int32_t* tiles,
                                  int32_t* sub_bin, int32_t* sub_start, int32_t* sub_len,
                                  int32_t* totals, hipStream_t s) {
  const int64_t nt = bin_tiles(nbins);
  int32_t* tmax = tiles;
  int32_t* tsub = tiles + nt;
  int32_t* tne = tiles + 2 * nt;
  if (endpos) {
    hipLaunchKernelGGL(bin_tile_max_kernel, dim3((unsigned)nt), dim3(kBinBS), 0, s, endpos, nbins,
                       tmax);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(bin_tile_count_kernel, dim3((unsigned)nt), dim3(kBinBS), 0, s, endpos, bstart,
                     nbins, M, maxsub, tmax, nsub, tsub, tne);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(bin_tile_fill_kernel, dim3((unsigned)nt), dim3(kBinBS), 0, s, bstart, nsub,
                     nbins, maxsub, tsub, tne, sub_bin, sub_start, sub_len, totals);
  return hipGetLastError();
}

// ---- subproblems ----
__global__ void iota_kernel(int32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}

hipError_t launch_iota_i32(int32_t* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(iota_kernel, dim3(nblocks(n, 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace esn
