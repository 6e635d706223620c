// Bin sort of the nonuniform points (Sec. 4.1) and the work lists for
// spreading (Sec. 4.2).
//
//   sort_keys : fold each coordinate into [0, 2pi), rescale to fine-grid units
//               t = x n / 2pi (FP64), take the window cell floor(t) + sh (the
//               cell floor(w/2) after the window start); write the cell key
//               and the point's record (coordinates and index) in input
//               order.  Cells are numbered bin-major, so every bin (and, in
//               3D, every column or 2 x 2 column block of a bin) is a run of
//               keys.
//   sort      : stable LSD radix sort of the records by key (rocPRIM), so
//               points of one cell keep their input order.
//   ends      : where the sorted keys move on to another bin gives that bin's
//               end; the bins' starts follow by a running maximum.
//
// For small point sets the sort is a counting sort instead (the radix sort's
// fixed cost dominates there):
//   bin_count : as sort_keys, and count the point into its cell; the count
//               before the increment is the point's slot within the cell.
//   scan      : exclusive prefix sums of the counts = first position of a cell.
//   scatter   : place point j at start[cell] + slot, storing its record.
//   starts    : a bin starts where its first cell starts.
// Both then split each bin's points into runs of at most maxsub (subproblems),
// by tiles of bins: counts per tile, then offsets from the tiles before.
#include <cstring>
#include <rocprim/device/device_radix_sort.hpp>

#include "device_common.hpp"

namespace esn {

constexpr double kInvTwoPi = 0.15915494309189533577;  // 1 / (2 pi)
constexpr double kThreePi = 9.42477796076937971539;   // 3 pi

// Fold x into [0, 2pi) and rescale to t = x n / 2pi in [0, n), in FP64.
__device__ __forceinline__ double fold_rescale(double x, int64_t n) {
  const double dn = (double)n;
  double t = x * (dn * kInvTwoPi);
  t -= dn * floor(t * (1.0 / dn));   // a rounding slip here is fixed below
  if (t < 0.0) t += dn;
  if (t >= dn) t -= dn;
  if (!(t >= 0.0 && t < dn)) t = 0.0;
  return t;
}

// Encode t for storage; returns the window cell (c + sh wrapped into [0, n),
// see window_cell) of the stored value.
__device__ __forceinline__ int encode_t(double t, int64_t n, int code, int fbits, int w,
                                        uint32_t* q_out, double* t_out) {
  if (code == kPtsFixed32) {
    // n 2^fbits <= 2^32, so the rounded value (ties to even) is an exact
    // integer below 2^32 once a round-up to the period is wrapped
    const double span = ldexp((double)n, fbits);
    double v = rint(ldexp(t, fbits));
    if (v >= span) v -= span;
    const uint32_t q = (uint32_t)v;
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

// Cell key of a point with coordinates xs[0 .. dim-1] (see SortArgs); also
// returns the encoded coordinates.  Cells are window cells.  In 3D the cells
// of a bin are ordered by z within each (x, y) column; with a.blocked the
// columns come in 2 x 2 blocks and a block's four columns are merged in z
// order (cell (lx, ly, lz) at 4 (lz + b2 (block)) + 2 (ly & 1) + (lx & 1)),
// so that each block's points with z cells 2j, 2j + 1 are one run.
__device__ __forceinline__ int point_key_of(const SortArgs& a, const double* xs, int* flag,
                                            uint32_t* q, double* t) {
  int cell[3] = {0, 0, 0};
#pragma unroll
  for (int m = 0; m < 3; m++) {
    if (m >= a.dim) break;
    const double x = xs[m];
    if (!isfinite(x)) *flag |= 1;
    else if (a.chkbnds && fabs(x) > kThreePi) *flag |= 2;
    const double tt = isfinite(x) ? fold_rescale(x, a.n[m]) : 0.0;
    cell[m] = encode_t(tt, a.n[m], a.pts_code, a.fbits[m], a.w, &q[m], &t[m]);
  }
  const int bx = cell[0] / a.b[0], by = cell[1] / a.b[1], bz = cell[2] / a.b[2];
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
  } else {
    local = lx + a.b[0] * ly;
  }
  return bin * cpb + local;
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

// Four consecutive points per thread: their coordinates come in one 16- or
// 32-byte load per dimension and their keys go out in one 16-byte store
// (a.vec4: every coordinate array is 16-byte aligned (32 for FP64); the last
// partial group takes the scalar path).
template <typename CTy>
__global__ void sort_keys_kernel(const SortArgs a) {
  const int64_t j0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (j0 >= a.M) return;
  int flag = 0;
  uint32_t q[3];
  double t[3];
  if (a.vec4 && j0 + 4 <= a.M) {
    double xs[4][3] = {};
#pragma unroll
    for (int m = 0; m < 3; m++) {
      if (m >= a.dim) break;
      const CTy* src = static_cast<const CTy*>(a.x[m]) + j0;
      if constexpr (sizeof(CTy) == 4) {
        const float4 v = *reinterpret_cast<const float4*>(src);
        xs[0][m] = v.x; xs[1][m] = v.y; xs[2][m] = v.z; xs[3][m] = v.w;
      } else {
        const double2 v0 = reinterpret_cast<const double2*>(src)[0];
        const double2 v1 = reinterpret_cast<const double2*>(src)[1];
        xs[0][m] = v0.x; xs[1][m] = v0.y; xs[2][m] = v1.x; xs[3][m] = v1.y;
      }
    }
    uint32_t k[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      k[u] = (uint32_t)point_key_of(a, xs[u], &flag, q, t);
      write_record(a, j0 + u, q, t, j0 + u);
    }
    *reinterpret_cast<uint4*>(a.key + j0) = make_uint4(k[0], k[1], k[2], k[3]);
  } else {
    for (int64_t j = j0; j < j0 + 4 && j < a.M; j++) {
      a.key[j] = (uint32_t)point_key<CTy>(a, j, &flag, q, t);
      write_record(a, j, q, t, j);
    }
  }
  if (flag) atomicOr(a.flags, flag);
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

hipError_t launch_sort_keys(const SortArgs& a, hipStream_t s) {
  if (a.M <= 0) return hipSuccess;
  const unsigned nb = nblocks((a.M + 3) / 4, 256);
  if (a.coord_prec == ESN_SINGLE)
    hipLaunchKernelGGL(sort_keys_kernel<float>, dim3(nb), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(sort_keys_kernel<double>, dim3(nb), dim3(256), 0, s, a);
  return hipGetLastError();
}

// The sorted records as rocPRIM values.
struct alignas(16) Rec16 { uint32_t w[4]; };
struct alignas(16) Rec32 { uint32_t w[8]; };

template <typename R>
static hipError_t sort_records_t(uint32_t* key[2], unsigned char* rec[2], int* sel, int64_t M,
                                 int key_bits, void* tmp, size_t* tmp_bytes, hipStream_t s) {
  rocprim::double_buffer<uint32_t> k(key[0], key[1]);
  rocprim::double_buffer<R> v(reinterpret_cast<R*>(rec[0]), reinterpret_cast<R*>(rec[1]));
  hipError_t e = rocprim::radix_sort_pairs(tmp, *tmp_bytes, k, v, (unsigned)M, 0u,
                                           (unsigned)key_bits, s);
  if (e != hipSuccess || !tmp) return e;
  *sel = v.current() == reinterpret_cast<R*>(rec[0]) ? 0 : 1;
  if ((k.current() == key[0] ? 0 : 1) != *sel) return hipErrorUnknown;
  return hipSuccess;
}

size_t sort_tmp_bytes(int64_t M, int key_bits, int rec_bytes) {
  size_t bytes = 0;
  uint32_t* k[2] = {nullptr, nullptr};
  unsigned char* r[2] = {nullptr, nullptr};
  int sel = 0;
  const hipError_t e =
      rec_bytes == 16 ? sort_records_t<Rec16>(k, r, &sel, M, key_bits, nullptr, &bytes, 0)
                      : sort_records_t<Rec32>(k, r, &sel, M, key_bits, nullptr, &bytes, 0);
  return e == hipSuccess ? bytes : 0;
}

hipError_t sort_records(uint32_t* key[2], unsigned char* rec[2], int* sel, int64_t M,
                        int key_bits, int rec_bytes, void* tmp, size_t tmp_bytes, hipStream_t s) {
  *sel = 0;
  if (M <= 1 || key_bits <= 0) return hipSuccess;
  size_t bytes = tmp_bytes;
  return rec_bytes == 16 ? sort_records_t<Rec16>(key, rec, sel, M, key_bits, tmp, &bytes, s)
                         : sort_records_t<Rec32>(key, rec, sel, M, key_bits, tmp, &bytes, s);
}

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
