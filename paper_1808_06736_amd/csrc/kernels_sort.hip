// Bin sort of the nonuniform points (Sec. 4.1) and the work lists for
// spreading (Sec. 4.2).
//
//   sort_keys : fold each coordinate into [0, 2pi), rescale to fine-grid units
//               t = x n / 2pi (FP64), take the cell floor(t); write the cell
//               key and the point's record (coordinates and index) in input
//               order.  Cells are numbered bin-major, so every bin (and, in
//               3D, every column of a bin) is a run of keys.
//   sort      : stable LSD radix sort of the records by key (rocPRIM), so
//               points of one cell keep their input order.
//   bounds    : the run of each bin in the sorted keys gives its point count.
//
// For small point sets the sort is a counting sort instead (the radix sort's
// fixed cost dominates there):
//   bin_count : as sort_keys, and count the point into its cell; the count
//               before the increment is the point's slot within the cell.
//   scan      : exclusive prefix sums of the counts = first position of a cell.
//   scatter   : place point j at start[cell] + slot, storing its record.
//   scan      : exclusive prefix sums of the bin counts = first position of a bin.
//   subprob   : split each bin's points into runs of at most maxsub.
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

// Encode t for storage; returns the cell floor(t) that the stored value decodes to.
__device__ __forceinline__ int encode_t(double t, int64_t n, int code, int fbits,
                                        uint32_t* q_out, double* t_out) {
  if (code == kPtsFixed32) {
    const uint64_t span = (uint64_t)n << fbits;
    uint64_t q = (uint64_t)llrint(ldexp(t, fbits));
    if (q >= span) q -= span;
    *q_out = (uint32_t)q;
    return (int)(q >> fbits);
  }
  *t_out = t;
  return (int)floor(t);
}

template <typename CTy>
__device__ __forceinline__ double load_coord(const void* p, int64_t j) {
  return (double)static_cast<const CTy*>(p)[j];
}

// Cell key of point j (see SortArgs); also returns the encoded coordinates.
template <typename CTy>
__device__ __forceinline__ int point_key(const SortArgs& a, int64_t j, int* flag, uint32_t* q,
                                         double* t) {
  int cell[3] = {0, 0, 0};
  for (int m = 0; m < a.dim; m++) {
    const double x = load_coord<CTy>(a.x[m], j);
    if (!isfinite(x)) *flag |= 1;
    else if (a.chkbnds && fabs(x) > kThreePi) *flag |= 2;
    const double tt = isfinite(x) ? fold_rescale(x, a.n[m]) : 0.0;
    cell[m] = encode_t(tt, a.n[m], a.pts_code, a.fbits[m], &q[m], &t[m]);
  }
  const int bx = cell[0] / a.b[0], by = cell[1] / a.b[1], bz = cell[2] / a.b[2];
  const int lx = cell[0] - bx * a.b[0], ly = cell[1] - by * a.b[1], lz = cell[2] - bz * a.b[2];
  const int bin = bx + a.nb[0] * (by + a.nb[1] * bz);
  const int cpb = a.b[0] * a.b[1] * a.b[2];
  int local;
  if (a.dim == 3) local = lz + a.b[2] * (lx + a.b[0] * ly);
  else local = lx + a.b[0] * ly;
  return bin * cpb + local;
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
__global__ void sort_keys_kernel(const SortArgs a) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.M) return;
  int flag = 0;
  uint32_t q[3];
  double t[3];
  const int key = point_key<CTy>(a, j, &flag, q, t);
  if (flag) atomicOr(a.flags, flag);
  a.key[j] = (uint32_t)key;
  write_record(a, j, q, t, j);
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

__global__ void bin_bounds_kernel(const uint32_t* __restrict__ skey, int64_t M, uint32_t cpb,
                                  int32_t* __restrict__ bcount) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  // bin b occupies sorted positions [start, end): add end at its last
  // position and subtract start at its first, so bcount[b] = end - start
  const uint32_t b = skey[i] / cpb;
  if (i == 0 || skey[i - 1] / cpb != b) atomicSub(&bcount[b], (int32_t)i);
  if (i == M - 1 || skey[i + 1] / cpb != b) atomicAdd(&bcount[b], (int32_t)(i + 1));
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
  if (a.coord_prec == ESN_SINGLE)
    hipLaunchKernelGGL(sort_keys_kernel<float>, dim3(nblocks(a.M, 256)), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(sort_keys_kernel<double>, dim3(nblocks(a.M, 256)), dim3(256), 0, s, a);
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

hipError_t launch_bin_bounds(const uint32_t* skey, int64_t M, int cpb, int32_t* bcount,
                             hipStream_t s) {
  if (M <= 0) return hipSuccess;
  hipLaunchKernelGGL(bin_bounds_kernel, dim3(nblocks(M, 256)), dim3(256), 0, s, skey, M,
                     (uint32_t)cpb, bcount);
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

// ---- subproblems ----
__global__ void subprob_count_kernel(const int32_t* __restrict__ bstart,
                                     int32_t* __restrict__ nsub, int64_t nbins, int maxsub,
                                     int32_t* nonempty) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbins) return;
  const int cnt = bstart[b + 1] - bstart[b];
  nsub[b] = (cnt + maxsub - 1) / maxsub;
  if (cnt > 0) atomicAdd(nonempty, 1);
}

__global__ void subprob_fill_kernel(const int32_t* __restrict__ bstart,
                                    const int32_t* __restrict__ nsub,
                                    const int32_t* __restrict__ subofs, int64_t nbins,
                                    int maxsub, int32_t* __restrict__ sub_bin,
                                    int32_t* __restrict__ sub_start,
                                    int32_t* __restrict__ sub_len) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbins) return;
  const int ns = nsub[b];
  const int o = subofs[b];
  const int st = bstart[b];
  const int cnt = bstart[b + 1] - st;
  for (int k = 0; k < ns; k++) {
    sub_bin[o + k] = (int32_t)b;
    sub_start[o + k] = st + k * maxsub;
    sub_len[o + k] = min(maxsub, cnt - k * maxsub);
  }
}

__global__ void iota_kernel(int32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}

hipError_t launch_subprob_count(const int32_t* bstart, int32_t* nsub, int64_t nbins, int maxsub,
                                int32_t* nonempty, hipStream_t s) {
  hipLaunchKernelGGL(subprob_count_kernel, dim3(nblocks(nbins, 256)), dim3(256), 0, s, bstart,
                     nsub, nbins, maxsub, nonempty);
  return hipGetLastError();
}

hipError_t launch_subprob_fill(const int32_t* bstart, const int32_t* nsub, const int32_t* subofs,
                               int64_t nbins, int maxsub, int32_t* sub_bin, int32_t* sub_start,
                               int32_t* sub_len, hipStream_t s) {
  hipLaunchKernelGGL(subprob_fill_kernel, dim3(nblocks(nbins, 256)), dim3(256), 0, s, bstart,
                     nsub, subofs, nbins, maxsub, sub_bin, sub_start, sub_len);
  return hipGetLastError();
}

hipError_t launch_iota_i32(int32_t* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(iota_kernel, dim3(nblocks(n, 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace esn
