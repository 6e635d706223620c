// Plan object and the C ABI (include/esnufft.h): makeplan / setpts / execute /
// destroy, the spread-only and interp-only steps, and the one-shot calls.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <mutex>
#include <vector>

#include "esn_internal.hpp"

using namespace esn;

namespace {

constexpr size_t kLdsBudgetCap = 64 * 1024;   // bytes of LDS one tile may use
// the 2D matrix-core kernels run 256-thread blocks: two of them per CU share its
// 160 KiB of LDS
constexpr size_t kLdsBudget2dCap = 80 * 1024;
// Points per set: permutation indices are int32, and the spreading and
// interpolation kernels form record indices up to a few hundred past a
// subproblem's start in 32-bit ints, so the limit keeps 2^16 of headroom.
constexpr int64_t kMaxPoints = ((int64_t)1 << 31) - ((int64_t)1 << 16);

size_t csize(int prec) { return prec == ESN_DOUBLE ? 2 * sizeof(double) : 2 * sizeof(float); }

int64_t nf_total(const esn_plan_s* p) { return p->nf[0] * p->nf[1] * p->nf[2]; }
int64_t n_total(const esn_plan_s* p) { return p->N[0] * p->N[1] * p->N[2]; }

size_t lds_budget(int device) {
  static int cached_dev = -1;
  static size_t cached = 0;
  if (cached_dev != device) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) !=
            hipSuccess ||
        v <= 0)
      v = 64 * 1024;
    cached = (size_t)v;
    cached_dev = device;
  }
  return std::min(cached, kLdsBudgetCap);
}

size_t lds_budget_2d(int device) {
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) !=
          hipSuccess ||
      v <= 0)
    v = 64 * 1024;
  return std::min((size_t)v, kLdsBudget2dCap);
}

int ceil_log2(int64_t n) {
  int k = 0;
  while (((int64_t)1 << k) < n) k++;
  return k;
}

// Device allocations of a plan, with their sizes kept for accounting.
// Plan memory comes from the stream-ordered allocator on the plan's stream:
// unlike hipMalloc / hipFree, allocating and freeing it does not wait for the
// whole device, so plans made and destroyed by one worker of a request loop
// do not stall the others.  A plan's first use of an allocation is on its own
// stream, and plan creation ends with a synchronisation of that stream, so
// the memory is ready for any stream the plan moves to.
// Memory given back to the stream-ordered allocator stays in its pool up to
// this much (per device) instead of returning to the system at the next
// synchronisation, so that plans that make and free their working buffers at
// every request (a request loop's cached plans) reuse pool memory.
constexpr uint64_t kPoolKeepBytes = (uint64_t)16 << 30;

void keep_pool_memory(int device) {
  static std::mutex mu;
  static std::vector<int> done;
  std::lock_guard<std::mutex> lk(mu);
  if (std::find(done.begin(), done.end(), device) != done.end()) return;
  done.push_back(device);
  hipMemPool_t pool = nullptr;
  if (hipDeviceGetDefaultMemPool(&pool, device) != hipSuccess || !pool) {
    (void)hipGetLastError();
    return;
  }
  uint64_t keep = kPoolKeepBytes;
  if (hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep) != hipSuccess)
    (void)hipGetLastError();
}

int dalloc(esn_plan_s* p, void** ptr, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (hipMallocAsync(ptr, bytes, p->stream) != hipSuccess) {
    *ptr = nullptr;
    (void)hipGetLastError();
    return ESN_ERR_ALLOC;
  }
  p->allocs.emplace_back(*ptr, bytes);
  p->device_bytes += (int64_t)bytes;
  return ESN_OK;
}

void dfree(esn_plan_s* p, void** ptr) {
  if (*ptr) {
    for (size_t i = 0; i < p->allocs.size(); i++) {
      if (p->allocs[i].first == *ptr) {
        p->device_bytes -= (int64_t)p->allocs[i].second;
        p->allocs.erase(p->allocs.begin() + i);
        break;
      }
    }
    (void)hipFreeAsync(*ptr, p->stream);
  }
  *ptr = nullptr;
}

// Small pinned host slots for the plans' read-backs (32 bytes each), carved
// from pinned pages that stay for the process (hipHostFree would wait for
// the device).
std::mutex g_pin_mu;
std::vector<int32_t*> g_pin_free;

int32_t* pinned_slot_get() {
  std::lock_guard<std::mutex> lk(g_pin_mu);
  if (g_pin_free.empty()) {
    void* page = nullptr;
    if (hipHostMalloc(&page, 4096, hipHostMallocDefault) != hipSuccess) return nullptr;
    for (int i = 0; i < 4096 / 32; i++) g_pin_free.push_back(static_cast<int32_t*>(page) + 8 * i);
  }
  int32_t* slot = g_pin_free.back();
  g_pin_free.pop_back();
  return slot;
}

void pinned_slot_put(int32_t* slot) {
  if (!slot) return;
  std::lock_guard<std::mutex> lk(g_pin_mu);
  g_pin_free.push_back(slot);
}

#define ESN_HIP(call)                         \
  do {                                        \
    hipError_t e_ = (call);                   \
    if (e_ != hipSuccess) return ESN_ERR_HIP; \
  } while (0)

#define ESN_TRY(call)               \
  do {                              \
    int s_ = (call);                \
    if (s_ >= 2) return s_;         \
  } while (0)

void default_bins(int dim, int* b) {
  if (dim == 1) { b[0] = 1024; b[1] = 1; b[2] = 1; }
  else if (dim == 2) { b[0] = 32; b[1] = 32; b[2] = 1; }
  else { b[0] = 8; b[1] = 8; b[2] = 8; }
}

GeomArgs make_geom(const esn_plan_s* p, int ntr) {
  GeomArgs g;
  for (int m = 0; m < 3; m++) {
    g.n[m] = p->nf[m];
    g.b[m] = p->bin[m];
    g.nb[m] = p->nb[m];
    g.fbits[m] = p->fbits[m];
  }
  g.pts_code = p->pts_code;
  g.beta = p->par.beta;
  g.M = p->M;
  g.ntr = ntr;
  g.cstride = p->M;
  g.gstride = nf_total(p);
  g.pts = p->d_pts;
  g.sub_bin = p->d_sub_bin;
  g.sub_start = p->d_sub_start;
  g.sub_len = p->d_sub_len;
  g.nsub = p->nsub;
  g.ktab = p->kerevalmeth == 2 ? p->d_ktab : nullptr;
  return g;
}

void free_points(esn_plan_s* p) {
  dfree(p, (void**)&p->d_pts);
  dfree(p, (void**)&p->d_ckey);
  dfree(p, &p->d_rscratch);
  dfree(p, (void**)&p->d_slot);
  p->rscratch_bytes = 0;
  p->cap_M = p->cap_count = 0;
}

void free_subs(esn_plan_s* p) {
  dfree(p, (void**)&p->d_sub_bin);
  dfree(p, (void**)&p->d_sub_start);
  dfree(p, (void**)&p->d_sub_len);
  p->cap_sub = 0;
}

// The fine grid (chunk transforms) and the FFT work buffers, made again after
// plan_trim gave them back.
int ensure_exec_buffers(esn_plan_s* p) {
  if (!p->spread_only && !p->d_grid &&
      dalloc(p, &p->d_grid, (size_t)nf_total(p) * csize(p->prec) * p->chunk) != ESN_OK)
    return ESN_ERR_ALLOC;
  for (FFTPlan* f : {&p->fft, &p->fft_tail, &p->fft_adj, &p->fft_adj_tail}) {
    const bool had = f->work != nullptr;
    const int rc = fft_ensure_work(f);
    if (rc != ESN_OK) return rc;
    if (!had && f->work) p->device_bytes += (int64_t)f->work_bytes;
  }
  return ESN_OK;
}



// The next timing record of a debug plan (its events created on first use),
// or null when timing is off or an event cannot be made.
TimingRec* timing_next(esn_plan_s* p, int kind) {
  if (!p->opts.debug) return nullptr;
  if (p->ring.empty()) p->ring.resize(kTimingRing);
  TimingRec& r = p->ring[p->ring_count % kTimingRing];
  // timing-only events: no system-scope fence (cache writeback and
  // invalidation) when they are reached
  for (auto& e : r.e)
    if (!e && hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess)
      return nullptr;
  r.kind = kind;
  r.vals = esn_stats{};
  p->ring_count++;
  return &r;
}

// Stage times of one record (waits for its last event).
int timing_values(TimingRec& r, esn_stats* out) {
  *out = esn_stats{};
  float a = 0, b = 0, c = 0, t = 0;
  switch (r.kind) {
    case 1:
      if (hipEventSynchronize(r.e[1]) != hipSuccess ||
          hipEventElapsedTime(&t, r.e[0], r.e[1]) != hipSuccess)
        return ESN_ERR_HIP;
      out->t_setpts = t;
      return ESN_OK;
    case 2:
    case 3:
      if (hipEventSynchronize(r.e[4]) != hipSuccess ||
          hipEventElapsedTime(&a, r.e[0], r.e[1]) != hipSuccess ||
          hipEventElapsedTime(&b, r.e[1], r.e[2]) != hipSuccess ||
          hipEventElapsedTime(&c, r.e[2], r.e[3]) != hipSuccess ||
          hipEventElapsedTime(&t, r.e[5], r.e[4]) != hipSuccess)
        return ESN_ERR_HIP;
      // type 1 direction: spread, FFT, deconvolve; type 2: amplify, FFT, interpolate
      out->t_spread_or_interp = r.kind == 2 ? a : c;
      out->t_deconv_or_amplify = r.kind == 2 ? c : a;
      out->t_fft = b;
      out->t_execute = t;
      return ESN_OK;
    case 4:
      *out = r.vals;
      return ESN_OK;
    default:
      return ESN_OK;
  }
}

void destroy_all(esn_plan_s* p) {
  (void)hipStreamSynchronize(p->stream);
  free_points(p);
  free_subs(p);
  for (int m = 0; m < 3; m++) dfree(p, (void**)&p->d_pf[m]);
  dfree(p, &p->d_grid);
  dfree(p, (void**)&p->d_bend);
  dfree(p, (void**)&p->d_bstart);
  dfree(p, (void**)&p->d_count);
  dfree(p, (void**)&p->d_sstart);
  dfree(p, (void**)&p->d_cell_scan_tmp);
  dfree(p, (void**)&p->d_nsub);
  dfree(p, (void**)&p->d_tiles);
  dfree(p, (void**)&p->d_flags);
  dfree(p, &p->d_ktab);
  pinned_slot_put(p->h_pinned);
  p->h_pinned = nullptr;
  fft_destroy(&p->fft);
  fft_destroy(&p->fft_tail);
  fft_destroy(&p->fft_adj);
  fft_destroy(&p->fft_adj_tail);
  for (auto& e : p->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& r : p->ring)
    for (auto& e : r.e)
      if (e) (void)hipEventDestroy(e);
  // anything still tracked (none is expected)
  for (auto& a : p->allocs) (void)hipFreeAsync(a.first, p->stream);
  p->allocs.clear();
  p->device_bytes = 0;
}

}  // namespace

extern "C" void esn_default_opts(esn_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->debug = 0;
  o->chkbnds = 1;
  o->modeord = 0;
  o->upsampfac = 2.0;
  o->sort = 1;
}

extern "C" const char* esn_strerror(int s) {
  switch (s) {
    case ESN_OK: return "success";
    case ESN_WARN_EPS_TOO_SMALL: return "warning: tolerance beyond what the precision supports";
    case ESN_ERR_BAD_ARG: return "invalid argument";
    case ESN_ERR_PTS_OUT_OF_RANGE: return "a point coordinate lies outside [-3pi, 3pi]";
    case ESN_ERR_NAN_PTS: return "a point coordinate is NaN or infinite";
    case ESN_ERR_BUDGET: return "request exceeds the device memory budget";
    case ESN_ERR_ALLOC: return "device memory allocation failed";
    case ESN_ERR_FFT_PLAN: return "rocFFT plan or execution failed";
    case ESN_ERR_HIP: return "HIP runtime error";
    case ESN_ERR_UNSUPPORTED: return "unsupported request";
    case ESN_ERR_NO_POINTS: return "no points set (call esn_setpts first)";
    case ESN_ERR_QUEUE: return "unknown ticket or server stopped";
    default: return "unknown status";
  }
}

extern "C" int esn_makeplan(int type, int dim, const int64_t* nmodes, int isign, int ntransf,
                            double eps, int prec, esn_plan* out, const esn_opts* opts,
                            void* stream) {
  if (!out) return ESN_ERR_BAD_ARG;
  *out = nullptr;
  if (type == 3) return t3_makeplan(dim, isign, ntransf, eps, prec, out, opts, stream);
  return esn::make_plan(type, dim, nmodes, isign, ntransf, eps, prec, out, opts, stream, false);
}

int esn::make_plan(int type, int dim, const int64_t* nmodes, int isign, int ntransf, double eps,
                   int prec, esn_plan* out, const esn_opts* opts, void* stream, bool spread_only) {
  if (!out) return ESN_ERR_BAD_ARG;
  *out = nullptr;
  if ((type != 1 && type != 2) || dim < 1 || dim > 3 || !nmodes || ntransf < 1 ||
      (isign != 1 && isign != -1))
    return ESN_ERR_BAD_ARG;
  esn_opts o;
  if (opts) o = *opts;
  else esn_default_opts(&o);
  if (o.modeord != 0 && o.modeord != 1) return ESN_ERR_BAD_ARG;
  esn_params par;
  int st = esn_choose_params(eps, prec, dim, nmodes, o.upsampfac, &par);
  if (st >= 2) return st;
  for (int m = 0; m < dim; m++)
    if (nmodes[m] > (int64_t)1 << 30 || par.nf[m] > (int64_t)1 << 31) return ESN_ERR_BAD_ARG;
  if (o.bin[0] < 0 || o.bin[1] < 0 || o.bin[2] < 0 || o.maxsubprob < 0 ||
      o.ntransf_chunk < 0 || o.block < 0 || o.block > 1024 ||
      (o.block != 0 && o.block % 64 != 0) || o.spread_method < 0 || o.spread_method > 3 ||
      o.interp_method < 0 || o.interp_method > 3 || o.sort < 0 || o.sort > 3 ||
      o.kerevalmeth < 0 || o.kerevalmeth > 2)
    return ESN_ERR_BAD_ARG;

  esn_plan_s* p = new (std::nothrow) esn_plan_s();
  if (!p) return ESN_ERR_ALLOC;
  p->type = type;
  p->dim = dim;
  p->isign = isign;
  p->ntransf = ntransf;
  p->prec = prec;
  p->eps = eps;
  p->par = par;
  p->opts = o;
  p->warn = st;
  p->stream = (hipStream_t)stream;
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return ESN_ERR_HIP;
  }
  keep_pool_memory(p->device);
  for (int m = 0; m < 3; m++) {
    p->N[m] = m < dim ? nmodes[m] : 1;
    p->nf[m] = par.nf[m];
  }
  const int w = par.w;

  // ---- point storage ----
  bool fixed = prec == ESN_SINGLE;
  for (int m = 0; m < dim; m++)
    if (p->nf[m] > 8192) fixed = false;
  p->pts_code = fixed ? kPtsFixed32 : kPtsF64;
  for (int m = 0; m < 3; m++) p->fbits[m] = m < dim ? 32 - ceil_log2(p->nf[m]) : 24;

  // ---- bins, subproblems, methods, chunk ----
  default_bins(dim, p->bin);
  // 2D tiles: small bins keep several waves per CU on the LDS tiles (measured
  // on 1e7 uniform points, 2000^2 grids: 16 x 8 spreads in half the time of
  // 32 x 32; interpolation is best at 16 x 16)
  if (dim == 2) {
    p->bin[0] = 16;
    p->bin[1] = type == 1 ? 8 : 16;
  }
  // the matrix-core kernels (3D single precision, w <= 7) work best on small
  // bins: 8 x 4 x 4 (measured at M = 1e7 on 256^3 and 288^3 fine grids, with
  // clustered, uniform and half-box uniform points, for both kernels)
  const bool mfma_candidate = dim == 3 && prec == ESN_SINGLE && w <= 7 && o.sort &&
                              o.spread_method != 1 && o.spread_method != 2 &&
                              o.interp_method != 1 && o.interp_method != 2;
  if (mfma_candidate) {
    p->bin[0] = 8;
    p->bin[1] = 4;
    p->bin[2] = 4;
  }
  for (int m = 0; m < dim; m++) {
    if (o.bin[m] > 0) p->bin[m] = o.bin[m];
    p->bin[m] = (int)std::min<int64_t>(p->bin[m], p->nf[m]);
  }
  const size_t budget = lds_budget(p->device);
  const size_t budget2d = lds_budget_2d(p->device);
  bool user_bins = o.bin[0] > 0 || o.bin[1] > 0 || o.bin[2] > 0;
  while (!user_bins && tile_lds_bytes(prec, dim, w, p->bin, 1) > budget) {
    int mx = 0;
    for (int m = 1; m < dim; m++)
      if (p->bin[m] > p->bin[mx]) mx = m;
    if (p->bin[mx] <= 1) break;
    p->bin[mx] /= 2;
  }
  for (int m = 0; m < 3; m++) {
    if (m >= dim) p->bin[m] = 1;
    p->nb[m] = (int)((p->nf[m] + p->bin[m] - 1) / p->bin[m]);
  }
  p->nbins = (int64_t)p->nb[0] * p->nb[1] * p->nb[2];
  if (p->nbins > (int64_t)1 << 30) {
    delete p;
    return ESN_ERR_BAD_ARG;
  }
  p->maxsub = o.maxsubprob > 0 ? o.maxsubprob : 1024;
  p->block = o.block > 0 ? o.block : 256;
  const bool tile_fits = tile_lds_bytes(prec, dim, w, p->bin, 1) <= budget;
  // matrix-core spreading / interpolation: 3D single precision, w <= 7,
  // fixed-point coordinates, even bin sizes, one transform per launch (method 3)
  const bool mfma3d_ok = dim == 3 && prec == ESN_SINGLE && w <= 7 && o.sort &&
                         p->pts_code == kPtsFixed32 && p->bin[0] % 2 == 0 &&
                         p->bin[1] % 2 == 0 && p->bin[2] % 2 == 0 &&
                         mfma_spread_lds_bytes(w, p->bin) <= budget &&
                         mfma_interp_lds_bytes(p->bin) <= budget;
  // 2D on the matrix cores: w <= 13, bins of whole blocks of window cells
  const int bs2 = mfma2d_block(w);
  const bool mfma2d_ok = dim == 2 && w <= 13 && o.sort && p->bin[0] % bs2 == 0 &&
                         p->bin[1] % bs2 == 0 &&
                         mfma2d_lds_bytes(prec, w, p->bin, 1, true) <= budget2d;
  const bool mfma_ok = mfma3d_ok || mfma2d_ok;
  // defaults: the matrix cores where they measured faster than the LDS tiles
  // (3D single precision both ways; 2D double precision spreading, 1e7 points
  // on a 2000^2 grid at w = 10: 1.13 ms against 2.40 ms).  In 2D single
  // precision spreading the two tie (0.46 ms at w = 6) and interpolation is
  // faster on the LDS tiles (0.29 / 0.48 ms against 0.42 / 0.89 ms).
  const bool mfma_spread = mfma3d_ok || (mfma2d_ok && prec == ESN_DOUBLE);
  const bool mfma_interp = mfma3d_ok;
  p->spread_method =
      o.spread_method ? o.spread_method : (mfma_spread ? 3 : (tile_fits ? 1 : 2));
  p->interp_method =
      o.interp_method ? o.interp_method : (mfma_interp ? 3 : (tile_fits ? 1 : 2));
  if ((p->spread_method == 3 || p->interp_method == 3) && !mfma_ok) {
    delete p;
    return ESN_ERR_BAD_ARG;
  }
  const bool mfma = (type == 1 && p->spread_method == 3) || (type == 2 && p->interp_method == 3);
  if (mfma && dim == 3 && o.maxsubprob <= 0) p->maxsub = type == 1 ? 1024 : 512;
  if (!o.sort) p->spread_method = p->interp_method = 2;
  if (!tile_fits) {
    if (p->spread_method == 1 || p->interp_method == 1) {
      delete p;
      return ESN_ERR_BAD_ARG;   // requested LDS method cannot hold one tile
    }
  }
  const bool uses_lds = (type == 1 && (p->spread_method == 1 || p->spread_method == 3)) ||
                        (type == 2 && (p->interp_method == 1 || p->interp_method == 3));
  int chunk = o.ntransf_chunk > 0 ? o.ntransf_chunk : ntransf;
  // 3D matrix-core kernels: one transform per launch.  (Two per launch, the
  // staged weights shared and a tile each, measured 1.05x (spreading) and
  // 0.96x (interpolation) against one at a time on the 1e7-point clustered
  // set: the weights are a small part of these kernels, and the second tile
  // halves the blocks per CU.)
  if (mfma && dim == 3) chunk = 1;
  if (mfma && dim == 2) {
    // transforms share a launch's staged weights, each with its own LDS tile
    int lim = 1;
    while (lim < ntransf && mfma2d_lds_bytes(prec, w, p->bin, lim + 1, type == 1) <= budget2d)
      lim++;
    if (o.ntransf_chunk <= 0) chunk = std::min(chunk, lim);
    else if (mfma2d_lds_bytes(prec, w, p->bin, std::min(chunk, ntransf), type == 1) > budget2d) {
      delete p;
      return ESN_ERR_BAD_ARG;
    }
  } else if (uses_lds) {
    size_t one = tile_lds_bytes(prec, dim, w, p->bin, 1);
    int lim = (int)std::max<size_t>(1, budget / one);
    if (o.ntransf_chunk <= 0) chunk = std::min(chunk, lim);
    else if (tile_lds_bytes(prec, dim, w, p->bin, std::min(chunk, ntransf)) > budget) {
      delete p;
      return ESN_ERR_BAD_ARG;
    }
  }
  // keep the fused grids within 16 GiB
  const size_t gbytes = (size_t)nf_total(p) * csize(prec);
  int memlim = (int)std::max<size_t>(1, ((size_t)16 << 30) / std::max<size_t>(gbytes, 1));
  chunk = std::max(1, std::min({chunk, ntransf, memlim}));
  p->chunk = chunk;
  p->tail = ntransf % chunk;


  int rc = ESN_OK;
  hipStream_t s = p->stream;
  auto fail = [&](int code) {
    destroy_all(p);
    delete p;
    return code;
  };

  // ---- kernel evaluation: exp and sqrt at every weight, or the piecewise
  // polynomial table of Sec. 5.3.  Automatic: the table in double precision,
  // where exp and sqrt are long FP64 instruction sequences, and exp and sqrt
  // in single precision, where each is one hardware instruction.
  p->kerevalmeth = o.kerevalmeth ? o.kerevalmeth : (prec == ESN_DOUBLE ? 2 : 1);
  if (p->kerevalmeth == 2) {
    std::vector<double> tab((size_t)w * (w + kPolyExtra + 1));
    if (esn_kernel_poly(w, par.beta, tab.data()) != ESN_OK) return fail(ESN_ERR_BAD_ARG);
    if (prec == ESN_DOUBLE) {
      if (dalloc(p, &p->d_ktab, tab.size() * sizeof(double)) != ESN_OK ||
          hipMemcpyAsync(p->d_ktab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, s) !=
              hipSuccess)
        return fail(ESN_ERR_ALLOC);
    } else {
      const std::vector<float> tf(tab.begin(), tab.end());
      if (dalloc(p, &p->d_ktab, tf.size() * sizeof(float)) != ESN_OK ||
          hipMemcpyAsync(p->d_ktab, tf.data(), tf.size() * sizeof(float), hipMemcpyHostToDevice, s) !=
              hipSuccess)
        return fail(ESN_ERR_ALLOC);
    }
  }

  // ---- correction factors p(k) per dim (FP64 quadrature on the GPU) ----
  {
    std::vector<double> nodes, weights;
    gauss_legendre_positive(par.nquad, &nodes, &weights);
    double* d_q = nullptr;
    if (dalloc(p, (void**)&d_q, sizeof(double) * 2 * par.nquad) != ESN_OK) return fail(ESN_ERR_ALLOC);
    std::vector<double> qw(nodes);
    qw.insert(qw.end(), weights.begin(), weights.end());
    if (hipMemcpyAsync(d_q, qw.data(), sizeof(double) * qw.size(), hipMemcpyHostToDevice, s) !=
        hipSuccess)
      return fail(ESN_ERR_HIP);
    for (int m = 0; m < 3; m++) {
      int64_t K = p->N[m] / 2 + 1;
      if (dalloc(p, (void**)&p->d_pf[m], sizeof(double) * K) != ESN_OK) return fail(ESN_ERR_ALLOC);
      if (m < dim) {
        if (launch_fseries(w, par.beta, d_q, d_q + par.nquad, par.nquad, p->nf[m], p->N[m],
                           p->d_pf[m], s) != hipSuccess)
          return fail(ESN_ERR_HIP);
      } else {
        const double one = 1.0;
        if (hipMemcpyAsync(p->d_pf[m], &one, sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess)
          return fail(ESN_ERR_HIP);
      }
    }
    if (hipStreamSynchronize(s) != hipSuccess) return fail(ESN_ERR_HIP);
    dfree(p, (void**)&d_q);
  }

  // ---- fine grid and FFT plans (none for a plan that only spreads into
  // caller grids) ----
  if (!spread_only) {
    if (dalloc(p, &p->d_grid, gbytes * chunk) != ESN_OK) return fail(ESN_ERR_ALLOC);
    rc = fft_make(&p->fft, dim, p->nf, p->N, type, chunk, prec, isign, s);
    if (rc != ESN_OK) return fail(rc);
    if (p->tail) {
      rc = fft_make(&p->fft_tail, dim, p->nf, p->N, type, p->tail, prec, isign, s);
      if (rc != ESN_OK) return fail(rc);
    }
    p->device_bytes += (int64_t)(p->fft.work_bytes + p->fft_tail.work_bytes);
  }
  p->spread_only = spread_only;

  // ---- per-cell / per-bin arrays ----
  {
    const int64_t cpb = (int64_t)p->bin[0] * p->bin[1] * p->bin[2];
    const int64_t ncells = p->nbins * cpb;
    if (ncells + 1 > (int64_t)1 << 31) return fail(ESN_ERR_BAD_ARG);
    p->ncells = ncells;
    p->key_bits = 0;
    while (((int64_t)1 << p->key_bits) < ncells) p->key_bits++;
    if (dalloc(p, (void**)&p->d_bend, 4 * p->nbins) ||
        dalloc(p, (void**)&p->d_bstart, 4 * (p->nbins + 1)) ||
        dalloc(p, (void**)&p->d_nsub, 4 * p->nbins) ||
        dalloc(p, (void**)&p->d_tiles, 4 * 3 * bin_tiles(p->nbins)) ||
        dalloc(p, (void**)&p->d_flags, 4 * 4))
      return fail(ESN_ERR_ALLOC);
  }
  if (!(p->h_pinned = pinned_slot_get()))
    return fail(ESN_ERR_ALLOC);
  // the plan's memory (stream-ordered) and tables are ready for any stream
  if (hipStreamSynchronize(s) != hipSuccess) return fail(ESN_ERR_HIP);
  *out = p;
  return p->warn;
}

// Geometry of the plan's bin sort for M points with coordinates xs.
static SortArgs sort_args(const esn_plan_s* p, int64_t M, int coord_prec, const void* const* xs) {
  SortArgs a;
  std::memset(&a, 0, sizeof(a));
  a.dim = p->dim;
  a.M = M;
  a.coord_prec = coord_prec;
  for (int m = 0; m < 3; m++) {
    a.x[m] = (xs && m < p->dim) ? xs[m] : nullptr;
    a.n[m] = p->nf[m];
    a.inv_n[m] = 1.0 / (double)p->nf[m];
    a.scale[m] = (double)p->nf[m] * 0.15915494309189533577;   // n / 2pi
    a.span[m] = std::ldexp((double)p->nf[m], p->fbits[m]);
    a.pow2f[m] = std::ldexp(1.0, p->fbits[m]);
    a.b[m] = p->bin[m];
    a.nb[m] = p->nb[m];
    a.fbits[m] = p->fbits[m];
  }
  a.pts_code = p->pts_code;
  a.chkbnds = p->opts.chkbnds;
  a.w = p->par.w;
  a.blocked = p->dim == 3 && p->bin[0] % 2 == 0 && p->bin[1] % 2 == 0;
  {
    const int bs2 = mfma2d_block(p->par.w);
    a.blocked2d = (p->dim == 2 && p->bin[0] % bs2 == 0 && p->bin[1] % bs2 == 0) ? bs2 : 0;
  }
  a.bpow2 = 1;
  for (int m = 0; m < 3; m++) {
    int sh = 0;
    while ((1 << sh) < p->bin[m]) sh++;
    a.bshift[m] = sh;
    if ((1 << sh) != p->bin[m]) a.bpow2 = 0;
  }
  return a;
}

extern "C" int esn_setpts(esn_plan p, int64_t M, int coord_prec, const void* x, const void* y,
                          const void* z) {
  const void* xs[3] = {x, y, z};
  return esn::setpts_impl(p, M, coord_prec, xs, nullptr, 0);
}

// setpts; with ext_scratch set, the sort's scratch is ext_scratch
// (ext_bytes bytes), the sort is the radix sort, and nothing is allocated:
// the plan must already hold room for M points and their subproblems.
int esn::setpts_impl(esn_plan p, int64_t M, int coord_prec, const void* const* xs,
                     void* ext_scratch, size_t ext_bytes) {
  if (!p || p->type == 3 || M < 0 || M > kMaxPoints) return ESN_ERR_BAD_ARG;
  if (coord_prec != ESN_SINGLE && coord_prec != ESN_DOUBLE) return ESN_ERR_BAD_ARG;
  if (M > 0)
    for (int m = 0; m < p->dim; m++)
      if (!xs[m]) return ESN_ERR_BAD_ARG;
  const bool noalloc = ext_scratch != nullptr;
  // bin sort method: the radix sort's fixed cost dominates for small point
  // sets, the counting sort's scattered atomics for large ones
  int method = 0;
  if (noalloc)
    method = p->opts.sort ? 2 : 0;
  else if (p->opts.sort == 1)
    method = (M < ((int64_t)1 << 21) && p->ncells < ((int64_t)1 << 23)) ? 3 : 2;
  else if (p->opts.sort >= 2)
    method = p->opts.sort;
  const size_t rbytes = (size_t)pts_record_bytes(p->pts_code);
  void* scratch = p->d_rscratch;
  size_t scratch_bytes = p->rscratch_bytes;
  if (noalloc) {
    if (M > p->cap_M) return ESN_ERR_BAD_ARG;
    if (method && std::min<int64_t>(p->nbins, M) + M / p->maxsub + 1 > p->cap_sub)
      return ESN_ERR_BAD_ARG;
    if (method == 2 && radix_scratch_bytes(M, p->key_bits, (int)rbytes) > ext_bytes)
      return ESN_ERR_BAD_ARG;
    scratch = ext_scratch;
    scratch_bytes = ext_bytes;
  }
  ESN_HIP(hipSetDevice(p->device));
  hipStream_t s = p->stream;
  p->M = -1;
  TimingRec* tr = timing_next(p, 1);
  if (tr) ESN_HIP(hipEventRecord(tr->e[0], s));
  if (M > p->cap_M) {
    free_points(p);
    if (dalloc(p, (void**)&p->d_pts, rbytes * M)) return ESN_ERR_ALLOC;
    p->cap_M = M;
  }
  if (method == 2 && !noalloc) {
    const size_t need = radix_scratch_bytes(p->cap_M, p->key_bits, (int)rbytes);
    if (need > p->rscratch_bytes) {
      dfree(p, &p->d_rscratch);
      p->rscratch_bytes = 0;
      if (dalloc(p, &p->d_rscratch, need)) return ESN_ERR_ALLOC;
      p->rscratch_bytes = need;
    }
    scratch = p->d_rscratch;
    scratch_bytes = p->rscratch_bytes;
  }
  if (method == 3) {
    if (!p->d_count) {
      if (dalloc(p, (void**)&p->d_count, 4 * (p->ncells + 1)) ||
          dalloc(p, (void**)&p->d_sstart, 4 * (p->ncells + 1)) ||
          dalloc(p, (void**)&p->d_cell_scan_tmp, 4 * (scan_tmp_elems(p->ncells + 1) + 1)))
        return ESN_ERR_ALLOC;
    }
    if (M > p->cap_count) {
      dfree(p, (void**)&p->d_slot);
      dfree(p, (void**)&p->d_ckey);
      if (dalloc(p, (void**)&p->d_slot, 4 * p->cap_M) || dalloc(p, (void**)&p->d_ckey, 4 * p->cap_M))
        return ESN_ERR_ALLOC;
      p->cap_count = p->cap_M;
    }
  }
  SortArgs a = sort_args(p, M, coord_prec, xs);
  a.key = p->d_ckey;
  a.slot = p->d_slot;
  a.count = p->d_count;
  a.sstart = p->d_sstart;
  a.pts = p->d_pts;
  a.flags = p->d_flags;
  ESN_HIP(hipMemsetAsync(p->d_flags, 0, 16, s));
  int nsub = 0;
  const int64_t cpb = (int64_t)p->bin[0] * p->bin[1] * p->bin[2];
  p->last_sort = method;
  if (method) {
    // every subproblem list fits min(nbins, M) + M / maxsub entries
    const int64_t cap = std::min<int64_t>(p->nbins, M) + M / p->maxsub + 1;
    if (cap > p->cap_sub) {
      free_subs(p);
      if (dalloc(p, (void**)&p->d_sub_bin, 4 * (size_t)cap) ||
          dalloc(p, (void**)&p->d_sub_start, 4 * (size_t)cap) ||
          dalloc(p, (void**)&p->d_sub_len, 4 * (size_t)cap))
        return ESN_ERR_ALLOC;
      p->cap_sub = cap;
    }
  }
  if (method == 2) {
    ESN_HIP(hipMemsetAsync(p->d_bend, 0, 4 * p->nbins, s));
    uint32_t* skey = nullptr;
    ESN_HIP(radix_sort_points(a, p->key_bits, p->d_pts, scratch, scratch_bytes, &skey, s));
    ESN_HIP(launch_bin_ends(skey, M, (int)cpb, p->d_bend, s));
    ESN_HIP(launch_bin_subproblems(p->d_bend, p->d_bstart, p->nbins, M, p->maxsub, p->d_nsub,
                                   p->d_tiles, p->d_sub_bin, p->d_sub_start, p->d_sub_len,
                                   p->d_flags + 1, s));
  } else if (method == 3) {
    ESN_HIP(hipMemsetAsync(p->d_count, 0, 4 * (p->ncells + 1), s));
    ESN_HIP(launch_bin_count(a, s));
    ESN_HIP(exclusive_scan_i32(p->d_count, p->d_sstart, p->ncells + 1, p->d_cell_scan_tmp, s));
    ESN_HIP(launch_scatter(a, s));
    ESN_HIP(launch_bin_starts(p->d_sstart, cpb, p->nbins, p->d_bstart, s));
    ESN_HIP(launch_bin_subproblems(nullptr, p->d_bstart, p->nbins, M, p->maxsub, p->d_nsub,
                                   p->d_tiles, p->d_sub_bin, p->d_sub_start, p->d_sub_len,
                                   p->d_flags + 1, s));
  } else {
    ESN_HIP(launch_encode_unsorted(a, s));
  }
  // error flags, subproblem and nonempty-bin totals
  ESN_HIP(hipMemcpyAsync(p->h_pinned, p->d_flags, 12, hipMemcpyDeviceToHost, s));
  ESN_HIP(hipStreamSynchronize(s));
  const int flags = p->h_pinned[0];
  if (flags & 1) return ESN_ERR_NAN_PTS;
  if (flags & 2) return ESN_ERR_PTS_OUT_OF_RANGE;
  if (method) {
    nsub = p->h_pinned[1];
    p->nbins_nonempty = p->h_pinned[2];
  } else {
    p->nbins_nonempty = 0;
  }
  p->nsub = nsub;
  p->M = M;
  if (tr) ESN_HIP(hipEventRecord(tr->e[1], s));
  return ESN_OK;
}

static int run_spread(esn_plan_s* p, int ntr, const void* c, void* grid) {
  GeomArgs g = make_geom(p, ntr);
  if (p->spread_method == 3) {
    if (p->dim == 2)
      ESN_HIP(launch_spread_mfma2d(p->prec, p->par.w, g, p->nsub, c, grid, p->stream));
    else
      ESN_HIP(launch_spread_mfma(p->par.w, g, p->nsub, c, grid, p->stream));
    return ESN_OK;
  }
  size_t lds = p->spread_method == 1 ? tile_lds_bytes(p->prec, p->dim, p->par.w, p->bin, ntr) : 0;
  ESN_HIP(launch_spread(p->spread_method, p->prec, p->dim, p->par.w, g, p->nsub, p->block, lds, c,
                        grid, p->stream));
  return ESN_OK;
}

static int run_interp(esn_plan_s* p, int ntr, const void* grid, void* c) {
  GeomArgs g = make_geom(p, ntr);
  if (p->interp_method == 3) {
    if (p->dim == 2)
      ESN_HIP(launch_interp_mfma2d(p->prec, p->par.w, g, p->nsub, grid, c, p->stream));
    else
      ESN_HIP(launch_interp_mfma(p->par.w, g, p->nsub, grid, c, p->stream));
    return ESN_OK;
  }
  size_t lds = p->interp_method == 1 ? tile_lds_bytes(p->prec, p->dim, p->par.w, p->bin, ntr, false) : 0;
  ESN_HIP(launch_interp(p->interp_method, p->prec, p->dim, p->par.w, g, p->nsub, p->block, lds, grid,
                        c, p->stream));
  return ESN_OK;
}

// The rocFFT plans of the opposite sign and the transforms per launch for
// the adjoint direction dir (3 - type), made on the first adjoint call.
static int make_adjoint(esn_plan_s* p) {
  if (p->fft_adj.plan) return ESN_OK;
  const int dir = 3 - p->type;
  const int method = dir == 1 ? p->spread_method : p->interp_method;
  int chunk = p->chunk;
  if (method == 3 && p->dim == 3) {
    chunk = 1;
  } else if (method == 3) {
    const size_t budget = lds_budget_2d(p->device);
    chunk = std::max(1, chunk);
    while (chunk > 1 && mfma2d_lds_bytes(p->prec, p->par.w, p->bin, chunk, dir == 1) > budget)
      chunk--;
  } else if (method == 1) {
    const size_t budget = lds_budget(p->device);
    const size_t one = tile_lds_bytes(p->prec, p->dim, p->par.w, p->bin, 1, dir == 1);
    chunk = std::max(1, std::min(chunk, (int)std::max<size_t>(1, budget / one)));
    while (chunk > 1 && tile_lds_bytes(p->prec, p->dim, p->par.w, p->bin, chunk, dir == 1) > budget)
      chunk--;
  }
  chunk = std::max(1, std::min(chunk, p->ntransf));
  const int tail = p->ntransf % chunk;
  int rc = fft_make(&p->fft_adj, p->dim, p->nf, p->N, 3 - p->type, chunk, p->prec, -p->isign,
                    p->stream);
  if (rc == ESN_OK && tail)
    rc = fft_make(&p->fft_adj_tail, p->dim, p->nf, p->N, 3 - p->type, tail, p->prec, -p->isign,
                  p->stream);
  if (rc != ESN_OK) {
    fft_destroy(&p->fft_adj);
    fft_destroy(&p->fft_adj_tail);
    return rc;
  }
  p->device_bytes += (int64_t)(p->fft_adj.work_bytes + p->fft_adj_tail.work_bytes);
  p->adj_chunk = chunk;
  p->adj_tail = tail;
  return ESN_OK;
}

// Transforms of direction dir (1: spread, FFT, deconvolve; 2: amplify, FFT,
// interpolate) on the plan's sorted points.  dir == type is the plan's own
// transform, the other direction its adjoint (opposite exponent sign).
static int execute_dir(esn_plan_s* p, int dir, void* c, void* f) {
  if (p->M < 0) return ESN_ERR_NO_POINTS;
  if ((p->M > 0 && !c) || !f) return ESN_ERR_BAD_ARG;
  ESN_HIP(hipSetDevice(p->device));
  const bool adj = dir != p->type;
  if (adj) ESN_TRY(make_adjoint(p));
  ESN_TRY(ensure_exec_buffers(p));
  const int chunk = adj ? p->adj_chunk : p->chunk;
  FFTPlan* fft_full = adj ? &p->fft_adj : &p->fft;
  FFTPlan* fft_last = adj ? &p->fft_adj_tail : &p->fft_tail;
  hipStream_t s = p->stream;
  const size_t cs = csize(p->prec);
  const int64_t G = nf_total(p), Nt = n_total(p);
  const double* pf[3] = {p->d_pf[0], p->d_pf[1], p->d_pf[2]};
  double t_a = 0, t_fft = 0, t_b = 0;
  // one chunk: events only, read when asked; several: timed chunk by chunk here
  const bool multi = p->ntransf > chunk;
  TimingRec* tr = timing_next(p, multi ? 4 : (dir == 1 ? 2 : 3));
  hipEvent_t* e = tr ? tr->e : nullptr;
  if (e) ESN_HIP(hipEventRecord(e[5], s));
  for (int c0 = 0; c0 < p->ntransf; c0 += chunk) {
    const int ntr = std::min(chunk, p->ntransf - c0);
    FFTPlan* fp = ntr == chunk ? fft_full : fft_last;
    char* cc = static_cast<char*>(c) + (size_t)c0 * p->M * cs;
    char* ff = static_cast<char*>(f) + (size_t)c0 * Nt * cs;
    // column FFT plans fold the correction (deconv / amplify) into their z
    // pass; its time then counts as FFT time
    ColModes cm;
    if (fp->modes) {
      cm.fstride = Nt;
      for (int m = 0; m < 3; m++) {
        cm.N[m] = p->N[m];
        cm.pf[m] = pf[m];
      }
      cm.n0 = p->nf[0];
      cm.n1 = p->nf[1];
      cm.modeord = p->opts.modeord;
    }
    if (dir == 1) {
      ESN_HIP(hipMemsetAsync(p->d_grid, 0, (size_t)ntr * G * cs, s));
      if (e) ESN_HIP(hipEventRecord(e[0], s));
      ESN_TRY(run_spread(p, ntr, cc, p->d_grid));
      if (e) ESN_HIP(hipEventRecord(e[1], s));
      if (fp->modes) {
        ESN_TRY(fft_exec_modes(fp, p->d_grid, ff, cm));
        if (e) ESN_HIP(hipEventRecord(e[2], s));
      } else {
        ESN_TRY(fft_exec(fp, p->d_grid));
        if (e) ESN_HIP(hipEventRecord(e[2], s));
        ESN_HIP(launch_deconv(p->prec, p->dim, p->N, p->nf, p->opts.modeord, ntr, p->d_grid, G,
                              ff, Nt, pf, s));
      }
    } else {
      if (e) ESN_HIP(hipEventRecord(e[0], s));
      if (fp->modes) {
        if (e) ESN_HIP(hipEventRecord(e[1], s));
        ESN_TRY(fft_exec_modes(fp, p->d_grid, ff, cm));
      } else {
        ESN_HIP(launch_amplify(p->prec, p->dim, p->N, p->nf, p->opts.modeord, ntr, p->d_grid, G,
                               ff, Nt, pf, s));
        if (e) ESN_HIP(hipEventRecord(e[1], s));
        ESN_TRY(fft_exec(fp, p->d_grid));
      }
      if (e) ESN_HIP(hipEventRecord(e[2], s));
      ESN_TRY(run_interp(p, ntr, p->d_grid, cc));
    }
    if (e) ESN_HIP(hipEventRecord(e[3], s));
    if (e && multi) {
      ESN_HIP(hipEventSynchronize(e[3]));
      float a = 0, b = 0, d = 0;
      ESN_HIP(hipEventElapsedTime(&a, e[0], e[1]));
      ESN_HIP(hipEventElapsedTime(&b, e[1], e[2]));
      ESN_HIP(hipEventElapsedTime(&d, e[2], e[3]));
      t_a += a; t_fft += b; t_b += d;
    }
  }
  if (e) {
    ESN_HIP(hipEventRecord(e[4], s));
    if (multi) {
      ESN_HIP(hipEventSynchronize(e[4]));
      float tot = 0;
      ESN_HIP(hipEventElapsedTime(&tot, e[5], e[4]));
      esn_stats& v = tr->vals;
      v.t_spread_or_interp = dir == 1 ? t_a : t_b;
      v.t_deconv_or_amplify = dir == 1 ? t_b : t_a;
      v.t_fft = t_fft;
      v.t_execute = tot;
    }
  }
  return p->warn;
}

extern "C" int esn_execute(esn_plan p, void* c, void* f) {
  if (!p) return ESN_ERR_BAD_ARG;
  if (p->type == 3) return t3_execute(p, c, f);
  if (p->spread_only) return ESN_ERR_BAD_ARG;
  return execute_dir(p, p->type, c, f);
}

extern "C" int esn_execute_adjoint(esn_plan p, void* c, void* f) {
  if (!p) return ESN_ERR_BAD_ARG;
  if (p->type == 3) return ESN_ERR_UNSUPPORTED;
  if (p->spread_only) return ESN_ERR_BAD_ARG;
  return execute_dir(p, 3 - p->type, c, f);
}

extern "C" int esn_spread(esn_plan p, const void* c, void* grid) {
  if (!p || p->type != 1 || !grid) return ESN_ERR_BAD_ARG;
  if (p->M < 0) return ESN_ERR_NO_POINTS;
  if (p->M > 0 && !c) return ESN_ERR_BAD_ARG;
  ESN_HIP(hipSetDevice(p->device));
  const size_t cs = csize(p->prec);
  const int64_t G = nf_total(p);
  ESN_HIP(hipMemsetAsync(grid, 0, (size_t)p->ntransf * G * cs, p->stream));
  for (int c0 = 0; c0 < p->ntransf; c0 += p->chunk) {
    const int ntr = std::min(p->chunk, p->ntransf - c0);
    ESN_TRY(run_spread(p, ntr, static_cast<const char*>(c) + (size_t)c0 * p->M * cs,
                       static_cast<char*>(grid) + (size_t)c0 * G * cs));
  }
  return ESN_OK;
}

extern "C" int esn_interp(esn_plan p, const void* grid, void* c) {
  if (!p || p->type != 2 || !grid) return ESN_ERR_BAD_ARG;
  if (p->M < 0) return ESN_ERR_NO_POINTS;
  if (p->M > 0 && !c) return ESN_ERR_BAD_ARG;
  ESN_HIP(hipSetDevice(p->device));
  const size_t cs = csize(p->prec);
  const int64_t G = nf_total(p);
  for (int c0 = 0; c0 < p->ntransf; c0 += p->chunk) {
    const int ntr = std::min(p->chunk, p->ntransf - c0);
    ESN_TRY(run_interp(p, ntr, static_cast<const char*>(grid) + (size_t)c0 * G * cs,
                       static_cast<char*>(c) + (size_t)c0 * p->M * cs));
  }
  return ESN_OK;
}

extern "C" int esn_get_info(esn_plan p, esn_info* o) {
  if (!p || !o) return ESN_ERR_BAD_ARG;
  std::memset(o, 0, sizeof(*o));
  o->type = p->type;
  o->dim = p->dim;
  o->isign = p->isign;
  o->ntransf = p->ntransf;
  o->prec = p->prec;
  o->w = p->par.w;
  o->nquad = p->par.nquad;
  o->modeord = p->opts.modeord;
  o->beta = p->par.beta;
  o->eps = p->eps;
  for (int m = 0; m < 3; m++) {
    o->nmodes[m] = p->N[m];
    o->nf[m] = p->nf[m];
    o->bin[m] = p->bin[m];
  }
  o->M = p->M;
  o->maxsubprob = p->maxsub;
  o->nsubprob = p->nsub;
  o->nbins_nonempty = p->nbins_nonempty;
  o->ntransf_chunk = p->chunk;
  o->spread_method = p->spread_method;
  o->interp_method = p->interp_method;
  o->point_code = p->pts_code;
  o->device_bytes = p->device_bytes;
  o->ndense_units = ((p->type == 1 && p->spread_method == 3) ||
                     (p->type == 2 && p->interp_method == 3)) ? p->nsub : 0;
  o->kerevalmeth = p->kerevalmeth;
  return ESN_OK;
}

extern "C" int esn_debug_sort(esn_plan p, int64_t* geom, int32_t* perm, uint32_t* key,
                              int32_t* bin_start, int32_t* sub) {
  if (!p || !geom || p->type == 3) return ESN_ERR_BAD_ARG;
  geom[0] = p->M;
  geom[1] = p->nbins;
  geom[2] = (int64_t)p->bin[0] * p->bin[1] * p->bin[2];
  geom[3] = p->nsub;
  geom[4] = p->last_sort;
  if (!perm && !key && !bin_start && !sub) return ESN_OK;
  if (p->M < 0) return ESN_ERR_NO_POINTS;
  if (p->last_sort == 0 && (bin_start || sub)) return ESN_ERR_BAD_ARG;
  ESN_HIP(hipSetDevice(p->device));
  hipStream_t s = p->stream;
  const int64_t M = p->M;
  if ((perm || key) && M > 0) {
    uint32_t* d_key = nullptr;
    int32_t* d_perm = nullptr;
    if (hipMalloc((void**)&d_key, 4 * M) != hipSuccess) return ESN_ERR_ALLOC;
    if (hipMalloc((void**)&d_perm, 4 * M) != hipSuccess) {
      (void)hipFree(d_key);
      return ESN_ERR_ALLOC;
    }
    const SortArgs a = sort_args(p, M, ESN_SINGLE, nullptr);
    int rc = ESN_OK;
    if (launch_record_keys(a, p->d_pts, d_key, d_perm, s) != hipSuccess ||
        (key && hipMemcpyAsync(key, d_key, 4 * M, hipMemcpyDeviceToHost, s) != hipSuccess) ||
        (perm && hipMemcpyAsync(perm, d_perm, 4 * M, hipMemcpyDeviceToHost, s) != hipSuccess) ||
        hipStreamSynchronize(s) != hipSuccess)
      rc = ESN_ERR_HIP;
    (void)hipFree(d_key);
    (void)hipFree(d_perm);
    if (rc != ESN_OK) return rc;
  }
  if (bin_start)
    ESN_HIP(hipMemcpyAsync(bin_start, p->d_bstart, 4 * (p->nbins + 1), hipMemcpyDeviceToHost, s));
  if (sub && p->nsub > 0) {
    std::vector<int32_t> b(p->nsub), st(p->nsub), ln(p->nsub);
    ESN_HIP(hipMemcpyAsync(b.data(), p->d_sub_bin, 4 * p->nsub, hipMemcpyDeviceToHost, s));
    ESN_HIP(hipMemcpyAsync(st.data(), p->d_sub_start, 4 * p->nsub, hipMemcpyDeviceToHost, s));
    ESN_HIP(hipMemcpyAsync(ln.data(), p->d_sub_len, 4 * p->nsub, hipMemcpyDeviceToHost, s));
    ESN_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < p->nsub; i++) {
      sub[3 * i] = b[i];
      sub[3 * i + 1] = st[i];
      sub[3 * i + 2] = ln[i];
    }
  }
  ESN_HIP(hipStreamSynchronize(s));
  return ESN_OK;
}

extern "C" int esn_plan_correction(esn_plan p, int m, double* out, int64_t len) {
  if (!p || !out || m < 0 || m >= p->dim || len != p->N[m] / 2 + 1) return ESN_ERR_BAD_ARG;
  ESN_HIP(hipSetDevice(p->device));
  ESN_HIP(hipMemcpyAsync(out, p->d_pf[m], sizeof(double) * len, hipMemcpyDeviceToHost, p->stream));
  ESN_HIP(hipStreamSynchronize(p->stream));
  return ESN_OK;
}

namespace esn {

// Stats of a plan's latest setpts and latest execute (types 1 and 2: read from
// the timing ring, waiting for those calls' events).
int plan_stats(esn_plan p, esn_stats* o) {
  if (p->type == 3) {
    *o = p->stats;
    return ESN_OK;
  }
  *o = esn_stats{};
  bool have_set = false, have_exec = false;
  const int64_t n = std::min<int64_t>(p->ring_count, kTimingRing);
  for (int64_t k = 0; k < n && !(have_set && have_exec); k++) {
    TimingRec& r = p->ring[(p->ring_count - 1 - k) % kTimingRing];
    esn_stats v;
    if (r.kind == 1 && !have_set) {
      if (timing_values(r, &v) != ESN_OK) return ESN_ERR_HIP;
      o->t_setpts = v.t_setpts;
      have_set = true;
    } else if (r.kind >= 2 && !have_exec) {
      if (timing_values(r, &v) != ESN_OK) return ESN_ERR_HIP;
      o->t_spread_or_interp = v.t_spread_or_interp;
      o->t_fft = v.t_fft;
      o->t_deconv_or_amplify = v.t_deconv_or_amplify;
      o->t_execute = v.t_execute;
      have_exec = true;
    }
  }
  return ESN_OK;
}

}  // namespace esn

extern "C" int esn_get_stats(esn_plan p, esn_stats* o) {
  if (!p || !o) return ESN_ERR_BAD_ARG;
  if (!p->opts.debug) return ESN_ERR_BAD_ARG;
  return plan_stats(p, o);
}

extern "C" int esn_get_stats_history(esn_plan p, esn_stats* out, int max, int* count) {
  if (!p || !out || !count || max < 0) return ESN_ERR_BAD_ARG;
  *count = 0;
  if (!p->opts.debug || p->type == 3) return ESN_ERR_BAD_ARG;
  const int64_t n = std::min<int64_t>(std::min<int64_t>(p->ring_count, kTimingRing), max);
  for (int64_t k = 0; k < n; k++) {
    TimingRec& r = p->ring[(p->ring_count - n + k) % kTimingRing];
    if (timing_values(r, &out[k]) != ESN_OK) return ESN_ERR_HIP;
  }
  *count = (int)n;
  return ESN_OK;
}

namespace esn {

int64_t plan_trim(esn_plan p) {
  if (!p) return 0;
  (void)hipStreamSynchronize(p->stream);
  free_points(p);
  free_subs(p);
  dfree(p, (void**)&p->d_count);
  dfree(p, (void**)&p->d_sstart);
  dfree(p, (void**)&p->d_cell_scan_tmp);
  dfree(p, &p->d_grid);
  for (FFTPlan* f : {&p->fft, &p->fft_tail, &p->fft_adj, &p->fft_adj_tail}) {
    if (f->work) p->device_bytes -= (int64_t)f->work_bytes;
    fft_trim(f);
  }
  p->M = -1;
  p->nsub = 0;
  return p->device_bytes;
}

int plan_set_stream(esn_plan p, hipStream_t s) {
  if (!p) return ESN_ERR_BAD_ARG;
  p->stream = s;
  for (FFTPlan* f : {&p->fft, &p->fft_tail, &p->fft_adj, &p->fft_adj_tail})
    if (fft_set_stream(f, s) != ESN_OK) return ESN_ERR_FFT_PLAN;
  return ESN_OK;
}

int64_t plan_estimate_bytes(int type, int dim, const int64_t* nmodes, double eps, int prec,
                            int64_t M) {
  esn_params par;
  if (esn_choose_params(eps, prec, dim, nmodes, 2.0, &par) >= 2) return -1;
  const int64_t cs = prec == ESN_DOUBLE ? 16 : 8;
  int64_t grid = cs, cells = 1;
  for (int m = 0; m < dim; m++) {
    grid *= par.nf[m];
    cells *= par.nf[m] + 64;      // bins may pad the grid
  }
  const int64_t rec = prec == ESN_DOUBLE ? 32 : 16;
  (void)type;
  return 2 * grid                 // fine grid + rocFFT work buffer
         + 8 * (cells + 1)        // bin counts and starts (at most one bin per cell)
         + M * (2 * rec + 8)      // sorted records, the sort's second record buffer and keys
         + (int64_t)(M / 256 + 1024) * 12   // subproblem lists
         + (1 << 20);             // factors, flags, small buffers
}

}  // namespace esn

extern "C" int esn_destroy(esn_plan p) {
  if (!p) return ESN_OK;
  (void)hipSetDevice(p->device);
  if (p->type == 3) t3_destroy(p);
  destroy_all(p);
  delete p;
  return ESN_OK;
}

// ---- one-shot calls ----
static int oneshot(int type, int dim, int64_t M, const double* x, const double* y,
                   const double* z, void* c, int isign, double eps, const int64_t* N, void* f,
                   int prec, const esn_opts* opts, void* stream) {
  esn_plan p = nullptr;
  int st = esn_makeplan(type, dim, N, isign, 1, eps, prec, &p, opts, stream);
  if (st >= 2) return st;
  int warn = st;
  st = esn_setpts(p, M, ESN_DOUBLE, x, y, z);
  if (st == ESN_OK) st = esn_execute(p, c, f);
  if (st < 2 && hipStreamSynchronize((hipStream_t)stream) != hipSuccess) st = ESN_ERR_HIP;
  esn_destroy(p);
  if (st >= 2) return st;
  return st ? st : warn;
}

extern "C" int esn_1d1(int64_t M, const double* x, const void* c, int isign, double eps,
                       int64_t N1, void* f, int prec, const esn_opts* opts, void* stream) {
  int64_t N[3] = {N1, 1, 1};
  return oneshot(1, 1, M, x, nullptr, nullptr, const_cast<void*>(c), isign, eps, N, f, prec, opts,
                 stream);
}
extern "C" int esn_1d2(int64_t M, const double* x, void* c, int isign, double eps, int64_t N1,
                       const void* f, int prec, const esn_opts* opts, void* stream) {
  int64_t N[3] = {N1, 1, 1};
  return oneshot(2, 1, M, x, nullptr, nullptr, c, isign, eps, N, const_cast<void*>(f), prec, opts,
                 stream);
}
extern "C" int esn_2d1(int64_t M, const double* x, const double* y, const void* c, int isign,
                       double eps, int64_t N1, int64_t N2, void* f, int prec,
                       const esn_opts* opts, void* stream) {
  int64_t N[3] = {N1, N2, 1};
  return oneshot(1, 2, M, x, y, nullptr, const_cast<void*>(c), isign, eps, N, f, prec, opts,
                 stream);
}
extern "C" int esn_2d2(int64_t M, const double* x, const double* y, void* c, int isign,
                       double eps, int64_t N1, int64_t N2, const void* f, int prec,
                       const esn_opts* opts, void* stream) {
  int64_t N[3] = {N1, N2, 1};
  return oneshot(2, 2, M, x, y, nullptr, c, isign, eps, N, const_cast<void*>(f), prec, opts,
                 stream);
}
extern "C" int esn_3d1(int64_t M, const double* x, const double* y, const double* z,
                       const void* c, int isign, double eps, int64_t N1, int64_t N2, int64_t N3,
                       void* f, int prec, const esn_opts* opts, void* stream) {
  int64_t N[3] = {N1, N2, N3};
  return oneshot(1, 3, M, x, y, z, const_cast<void*>(c), isign, eps, N, f, prec, opts, stream);
}
extern "C" int esn_3d2(int64_t M, const double* x, const double* y, const double* z, void* c,
                       int isign, double eps, int64_t N1, int64_t N2, int64_t N3,
                       const void* f, int prec, const esn_opts* opts, void* stream) {
  int64_t N[3] = {N1, N2, N3};
  return oneshot(2, 3, M, x, y, z, c, isign, eps, N, const_cast<void*>(f), prec, opts, stream);
}
