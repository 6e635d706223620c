// rocFFT wrapper: in-place, unnormalised, interleaved complex-to-complex FFTs of
// the fine grid (Sec. 3.1 step 2, eq. (dft1); Sec. 3.2 step 2, eq. (dft)),
// batched over the transforms of one fused launch.  The exponent sign equals
// the transform's isign: +1 -> rocFFT's inverse (backward, e^{+2 pi i lk/n}),
// -1 -> rocFFT's forward (e^{-2 pi i lk/n}).
//
// 3D transforms skip the y and z FFTs of the x columns that hold no mode
// (k1 mod n1 outside I_N1): half the grid or more for sigma = 2.  The result
// at the kept columns is that of the full 3D FFT, since the y and z FFTs act
// on each x column by itself.  In single precision, with y and z lengths
// 2^a 3^b 5^c (a >= 5) up to 512 and x a multiple of 32, those two passes are
// the column FFT kernels (kernels_fft.hip), one launch per pass over both kept
// runs; otherwise, on power-of-two grids, rocFFT's strided 2D plans, and on
// other grids the full 3D rocFFT plan.  2D transforms on such lengths run the
// x pass and the y pass on the kept columns the same way.  With column FFTs the correction
// (deconvolution for type 1, amplification for type 2) folds into the z pass
// (fft_exec_modes).
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "esn_internal.hpp"

namespace esn {

static std::once_flag g_rocfft_once;
static rocfft_status g_rocfft_setup = rocfft_status_success;

// rocFFT plan of `dim` lengths (fastest first) with optional strides.
static rocfft_plan make_one(int dim, const size_t* len, size_t batch, const size_t* stride,
                            size_t dist, int prec, int sign) {
  rocfft_plan_description d = nullptr;
  if (stride) {
    if (rocfft_plan_description_create(&d) != rocfft_status_success) return nullptr;
    if (rocfft_plan_description_set_data_layout(
            d, rocfft_array_type_complex_interleaved, rocfft_array_type_complex_interleaved,
            nullptr, nullptr, (size_t)dim, stride, dist, (size_t)dim, stride, dist) !=
        rocfft_status_success) {
      rocfft_plan_description_destroy(d);
      return nullptr;
    }
  }
  rocfft_plan p = nullptr;
  const rocfft_status st = rocfft_plan_create(
      &p, rocfft_placement_inplace,
      sign > 0 ? rocfft_transform_type_complex_inverse : rocfft_transform_type_complex_forward,
      prec == ESN_DOUBLE ? rocfft_precision_double : rocfft_precision_single, (size_t)dim, len,
      batch, d);
  if (d) rocfft_plan_description_destroy(d);
  return st == rocfft_status_success ? p : nullptr;
}

// Twiddle table of the column FFTs: exp(2 pi i e / ly), e < ly, then
// exp(2 pi i e / lz), e < lz, in FP64.
static int col_twiddles(FFTPlan* p, hipStream_t s) {
  std::vector<double2> tw((size_t)(p->ly + p->lz));
  for (int i = 0; i < p->ly + p->lz; i++) {
    const int len = i < p->ly ? p->ly : p->lz;
    const int e = i < p->ly ? i : i - p->ly;
    const double ang = 2.0 * M_PI * (double)e / (double)len;
    tw[(size_t)i] = make_double2(std::cos(ang), std::sin(ang));
  }
  // stream-ordered memory on the plan's stream (no wait for the whole device)
  if (hipMallocAsync((void**)&p->d_tw, tw.size() * sizeof(double2), s) != hipSuccess) {
    p->d_tw = nullptr;
    return ESN_ERR_ALLOC;
  }
  if (hipMemcpyAsync(p->d_tw, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice,
                     s) != hipSuccess)
    return ESN_ERR_HIP;
  return ESN_OK;
}

// rocFFT work buffer (one for every plan of p: they run one after another on
// the stream) and execution info on stream s.
static int finish_plan(FFTPlan* p, hipStream_t s) {
  if (!p->plan) return ESN_ERR_FFT_PLAN;
  size_t work = 0;
  for (rocfft_plan q : {p->plan, p->yz[0], p->yz[1]}) {
    if (!q) continue;
    size_t wb = 0;
    if (rocfft_plan_get_work_buffer_size(q, &wb) != rocfft_status_success) return ESN_ERR_FFT_PLAN;
    work = std::max(work, wb);
  }
  p->work_bytes = work;
  if (rocfft_execution_info_create(&p->info) != rocfft_status_success) return ESN_ERR_FFT_PLAN;
  if (work > 0) {
    if (hipMallocAsync(&p->work, work, s) != hipSuccess) {
      p->work = nullptr;
      return ESN_ERR_ALLOC;
    }
    if (rocfft_execution_info_set_work_buffer(p->info, p->work, work) != rocfft_status_success)
      return ESN_ERR_FFT_PLAN;
  }
  if (rocfft_execution_info_set_stream(p->info, (void*)s) != rocfft_status_success)
    return ESN_ERR_FFT_PLAN;
  return ESN_OK;
}

int fft_make(FFTPlan* p, int dim, const int64_t* nf, const int64_t* nmodes, int type, int batch,
             int prec, int sign, hipStream_t s) {
  std::call_once(g_rocfft_once, [] { g_rocfft_setup = rocfft_setup(); });
  if (g_rocfft_setup != rocfft_status_success) return ESN_ERR_FFT_PLAN;
  p->batch = batch;
  p->elem = prec == ESN_DOUBLE ? 16 : 8;
  p->grid = 1;
  for (int m = 0; m < dim; m++) p->grid *= nf[m];
  p->x_first = type == 1;
  // kept x runs: k1 = 0 .. ceil(N1/2) - 1 and n1 - floor(N1/2) .. n1 - 1
  const int64_t lo = (nmodes[0] + 1) / 2, hi = nmodes[0] / 2;
  // column FFTs where they apply; else rocFFT's strided (y, z) transforms,
  // which are fast only for power-of-two sizes (on a 256^3 grid x pass + kept
  // runs take 153 us against 191 us for the full 3D plan; on 288^3 789 us
  // against 487 us), and the full plan for other sizes
  auto pow2 = [](int64_t v) { return v > 0 && (v & (v - 1)) == 0; };
  const bool cols = dim >= 2 && lo + hi < nf[0] && prec == ESN_SINGLE &&
                    nf[0] % kColWidth == 0 && fft_cols_supported(nf[1]) &&
                    (dim == 2 || fft_cols_supported(nf[2])) && p->grid < ((int64_t)1 << 28);
  const bool prune =
      cols || (dim == 3 && lo + hi < nf[0] && pow2(nf[0]) && pow2(nf[1]) && pow2(nf[2]));
  p->stream = s;
  if (cols) {
    const int64_t n2 = dim == 3 ? nf[2] : 1;
    const size_t lx[1] = {(size_t)nf[0]};
    p->plan = make_one(1, lx, (size_t)batch * nf[1] * n2, nullptr, 0, prec, sign);
    // column blocks of 32 covering x = 0 .. lo - 1 and x = nf0 - hi .. nf0 - 1;
    // blocks that would cover a column twice merge into one range
    const int all = (int)(nf[0] / kColWidth);
    int ca = (int)((lo + kColWidth - 1) / kColWidth);
    int cb0 = (int)((nf[0] - hi) / kColWidth);
    if (hi == 0) cb0 = all;
    if (cb0 < ca) {
      ca = all;
      cb0 = all;
    }
    p->nchunks = ca + (all - cb0);
    p->cols = 1;
    // 2D: the y pass on the kept columns, no z pass; the correction stays in
    // its own kernels
    p->modes = dim == 3;
    p->ly = (int)nf[1];
    p->lz = dim == 3 ? (int)nf[2] : 0;
    ColFFTArgs a;
    a.chunks_a = ca;
    a.chunk_b0 = cb0;
    a.sign = sign;
    a.tstride = p->grid;
    // the y pass runs on every z plane; the z pass only on the y rows that
    // hold modes (k2 mod n2 in I_N2): type 1 runs it last, and only those rows
    // are read afterwards; type 2 runs it first, on the amplified grid whose
    // other rows are zero, so their z transforms are zero as well
    p->cy = a;
    p->cy.estride = nf[0];
    p->cy.pstride = nf[0] * nf[1];
    p->cy.nplanes = n2;
    p->cy.planes_a = n2;
    p->cy.plane_b0 = n2;
    p->cz = a;
    p->cz.estride = nf[0] * nf[1];
    p->cz.pstride = nf[0];
    const int64_t ylo = (nmodes[1] + 1) / 2, yhi = nmodes[1] / 2;
    if (ylo + yhi < nf[1]) {
      p->cz.planes_a = ylo;
      p->cz.plane_b0 = nf[1] - yhi;
      p->cz.nplanes = ylo + yhi;
    } else {
      p->cz.planes_a = p->cz.plane_b0 = p->cz.nplanes = nf[1];
    }
    // with the correction in the passes: the y pass keeps the y points that
    // hold modes, the z pass the z points
    p->nx = nf[0];
    p->cy_keep = p->cy;
    p->cy_keep.keep_lo = ylo;
    p->cy_keep.keep_hi = ylo + yhi < nf[1] ? yhi : nf[1] - ylo;
    p->cz_keep = p->cz;
    if (dim == 3) {
      const int64_t zlo = (nmodes[2] + 1) / 2, zhi = nmodes[2] / 2;
      p->cz_keep.keep_lo = zlo;
      p->cz_keep.keep_hi = zlo + zhi < nf[2] ? zhi : nf[2] - zlo;
    }
    const int rc = col_twiddles(p, s);
    if (rc != ESN_OK) return rc;
  } else if (prune) {
    const size_t lx[1] = {(size_t)nf[0]};
    p->plan = make_one(1, lx, (size_t)batch * nf[1] * nf[2], nullptr, 0, prec, sign);
    const size_t lyz[2] = {(size_t)nf[1], (size_t)nf[2]};
    const size_t syz[2] = {(size_t)nf[0], (size_t)(nf[0] * nf[1])};
    const int64_t runs[2] = {lo, hi};
    const int64_t offs[2] = {0, nf[0] - hi};
    for (int r = 0; r < 2; r++) {
      if (runs[r] <= 0) continue;
      p->yz[p->nyz] = make_one(2, lyz, (size_t)runs[r], syz, 1, prec, sign);
      p->yz_off[p->nyz] = offs[r];
      if (!p->yz[p->nyz]) return ESN_ERR_FFT_PLAN;
      p->nyz++;
    }
  } else {
    size_t lengths[3];
    for (int m = 0; m < dim; m++) lengths[m] = (size_t)nf[m];   // fastest first
    p->plan = make_one(dim, lengths, (size_t)batch, nullptr, 0, prec, sign);
  }
  return finish_plan(p, s);
}

int fft_make_padded(FFTPlan* p, int dim, const int64_t* L, const int64_t* N, int prec, int sign,
                    hipStream_t s) {
  int64_t grid = 1;
  for (int m = 0; m < dim; m++) grid *= L[m];
  const bool cols = dim == 3 && prec == ESN_SINGLE && L[0] % kColWidth == 0 && N[0] < L[0] &&
                    N[1] < L[1] && fft_cols_supported(L[1]) && fft_cols_supported(L[2]) &&
                    grid < ((int64_t)1 << 28);
  if (!cols) return fft_make(p, dim, L, L, 1, 1, prec, sign, s);   // full transform
  std::call_once(g_rocfft_once, [] { g_rocfft_setup = rocfft_setup(); });
  if (g_rocfft_setup != rocfft_status_success) return ESN_ERR_FFT_PLAN;
  p->batch = 1;
  p->elem = 8;
  p->grid = grid;
  p->stream = s;
  p->padded = 1;
  p->ly = (int)L[1];
  p->lz = (int)L[2];
  p->nx = L[0];
  // column blocks covering x = 0 .. N0 - 1
  p->nchunks = (int)((N[0] + kColWidth - 1) / kColWidth);
  ColFFTArgs a;
  a.chunks_a = p->nchunks;
  a.chunk_b0 = (int)(L[0] / kColWidth);
  a.sign = sign;
  a.tstride = grid;
  p->cy = a;   // every z plane
  p->cy.estride = L[0];
  p->cy.pstride = L[0] * L[1];
  p->cy.nplanes = p->cy.planes_a = p->cy.plane_b0 = L[2];
  p->cz = a;   // the y rows 0 .. N1 - 1
  p->cz.estride = L[0] * L[1];
  p->cz.pstride = L[0];
  p->cz.nplanes = p->cz.planes_a = N[1];
  p->cz.plane_b0 = L[1];
  const size_t lx[1] = {(size_t)L[0]};
  p->plan = make_one(1, lx, (size_t)(L[1] * L[2]), nullptr, 0, prec, sign);
  const int rc = col_twiddles(p, s);
  if (rc != ESN_OK) return rc;
  return finish_plan(p, s);
}

int fft_exec_padded(FFTPlan* p, void* data, int input_padded) {
  if (!p->padded) return fft_exec(p, data);
  float2* g = static_cast<float2*>(data);
  const ColModes none;
  void* in[1] = {data};
  auto xpass = [&] { return rocfft_execute(p->plan, in, nullptr, p->info) == rocfft_status_success; };
  auto ypass = [&] {
    return launch_fft_cols(g, p->ly, p->cy, p->d_tw, p->nchunks, 1, 0, 0, none, p->stream);
  };
  auto zpass = [&] {
    return launch_fft_cols(g, p->lz, p->cz, p->d_tw + p->ly, p->nchunks, 1, 0, 0, none,
                           p->stream);
  };
  if (input_padded) {
    // nonzero input in [0, N): z on its columns, y on its x columns, then x
    if (zpass() != hipSuccess || ypass() != hipSuccess) return ESN_ERR_HIP;
    return xpass() ? ESN_OK : ESN_ERR_FFT_PLAN;
  }
  // output needed in [0, N) only: x, y on those x columns, z on their y rows
  if (!xpass()) return ESN_ERR_FFT_PLAN;
  if (ypass() != hipSuccess || zpass() != hipSuccess) return ESN_ERR_HIP;
  return ESN_OK;
}

int fft_exec(FFTPlan* p, void* data) {
  auto run = [&](rocfft_plan q, void* ptr) {
    void* in[1] = {ptr};
    return rocfft_execute(q, in, nullptr, p->info) == rocfft_status_success;
  };
  if (p->cols) {
    float2* g = static_cast<float2*>(data);
    const ColModes none;
    auto ypass = [&] {
      return launch_fft_cols(g, p->ly, p->cy, p->d_tw, p->nchunks, p->batch, 0, 0, none,
                             p->stream);
    };
    auto zpass = [&] {
      return launch_fft_cols(g, p->lz, p->cz, p->d_tw + p->ly, p->nchunks, p->batch, 0, 0, none,
                             p->stream);
    };
    if (p->x_first) {   // type 1: x, y, z (kept y rows)
      if (!run(p->plan, data)) return ESN_ERR_FFT_PLAN;
      if (ypass() != hipSuccess || (p->lz && zpass() != hipSuccess)) return ESN_ERR_HIP;
    } else {            // type 2: z (kept y rows), y, x
      if ((p->lz && zpass() != hipSuccess) || ypass() != hipSuccess) return ESN_ERR_HIP;
      if (!run(p->plan, data)) return ESN_ERR_FFT_PLAN;
    }
    return ESN_OK;
  }
  if (!p->nyz) return run(p->plan, data) ? ESN_OK : ESN_ERR_FFT_PLAN;
  if (p->x_first && !run(p->plan, data)) return ESN_ERR_FFT_PLAN;
  for (int t = 0; t < p->batch; t++)
    for (int r = 0; r < p->nyz; r++) {
      char* base = static_cast<char*>(data) + (size_t)(t * p->grid + p->yz_off[r]) * p->elem;
      if (!run(p->yz[r], base)) return ESN_ERR_FFT_PLAN;
    }
  if (!p->x_first && !run(p->plan, data)) return ESN_ERR_FFT_PLAN;
  return ESN_OK;
}

int fft_exec_modes(FFTPlan* p, void* grid, void* f, const ColModes& cm) {
  if (!p->modes) return ESN_ERR_BAD_ARG;
  float2* g = static_cast<float2*>(grid);
  ColModes m = cm;
  m.f = static_cast<float2*>(f);
  const ColModes none;
  auto xpass = [&] {
    void* in[1] = {grid};
    return rocfft_execute(p->plan, in, nullptr, p->info) == rocfft_status_success;
  };
  if (p->x_first) {
    // type 1: x; y, storing the y rows that hold modes only (the z pass reads
    // no other); z on those rows, writing the modes with their factors
    if (!xpass()) return ESN_ERR_FFT_PLAN;
    if (launch_fft_cols(g, p->ly, p->cy_keep, p->d_tw, p->nchunks, p->batch, 0, 1, none,
                        p->stream) != hipSuccess ||
        launch_fft_cols(g, p->lz, p->cz_keep, p->d_tw + p->ly, p->nchunks, p->batch, 0, 2, m,
                        p->stream) != hipSuccess)
      return ESN_ERR_HIP;
    return ESN_OK;
  }
  // type 2: clear the x columns outside the column blocks (read by the x
  // pass); z on the y rows that hold modes, reading p_k f_k; y, reading those
  // rows only (the others are zero); x
  const int64_t x0 = (int64_t)p->cy.chunks_a * kColWidth, x1 = (int64_t)p->cy.chunk_b0 * kColWidth;
  if (launch_zero_cols(g, p->nx, p->grid / p->nx, x0, x1, p->batch, p->grid, p->stream) !=
          hipSuccess ||
      launch_fft_cols(g, p->lz, p->cz_keep, p->d_tw + p->ly, p->nchunks, p->batch, 2, 0, m,
                      p->stream) != hipSuccess ||
      launch_fft_cols(g, p->ly, p->cy_keep, p->d_tw, p->nchunks, p->batch, 1, 0, none,
                      p->stream) != hipSuccess)
    return ESN_ERR_HIP;
  return xpass() ? ESN_OK : ESN_ERR_FFT_PLAN;
}

void fft_destroy(FFTPlan* p) {
  if (p->info) rocfft_execution_info_destroy(p->info);
  for (rocfft_plan q : {p->plan, p->yz[0], p->yz[1]})
    if (q) rocfft_plan_destroy(q);
  if (p->work) (void)hipFreeAsync(p->work, p->stream);
  if (p->d_tw) (void)hipFreeAsync(p->d_tw, p->stream);
  *p = FFTPlan();
}

// Give back the rocFFT work buffer (a plan kept idle); fft_ensure_work makes
// it again before the next transform.
void fft_trim(FFTPlan* p) {
  if (p->work) (void)hipFreeAsync(p->work, p->stream);
  p->work = nullptr;
}

int fft_ensure_work(FFTPlan* p) {
  if (!p->info || p->work_bytes == 0 || p->work) return ESN_OK;
  if (hipMallocAsync(&p->work, p->work_bytes, p->stream) != hipSuccess) {
    p->work = nullptr;
    return ESN_ERR_ALLOC;
  }
  if (rocfft_execution_info_set_work_buffer(p->info, p->work, p->work_bytes) !=
      rocfft_status_success)
    return ESN_ERR_FFT_PLAN;
  return ESN_OK;
}

int fft_set_stream(FFTPlan* p, hipStream_t s) {
  p->stream = s;
  if (p->info && rocfft_execution_info_set_stream(p->info, (void*)s) != rocfft_status_success)
    return ESN_ERR_FFT_PLAN;
  return ESN_OK;
}

}  // namespace esn
