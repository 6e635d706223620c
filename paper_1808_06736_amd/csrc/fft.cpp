// rocFFT wrapper: in-place, unnormalised, interleaved complex-to-complex FFTs of
// the fine grid (Sec. 3.1 step 2, eq. (dft1); Sec. 3.2 step 2, eq. (dft)),
// batched over the transforms of one fused launch.  The exponent sign equals
// the transform's isign: +1 -> rocFFT's inverse (backward, e^{+2 pi i lk/n}),
// -1 -> rocFFT's forward (e^{-2 pi i lk/n}).
#include <mutex>

#include "esn_internal.hpp"

namespace esn {

static std::once_flag g_rocfft_once;
static rocfft_status g_rocfft_setup = rocfft_status_success;

int fft_make(FFTPlan* p, int dim, const int64_t* nf, int batch, int prec, int sign,
             hipStream_t s) {
  std::call_once(g_rocfft_once, [] { g_rocfft_setup = rocfft_setup(); });
  if (g_rocfft_setup != rocfft_status_success) return ESN_ERR_FFT_PLAN;
  size_t lengths[3];
  for (int m = 0; m < dim; m++) lengths[m] = (size_t)nf[m];   // fastest first
  rocfft_status st = rocfft_plan_create(
      &p->plan, rocfft_placement_inplace,
      sign > 0 ? rocfft_transform_type_complex_inverse : rocfft_transform_type_complex_forward,
      prec == ESN_DOUBLE ? rocfft_precision_double : rocfft_precision_single, (size_t)dim,
      lengths, (size_t)batch, nullptr);
  if (st != rocfft_status_success) {
    p->plan = nullptr;
    return ESN_ERR_FFT_PLAN;
  }
  st = rocfft_plan_get_work_buffer_size(p->plan, &p->work_bytes);
  if (st != rocfft_status_success) return ESN_ERR_FFT_PLAN;
  if (rocfft_execution_info_create(&p->info) != rocfft_status_success) return ESN_ERR_FFT_PLAN;
  if (p->work_bytes > 0) {
    if (hipMalloc(&p->work, p->work_bytes) != hipSuccess) {
      p->work = nullptr;
      return ESN_ERR_ALLOC;
    }
    if (rocfft_execution_info_set_work_buffer(p->info, p->work, p->work_bytes) !=
        rocfft_status_success)
      return ESN_ERR_FFT_PLAN;
  }
  if (rocfft_execution_info_set_stream(p->info, (void*)s) != rocfft_status_success)
    return ESN_ERR_FFT_PLAN;
  return ESN_OK;
}

int fft_exec(FFTPlan* p, void* data) {
  void* in[1] = {data};
  rocfft_status st = rocfft_execute(p->plan, in, nullptr, p->info);
  return st == rocfft_status_success ? ESN_OK : ESN_ERR_FFT_PLAN;
}

void fft_destroy(FFTPlan* p) {
  if (p->info) rocfft_execution_info_destroy(p->info);
  if (p->plan) rocfft_plan_destroy(p->plan);
  if (p->work) (void)hipFree(p->work);
  p->info = nullptr;
  p->plan = nullptr;
  p->work = nullptr;
  p->work_bytes = 0;
}

}  // namespace esn
