// Toeplitz form of the normal operator T = A^H W A, for the inverse NUFFT by
// conjugate gradients on the normal equations (Sec. 1, remark on the inverse
// NUFFT; the paper leaves that problem aside and notes that such solvers
// apply NUFFTs repeatedly).
//
// A is the type 2 transform of sign isign on M points, (A f)_j = sum_k f_k
// exp(isign i k.x_j), and W = diag(w_j).  Then (T f)_k = sum_k' t_{k - k'} f_k'
// with t_m = sum_j w_j exp(-isign i m.x_j), |m_i| <= N_i - 1: a Toeplitz
// matrix whose generating values are one type 1 transform (eq. (1), sign
// -isign) of the weights on 2 N_i modes per dimension.  Embedded in a circulant
// of period L_i = 2 N_i (the values in FFT order are its first column), T f is a
// circular convolution on the doubled grid: zero-pad f, FFT, multiply by the
// FFT of t, inverse FFT, keep N.  Set-up costs one type 1 transform; each
// application two FFTs of prod(2 N_i) points, against a type 2 and a type 1
// transform (with their spreading and interpolation) for A^H W A applied
// directly.  The forward FFT's input is zero outside [0, N) and only [0, N) of
// the inverse FFT is kept, so both may skip the other columns.
#include <cstring>

#include "esn_internal.hpp"

using namespace esn;

struct esn_toeplitz_s {
  int dim = 1, prec = ESN_SINGLE, device = 0;
  hipStream_t stream = nullptr;
  ToepArgs a;
  int64_t ltot = 1, ntot = 1;
  FFTPlan fwd;          // full transform (the generating values)
  FFTPlan pfwd, pbwd;   // of the zero-padded input, and for the output in [0, N)
  void* d_that = nullptr;   // FFT of the circulant's first column / prod(L)
  void* d_grid = nullptr;   // doubled work grid
};

namespace {

#define ESN_HIP(call)                             \
  do {                                            \
    if ((call) != hipSuccess) return ESN_ERR_HIP; \
  } while (0)

size_t csize_of(int prec) { return prec == ESN_DOUBLE ? 16 : 8; }

void toep_free(esn_toeplitz t) {
  if (!t) return;
  (void)hipStreamSynchronize(t->stream);
  fft_destroy(&t->fwd);
  fft_destroy(&t->pfwd);
  fft_destroy(&t->pbwd);
  if (t->d_that) (void)hipFree(t->d_that);
  if (t->d_grid) (void)hipFree(t->d_grid);
  delete t;
}

}  // namespace

extern "C" int esn_toeplitz_makeplan(int dim, const int64_t* nmodes, int isign, double eps,
                                     int prec, int64_t M, int coord_prec, const void* x,
                                     const void* y, const void* z, const void* weights,
                                     esn_toeplitz* out, const esn_opts* opts, void* stream) {
  if (!out) return ESN_ERR_BAD_ARG;
  *out = nullptr;
  if (dim < 1 || dim > 3 || !nmodes || (isign != 1 && isign != -1) || M < 0 ||
      (prec != ESN_SINGLE && prec != ESN_DOUBLE))
    return ESN_ERR_BAD_ARG;
  esn_opts o;
  if (opts) o = *opts;
  else esn_default_opts(&o);
  if (o.modeord != 0 && o.modeord != 1) return ESN_ERR_BAD_ARG;
  int64_t N2[3] = {1, 1, 1};
  for (int m = 0; m < dim; m++) {
    if (nmodes[m] < 1 || nmodes[m] > ((int64_t)1 << 29)) return ESN_ERR_BAD_ARG;
    N2[m] = 2 * nmodes[m];
  }
  esn_toeplitz t = new (std::nothrow) esn_toeplitz_s();
  if (!t) return ESN_ERR_ALLOC;
  t->dim = dim;
  t->prec = prec;
  t->stream = (hipStream_t)stream;
  for (int m = 0; m < 3; m++) {
    t->a.N[m] = m < dim ? nmodes[m] : 1;
    t->a.L[m] = N2[m];
    t->ltot *= N2[m];
    t->ntot *= t->a.N[m];
  }
  t->a.modeord = o.modeord;
  auto fail = [&](int code) {
    toep_free(t);
    return code;
  };
  if (hipGetDevice(&t->device) != hipSuccess) return fail(ESN_ERR_HIP);
  const size_t gbytes = (size_t)t->ltot * csize_of(prec);
  if (hipMalloc(&t->d_that, gbytes) != hipSuccess || hipMalloc(&t->d_grid, gbytes) != hipSuccess)
    return fail(ESN_ERR_ALLOC);

  // generating values t_m on 2N modes in FFT order (the circulant's first
  // column), from a type 1 plan of sign -isign on the points
  esn_opts o1 = o;
  o1.modeord = 1;
  esn_plan p1 = nullptr;
  int rc = make_plan(1, dim, N2, -isign, 1, eps, prec, &p1, &o1, stream, false);
  if (rc >= 2) return fail(rc);
  const int warn = rc;
  rc = esn_setpts(p1, M, coord_prec, x, y, z);
  void* ones = nullptr;
  if (rc == ESN_OK && !weights && M > 0) {
    if (hipMalloc(&ones, (size_t)M * csize_of(prec)) != hipSuccess ||
        launch_fill_ones(prec, ones, M, t->stream) != hipSuccess)
      rc = ESN_ERR_ALLOC;
  }
  if (rc == ESN_OK) rc = esn_execute(p1, const_cast<void*>(weights ? weights : ones), t->d_that);
  if (rc < 2 && hipStreamSynchronize(t->stream) != hipSuccess) rc = ESN_ERR_HIP;
  if (ones) (void)hipFree(ones);
  esn_destroy(p1);
  if (rc >= 2) return fail(rc);

  // its FFT, with the inverse transform's 1 / prod(L) folded in
  rc = fft_make(&t->fwd, dim, t->a.L, t->a.L, 1, 1, prec, -1, t->stream);
  // an application's input is zero outside [0, N) and only [0, N) of its
  // output is kept, so its transforms may skip the other columns
  if (rc == ESN_OK) rc = fft_make_padded(&t->pfwd, dim, t->a.L, t->a.N, prec, -1, t->stream);
  if (rc == ESN_OK) rc = fft_make_padded(&t->pbwd, dim, t->a.L, t->a.N, prec, +1, t->stream);
  if (rc != ESN_OK) return fail(rc);
  if (fft_exec(&t->fwd, t->d_that) != ESN_OK) return fail(ESN_ERR_FFT_PLAN);
  if (launch_scale(prec, t->d_that, t->ltot, 1.0 / (double)t->ltot, t->stream) != hipSuccess ||
      hipStreamSynchronize(t->stream) != hipSuccess)
    return fail(ESN_ERR_HIP);
  *out = t;
  return warn;
}

extern "C" int esn_toeplitz_apply(esn_toeplitz t, const void* f, void* g) {
  if (!t || !f || !g) return ESN_ERR_BAD_ARG;
  ESN_HIP(hipSetDevice(t->device));
  hipStream_t s = t->stream;
  ESN_HIP(launch_toep_pad(t->a, t->prec, f, t->d_grid, s));
  if (fft_exec_padded(&t->pfwd, t->d_grid, 1) != ESN_OK) return ESN_ERR_FFT_PLAN;
  ESN_HIP(launch_cmul(t->prec, t->d_grid, t->d_that, t->d_grid, t->ltot, 1, s));
  if (fft_exec_padded(&t->pbwd, t->d_grid, 0) != ESN_OK) return ESN_ERR_FFT_PLAN;
  ESN_HIP(launch_toep_extract(t->a, t->prec, t->d_grid, g, s));
  return ESN_OK;
}

extern "C" int esn_toeplitz_destroy(esn_toeplitz t) {
  if (!t) return ESN_OK;
  (void)hipSetDevice(t->device);
  toep_free(t);
  return ESN_OK;
}
