// Type 3 NUFFT (Sec. 3.3, eq. (3)): f_k = sum_j c_j exp(isign i s_k.x_j) for
// M sources x_j and N target frequencies s_k in R^d.
//
// setpts (esn_setpts3), per dimension i:
//   * bounds of the sources and targets; centres x0, s0 and half-widths X, S
//     (eq. (XS) after the translation of eq. (trans));
//   * step 0, eq. (ng): n = 2 sigma X S / pi + w, rounded up to an even
//     2^a 3^b 5^c size of at least 2w; gamma = n / (2 sigma S);
//   * step 1 geometry: sources x'' = (x - x0) / gamma lie at least w/2 cells
//     inside [-pi, pi) (eq. (cond1)); a spread-only type 1 plan sorts them;
//   * step 2 geometry: targets s'' = h gamma (s - s0), |s''| <= pi / sigma
//     (eq. (cond2)); a type 2 plan with n modes per dimension in FFT order
//     sorts them;
//   * per target, the correction of step 3, 1 / (w sum_q wq phi(zq)
//     cos((w/2) s'' zq)) per dimension (d p FP64 cosines), times the postphase
//     exp(isign i s.x0); per source the prephase exp(isign i s0.(x - x0)).
// execute (esn_execute): prephase the strengths, spread them onto the type 3
// grid (eq. (blt3)), evaluate that grid as a Fourier series at the targets with
// the type 2 plan (eq. (bkt3)), multiply by the per-target factors.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <future>
#include <vector>

#include "esn_internal.hpp"

namespace esn {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int64_t kT3MaxGrid = (int64_t)1 << 31;   // cells of the type 3 grid
// Points per set: permutation indices are int32, and the spreading and
// interpolation kernels form record indices up to a few hundred past a
// subproblem's start in 32-bit ints, so the limit keeps 2^16 of headroom.
constexpr int64_t kMaxPoints = ((int64_t)1 << 31) - ((int64_t)1 << 16);

#define ESN_HIP(call)                       \
  do {                                      \
    if ((call) != hipSuccess) return ESN_ERR_HIP; \
  } while (0)

int t3_alloc(esn_plan_s* p, void** ptr, size_t bytes) {
  if (*ptr) {
    (void)hipFree(*ptr);
    *ptr = nullptr;
  }
  if (bytes == 0) return ESN_OK;
  if (hipMalloc(ptr, bytes) != hipSuccess) {
    *ptr = nullptr;
    return ESN_ERR_ALLOC;
  }
  (void)p;
  return ESN_OK;
}

void t3_free(void** ptr) {
  if (*ptr) (void)hipFree(*ptr);
  *ptr = nullptr;
}

size_t csize(int prec) { return prec == ESN_DOUBLE ? 2 * sizeof(double) : 2 * sizeof(float); }

// Smallest even 2^a 3^b 5^c >= n.
int64_t next_smooth_even(int64_t n) {
  if (n < 2) n = 2;
  for (int64_t m = n + (n & 1);; m += 2) {
    int64_t r = m;
    for (int f : {2, 3, 5})
      while (r % f == 0) r /= f;
    if (r == 1) return m;
  }
}

// Bounds [xlo, xhi] of the dim source coordinate arrays (M values each) and
// [slo, shi] of the target arrays (N values each), from one launch and one
// copy to the host; ESN_ERR_NAN_PTS if a value is NaN or infinite.
int coord_bounds(esn_plan_s* p, const void* const* x, int64_t M, const void* const* sx, int64_t N,
                 int coord_prec, double* xlo, double* xhi, double* slo, double* shi) {
  hipStream_t s = p->stream;
  MinMaxSets a;
  std::memset(&a, 0, sizeof(a));
  int slot[6] = {-1, -1, -1, -1, -1, -1};
  for (int m = 0; m < p->dim; m++) {
    xlo[m] = xhi[m] = slo[m] = shi[m] = 0.0;
    if (M > 0) {
      slot[m] = a.count;
      a.x[a.count] = x[m];
      a.n[a.count++] = M;
    }
    if (N > 0) {
      slot[3 + m] = a.count;
      a.x[a.count] = sx[m];
      a.n[a.count++] = N;
    }
  }
  if (a.count == 0) return ESN_OK;
  double* out = p->d_t3_mm + 2 * (int64_t)6 * t3_minmax_blocks(kMaxPoints);
  if (launch_minmax(a, coord_prec, p->d_t3_mm, out, s) != hipSuccess ||
      hipMemcpyAsync(p->h_t3_mm, out, sizeof(double) * 2 * a.count, hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return ESN_ERR_HIP;
  for (int m = 0; m < p->dim; m++)
    for (int set = 0; set < 2; set++) {
      const int i = slot[3 * set + m];
      if (i < 0) continue;
      const double lo = p->h_t3_mm[2 * i], hi = p->h_t3_mm[2 * i + 1];
      if (!std::isfinite(lo) || !std::isfinite(hi)) return ESN_ERR_NAN_PTS;
      (set ? slo : xlo)[m] = lo;
      (set ? shi : xhi)[m] = hi;
    }
  return ESN_OK;
}

// Chebyshev coefficients a[0 .. kT3Cheb-1] of the correction sum
// g(u) = sum_q wphi_q cos(u z_q) (eqs. (pk1), (quad)) on |u| <= U, as a series
// in x = 2 (u / U)^2 - 1 (g is even): the interpolant at the kT3Cheb
// Chebyshev points, with cscale = 2 / U^2.  For w <= 16 and U <= pi w / 4 (the
// largest |u| that the dilation of eq. (ng) allows) its terms fall below FP64
// rounding relative to g well before the last.  U = 0 gives the constant g(0).
void t3_cheb(const std::vector<double>& zq, const std::vector<double>& wphi, double U, double* a,
             double* cscale) {
  auto g = [&](double u) {
    double s = 0.0;
    for (size_t q = 0; q < zq.size(); q++) s += wphi[q] * std::cos(u * zq[q]);
    return s;
  };
  for (int k = 0; k < kT3Cheb; k++) a[k] = 0.0;
  if (!(U > 0.0)) {
    a[0] = g(0.0);
    *cscale = 0.0;
    return;
  }
  constexpr int K = kT3Cheb;
  double G[K];
  for (int j = 0; j < K; j++) {
    const double x = std::cos(kPi * (j + 0.5) / K);
    G[j] = g(U * std::sqrt(0.5 * (x + 1.0)));
  }
  for (int k = 0; k < K; k++) {
    double s = 0.0;
    for (int j = 0; j < K; j++) s += G[j] * std::cos(kPi * k * (j + 0.5) / K);
    a[k] = (k == 0 ? 1.0 : 2.0) * s / K;
  }
  *cscale = 2.0 / (U * U);
}

}  // namespace

int t3_makeplan(int dim, int isign, int ntransf, double eps, int prec, esn_plan* out,
                const esn_opts* opts, void* stream) {
  if (dim < 1 || dim > 3 || ntransf < 1 || (isign != 1 && isign != -1)) return ESN_ERR_BAD_ARG;
  esn_opts o;
  if (opts) o = *opts;
  else esn_default_opts(&o);
  // the spreading plan's fine grid must be the type 3 grid itself, which a
  // type 1 plan with n/2 modes gives only at sigma = 2
  if (o.upsampfac != 2.0) return ESN_ERR_BAD_ARG;
  // the kernel parameters: w, beta and the quadrature follow from eps alone
  int64_t ones[3] = {1, 1, 1};
  esn_params par;
  const int st = esn_choose_params(eps, prec, dim, ones, o.upsampfac, &par);
  if (st >= 2) return st;
  esn_plan_s* p = new (std::nothrow) esn_plan_s();
  if (!p) return ESN_ERR_ALLOC;
  p->type = 3;
  p->dim = dim;
  p->isign = isign;
  p->ntransf = ntransf;
  p->prec = prec;
  p->eps = eps;
  p->par = par;
  p->opts = o;
  p->warn = st;
  p->stream = (hipStream_t)stream;
  p->spread_only = false;
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return ESN_ERR_HIP;
  }
  for (int m = 0; m < 3; m++) p->N[m] = p->nf[m] = 1;
  // quadrature of the correction factors: nodes and weights * phi(node), FP64
  std::vector<double> wq;
  gauss_legendre_positive(par.nquad, &p->t3_zq, &wq);
  p->t3_wphi.resize(par.nquad);
  for (int j = 0; j < par.nquad; j++)
    p->t3_wphi[j] =
        wq[j] * std::exp(par.beta * (std::sqrt(1.0 - p->t3_zq[j] * p->t3_zq[j]) - 1.0));
  // the side stream (default priority) and its ordering event for setpts3
  if (hipStreamCreateWithFlags(&p->t3_side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&p->t3_ready, hipEventDisableTiming) != hipSuccess) {
    t3_destroy(p);
    delete p;
    return ESN_ERR_HIP;
  }
  // per-block partials of up to six arrays, then the six (min, max) pairs
  const int nb = t3_minmax_blocks(kMaxPoints);
  if (t3_alloc(p, (void**)&p->d_t3_mm, sizeof(double) * 2 * 6 * (nb + 1)) ||
      hipHostMalloc((void**)&p->h_t3_mm, sizeof(double) * 2 * 6, hipHostMallocDefault) !=
          hipSuccess) {
    t3_destroy(p);
    delete p;
    return ESN_ERR_ALLOC;
  }
  if (o.debug) {
    for (auto& e : p->ev)
      if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
        t3_destroy(p);
        delete p;
        return ESN_ERR_HIP;
      }
  }
  *out = p;
  return st;
}

extern "C" int esn_setpts3(esn_plan p, int64_t M, int coord_prec, const void* x, const void* y,
                           const void* z, int64_t N, const void* s, const void* t,
                           const void* u) {
  if (!p || p->type != 3 || M < 0 || M > kMaxPoints || N < 0 || N > kMaxPoints)
    return ESN_ERR_BAD_ARG;
  if (coord_prec != ESN_SINGLE && coord_prec != ESN_DOUBLE) return ESN_ERR_BAD_ARG;
  const void* xs[3] = {x, y, z};
  const void* ss[3] = {s, t, u};
  for (int m = 0; m < p->dim; m++)
    if ((M > 0 && !xs[m]) || (N > 0 && !ss[m])) return ESN_ERR_BAD_ARG;
  ESN_HIP(hipSetDevice(p->device));
  hipStream_t st = p->stream;
  p->M = -1;
  p->t3_N = -1;
  const int dim = p->dim, w = p->par.w;
  if (p->opts.debug) ESN_HIP(hipEventRecord(p->ev[5], st));
  const double sigma = p->opts.upsampfac;

  // ---- centres, half-widths, grid sizes and dilations (steps 0 and 1) ----
  double xlo[3], xhi[3], slo[3], shi[3];
  int rc = coord_bounds(p, xs, M, ss, N, coord_prec, xlo, xhi, slo, shi);
  if (rc != ESN_OK) return rc;
  int64_t n[3] = {1, 1, 1};
  double gam[3] = {1, 1, 1}, x0[3] = {0, 0, 0}, s0[3] = {0, 0, 0}, Sh[3] = {0, 0, 0};
  int64_t cells = 1;
  for (int m = 0; m < dim; m++) {
    x0[m] = 0.5 * (xlo[m] + xhi[m]);
    s0[m] = 0.5 * (slo[m] + shi[m]);
    const double X = 0.5 * (xhi[m] - xlo[m]), S = 0.5 * (shi[m] - slo[m]);
    Sh[m] = S;
    const double want = std::max(2.0 * sigma / kPi * X * S + w, 2.0 * w);
    if (!(want < (double)kT3MaxGrid)) return ESN_ERR_BUDGET;
    n[m] = next_smooth_even((int64_t)std::ceil(want));
    // gamma from eq. (ng); with no spread of target frequencies any dilation
    // that keeps the sources w/2 cells inside the box will do (eq. (cond1))
    if (S > 0.0) gam[m] = (double)n[m] / (2.0 * sigma * S);
    else if (X > 0.0) gam[m] = X / (kPi * (1.0 - (double)w / (double)n[m]));
    else gam[m] = 1.0;
    cells *= n[m];
    if (cells > kT3MaxGrid) return ESN_ERR_BUDGET;
  }

  // ---- the two inner plans, remade when the grid changes ----
  bool same = p->t3_spread && p->t3_inner;
  for (int m = 0; m < dim; m++) same = same && n[m] == p->t3_n[m];
  if (!same) {
    if (p->t3_spread) esn_destroy(p->t3_spread);
    if (p->t3_inner) esn_destroy(p->t3_inner);
    p->t3_spread = p->t3_inner = nullptr;
    esn_opts o = p->opts;
    o.modeord = 1;   // the inner type 2 reads the grid as modes in FFT order
    int64_t half[3] = {1, 1, 1};
    for (int m = 0; m < dim; m++) half[m] = n[m] / 2;   // its fine grid is then n
    rc = make_plan(1, dim, half, 1, p->ntransf, p->eps, p->prec, &p->t3_spread, &o, st, true);
    if (rc >= 2) return rc;
    rc = make_plan(2, dim, n, p->isign, p->ntransf, p->eps, p->prec, &p->t3_inner, &o, st, false);
    if (rc >= 2) return rc;
    for (int m = 0; m < dim; m++)
      if (p->t3_spread->nf[m] != n[m]) return ESN_ERR_BAD_ARG;
    for (int m = 0; m < 3; m++) p->t3_n[m] = m < dim ? n[m] : 1;
    const size_t gbytes = (size_t)p->ntransf * cells * csize(p->prec);
    if (t3_alloc(p, &p->d_t3_grid, gbytes)) return ESN_ERR_ALLOC;
    p->t3_cap_grid = cells;
  }
  for (int m = 0; m < 3; m++) {
    p->t3_x0[m] = x0[m];
    p->t3_s0[m] = s0[m];
    p->t3_gam[m] = gam[m];
    p->nf[m] = p->t3_n[m];
  }

  // ---- per-point and per-target arrays ----
  const size_t cs = csize(p->prec);
  if (M > p->t3_cap_M) {
    if (t3_alloc(p, &p->d_t3_pre, cs * M) ||
        t3_alloc(p, &p->d_t3_c, cs * M * (size_t)p->ntransf))
      return ESN_ERR_ALLOC;
    p->t3_cap_M = M;
  }
  if (N > p->t3_cap_N) {
    if (t3_alloc(p, &p->d_t3_post, cs * N)) return ESN_ERR_ALLOC;
    p->t3_cap_N = N;
  }
  const int64_t nxy = std::max<int64_t>(std::max(M, N), 1);
  if (nxy > p->t3_cap_xy) {
    if (t3_alloc(p, (void**)&p->d_t3_xy, sizeof(double) * 6 * nxy)) return ESN_ERR_ALLOC;
    p->t3_cap_xy = nxy;
  }

  // ---- sources: rescale, prephase, sort (step 1) ----
  T3Args a;
  std::memset(&a, 0, sizeof(a));
  a.dim = dim;
  a.isign = p->isign;
  a.w = w;
  for (int m = 0; m < 3; m++) {
    a.x0[m] = x0[m];
    a.s0[m] = s0[m];
    a.inv_gam[m] = 1.0 / gam[m];
    a.hgam[m] = 2.0 * kPi / (double)p->t3_n[m] * gam[m];
    a.out[m] = p->d_t3_xy + m * p->t3_cap_xy;
    // the targets' u = (w/2) s'' lie in [-U, U]
    t3_cheb(p->t3_zq, p->t3_wphi, m < dim ? 0.5 * w * a.hgam[m] * Sh[m] : 0.0, a.cheb[m],
            &a.cscale[m]);
  }
  a.n = M;
  ESN_HIP(launch_t3_sources(a, coord_prec, p->prec, xs, p->d_t3_pre, st));

  // ---- targets: rescale, correction and postphase (steps 2 and 3) ----
  T3Args b = a;
  b.n = N;
  for (int m = 0; m < 3; m++) b.out[m] = p->d_t3_xy + (3 + m) * p->t3_cap_xy;
  ESN_HIP(launch_t3_targets(b, coord_prec, p->prec, ss, p->d_t3_post, st));

  // ---- both sorts at once: the sources' on the plan's stream, the targets'
  // on the side stream from a second host thread (each setpts waits for its
  // own stream at its end) ----
  ESN_HIP(hipEventRecord(p->t3_ready, st));
  ESN_HIP(hipStreamWaitEvent(p->t3_side, p->t3_ready, 0));
  if (plan_set_stream(p->t3_inner, p->t3_side) != ESN_OK) return ESN_ERR_FFT_PLAN;
  std::future<int> inner = std::async(std::launch::async, [&]() {
    return esn_setpts(p->t3_inner, N, ESN_DOUBLE, b.out[0], dim > 1 ? b.out[1] : nullptr,
                      dim > 2 ? b.out[2] : nullptr);
  });
  const int rc_src = esn_setpts(p->t3_spread, M, ESN_DOUBLE, a.out[0],
                                dim > 1 ? a.out[1] : nullptr, dim > 2 ? a.out[2] : nullptr);
  const int rc_tgt = inner.get();
  if (plan_set_stream(p->t3_inner, st) != ESN_OK) return ESN_ERR_FFT_PLAN;
  if (rc_src != ESN_OK) return rc_src;
  if (rc_tgt != ESN_OK) return rc_tgt;
  p->M = M;
  p->t3_N = N;
  if (p->opts.debug) {
    ESN_HIP(hipEventRecord(p->ev[0], st));
    ESN_HIP(hipEventSynchronize(p->ev[0]));
    float ms = 0;
    ESN_HIP(hipEventElapsedTime(&ms, p->ev[5], p->ev[0]));
    p->stats.t_setpts = ms;
  }
  return ESN_OK;
}

int t3_execute(esn_plan p, void* c, void* f) {
  if (p->M < 0 || p->t3_N < 0) return ESN_ERR_NO_POINTS;
  if ((p->M > 0 && !c) || (p->t3_N > 0 && !f)) return ESN_ERR_BAD_ARG;
  ESN_HIP(hipSetDevice(p->device));
  hipStream_t st = p->stream;
  if (p->t3_N == 0) return p->warn;
  const bool dbg = p->opts.debug != 0;
  if (dbg) ESN_HIP(hipEventRecord(p->ev[0], st));
  // step 1: prephased strengths spread onto the type 3 grid
  ESN_HIP(launch_cmul(p->prec, c, p->d_t3_pre, p->d_t3_c, p->M, p->ntransf, st));
  if (dbg) ESN_HIP(hipEventRecord(p->ev[1], st));
  int rc = esn_spread(p->t3_spread, p->d_t3_c, p->d_t3_grid);
  if (rc >= 2) return rc;
  if (dbg) ESN_HIP(hipEventRecord(p->ev[2], st));
  // step 2: the grid as Fourier coefficients, evaluated at the rescaled targets
  rc = esn_execute(p->t3_inner, f, p->d_t3_grid);
  if (rc >= 2) return rc;
  if (dbg) ESN_HIP(hipEventRecord(p->ev[3], st));
  // step 3: correction and postphase
  ESN_HIP(launch_cmul(p->prec, f, p->d_t3_post, f, p->t3_N, p->ntransf, st));
  if (dbg) {
    ESN_HIP(hipEventRecord(p->ev[4], st));
    ESN_HIP(hipEventSynchronize(p->ev[4]));
    float sp = 0, in = 0, tot = 0;
    ESN_HIP(hipEventElapsedTime(&sp, p->ev[1], p->ev[2]));
    ESN_HIP(hipEventElapsedTime(&in, p->ev[2], p->ev[3]));
    ESN_HIP(hipEventElapsedTime(&tot, p->ev[0], p->ev[4]));
    p->stats.t_spread_or_interp = sp;   // step 1 spreading
    p->stats.t_fft = in;                // step 2: the inner type 2 transform
    esn_stats inner;
    if (plan_stats(p->t3_inner, &inner) != ESN_OK) return ESN_ERR_HIP;
    p->stats.t_deconv_or_amplify = inner.t_spread_or_interp;   // its interpolation
    p->stats.t_execute = tot;
  }
  return p->warn;
}

void t3_destroy(esn_plan p) {
  (void)hipStreamSynchronize(p->stream);
  if (p->t3_spread) esn_destroy(p->t3_spread);
  if (p->t3_inner) esn_destroy(p->t3_inner);
  p->t3_spread = p->t3_inner = nullptr;
  t3_free(&p->d_t3_pre);
  t3_free(&p->d_t3_post);
  t3_free(&p->d_t3_grid);
  t3_free(&p->d_t3_c);
  t3_free((void**)&p->d_t3_xy);
  t3_free((void**)&p->d_t3_mm);
  if (p->t3_ready) (void)hipEventDestroy(p->t3_ready);
  if (p->t3_side) (void)hipStreamDestroy(p->t3_side);
  p->t3_ready = nullptr;
  p->t3_side = nullptr;
  if (p->h_t3_mm) (void)hipHostFree(p->h_t3_mm);
  p->h_t3_mm = nullptr;
}

}  // namespace esn
