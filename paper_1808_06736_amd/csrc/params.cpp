// Host-side plan arithmetic: kernel width and shape, fine-grid sizes and the
// Gauss-Legendre rule behind the kernel's Fourier transform.  All FP64.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "esn_internal.hpp"

namespace esn {

// Kernel width from the tolerance, eq. (params): w = ceil(log10(1/eps)) + 1,
// i.e. one more than the number of requested digits.  A tiny guard keeps exact
// powers of ten (1e-6 -> 6 digits) from rounding up by one ulp of log10.
// Clamped to [2, kMaxW].  Returns false when clamping at the top was needed.
bool width_from_eps(double eps, int* w_out) {
  double digits = std::log10(1.0 / eps);
  int w = (int)std::ceil(digits - 1e-10) + 1;
  bool ok = true;
  if (w < 2) w = 2;
  if (w > kMaxW) { w = kMaxW; ok = false; }
  *w_out = w;
  return ok;
}

// Low upsampling, sigma = 5/4.  The paper names the option but fixes no
// parameters for it; they follow here from its own recipe.  beta is eq. (gam),
// beta = gamma pi w (1 - 1/(2 sigma)), with the safety factor gamma = 0.976
// that turns eq. (gam) into the factor 2.30 of eq. (params) at sigma = 2; at
// sigma = 5/4 this is 1.8397 w.  The width grows with the digits at the rate
// of eq. (ESerr) without its algebraic factor: 1 / (pi gamma sqrt(1 - 1/sigma -
// (1/gamma^2 - 1) / (4 sigma^2))) per unit of ln(1/eps), 1.7136 per decade,
// plus a constant 0.6 fitted so that the aliasing bound of eq. (epsest) stays
// within 5 eps over eps = 1e-1 .. 1e-9, as the sigma = 2 rule keeps it within
// 2 to 9 eps for w <= 13.
constexpr double kSafety = 0.976;
constexpr double kSigmaLow = 1.25;
constexpr double kLowWidthConst = 0.6;

double beta_for(int w, double sigma) {
  if (sigma == 2.0) return 2.30 * w;   // eq. (params)
  return kSafety * M_PI * w * (1.0 - 0.5 / sigma);
}

bool width_from_eps_low(double eps, int* w_out) {
  const double sigma = kSigmaLow;
  const double rate = M_PI * kSafety *
                      std::sqrt(1.0 - 1.0 / sigma - (1.0 / (kSafety * kSafety) - 1.0) /
                                                        (4.0 * sigma * sigma));
  const double per_decade = std::log(10.0) / rate;
  int w = (int)std::ceil(per_decade * std::log10(1.0 / eps) + kLowWidthConst - 1e-10);
  bool ok = true;
  if (w < 2) w = 2;
  if (w > kMaxW) { w = kMaxW; ok = false; }
  *w_out = w;
  return ok;
}

// Smallest integer >= n of the form 2^a 3^b 5^c (Sec. 3.1: FFT-friendly sizes).
int64_t next_smooth235(int64_t n) {
  if (n <= 1) return 1;
  for (int64_t m = n;; m++) {
    int64_t r = m;
    while (r % 2 == 0) r /= 2;
    while (r % 3 == 0) r /= 3;
    while (r % 5 == 0) r /= 5;
    if (r == 1) return m;
  }
}

// Fine grid size of one dimension (Sec. 3.1 and its d > 1 case):
// n >= sigma N, n >= 2w, n = 2^a 3^b 5^c.
int64_t fine_size(int64_t N, double sigma, int w) {
  int64_t need = (int64_t)std::ceil(sigma * (double)N - 1e-9);
  if (need < 2 * w) need = 2 * w;
  return next_smooth235(need);
}

// Legendre polynomial P_n(x) and its derivative by the three-term recurrence.
static void legendre(int n, double x, double* pn, double* dpn) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { *pn = 1.0; *dpn = 0.0; return; }
  for (int k = 2; k <= n; k++) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  *pn = p1;
  *dpn = n * (x * p1 - p0) / (x * x - 1.0);
}

// The p positive nodes and their weights of the 2p-node Gauss-Legendre rule
// on [-1, 1] (used by eq. (quad)): roots of P_{2p} by Newton's method from the
// asymptotic guesses cos(pi (i - 1/4) / (2p + 1/2)), weights
// 2 / ((1 - x^2) P'_{2p}(x)^2).  Nodes come out in decreasing order.
void gauss_legendre_positive(int p, std::vector<double>* nodes,
                             std::vector<double>* weights) {
  const int n = 2 * p;
  nodes->resize(p);
  weights->resize(p);
  for (int i = 1; i <= p; i++) {
    double x = std::cos(M_PI * (i - 0.25) / (n + 0.5));
    double pn = 0, dpn = 1;
    for (int it = 0; it < 100; it++) {
      legendre(n, x, &pn, &dpn);
      double dx = pn / dpn;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    legendre(n, x, &pn, &dpn);
    (*nodes)[i - 1] = x;
    (*weights)[i - 1] = 2.0 / ((1.0 - x * x) * dpn * dpn);
  }
}

// Number of positive quadrature nodes: p >= 1.5 w + 2 (Sec. 3.1, after eq. (quad)).
int quad_nodes_for_width(int w) { return (int)std::ceil(1.5 * w + 2.0); }

}  // namespace esn

extern "C" int esn_choose_params(double eps, int prec, int dim, const int64_t* nmodes,
                                 double upsampfac, esn_params* out) {
  if (!out || !nmodes || dim < 1 || dim > 3) return ESN_ERR_BAD_ARG;
  if (!(eps > 0.0) || !std::isfinite(eps)) return ESN_ERR_BAD_ARG;
  if (prec != ESN_SINGLE && prec != ESN_DOUBLE) return ESN_ERR_BAD_ARG;
  if (upsampfac != 2.0 && upsampfac != esn::kSigmaLow) return ESN_ERR_BAD_ARG;
  for (int m = 0; m < dim; m++)
    if (nmodes[m] < 1) return ESN_ERR_BAD_ARG;
  int w = 0;
  const bool ok = upsampfac == 2.0 ? esn::width_from_eps(eps, &w) : esn::width_from_eps_low(eps, &w);
  int status = ESN_OK;
  if (!ok || eps < 1e-15 || (prec == ESN_SINGLE && eps < 1e-6))
    status = ESN_WARN_EPS_TOO_SMALL;
  out->w = w;
  out->beta = esn::beta_for(w, upsampfac);
  out->nquad = esn::quad_nodes_for_width(w);
  for (int m = 0; m < 3; m++)
    out->nf[m] = (m < dim) ? esn::fine_size(nmodes[m], upsampfac, w) : 1;
  return status;
}

extern "C" int esn_gauss_legendre(int p, double* nodes, double* weights) {
  if (p < 1 || p > 4096 || !nodes || !weights) return ESN_ERR_BAD_ARG;
  std::vector<double> q, w;
  esn::gauss_legendre_positive(p, &q, &w);
  for (int i = 0; i < p; i++) {
    nodes[i] = q[i];
    weights[i] = w[i];
  }
  return ESN_OK;
}

extern "C" int esn_correction_factors(int w, double beta, int nquad, int64_t nf, int64_t N,
                                      double* out) {
  if (w < 2 || w > esn::kMaxW || nquad < 1 || nf < 1 || N < 1 || N > nf || !out)
    return ESN_ERR_BAD_ARG;
  std::vector<double> q, wq;
  esn::gauss_legendre_positive(nquad, &q, &wq);
  const double alpha = M_PI * (double)w / (double)nf;   // eq. (al)
  for (int64_t k = 0; k <= N / 2; k++) {
    double s = 0.0;
    for (int j = 0; j < nquad; j++) {
      const double phi = std::exp(beta * (std::sqrt(1.0 - q[j] * q[j]) - 1.0));
      s += wq[j] * phi * std::cos(alpha * (double)k * q[j]);
    }
    out[k] = 1.0 / ((double)w * s);
  }
  return ESN_OK;
}

// Piecewise polynomial form of the ES kernel (Sec. 5.3): the support [-1, 1]
// of phi(z) = exp(beta (sqrt(1 - z^2) - 1)) is split into w equal intervals,
// one per window cell, and each is replaced by a polynomial of degree w + 3
// in the local variable t in [-1, 1], z = (k + (t + 1) / 2 - w / 2) (2 / w) on
// interval k.  The polynomial interpolates phi at the degree + 1 Chebyshev
// points of the interval (FP64 values) and is converted to monomials in t in
// long double.  A window's w ordinates share one t, so its w weights are w
// Horner evaluations with the same argument.
extern "C" int esn_kernel_poly(int w, double beta, double* coeffs) {
  if (w < 2 || w > 16 || !(beta > 0.0) || !coeffs) return ESN_ERR_BAD_ARG;
  const int P = w + esn::kPolyExtra;   // degree
  const int n = P + 1;                 // interpolation points
  std::vector<double> vals(n);
  std::vector<long double> cheb(n), mono(n), tkm1(n), tk(n), tkp1(n);
  for (int k = 0; k < w; k++) {
    for (int i = 0; i < n; i++) {
      const double t = std::cos(M_PI * (i + 0.5) / n);
      const double z = (k + 0.5 * (t + 1.0) - 0.5 * w) * (2.0 / w);
      const double a = std::max(0.0, 1.0 - z * z);
      vals[i] = std::abs(z) <= 1.0 ? std::exp(beta * (std::sqrt(a) - 1.0)) : 0.0;
    }
    // Chebyshev coefficients of the interpolant (discrete cosine transform)
    for (int j = 0; j < n; j++) {
      long double acc = 0.0L;
      for (int i = 0; i < n; i++)
        acc += (long double)vals[i] * std::cos((long double)M_PI * j * (i + 0.5L) / n);
      cheb[j] = (j == 0 ? 1.0L : 2.0L) * acc / n;
    }
    // sum_j cheb[j] T_j(t) in monomials, with T_{j+1} = 2 t T_j - T_{j-1}
    std::fill(mono.begin(), mono.end(), 0.0L);
    std::fill(tkm1.begin(), tkm1.end(), 0.0L);
    std::fill(tk.begin(), tk.end(), 0.0L);
    tkm1[0] = 1.0L;   // T_0
    tk[1] = 1.0L;     // T_1
    mono[0] += cheb[0];
    if (n > 1)
      for (int i = 0; i < n; i++) mono[i] += cheb[1] * tk[i];
    for (int j = 2; j < n; j++) {
      std::fill(tkp1.begin(), tkp1.end(), 0.0L);
      for (int i = 0; i + 1 < n; i++) tkp1[i + 1] += 2.0L * tk[i];
      for (int i = 0; i < n; i++) tkp1[i] -= tkm1[i];
      for (int i = 0; i < n; i++) mono[i] += cheb[j] * tkp1[i];
      tkm1.swap(tk);
      tk.swap(tkp1);
    }
    for (int i = 0; i < n; i++) coeffs[k * n + i] = (double)mono[i];
  }
  return ESN_OK;
}

