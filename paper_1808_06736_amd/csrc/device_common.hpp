// Device helpers shared by the spread / interp kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "esn_internal.hpp"

namespace esn {

template <typename T> struct CT;                    // complex type of precision T
template <> struct CT<float> { using type = float2; };
template <> struct CT<double> { using type = double2; };
template <typename T> using cplx_t = typename CT<T>::type;

// A sorted point's coordinate in one dimension, split into the fine-grid cell
// c = floor(t) (c in [0, n)) and the offset within it, f = t - c in [0, 1).
template <typename T>
struct Coord {
  int cell;
  T f;
};

// Window shift sh in {0, 1} of a coordinate whose offset in its cell is
// fr 2^-fbits (fixed point) or f (FP64): w even: f > 0; w odd: f > 1/2 (see
// the window comment below), decided exactly on the stored bits.
__host__ __device__ __forceinline__ int window_shift_fixed(uint32_t fr, int fbits, int w) {
  return (w & 1) ? (fr > (1u << (fbits - 1)) ? 1 : 0) : (fr != 0u ? 1 : 0);
}
__host__ __device__ __forceinline__ int window_shift_f64(double f, int w) {
  return (w & 1) ? (f > 0.5 ? 1 : 0) : (f > 0.0 ? 1 : 0);
}

// Window cell of a coordinate: c + sh wrapped into [0, n).  Its window starts
// floor(w/2) cells before it, so points are binned by it: a bin's windows all
// start in the bin's cells moved back by floor(w/2).  (c = n - 1 with sh = 1
// wraps to 0; the window n - floor(w/2) .. is then taken as -floor(w/2) ..,
// the same cells of the periodic grid.)
__host__ __device__ __forceinline__ int window_cell(int cell, int sh, int64_t n) {
  const int k = cell + sh;
  return k >= n ? k - (int)n : k;
}

// Coordinate of a fixed-point value v (cell in the high bits, fbits bits of
// fraction) or of an FP64 value t.
template <typename T>
__device__ __forceinline__ Coord<T> decode_fixed(uint32_t v, int fbits, int* sh_out, int w) {
  Coord<T> r;
  const uint32_t mask = (fbits >= 32) ? 0xffffffffu : ((1u << fbits) - 1u);
  const uint32_t fr = v & mask;
  r.cell = (int)(fbits >= 32 ? 0u : (v >> fbits));
  // the fraction fr * 2^-fbits (exact in float when fbits <= 24)
  if constexpr (sizeof(T) == 4) r.f = ldexpf((float)fr, -fbits);
  else r.f = ldexp((double)fr, -fbits);
  *sh_out = window_shift_fixed(fr, fbits, w);
  return r;
}
template <typename T>
__device__ __forceinline__ Coord<T> decode_f64(double t, int* sh_out, int w) {
  Coord<T> r;
  const double c = floor(t);
  const double f = t - c;                      // exact in FP64
  r.cell = (int)c;
  r.f = (T)f;
  *sh_out = window_shift_f64(f, w);
  return r;
}

// Coordinate m of sorted point i from its record.
template <typename T>
__device__ __forceinline__ Coord<T> decode_coord(const unsigned char* pts, int code, int fbits,
                                                 int64_t i, int m, int* sh_out, int w) {
  if (code == kPtsFixed32)
    return decode_fixed<T>(reinterpret_cast<const uint32_t*>(pts + i * 16)[m], fbits, sh_out, w);
  return decode_f64<T>(reinterpret_cast<const double*>(pts + i * 32)[m], sh_out, w);
}

// Original index of sorted point i.
__device__ __forceinline__ int64_t point_perm(const unsigned char* pts, int code, int64_t i) {
  return code == kPtsFixed32 ? reinterpret_cast<const int32_t*>(pts + i * 16)[3]
                             : reinterpret_cast<const int32_t*>(pts + i * 32)[6];
}

// Window of a point at fine-grid coordinate t = c + f: the w cells
// l0 .. l0 + w - 1 with l0 = ceil(t - w/2) = c - floor(w/2) + sh, where
// sh in {0, 1} is decided exactly from f (w even: f > 0; w odd: f > 1/2).
// When t - w/2 is an integer the left end of the closed support (z = -1) is
// the first window cell and the right end (z = +1) is left out.
//
// ES kernel values at the window, eq. (ES) rescaled by alpha = w h / 2
// (eqs. (al), (psi1)):  ker[k] = phi((l0 + k - t) / (w/2)),
// phi(z) = exp(beta (sqrt(1 - z^2) - 1)).
template <int W>
__device__ __forceinline__ void es_weights_f32(int sh, float f, float beta, float* ker) {
  // offset of the first window cell from t, in [-W/2, -W/2 + 1]
  const float off = (float)(sh - W / 2) - f;
  const float s = 2.0f / (float)W;
#pragma unroll
  for (int k = 0; k < W; k++) {
    float z = (off + (float)k) * s;
    float a = fmaxf(1.0f - z * z, 0.0f);
    ker[k] = __expf(beta * (__fsqrt_rn(a) - 1.0f));
  }
}

template <int W>
__device__ __forceinline__ void es_weights_f64(int sh, double f, double beta, double* ker) {
  const double off = (double)(sh - W / 2) - f;
  const double s = 2.0 / (double)W;
#pragma unroll
  for (int k = 0; k < W; k++) {
    double z = (off + (double)k) * s;
    double a = fmax(1.0 - z * z, 0.0);
    ker[k] = exp(beta * (sqrt(a) - 1.0));
  }
}

template <int W, typename T>
__device__ __forceinline__ void es_weights_t(int sh, T f, T beta, T* ker) {
  if constexpr (sizeof(T) == 4) es_weights_f32<W>(sh, f, beta, ker);
  else es_weights_f64<W>(sh, f, beta, ker);
}

// The same from the piecewise polynomial table c[W][W + kPolyExtra + 1]
// (Sec. 5.3): window cell k lies in interval k at the local coordinate
// t = 2 u - 1, u = l0 - t_point + W/2 in [0, 1) (the same for all k), and its
// weight is interval k's polynomial at t (Horner's scheme).  c is the same for
// every thread, so its values come through scalar loads.
template <int W, typename T>
__device__ __forceinline__ void es_weights_poly(int sh, T f, const T* __restrict__ cg, T* ker) {
  constexpr int P = W + kPolyExtra;
  // read-only for the whole launch: through the constant address space, so the
  // uniform loads become scalar loads even after the kernel's own stores
  typedef const __attribute__((address_space(4))) T* ConstPtr;
  const ConstPtr c = (ConstPtr)cg;
  const T u = (T)sh - f + ((W & 1) ? (T)0.5 : (T)0);
  const T t = (T)2 * u - (T)1;
#pragma unroll
  for (int k = 0; k < W; k++) {
    T acc = c[k * (P + 1) + P];
#pragma unroll
    for (int j = P - 1; j >= 0; j--) acc = fma(acc, t, c[k * (P + 1) + j]);
    ker[k] = acc;
  }
}

// Kernel values by the plan's method: the table when ktab is set, else exp and sqrt.
template <int W, typename T>
__device__ __forceinline__ void es_weights_any(int sh, T f, T beta, const void* ktab, T* ker) {
  if (ktab) es_weights_poly<W, T>(sh, f, static_cast<const T*>(ktab), ker);
  else es_weights_t<W, T>(sh, f, beta, ker);
}

// Periodic wrap of an index that lies in [-n, 2n).
__device__ __forceinline__ int64_t wrap_once(int64_t g, int64_t n) {
  if (g < 0) g += n;
  if (g >= n) g -= n;
  return g;
}

// Periodic wrap of any index.
__device__ __forceinline__ int64_t wrap_any(int64_t g, int64_t n) {
  g %= n;
  return g < 0 ? g + n : g;
}

}  // namespace esn
