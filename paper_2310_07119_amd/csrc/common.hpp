// Device-side complex arithmetic and small helpers shared by the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tw {

template <class T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};

template <class T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {  // a * conj(b)
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
template <class T>
__device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return {a.re * s, a.im * s}; }
// multiply by -i (forward) or +i (inverse)
template <class T, bool INV>
__device__ __forceinline__ cx<T> mul_mi(cx<T> a) {
  if constexpr (INV) return {-a.im, a.re};
  else return {a.im, -a.re};
}
template <class T>
__device__ __forceinline__ T abs2(cx<T> a) { return a.re * a.re + a.im * a.im; }

// Complex value of precision T times an FP64 factor, computed in FP64 and rounded
// back to T (exact for T = double).
template <class T>
__device__ __forceinline__ cx<T> mul_d(cx<T> a, cx<double> f) {
  double r = (double)a.re * f.re - (double)a.im * f.im;
  double i = (double)a.re * f.im + (double)a.im * f.re;
  return {(T)r, (T)i};
}
template <class T>
__device__ __forceinline__ cx<T> mul_d(cx<T> a, double f) {
  return {(T)((double)a.re * f), (T)((double)a.im * f)};
}

// exp(-i * arg) for an FP64 argument, in both storage precisions.
//
// The argument is reduced by quarter turns, arg = k pi/2 + r with |r| <= pi/4,
// using pi/2 split into three parts (the first two with 33 significant bits,
// so k * part is exact for |k| < 2^20: Cody and Waite's reduction). sin r and
// cos r are Taylor series, truncated where the next term is below one unit in
// the last place of the storage precision (FP64: through r^17 and r^16; FP32:
// through r^9 and r^10), and the quadrant k mod 4 maps them to sin and cos of
// arg. Arguments beyond 10^6 (never reached by kick phases) take the library
// sincos.
__device__ __forceinline__ double quarter_turns(double arg, int& q) {
  const double k = rint(arg * 0.63661977236758134308);  // 2/pi
  q = (int)((long long)k & 3);
  return ((arg - k * 1.5707963267341256) - k * 6.077100506303966e-11) - k * 2.0222662487959506e-21;
}

// (cos, sin) of the reduced angle mapped to the quadrant: returns exp(-i arg).
template <class T>
__device__ __forceinline__ cx<T> quadrant(T c, T s, int q) {
  T cosx, sinx;
  switch (q) {
    case 0: cosx = c; sinx = s; break;
    case 1: cosx = -s; sinx = c; break;
    case 2: cosx = -c; sinx = -s; break;
    default: cosx = s; sinx = -c; break;
  }
  return {cosx, -sinx};
}

__device__ __forceinline__ void sincos_series(double x, double& s, double& c) {
  const double x2 = x * x;
  double ps = -1.0 / 355687428096000.0;
  ps = ps * x2 + 1.0 / 1307674368000.0;
  ps = ps * x2 - 1.0 / 6227020800.0;
  ps = ps * x2 + 1.0 / 39916800.0;
  ps = ps * x2 - 1.0 / 362880.0;
  ps = ps * x2 + 1.0 / 5040.0;
  ps = ps * x2 - 1.0 / 120.0;
  ps = ps * x2 + 1.0 / 6.0;
  double pc = 1.0 / 20922789888000.0;
  pc = pc * x2 - 1.0 / 87178291200.0;
  pc = pc * x2 + 1.0 / 479001600.0;
  pc = pc * x2 - 1.0 / 3628800.0;
  pc = pc * x2 + 1.0 / 40320.0;
  pc = pc * x2 - 1.0 / 720.0;
  pc = pc * x2 + 1.0 / 24.0;
  pc = pc * x2 - 0.5;
  s = x - x * x2 * ps;
  c = 1.0 + x2 * pc;
}

__device__ __forceinline__ void sincos_series(float x, float& s, float& c) {
  const float x2 = x * x;
  float ps = 1.f / 362880.f;
  ps = ps * x2 - 1.f / 5040.f;
  ps = ps * x2 + 1.f / 120.f;
  ps = ps * x2 - 1.f / 6.f;
  float pc = -1.f / 3628800.f;
  pc = pc * x2 + 1.f / 40320.f;
  pc = pc * x2 - 1.f / 720.f;
  pc = pc * x2 + 1.f / 24.f;
  pc = pc * x2 - 0.5f;
  s = x + x * x2 * ps;
  c = 1.f + x2 * pc;
}

// exp(-i x) for |x| <= 2^-5 (FP64): typical kick phases are far below pi/4,
// and the series through x^7 / x^8 already leave a remainder below
// x^9/9! < 2^-64 |x|
__device__ __forceinline__ cx<double> expmi_small(double x) {
  const double x2 = x * x;
  const double ps = ((-1.0 / 5040.0) * x2 + 1.0 / 120.0) * x2 - 1.0 / 6.0;
  const double pc = (((1.0 / 40320.0) * x2 - 1.0 / 720.0) * x2 + 1.0 / 24.0) * x2 - 0.5;
  return {1.0 + x2 * pc, -(x + x * x2 * ps)};
}

template <class T>
__device__ __forceinline__ cx<T> expmi(double arg) {
  T s, c;
  if constexpr (sizeof(T) == 8) {
    if (fabs(arg) <= 0.03125) return expmi_small(arg);
  }
  if (fabs(arg) <= 0.78539816339744830962) {  // small kick phases
    sincos_series((T)arg, s, c);
    return {c, -s};
  }
  if (fabs(arg) <= 1.0e6) {
    int q;
    const double r = quarter_turns(arg, q);
    sincos_series((T)r, s, c);
    return quadrant<T>(c, s, q);
  }
  if constexpr (sizeof(T) == 8) {
    double sd, cd;
    sincos(arg, &sd, &cd);
    return {(T)cd, (T)(-sd)};
  } else {
    const double two_pi = 6.283185307179586476925286766559;
    const double r = arg - two_pi * rint(arg * (1.0 / two_pi));
    float sf, cf;
    sincosf((float)r, &sf, &cf);
    return {cf, -sf};
  }
}

// The kick psi <- psi exp(-i arg) (Sec. "Integrating the equations of motion").
// FP64: the product with the factor of expmi. FP32: exp(-i arg) = (-i)^q
// exp(-i r) with arg = q pi/2 + r, |r| <= pi/4 (FP64 reduction): the quarter
// turns are exact swaps and sign changes, and exp(-i r) is applied as three
// shears, x -= t y, y -= s x, x -= t y with s = sin r, t = tan(r/2) =
// s / (1 + cos r), each of determinant 1 whatever s and t round to. A factor
// formed as (cos, sin) rounded to float instead has |f|^2 - 1 up to 6e-8 (for
// |r| below 2.4e-4 cos rounds to exactly 1 and every kick grew the norm by r^2).
__device__ __forceinline__ void sincos_m1_series(float x, float& s, float& cm1) {
  const float x2 = x * x;
  float ps = 1.f / 362880.f;
  ps = ps * x2 - 1.f / 5040.f;
  ps = ps * x2 + 1.f / 120.f;
  ps = ps * x2 - 1.f / 6.f;
  float pc = -1.f / 3628800.f;
  pc = pc * x2 + 1.f / 40320.f;
  pc = pc * x2 - 1.f / 720.f;
  pc = pc * x2 + 1.f / 24.f;
  pc = pc * x2 - 0.5f;
  s = x + x * x2 * ps;
  cm1 = x2 * pc;
}

// Rotation of w by -x for |x| <= 2^-5 as the three shears above, with sin x
// and tan(x/2) from their series (the next terms are below 1e-12 relative).
__device__ __forceinline__ cx<float> rotate_small(cx<float> w, float x) {
  const float x2 = x * x, xx2 = x * x2;
  const float s = __builtin_fmaf(xx2, __builtin_fmaf(x2, 1.f / 120.f, -1.f / 6.f), x);
  const float t = __builtin_fmaf(0.5f * xx2, __builtin_fmaf(x2, 1.f / 120.f, 1.f / 12.f), 0.5f * x);
  const float x1 = __builtin_fmaf(t, w.im, w.re);
  const float y1 = __builtin_fmaf(-s, x1, w.im);
  return {__builtin_fmaf(t, y1, x1), y1};
}

template <class T>
__device__ __forceinline__ cx<T> kick_rotate(cx<T> v, double arg) {
  if constexpr (sizeof(T) == 8) {
    return cmul(v, expmi<T>(arg));
  } else {
    int q = 0;
    double r = arg;
    if (fabs(arg) > 0.78539816339744830962) {
      if (fabs(arg) > 1.0e6) {
        const double two_pi = 6.283185307179586476925286766559;
        r = arg - two_pi * rint(arg * (1.0 / two_pi));
      }
      r = quarter_turns(r, q);
    }
    cx<float> w = v;
    switch (q) {  // times (-i)^q
      case 1: w = {v.im, -v.re}; break;
      case 2: w = {-v.re, -v.im}; break;
      case 3: w = {-v.im, v.re}; break;
      default: break;
    }
    if (fabs(r) <= 0.03125) return rotate_small(w, (float)r);
    float s, cm1;
    sincos_m1_series((float)r, s, cm1);
    const float t = s * __builtin_amdgcn_rcpf(2.f + cm1);
    // rotation by -r
    const float x1 = __builtin_fmaf(t, w.im, w.re);
    const float y1 = __builtin_fmaf(-s, x1, w.im);
    const float x2 = __builtin_fmaf(t, y1, x1);
    return {x2, y1};
  }
}

// The kick of one field's R values held by a thread, v_m <- v_m exp(-i kick V_m),
// with V_m the real (im = false) or imaginary part of the pair-packed
// potential pot[m]. FP64: kick_rotate of each value. FP32: the phases are
// formed in FP32 with the kick factor split into two floats (kick = k_hi +
// k_lo, so the phase carries one rounding and no bias from rounding the kick
// factor); when all R lie within 2^-5 (kick phases are small) each value
// takes rotate_small, otherwise each takes kick_rotate with its FP64 phase.
// One branch per field instead of one per value.
template <class T, int R>
__device__ __forceinline__ void kick_values(cx<T> (&v)[R], const cx<T> (&pot)[R], bool im, double kick) {
  if constexpr (sizeof(T) == 8) {
    // one branch per field: the short series for all R when every phase is
    // below 2^-5 (the same values kick_rotate gives them)
    double x[R];
    bool small = true;
#pragma unroll
    for (int m = 0; m < R; ++m) {
      x[m] = kick * (im ? pot[m].im : pot[m].re);
      small = small && fabs(x[m]) <= 0.03125;
    }
    if (small) {
#pragma unroll
      for (int m = 0; m < R; ++m) v[m] = cmul(v[m], expmi_small(x[m]));
    } else {
#pragma unroll
      for (int m = 0; m < R; ++m) v[m] = kick_rotate<T>(v[m], x[m]);
    }
  } else {
    const float kh = (float)kick, kl = (float)(kick - (double)kh);
    float x[R];
    bool small = true;
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const float p = im ? pot[m].im : pot[m].re;
      x[m] = __builtin_fmaf(kh, p, kl * p);
      small = small && fabsf(x[m]) <= 0.03125f;
    }
    if (small) {
#pragma unroll
      for (int m = 0; m < R; ++m) v[m] = rotate_small(v[m], x[m]);
    } else {
#pragma unroll
      for (int m = 0; m < R; ++m) v[m] = kick_rotate<T>(v[m], kick * (double)(im ? pot[m].im : pot[m].re));
    }
  }
}

// Green's function factor of the Poisson solve at |k|^2 = k2 (zero mode
// removed), -4 pi G / (|k|^2 N) with green = -4 pi G / N, in FP64 (applied with
// mul_d). FP64 passes divide; FP32 passes take the hardware reciprocal
// estimate refined by two Newton steps, exact far below FP32 resolution (a
// per-mode error of FP32 size would bias the potential the same way every step).
template <class T>
__device__ __forceinline__ double green_factor(double k2, double green) {
  if constexpr (sizeof(T) == 8) {
    return (k2 == 0.0) ? 0.0 : green / k2;
  } else {
    double r = __builtin_amdgcn_rcp(k2);
    r = __builtin_fma(r, __builtin_fma(-k2, r, 1.0), r);
    r = __builtin_fma(r, __builtin_fma(-k2, r, 1.0), r);
    return (k2 == 0.0) ? 0.0 : green * r;
  }
}

}  // namespace tw
