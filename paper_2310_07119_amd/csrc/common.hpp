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

// exp(-i * arg) for an FP64 argument. FP64 storage: FP64 sincos.
// FP32 storage: the argument is reduced modulo 2 pi in FP64 and the reduced
// angle is evaluated in FP32.
template <class T>
__device__ __forceinline__ cx<T> expmi(double arg);
template <>
__device__ __forceinline__ cx<double> expmi<double>(double arg) {
  double s, c;
  sincos(arg, &s, &c);
  return {c, -s};
}
template <>
__device__ __forceinline__ cx<float> expmi<float>(double arg) {
  const double two_pi = 6.283185307179586476925286766559;
  double r = arg - two_pi * rint(arg * (1.0 / two_pi));
  float s, c;
  sincosf((float)r, &s, &c);
  return {c, -s};
}

}  // namespace tw
