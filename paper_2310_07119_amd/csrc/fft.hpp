// Batched 1D complex FFT of a pencil held across TPP threads of a workgroup.
//
// Layout: a pencil of N points is spread over TPP = N/R threads; thread t holds
// points t + TPP*m (m = 0..R-1) in registers, both on input and on output
// ("natural" layout), so pointwise work in Fourier space indexes k = t + TPP*m.
// The transform is a Stockham autosort FFT (every stage reads in natural
// order and writes in natural order, no bit reversal): stage s of radix Rs
// with Ns = product of earlier radices computes, for each butterfly j in
// [0, N/Rs), the Rs-point DFT of inputs x[j + r N/Rs] * W_N^(r (j mod Ns) N/(Ns Rs))
// and writes output r to (j div Ns) Ns Rs + (j mod Ns) + r Ns. With every radix
// dividing R, a thread's butterflies of the first stage read only its own
// registers and those of the last stage write only its own registers, so an
// S-stage transform needs S-1 exchanges through LDS.
//
// Forward: X_k = sum_n x_n exp(-2 pi i k n / N). Inverse: conjugate twiddles,
// no 1/N (callers fold normalisation into their pointwise factors).
//
// LDS: element i of a pencil lives at lds_pad(i) = i + i/8, and consecutive
// pencils are fft_lds_stride(N) = N + N/8 + 1 elements apart. The first
// stage writes with a stride of R = 8 elements; the padding turns it into an
// odd stride so the lanes of one LDS cycle hit distinct banks.
//
// SYNC_WAVE: every pencil is owned by the lanes of a single wavefront, so the
// exchanges only need wavefront-level ordering; otherwise a workgroup barrier.
#pragma once
#include "common.hpp"
#include <utility>

namespace tw {

// ---------------------------------------------------------------- plans
// Power-of-two lengths: 8 points per thread (N <= 512, at most 64 threads per
// pencil), 16 for N = 1024 (so a pencil never spans two wavefronts); radix-8
// stages and one smaller last stage.
__host__ __device__ constexpr int fft_points_per_thread(int N) { return N > 512 ? 16 : (N >= 8 ? 8 : N); }
__host__ __device__ constexpr int fft_threads(int N) { return N / fft_points_per_thread(N); }
__host__ __device__ constexpr int fft_lds_stride(int N) { return N + N / 8 + 1; }
__host__ __device__ constexpr int lds_pad(int i) { return i + (i >> 3); }

__host__ __device__ constexpr int fft_next_radix(int rem) { return (rem % 8 == 0) ? 8 : rem; }
__host__ __device__ constexpr int fft_num_stages(int N, int R) {
  int s = 0;
  int rem = N;
  while (rem > 1) {
    rem /= fft_next_radix(rem);
    ++s;
  }
  return s;
}
__host__ __device__ constexpr int fft_stage_radix(int N, int R, int stage) {
  int rem = N;
  for (int s = 0; s < stage; ++s) rem /= fft_next_radix(rem);
  return fft_next_radix(rem);
}
__host__ __device__ constexpr int fft_stage_ns(int N, int R, int stage) {
  int ns = 1;
  for (int s = 0; s < stage; ++s) ns *= fft_stage_radix(N, R, s);
  return ns;
}

// ----------------------------------------------------------- butterflies
// In-place DFT of the RAD values v[i0 + r*step], r = 0..RAD-1.
template <class T, int RAD, bool INV>
struct Butterfly;

template <class T, bool INV>
struct Butterfly<T, 1, INV> {
  template <int RR>
  static __device__ __forceinline__ void run(cx<T> (&)[RR], int, int) {}
};

template <class T, bool INV>
struct Butterfly<T, 2, INV> {
  template <int RR>
  static __device__ __forceinline__ void run(cx<T> (&v)[RR], int i0, int step) {
    cx<T> a = v[i0], b = v[i0 + step];
    v[i0] = a + b;
    v[i0 + step] = a - b;
  }
};

template <class T, bool INV>
struct Butterfly<T, 4, INV> {
  static __device__ __forceinline__ void dft4(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3) {
    cx<T> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = mul_mi<T, INV>(a1 - a3);
    a0 = t0 + t2;
    a2 = t0 - t2;
    a1 = t1 + t3;
    a3 = t1 - t3;
  }
  template <int RR>
  static __device__ __forceinline__ void run(cx<T> (&v)[RR], int i0, int step) {
    dft4(v[i0], v[i0 + step], v[i0 + 2 * step], v[i0 + 3 * step]);
  }
};

template <class T, bool INV>
struct Butterfly<T, 8, INV> {
  template <int RR>
  static __device__ __forceinline__ void run(cx<T> (&v)[RR], int i0, int step) {
    // even/odd split: X_k = E_k + W8^k O_k, X_{k+4} = E_k - W8^k O_k
    cx<T> e0 = v[i0], e1 = v[i0 + 2 * step], e2 = v[i0 + 4 * step], e3 = v[i0 + 6 * step];
    cx<T> o0 = v[i0 + step], o1 = v[i0 + 3 * step], o2 = v[i0 + 5 * step], o3 = v[i0 + 7 * step];
    Butterfly<T, 4, INV>::dft4(e0, e1, e2, e3);
    Butterfly<T, 4, INV>::dft4(o0, o1, o2, o3);
    const T h = (T)0.70710678118654752440084436210485;
    // W8^1 = (1 -+ i)/sqrt2, W8^2 = -+i, W8^3 = (-1 -+ i)/sqrt2 (forward sign first)
    cx<T> w1o1, w2o2, w3o3;
    if constexpr (!INV) {
      w1o1 = {h * (o1.re + o1.im), h * (o1.im - o1.re)};
      w3o3 = {h * (o3.im - o3.re), -h * (o3.re + o3.im)};
    } else {
      w1o1 = {h * (o1.re - o1.im), h * (o1.im + o1.re)};
      w3o3 = {-h * (o3.re + o3.im), h * (o3.re - o3.im)};
    }
    w2o2 = mul_mi<T, INV>(o2);
    v[i0] = e0 + o0;
    v[i0 + 4 * step] = e0 - o0;
    v[i0 + step] = e1 + w1o1;
    v[i0 + 5 * step] = e1 - w1o1;
    v[i0 + 2 * step] = e2 + w2o2;
    v[i0 + 6 * step] = e2 - w2o2;
    v[i0 + 3 * step] = e3 + w3o3;
    v[i0 + 7 * step] = e3 - w3o3;
  }
};

// ---------------------------------------------------------------- stages
template <bool SYNC_WAVE>
__device__ __forceinline__ void fft_sync() {
  if constexpr (SYNC_WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

template <class T, int N, int TPP, bool INV, bool SW, int S>
struct FftStage {
  static constexpr int R = N / TPP;
  static constexpr int NS = fft_num_stages(N, R);
  static constexpr int RS = fft_stage_radix(N, R, S);
  static constexpr int NSB = fft_stage_ns(N, R, S);  // Ns: product of earlier radices
  static constexpr int NB = R / RS;                   // butterflies per thread
  static_assert(R % RS == 0, "every stage radix must divide the points per thread");

  static __device__ __forceinline__ void run(cx<T> (&v)[R], cx<T>* lds, int t, const cx<T>* __restrict__ twd) {
    if constexpr (S > 0) {
      fft_sync<SW>();  // previous stage's LDS writes are visible
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int j = t + TPP * i;
#pragma unroll
        for (int r = 0; r < RS; ++r) v[i + r * NB] = lds[lds_pad(j + r * (N / RS))];
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int j = t + TPP * i;
      if constexpr (NSB > 1) {
        const int jm = j % NSB;
#pragma unroll
        for (int r = 1; r < RS; ++r) {
          const cx<T> w = twd[r * jm * (N / (NSB * RS))];
          v[i + r * NB] = INV ? cmulc(v[i + r * NB], w) : cmul(v[i + r * NB], w);
        }
      }
      Butterfly<T, RS, INV>::run(v, i, NB);
    }
    if constexpr (S < NS - 1) {
      fft_sync<SW>();  // every lane has consumed the previous contents
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int j = t + TPP * i;
        const int base = (j / NSB) * NSB * RS + (j % NSB);
#pragma unroll
        for (int r = 0; r < RS; ++r) lds[lds_pad(base + r * NSB)] = v[i + r * NB];
      }
      FftStage<T, N, TPP, INV, SW, S + 1>::run(v, lds, t, twd);
    }
  }
};

// Transform the pencil held in v (natural layout) in place. `lds` is this
// pencil's private buffer of fft_lds_stride(N) elements. With SYNC_WAVE =
// false every thread of the workgroup must make the same calls (the stage
// barriers are workgroup-wide). twd[e] = W_N^e.
template <class T, int N, bool INV, bool SYNC_WAVE>
__device__ __forceinline__ void fft_pencil(cx<T> (&v)[N / fft_threads(N)], cx<T>* lds, int t,
                                           const cx<T>* __restrict__ twd) {
  FftStage<T, N, fft_threads(N), INV, SYNC_WAVE, 0>::run(v, lds, t, twd);
}

}  // namespace tw
