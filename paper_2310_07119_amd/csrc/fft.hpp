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
// Lengths with compiled pass kernels (X-macro); 1D resident kernels also take 8.
#define TW_PASS_LENGTHS(X) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(1024)
#define TW_STEP1D_LENGTHS(X) X(8) TW_PASS_LENGTHS(X)
// Supported lengths: powers of two 8..1024 and 3*2^k (24, 48, 96, 192, 384).
// Powers of two: 8 points per thread (N <= 512, at most 64 threads per pencil),
// 16 for N = 1024 (so a pencil never spans two wavefronts); radix-8 stages and
// one smaller last stage. 3*2^k: 12 points per thread, radix-4 stages, then
// radix 2 if needed, then one radix-6 stage (e.g. 96 = 4*4*6, 48 = 4*2*6).
__host__ __device__ constexpr bool fft_is_pow2(int N) { return N > 0 && (N & (N - 1)) == 0; }
__host__ __device__ constexpr bool fft_length_ok(int N) {
  return (fft_is_pow2(N) && N >= 8 && N <= 1024) || N == 24 || N == 48 || N == 96 || N == 192 || N == 384;
}
__host__ __device__ constexpr int fft_points_per_thread(int N) {
  return fft_is_pow2(N) ? (N > 512 ? 16 : (N >= 8 ? 8 : N)) : 12;
}
__host__ __device__ constexpr int fft_threads(int N) { return N / fft_points_per_thread(N); }
__host__ __device__ constexpr int fft_lds_stride(int N) { return N + N / 8 + 1; }
__host__ __device__ constexpr int lds_pad(int i) { return i + (i >> 3); }

// radix of the next stage when `rem` points of the transform are left
__host__ __device__ constexpr int fft_next_radix(int N, int rem) {
  if (fft_is_pow2(N)) return (rem % 8 == 0) ? 8 : rem;
  if (rem == 6) return 6;
  if (rem == 12) return 2;
  return 4;
}
__host__ __device__ constexpr int fft_num_stages(int N, int R) {
  int s = 0;
  int rem = N;
  while (rem > 1) {
    rem /= fft_next_radix(N, rem);
    ++s;
  }
  return s;
}
__host__ __device__ constexpr int fft_stage_radix(int N, int R, int stage) {
  int rem = N;
  for (int s = 0; s < stage; ++s) rem /= fft_next_radix(N, rem);
  return fft_next_radix(N, rem);
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
struct Butterfly<T, 3, INV> {
  // X0 = a+b+c; X1,2 = a - (b+c)/2 -+ i (sqrt3/2)(b-c) for the forward sign
  static __device__ __forceinline__ void dft3(cx<T>& a, cx<T>& b, cx<T>& c) {
    // x sqrt3/2; in FP32 with a float-pair constant rounded once (see the
    // radix-8 butterfly)
    auto h = [](T x) -> T {
      if constexpr (sizeof(T) == 4) {
        return __builtin_fmaf(0.8660254f, x, 1.5543625e-08f * x);
      } else {
        return (T)0.86602540378443864676372317075294 * x;
      }
    };
    const cx<T> t = b + c;
    const cx<T> m = {a.re - (T)0.5 * t.re, a.im - (T)0.5 * t.im};
    const cx<T> d = b - c;
    const cx<T> q = INV ? cx<T>{-h(d.im), h(d.re)} : cx<T>{h(d.im), -h(d.re)};
    a = a + t;
    b = m + q;
    c = m - q;
  }
  template <int RR>
  static __device__ __forceinline__ void run(cx<T> (&v)[RR], int i0, int step) {
    dft3(v[i0], v[i0 + step], v[i0 + 2 * step]);
  }
};

template <class T, bool INV>
struct Butterfly<T, 6, INV> {
  // even/odd split: X_k = E_k + W6^k O_k, X_{k+3} = E_k - W6^k O_k (k = 0, 1, 2)
  template <int RR>
  static __device__ __forceinline__ void run(cx<T> (&v)[RR], int i0, int step) {
    cx<T> e0 = v[i0], e1 = v[i0 + 2 * step], e2 = v[i0 + 4 * step];
    cx<T> o0 = v[i0 + step], o1 = v[i0 + 3 * step], o2 = v[i0 + 5 * step];
    Butterfly<T, 3, INV>::dft3(e0, e1, e2);
    Butterfly<T, 3, INV>::dft3(o0, o1, o2);
    // W6 = 1/2 -+ i sqrt3/2, W6^2 = -1/2 -+ i sqrt3/2 (forward sign first)
    cx<T> p1, p2;
    if constexpr (sizeof(T) == 4) {
      // x sqrt3/2 as a float pair rounded once (a single float constant
      // makes |W6| differ from 1 by 2.7e-8 and scales every transform's norm)
      auto h = [](float x) { return __builtin_fmaf(0.8660254f, x, 1.5543625e-08f * x); };
      if constexpr (!INV) {
        p1 = {0.5f * o1.re + h(o1.im), 0.5f * o1.im - h(o1.re)};
        p2 = {h(o2.im) - 0.5f * o2.re, -0.5f * o2.im - h(o2.re)};
      } else {
        p1 = {0.5f * o1.re - h(o1.im), 0.5f * o1.im + h(o1.re)};
        p2 = {-0.5f * o2.re - h(o2.im), h(o2.re) - 0.5f * o2.im};
      }
    } else {
      const T h = (T)0.86602540378443864676372317075294;
      const cx<T> w1 = INV ? cx<T>{(T)0.5, h} : cx<T>{(T)0.5, -h};
      const cx<T> w2 = INV ? cx<T>{(T)-0.5, h} : cx<T>{(T)-0.5, -h};
      p1 = cmul(o1, w1);
      p2 = cmul(o2, w2);
    }
    v[i0] = e0 + o0;
    v[i0 + 3 * step] = e0 - o0;
    v[i0 + step] = e1 + p1;
    v[i0 + 4 * step] = e1 - p1;
    v[i0 + 2 * step] = e2 + p2;
    v[i0 + 5 * step] = e2 - p2;
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
    // x / sqrt2. In FP32 the constant is a float pair (hi + lo = 1/sqrt2 to
    // about 2^-50) and the product is rounded once; a single float constant is
    // 1.7e-8 (relative) short and shrinks every transform's output norm by a
    // fixed fraction, which accumulated to most of the FP32 norm drift over
    // long runs.
    auto h = [](T x) -> T {
      if constexpr (sizeof(T) == 4) {
        return __builtin_fmaf(0.70710677f, x, 1.21016175e-08f * x);
      } else {
        return (T)0.70710678118654752440084436210485 * x;
      }
    };
    // W8^1 = (1 -+ i)/sqrt2, W8^2 = -+i, W8^3 = (-1 -+ i)/sqrt2 (forward sign first)
    cx<T> w1o1, w2o2, w3o3;
    if constexpr (!INV) {
      w1o1 = {h(o1.re + o1.im), h(o1.im - o1.re)};
      w3o3 = {h(o3.im - o3.re), -h(o3.re + o3.im)};
    } else {
      w1o1 = {h(o1.re - o1.im), h(o1.im + o1.re)};
      w3o3 = {-h(o3.re + o3.im), h(o3.re - o3.im)};
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

// ------------------------------------------------------- FP32 rotations
// FP32 twiddle multiplications are rotations by three shears, exp(i phi) =
// X(-t) Y(s) X(-t) with t = tan(phi/2), s = sin phi, X(a) = [[1, a], [0, 1]],
// Y(b) = [[1, 0], [b, 1]] (Paeth's decomposition). Every shear has
// determinant 1 whatever t and s round to, so the product changes no input's
// norm systematically. A float pair (cos, sin) instead has |w|^2 - 1 up to
// 6e-8 (near the axes no neighbouring pair does better), and the FP32
// transforms shrank the fields' norms by 1e-9 to 1e-8 per transform depending
// on where the field's energy sat. The FP32 table holds (t, s) of the angle
// reduced to |phi| <= pi/2; entries whose angle was beyond pi/2 are -exp(i phi)
// (flip), which the index tells: 4e in (N, 3N). Inverse transforms rotate by -phi.
__host__ __device__ constexpr bool twiddle_flip(int e, int N) { return 4 * e > N && 4 * e < 3 * N; }

template <bool INV>
__device__ __forceinline__ cx<float> shear_rotate(cx<float> v, float t, float s, bool flip) {
  const float tt = INV ? t : -t;
  const float ss = INV ? -s : s;
  const float x1 = __builtin_fmaf(tt, v.im, v.re);
  const float y1 = __builtin_fmaf(ss, x1, v.im);
  const float x2 = __builtin_fmaf(tt, y1, x1);
  return flip ? cx<float>{-x2, -y1} : cx<float>{x2, y1};
}

// --------------------------------------------------------- twiddle cache
// Per-thread twiddles of every stage, loaded once from the table into
// registers (a thread's butterfly indices are the same for every pencil it
// transforms). Stage s, butterfly i, input r >= 1 uses W_N^(r (j mod Ns) N/(Ns Rs)).
// With CACHED = false only the table pointer is kept and each stage reads its
// twiddles when it runs (fewer registers, more memory latency per stage).
// FP64 tables hold (cos, sin); FP32 tables the shear pairs above.
template <class T, int N, bool CACHED_ = true>
struct TwiddleCache {
  static constexpr bool CACHED = CACHED_;
  static constexpr int TPP = fft_threads(N);
  static constexpr int R = N / TPP;
  static constexpr int NS = fft_num_stages(N, R);
  static constexpr int stage_count(int s) {
    return fft_stage_ns(N, R, s) > 1 ? (R / fft_stage_radix(N, R, s)) * (fft_stage_radix(N, R, s) - 1) : 0;
  }
  static constexpr int stage_offset(int s) {
    int o = 0;
    for (int q = 0; q < s; ++q) o += stage_count(q);
    return o;
  }
  static constexpr int COUNT = stage_offset(NS);
  static constexpr int SIZE = (CACHED && COUNT > 0) ? COUNT : 1;
  cx<T> w[SIZE];
  const cx<T>* table;
  int t_;

  __device__ __forceinline__ void load(const cx<T>* __restrict__ twd, int t) {
    table = twd;
    t_ = t;
    if constexpr (CACHED) load_stage<0>(twd, t);
  }
  // table index of the twiddle of stage S, butterfly i, input r
  template <int S>
  __device__ __forceinline__ int index(int i, int r) const {
    constexpr int RS = fft_stage_radix(N, R, S);
    constexpr int NSB = fft_stage_ns(N, R, S);
    return r * ((t_ + TPP * i) % NSB) * (N / (NSB * RS));
  }
  // twiddle for stage S, butterfly i, input r
  template <int S>
  __device__ __forceinline__ cx<T> get(int i, int r) const {
    if constexpr (CACHED) {
      return w[stage_offset(S) + i * (fft_stage_radix(N, R, S) - 1) + (r - 1)];
    } else {
      return table[index<S>(i, r)];
    }
  }
  // v <- v W (forward) or v conj(W) (inverse) for stage S, butterfly i, input r
  template <int S, bool INV>
  __device__ __forceinline__ void apply(cx<T>& v, int i, int r) const {
    const cx<T> w = get<S>(i, r);
    if constexpr (sizeof(T) == 8) {
      v = INV ? cmulc(v, w) : cmul(v, w);
    } else {
      v = shear_rotate<INV>(v, w.re, w.im, twiddle_flip(index<S>(i, r), N));
    }
  }
  template <int S>
  __device__ __forceinline__ void load_stage(const cx<T>* __restrict__ twd, int t) {
    if constexpr (S < NS) {
      constexpr int RS = fft_stage_radix(N, R, S);
      constexpr int NSB = fft_stage_ns(N, R, S);
      constexpr int NB = R / RS;
      if constexpr (NSB > 1) {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          const int jm = (t + TPP * i) % NSB;
#pragma unroll
          for (int r = 1; r < RS; ++r) w[stage_offset(S) + i * (RS - 1) + (r - 1)] = twd[r * jm * (N / (NSB * RS))];
        }
      }
      load_stage<S + 1>(twd, t);
    }
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

  template <class TC>
  static __device__ __forceinline__ void run(cx<T> (&v)[R], cx<T>* lds, int t, const TC& tc) {
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
      if constexpr (NSB > 1) {
#pragma unroll
        for (int r = 1; r < RS; ++r) tc.template apply<S, INV>(v[i + r * NB], i, r);  // TwiddleCache<T, N, cached>
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
      FftStage<T, N, TPP, INV, SW, S + 1>::run(v, lds, t, tc);
    }
  }
};

// Two pencils transformed in lockstep (each in its own LDS buffer): one pair
// of synchronisations per stage serves both, and the two butterflies of a
// stage are independent work for the scheduler to interleave.
template <class T, int N, int TPP, bool INV, bool SW, int S>
struct FftStage2 {
  using One = FftStage<T, N, TPP, INV, SW, S>;
  static constexpr int R = One::R, NS = One::NS, RS = One::RS, NSB = One::NSB, NB = One::NB;

  template <class TC>
  static __device__ __forceinline__ void run(cx<T> (&a)[R], cx<T> (&b)[R], cx<T>* la, cx<T>* lb, int t,
                                             const TC& tc) {
    if constexpr (S > 0) {
      fft_sync<SW>();
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int j = t + TPP * i;
#pragma unroll
        for (int r = 0; r < RS; ++r) {
          a[i + r * NB] = la[lds_pad(j + r * (N / RS))];
          b[i + r * NB] = lb[lds_pad(j + r * (N / RS))];
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      if constexpr (NSB > 1) {
#pragma unroll
        for (int r = 1; r < RS; ++r) {
          tc.template apply<S, INV>(a[i + r * NB], i, r);
          tc.template apply<S, INV>(b[i + r * NB], i, r);
        }
      }
      Butterfly<T, RS, INV>::run(a, i, NB);
      Butterfly<T, RS, INV>::run(b, i, NB);
    }
    if constexpr (S < NS - 1) {
      fft_sync<SW>();
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int j = t + TPP * i;
        const int base = (j / NSB) * NSB * RS + (j % NSB);
#pragma unroll
        for (int r = 0; r < RS; ++r) {
          la[lds_pad(base + r * NSB)] = a[i + r * NB];
          lb[lds_pad(base + r * NSB)] = b[i + r * NB];
        }
      }
      FftStage2<T, N, TPP, INV, SW, S + 1>::run(a, b, la, lb, t, tc);
    }
  }
};

// Transform the pencil held in v (natural layout) in place. `lds` is this
// pencil's private buffer of fft_lds_stride(N) elements. With SYNC_WAVE =
// false every thread of the workgroup must make the same calls (the stage
// barriers are workgroup-wide). `tc` holds this thread's twiddles (loaded from
// the table twd[e] = W_N^e by TwiddleCache::load).
template <class T, int N, bool INV, bool SYNC_WAVE, bool CACHED>
__device__ __forceinline__ void fft_pencil(cx<T> (&v)[N / fft_threads(N)], cx<T>* lds, int t,
                                           const TwiddleCache<T, N, CACHED>& tc) {
  FftStage<T, N, fft_threads(N), INV, SYNC_WAVE, 0>::run(v, lds, t, tc);
}
// The same for two pencils at once (buffers la and lb).
template <class T, int N, bool INV, bool SYNC_WAVE, bool CACHED>
__device__ __forceinline__ void fft_pencil2(cx<T> (&a)[N / fft_threads(N)], cx<T> (&b)[N / fft_threads(N)],
                                            cx<T>* la, cx<T>* lb, int t, const TwiddleCache<T, N, CACHED>& tc) {
  FftStage2<T, N, fft_threads(N), INV, SYNC_WAVE, 0>::run(a, b, la, lb, t, tc);
}

}  // namespace tw
