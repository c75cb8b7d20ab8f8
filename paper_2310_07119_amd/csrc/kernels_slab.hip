// xy-plane passes for D = 3: one workgroup holds one z-plane (N x N points)
// of a field in LDS and transforms it along x and along y before a single
// write-back, so a drift along both in-plane axes, or the in-plane half of
// the density / Poisson transforms, costs one HBM round trip instead of two.
//
// With these passes a 3D step is three HBM passes (Sec. "Integrating the
// equations of motion": drift, potential from the density, kick, drift; the
// drift is separable per axis and the axis order of the merged drifts
// alternates between steps):
//   kind B: plane drift(x, y) + density + FFT_xy  |  z-pencil FFT_z, Green, IFFT_z
//           |  plane IFFT_xy -> V, kick, drift(x, y)
//   kind A: z-pencil drift_z + density + FFT_z  |  plane FFT_xy, Green, IFFT_xy
//           |  z-pencil IFFT_z -> V, kick, drift_z
// The z-pencil passes are the strided pencil passes of the other kernels.
//
// LDS layout: the plane is N rows of fft_lds_stride(N) complex elements;
// point (x, y) lives at y * LS + lds_pad(x). Row transforms use a row's own
// slot as their exchange buffer (wavefront-local: a pencil's threads share one
// wavefront); column transforms run after every column has been read into
// registers, each in the slot of its column index. Between the two, the data
// moves through the plane layout (two workgroup barriers per transpose).
#include "common.hpp"
#include "fft.hpp"
#include "internal.hpp"
#include "pass_common.hpp"

namespace tw {

template <class T, int N>
struct SlabCfg {
  static constexpr int TPP = fft_threads(N);
  static constexpr int R = N / TPP;
  static constexpr int LS = fft_lds_stride(N);
  static constexpr int PENCIL_THREADS = N * TPP;                 // every pencil of one axis at once
  // the whole plane is in registers across a transpose: two pencils per
  // thread at 128 x 128 (1024 threads)
  static constexpr int threads_for(int p) { return p > 1024 ? threads_for(p / 2) : p; }
  static constexpr int THREADS = threads_for(PENCIL_THREADS);
  static constexpr int PPT = PENCIL_THREADS / THREADS;           // pencils per thread
  static constexpr int PSTEP = THREADS / TPP;                    // pencil index step between them
  // plane, reduction slots, and the drift factors along x and y (16 bytes each)
  static constexpr size_t LDS = (size_t)N * LS * sizeof(cx<T>) + 16 * sizeof(double) + 2 * (size_t)N * 16;
  // 1024 threads leave 128 VGPRs per thread: twiddles are then read from the
  // table at each stage instead of being held in registers
  static constexpr bool TW_CACHED = THREADS < 1024;
  static_assert(PENCIL_THREADS % THREADS == 0 && THREADS % TPP == 0, "plane shape");
  static_assert(TPP <= 64, "a pencil must fit one wavefront");
};

__device__ __forceinline__ void slab_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// One workgroup: plane `plane` of pair slot `by` (relative to a.pair0).
template <class T, int N, int MODE>
__device__ __forceinline__ void slab_body(const PassArgs& a, unsigned plane, int64_t by) {
  using Cfg = SlabCfg<T, N>;
  constexpr int TPP = Cfg::TPP, R = Cfg::R, LS = Cfg::LS, PPT = Cfg::PPT, PSTEP = Cfg::PSTEP;
  constexpr int64_t NN = (int64_t)N * N;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* S = reinterpret_cast<cx<T>*>(smem_raw);
  double* red = reinterpret_cast<double*>(smem_raw + (size_t)N * LS * sizeof(cx<T>));
  // drift factors staged in LDS and read where they are applied: FP64 (cos,
  // sin)/n, or for FP32 planes each factor as a pair of floats (f = hi + lo
  // to 2^-48), applied with FP32 arithmetic. FP64 factors multiplied in FP64
  // kept their conversions and products live across the transforms and made
  // the 128-point FP32 planes spill.
  unsigned char* phl = smem_raw + (size_t)N * LS * sizeof(cx<T>) + 16 * sizeof(double);

  const int tid = threadIdx.x;
  const int t = tid % TPP;
  const int q0 = tid / TPP;  // first pencil (row y, or column x) of this thread; then + PSTEP * j
  const int64_t pair = a.pair0 + by;
  const int64_t fA = 2 * pair, fB = 2 * pair + 1;
  const bool hasB = fB < a.nfield;
  const int64_t off = (int64_t)plane * NN;

  TwiddleCache<T, N, Cfg::TW_CACHED> tc;
  tc.load(reinterpret_cast<const cx<T>*>(a.twd), t);
  if constexpr (MODE == SLAB_DRIFT || MODE == SLAB_DRIFT_RHO || MODE == SLAB_KICK_DRIFT) {
    const cx<double>* p1 = reinterpret_cast<const cx<double>*>(a.phase);
    const cx<double>* p2 = reinterpret_cast<const cx<double>*>(a.phase2);
    for (int e = tid; e < 2 * N; e += Cfg::THREADS) {
      const cx<double> f = e < N ? p1[e] : p2[e - N];
      if constexpr (sizeof(T) == 8) {
        reinterpret_cast<cx<double>*>(phl)[e] = f;
      } else {
        const float hr = (float)f.re, hi = (float)f.im;
        reinterpret_cast<float4*>(phl)[e] = make_float4(hr, hi, (float)(f.re - (double)hr), (float)(f.im - (double)hi));
      }
    }
    slab_barrier();
  }

  using Regs = cx<T>[PPT][R];
  auto load_rows = [&](const cx<T>* f, Regs& v) {
#pragma unroll
    for (int j = 0; j < PPT; ++j)
#pragma unroll
      for (int m = 0; m < R; ++m) v[j][m] = f[off + (int64_t)(q0 + PSTEP * j) * N + t + TPP * m];
  };
  auto store_rows = [&](cx<T>* f, const Regs& v) {
#pragma unroll
    for (int j = 0; j < PPT; ++j)
#pragma unroll
      for (int m = 0; m < R; ++m) f[off + (int64_t)(q0 + PSTEP * j) * N + t + TPP * m] = v[j][m];
  };
  // transform every pencil this thread holds, pencil q in exchange slot q
  auto fft_all = [&](Regs& v, bool inv) {
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      cx<T>* slot = S + (q0 + PSTEP * j) * LS;
      if (inv) fft_pencil<T, N, true, true, Cfg::TW_CACHED>(v[j], slot, t, tc);
      else fft_pencil<T, N, false, true, Cfg::TW_CACHED>(v[j], slot, t, tc);
    }
  };
  auto phase_all = [&](Regs& v, int table) {
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int e = table * N + t + TPP * m;
      if constexpr (sizeof(T) == 8) {
        const cx<double> f = reinterpret_cast<const cx<double>*>(phl)[e];
#pragma unroll
        for (int j = 0; j < PPT; ++j) v[j][m] = mul_d(v[j][m], f);
      } else {
        const float4 f = reinterpret_cast<const float4*>(phl)[e];  // (hi.re, hi.im, lo.re, lo.im)
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
          const cx<float> x = v[j][m];
          const float cre = __builtin_fmaf(x.re, f.z, -x.im * f.w);
          const float cim = __builtin_fmaf(x.re, f.w, x.im * f.z);
          const float re = __builtin_fmaf(x.re, f.x, __builtin_fmaf(-x.im, f.y, cre));
          const float im = __builtin_fmaf(x.re, f.y, __builtin_fmaf(x.im, f.x, cim));
          v[j][m] = {re, im};
        }
      }
    }
  };
  // rows in registers -> columns in registers (and back): through the plane layout
  auto rows_to_cols = [&](Regs& v) {
    slab_barrier();  // every row's exchanges are done before the plane is rewritten
#pragma unroll
    for (int j = 0; j < PPT; ++j)
#pragma unroll
      for (int m = 0; m < R; ++m) S[(q0 + PSTEP * j) * LS + lds_pad(t + TPP * m)] = v[j][m];
    slab_barrier();
#pragma unroll
    for (int j = 0; j < PPT; ++j)
#pragma unroll
      for (int m = 0; m < R; ++m) v[j][m] = S[(t + TPP * m) * LS + lds_pad(q0 + PSTEP * j)];
    slab_barrier();  // every column is read before column exchanges reuse the plane
  };
  auto cols_to_rows = [&](Regs& v) {
    slab_barrier();
#pragma unroll
    for (int j = 0; j < PPT; ++j)
#pragma unroll
      for (int m = 0; m < R; ++m) S[(t + TPP * m) * LS + lds_pad(q0 + PSTEP * j)] = v[j][m];
    slab_barrier();
#pragma unroll
    for (int j = 0; j < PPT; ++j)
#pragma unroll
      for (int m = 0; m < R; ++m) v[j][m] = S[(q0 + PSTEP * j) * LS + lds_pad(t + TPP * m)];
    // the next row exchanges touch only the rows this wavefront just read
  };
  // drift along x (rows) then y (columns); rows in, rows out
  auto drift_xy = [&](Regs& v) {
    fft_all(v, false);
    phase_all(v, 0);
    fft_all(v, true);
    rows_to_cols(v);
    fft_all(v, false);
    phase_all(v, 1);
    fft_all(v, true);
    cols_to_rows(v);
  };
  cx<T>* zp = reinterpret_cast<cx<T>*>(a.z) + pair * a.ncell;

  if constexpr (MODE == SLAB_DRIFT) {
    Regs v;
    load_rows(field_ptr<T>(a, fA), v);
    drift_xy(v);
    store_rows(field_ptr<T>(a, fA), v);
    if (hasB) {
      load_rows(field_ptr<T>(a, fB), v);
      drift_xy(v);
      store_rows(field_ptr<T>(a, fB), v);
    }
  } else if constexpr (MODE == SLAB_DRIFT_RHO) {
    Regs v;
    T ra[PPT][R];
    load_rows(field_ptr<T>(a, fA), v);
    drift_xy(v);
    store_rows(field_ptr<T>(a, fA), v);
    {
      const double mean = a.rho_mean ? a.rho_mean[fA] : 0.0;
#pragma unroll
      for (int j = 0; j < PPT; ++j)
#pragma unroll
        for (int m = 0; m < R; ++m) ra[j][m] = (T)(a.m_tot * (double)abs2(v[j][m]) - mean);
    }
    if (hasB) {
      load_rows(field_ptr<T>(a, fB), v);
      drift_xy(v);
      store_rows(field_ptr<T>(a, fB), v);
      const double mean = a.rho_mean ? a.rho_mean[fB] : 0.0;
#pragma unroll
      for (int j = 0; j < PPT; ++j)
#pragma unroll
        for (int m = 0; m < R; ++m) v[j][m] = {ra[j][m], (T)(a.m_tot * (double)abs2(v[j][m]) - mean)};
    } else {
#pragma unroll
      for (int j = 0; j < PPT; ++j)
#pragma unroll
        for (int m = 0; m < R; ++m) v[j][m] = {ra[j][m], (T)0};
    }
    // z = rho_A + i rho_B, forward along x and y
    fft_all(v, false);
    rows_to_cols(v);
    fft_all(v, false);
    cols_to_rows(v);
    store_rows(zp, v);
  } else if constexpr (MODE == SLAB_POISSON) {
    // z holds the pair density transformed along z: forward along x and y,
    // Green's function -4 pi G / (|k|^2 N) (V_0 = 0), inverse along y and x
    Regs v;
    load_rows(zp, v);
    fft_all(v, false);
    rows_to_cols(v);
    fft_all(v, false);
    const double k2z = a.k2[2][plane];
    const double* __restrict__ k2x = a.k2[0];
    const double* __restrict__ k2y = a.k2[1];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const double k2o = k2z + k2x[q0 + PSTEP * j];
#pragma unroll
      for (int m = 0; m < R; ++m) {
        v[j][m] = mul_d(v[j][m], green_factor<T>(k2o + k2y[t + TPP * m], a.green));
      }
    }
    fft_all(v, true);
    cols_to_rows(v);
    fft_all(v, true);
    store_rows(zp, v);
  } else if constexpr (MODE == SLAB_KICK_DRIFT) {
    // z holds the potential pair transformed along x and y: inverse along both
    Regs zv;
    load_rows(zp, zv);
    fft_all(zv, true);
    rows_to_cols(zv);
    fft_all(zv, true);
    cols_to_rows(zv);
    if (a.vmax) {
      double mx = 0.0;
#pragma unroll
      for (int j = 0; j < PPT; ++j)
#pragma unroll
        for (int m = 0; m < R; ++m)
          mx = fmax(mx, fmax(fabs((double)zv[j][m].re), hasB ? fabs((double)zv[j][m].im) : 0.0));
      mx = block_max(mx, red);
      if (tid == 0) record_max(a.vmax + ((plane + (unsigned)by) & (kVmaxBuckets - 1)), mx);
    }
    // Planes of two pencils per thread park the potentials in the pair
    // scratch during the first field's drift instead of holding them in
    // registers (the 128-point FP32 kick pass spilled 112 registers), and read
    // them back for the second field: 8 more bytes per pair and cell.
    constexpr bool PARK = PPT > 1;
    if (a.store_v || PARK) store_rows(zp, zv);  // the potentials (also for the test particles)
    const double kick = a.kick_dev ? a.kick_dev[0] : a.kick;
    Regs v;
    load_rows(field_ptr<T>(a, fA), v);
#pragma unroll
    for (int j = 0; j < PPT; ++j) kick_values<T, R>(v[j], zv[j], false, kick);
    drift_xy(v);
    store_rows(field_ptr<T>(a, fA), v);
    if (hasB) {
      if constexpr (PARK) load_rows(zp, zv);
      load_rows(field_ptr<T>(a, fB), v);
#pragma unroll
      for (int j = 0; j < PPT; ++j) kick_values<T, R>(v[j], zv[j], true, kick);
      drift_xy(v);
      store_rows(field_ptr<T>(a, fB), v);
    }
  }
}

template <class T, int N, int MODE>
__global__ void __launch_bounds__((SlabCfg<T, N>::THREADS)) slab_kernel(PassArgs a) {
  slab_body<T, N, MODE>(a, blockIdx.x, pair_slot(a));
}

template <class T, int N>
static hipError_t launch_slab_tn(int mode, const PassArgs& a, hipStream_t s, int ny) {
  using Cfg = SlabCfg<T, N>;
  const dim3 grid((unsigned)a.n[2], (unsigned)ny);
  const dim3 block(Cfg::THREADS);
  auto go = [&](auto kern) -> hipError_t {
    if constexpr (Cfg::LDS > 64 * 1024) {
      hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void*>(kern), Cfg::LDS);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, grid, block, Cfg::LDS, s, a);
    return hipGetLastError();
  };
  switch (mode) {
    case SLAB_DRIFT: return go(slab_kernel<T, N, SLAB_DRIFT>);
    case SLAB_DRIFT_RHO: return go(slab_kernel<T, N, SLAB_DRIFT_RHO>);
    case SLAB_POISSON: return go(slab_kernel<T, N, SLAB_POISSON>);
    case SLAB_KICK_DRIFT: return go(slab_kernel<T, N, SLAB_KICK_DRIFT>);
    default: return hipErrorInvalidValue;
  }
}

// Plane lengths with compiled plane kernels: FP32 up to 128 x 128, FP64 up to
// 64 x 64 (the plane must fit one workgroup's LDS).
#define TW_SLAB_LENGTHS_F32(X) X(16) X(32) X(64) X(96) X(128)
#define TW_SLAB_LENGTHS_F64(X) X(16) X(32) X(64)

size_t slab_lds_bytes(int n, bool fp32) {
  if (fp32) {
    switch (n) {
#define TW_CASE(L) \
  case L: return SlabCfg<float, L>::LDS;
      TW_SLAB_LENGTHS_F32(TW_CASE)
#undef TW_CASE
      default: return 0;
    }
  }
  switch (n) {
#define TW_CASE(L) \
  case L: return SlabCfg<double, L>::LDS;
    TW_SLAB_LENGTHS_F64(TW_CASE)
#undef TW_CASE
    default: return 0;
  }
}

hipError_t launch_slab(const Plan& P, int mode, const PassArgs& a, hipStream_t s, int ny) {
  if (ny <= 0) return hipSuccess;
  if (a.n[0] != a.n[1] || a.stride != 1) return hipErrorInvalidValue;
  if (P.fp32) {
    switch (a.n[0]) {
#define TW_CASE(L) \
  case L: return launch_slab_tn<float, L>(mode, a, s, ny);
      TW_SLAB_LENGTHS_F32(TW_CASE)
#undef TW_CASE
      default: return hipErrorInvalidValue;
    }
  }
  switch (a.n[0]) {
#define TW_CASE(L) \
  case L: return launch_slab_tn<double, L>(mode, a, s, ny);
    TW_SLAB_LENGTHS_F64(TW_CASE)
#undef TW_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tw
