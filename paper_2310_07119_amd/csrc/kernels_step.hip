// Split-step kernels: per-axis pencil passes for D >= 2, a resident whole-run
// kernel for D = 1, drift phase tables and per-field density means.
//
// The step (Sec. "Integrating the equations of motion"): drift, potential from
// the drifted field's density, kick, drift. The kinetic propagator is
// separable, exp(-i hbar |k|^2 tau/2) = prod_d exp(-i hbar k_d^2 tau/2), so a
// D-dim drift is a product of 1D drifts along each axis, each done as
// FFT -> pointwise factor -> inverse FFT inside one pass with the pencil held
// in registers/LDS. The Poisson solve (V_k = -4 pi G rho_k/|k|^2, V_0 = 0) is
// not separable and needs the full D-dim transform of rho; two realizations
// share one complex transform (z = rho_A + i rho_B; the Green's function is
// real and even, so V_A = Re, V_B = Im of the inverse).
#include "common.hpp"
#include "fft.hpp"
#include "internal.hpp"
#include "pass_common.hpp"
#include "pass_rows.hpp"

#include <type_traits>

namespace tw {

template <class T, int N, int MODE, bool ROWS>
__global__ void __launch_bounds__((pass_threads<T, N, ROWS>())) pass_kernel(PassArgs a) {
  pass_body<T, N, MODE, ROWS>(a, blockIdx.x, gridDim.x, pair_slot(a));
}

template <class T, int N, bool ROWS>
static hipError_t launch_pass_tnr(int mode, const PassArgs& a, hipStream_t s, int ny) {
  constexpr int C = pencils_per_group<T, N, ROWS>();
  const int64_t npencils = a.ncell / N;
  dim3 grid((unsigned)((npencils + C - 1) / C), (unsigned)ny);
  dim3 block(pass_threads<T, N, ROWS>());
  auto go = [&](auto mode_c) -> hipError_t {
    constexpr int M = decltype(mode_c)::value;
    constexpr size_t LDS = pass_lds_bytes<T, N, ROWS, M>();
    const void* kern = reinterpret_cast<const void*>(pass_kernel<T, N, M, ROWS>);
    if constexpr (LDS > 64 * 1024) {
      hipError_t e = ensure_dynamic_lds(kern, LDS);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((pass_kernel<T, N, M, ROWS>), grid, block, LDS, s, a);
    return hipGetLastError();
  };
  switch (mode) {
#define TW_MODE(M) \
  case M: return go(std::integral_constant<int, M>{});
    TW_MODE(PASS_DRIFT)
    TW_MODE(PASS_DRIFT_RHO)
    TW_MODE(PASS_ZFWD)
    TW_MODE(PASS_ZPOISSON)
    TW_MODE(PASS_ZINV)
    TW_MODE(PASS_KICK_DRIFT)
    TW_MODE(PASS_RHO)
    TW_MODE(PASS_KIN_SUM)
    TW_MODE(PASS_POT_SUM)
#undef TW_MODE
    default: return hipErrorInvalidValue;
  }
}

template <class T, int N>
static hipError_t launch_pass_tn(int mode, const PassArgs& a, hipStream_t s, int ny) {
  return a.stride == 1 ? launch_pass_tnr<T, N, true>(mode, a, s, ny) : launch_pass_tnr<T, N, false>(mode, a, s, ny);
}

template <class T>
static hipError_t launch_pass_t(int mode, const PassArgs& a, hipStream_t s, int ny) {
  switch (a.n[a.axis]) {
#define TW_CASE(L) \
  case L: return launch_pass_tn<T, L>(mode, a, s, ny);
    TW_PASS_LENGTHS(TW_CASE)
#undef TW_CASE
    default: return hipErrorInvalidValue;
  }
}

bool pass_length_supported(int n) {
  switch (n) {
#define TW_CASE(L) case L:
    TW_PASS_LENGTHS(TW_CASE)
#undef TW_CASE
    return true;
    default: return false;
  }
}

int pass_pencils_per_group(int n, bool fp32, bool rows, int variant) {
  auto pick = [&](auto tag, auto r) -> int {
    using T = decltype(tag);
    constexpr bool RW = decltype(r)::value;
    switch (n) {
#define TW_CASE(L) \
  case L: return pencils_per_group<T, L, RW>();
      TW_PASS_LENGTHS(TW_CASE)
#undef TW_CASE
      default: return 0;
    }
  };
  if (!rows && variant == 1) return cols_pencils_per_group(n, fp32);
  if (fp32) return rows ? pick(float{}, std::true_type{}) : pick(float{}, std::false_type{});
  return rows ? pick(double{}, std::true_type{}) : pick(double{}, std::false_type{});
}

hipError_t launch_pass(const Plan& P, int mode, const PassArgs& a, hipStream_t s, int ny) {
  if (ny <= 0) return hipSuccess;
  if (a.stride != 1 && a.variant == 1) return launch_pass_cols(P, mode, a, s, ny);
  return P.fp32 ? launch_pass_t<float>(mode, a, s, ny) : launch_pass_t<double>(mode, a, s, ny);
}

// ------------------------------------------------------------------ 1D resident
// D = 1: a whole field fits in one workgroup's registers and LDS, so all steps
// run inside one launch with no HBM traffic between steps. Each field is
// transformed on its own (complex transform of the real density).
template <class T, int N>
__host__ __device__ constexpr int fields_per_group_1d() {
  constexpr int TPP = fft_threads(N);
  return TPP >= 64 ? 1 : 64 / TPP;
}

template <class T, int N>
__global__ void __launch_bounds__((fields_per_group_1d<T, N>() * fft_threads(N))) step1d_kernel(void* psi, void* psi_cl, int64_t n_real, int64_t nfield,
                                                       int64_t nsteps, const cx<T>* __restrict__ twd,
                                                       const double* __restrict__ k2,
                                                       const cx<double>* __restrict__ ph_half,
                                                       const cx<double>* __restrict__ ph_full, double green,
                                                       double kick, double m_tot,
                                                       const double* __restrict__ rho_mean) {
  constexpr int TPP = fft_threads(N);
  constexpr int R = N / TPP;
  constexpr int C = fields_per_group_1d<T, N>();
  __shared__ cx<T> lds_all[C * fft_lds_stride(N)];
  const int c = threadIdx.x / TPP;
  const int t = threadIdx.x % TPP;
  cx<T>* lds = lds_all + c * fft_lds_stride(N);
  const int64_t f = (int64_t)blockIdx.x * C + c;
  const bool active = f < nfield;
  cx<T>* fp = !active ? nullptr
              : (f < n_real ? reinterpret_cast<cx<T>*>(psi) + f * N : reinterpret_cast<cx<T>*>(psi_cl));
  const double mean = (active && rho_mean) ? rho_mean[f] : 0.0;
  TwiddleCache<T, N> tc;
  tc.load(twd, t);

  cx<T> v[R];
#pragma unroll
  for (int m = 0; m < R; ++m) v[m] = active ? fp[t + TPP * m] : cx<T>{(T)0, (T)0};
  double g[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const double kk = k2[t + TPP * m];
    g[m] = (kk == 0.0) ? 0.0 : green / kk;
  }
  auto drift = [&](const cx<double>* ph) {
    fft_pencil<T, N, false, true>(v, lds, t, tc);
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = mul_d(v[m], ph[t + TPP * m]);
    fft_pencil<T, N, true, true>(v, lds, t, tc);
  };

  drift(ph_half);
  for (int64_t s = 0; s < nsteps; ++s) {
    cx<T> zv[R];
#pragma unroll
    for (int m = 0; m < R; ++m) zv[m] = {(T)(m_tot * (double)abs2(v[m]) - mean), (T)0};
    fft_pencil<T, N, false, true>(zv, lds, t, tc);
#pragma unroll
    for (int m = 0; m < R; ++m) zv[m] = mul_d(zv[m], g[m]);
    fft_pencil<T, N, true, true>(zv, lds, t, tc);
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = kick_rotate<T>(v[m], (kick * (double)zv[m].re));
    drift(s + 1 < nsteps ? ph_full : ph_half);
  }
  if (active) {
#pragma unroll
    for (int m = 0; m < R; ++m) fp[t + TPP * m] = v[m];
  }
}

template <class T, int N>
static hipError_t launch_step1d_tn(const Plan& P, void* psi, void* psi_cl, int64_t nfield, int64_t nsteps,
                                   const void* ph_half, const void* ph_full, double kick, hipStream_t s) {
  constexpr int TPP = fft_threads(N);
  constexpr int C = fields_per_group_1d<T, N>();
  dim3 grid((unsigned)((nfield + C - 1) / C)), block(C * TPP);
  const double green = -4.0 * M_PI * P.p.G / (double)N;
  hipLaunchKernelGGL((step1d_kernel<T, N>), grid, block, 0, s, psi, psi_cl, (int64_t)P.p.n_real, nfield, nsteps,
                     reinterpret_cast<const cx<T>*>(P.twd[0]), P.k2[0],
                     reinterpret_cast<const cx<double>*>(ph_half), reinterpret_cast<const cx<double>*>(ph_full),
                     green, kick, P.p.m_tot, P.fp32 ? P.rho_mean : nullptr);
  return hipGetLastError();
}

template <class T>
static hipError_t launch_step1d_t(const Plan& P, void* psi, void* psi_cl, int64_t nfield, int64_t nsteps,
                                  const void* ph_half, const void* ph_full, double kick, hipStream_t s) {
  switch (P.n[0]) {
#define TW_CASE(L) \
  case L: return launch_step1d_tn<T, L>(P, psi, psi_cl, nfield, nsteps, ph_half, ph_full, kick, s);
    TW_STEP1D_LENGTHS(TW_CASE)
#undef TW_CASE
    default: return hipErrorInvalidValue;
  }
}

bool step1d_length_supported(int n) { return n == 8 || pass_length_supported(n); }

// D = 1 with device-chosen step sizes: one launch per step (each field still
// in one workgroup), so that the ensemble-wide max |V| of step n can size step
// n + 2 between launches (adapt_kernel). step < 0: only the potential of the
// fields on entry, its max |V| recorded, nothing stored. step >= 0: the
// opening half drift (step 0 only), density, potential (max |V| recorded),
// kick with the factor in kick_dev, then the drift of ph_step (merged with the
// next step's first half, or the closing half drift).
template <class T, int N>
__global__ void __launch_bounds__((fields_per_group_1d<T, N>() * fft_threads(N)))
    step1d_adapt_kernel(void* psi, void* psi_cl, int64_t n_real, int64_t nfield, int64_t step,
                        const cx<T>* __restrict__ twd, const double* __restrict__ k2,
                        const cx<double>* __restrict__ ph_open, const cx<double>* __restrict__ ph_step, double green,
                        const double* __restrict__ kick_dev, double m_tot, const double* __restrict__ rho_mean,
                        double* vmax) {
  constexpr int TPP = fft_threads(N);
  constexpr int R = N / TPP;
  constexpr int C = fields_per_group_1d<T, N>();
  __shared__ cx<T> lds_all[C * fft_lds_stride(N)];
  __shared__ double red[16];
  const int c = threadIdx.x / TPP;
  const int t = threadIdx.x % TPP;
  cx<T>* lds = lds_all + c * fft_lds_stride(N);
  const int64_t f = (int64_t)blockIdx.x * C + c;
  const bool active = f < nfield;
  cx<T>* fp = !active ? nullptr
              : (f < n_real ? reinterpret_cast<cx<T>*>(psi) + f * N : reinterpret_cast<cx<T>*>(psi_cl));
  const double mean = (active && rho_mean) ? rho_mean[f] : 0.0;
  TwiddleCache<T, N> tc;
  tc.load(twd, t);
  cx<T> v[R];
#pragma unroll
  for (int m = 0; m < R; ++m) v[m] = active ? fp[t + TPP * m] : cx<T>{(T)0, (T)0};
  auto drift = [&](const cx<double>* ph) {
    fft_pencil<T, N, false, true>(v, lds, t, tc);
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = mul_d(v[m], ph[t + TPP * m]);
    fft_pencil<T, N, true, true>(v, lds, t, tc);
  };
  if (step == 0) drift(ph_open);
  cx<T> zv[R];
#pragma unroll
  for (int m = 0; m < R; ++m) zv[m] = {(T)(m_tot * (double)abs2(v[m]) - mean), (T)0};
  fft_pencil<T, N, false, true>(zv, lds, t, tc);
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const double kk = k2[t + TPP * m];
    zv[m] = mul_d(zv[m], (kk == 0.0) ? 0.0 : green / kk);
  }
  fft_pencil<T, N, true, true>(zv, lds, t, tc);
  double mx = 0.0;
  if (active) {
#pragma unroll
    for (int m = 0; m < R; ++m) mx = fmax(mx, fabs((double)zv[m].re));
  }
  mx = block_max(mx, red);
  if (threadIdx.x == 0) record_max(vmax + (blockIdx.x & (kVmaxBuckets - 1)), mx);
  if (step < 0) return;
  const double kick = kick_dev[0];
#pragma unroll
  for (int m = 0; m < R; ++m) v[m] = kick_rotate<T>(v[m], kick * (double)zv[m].re);
  drift(ph_step);
  if (active) {
#pragma unroll
    for (int m = 0; m < R; ++m) fp[t + TPP * m] = v[m];
  }
}

template <class T, int N>
static hipError_t launch_step1d_adapt_tn(const Plan& P, void* psi, void* psi_cl, int64_t nfield, int64_t step,
                                         const void* ph_open, const void* ph_step, const double* kick_dev,
                                         double* vmax, hipStream_t s) {
  constexpr int TPP = fft_threads(N);
  constexpr int C = fields_per_group_1d<T, N>();
  dim3 grid((unsigned)((nfield + C - 1) / C)), block(C * TPP);
  const double green = -4.0 * M_PI * P.p.G / (double)N;
  hipLaunchKernelGGL((step1d_adapt_kernel<T, N>), grid, block, 0, s, psi, psi_cl, (int64_t)P.p.n_real, nfield, step,
                     reinterpret_cast<const cx<T>*>(P.twd[0]), P.k2[0], reinterpret_cast<const cx<double>*>(ph_open),
                     reinterpret_cast<const cx<double>*>(ph_step), green, kick_dev, P.p.m_tot,
                     P.fp32 ? P.rho_mean : nullptr, vmax);
  return hipGetLastError();
}

hipError_t launch_step1d_adapt(const Plan& P, void* psi, void* psi_cl, int64_t nfield, int64_t step,
                               const void* ph_open, const void* ph_step, const double* kick_dev, double* vmax,
                               hipStream_t s) {
  auto go = [&](auto tag) -> hipError_t {
    using T = decltype(tag);
    switch (P.n[0]) {
#define TW_CASE(L) \
  case L: return launch_step1d_adapt_tn<T, L>(P, psi, psi_cl, nfield, step, ph_open, ph_step, kick_dev, vmax, s);
      TW_STEP1D_LENGTHS(TW_CASE)
#undef TW_CASE
      default: return hipErrorInvalidValue;
    }
  };
  return P.fp32 ? go(float{}) : go(double{});
}

hipError_t launch_step1d(const Plan& P, void* psi, void* psi_cl, int64_t nfield, int64_t nsteps,
                         const void* ph_half, const void* ph_full, double kick, hipStream_t s) {
  return P.fp32 ? launch_step1d_t<float>(P, psi, psi_cl, nfield, nsteps, ph_half, ph_full, kick, s)
                : launch_step1d_t<double>(P, psi, psi_cl, nfield, nsteps, ph_half, ph_full, kick, s);
}

// ---------------------------------------------------------------- tables
// out[j] = exp(-i hbar k_j^2 tau / 2) / n  (FP64), k_j^2 from the axis table.
__global__ void phase_table_kernel(cx<double>* out, const double* __restrict__ k2, int n, double hbar, double tau) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double arg = hbar * k2[j] * tau * 0.5;
  double s, c;
  sincos(arg, &s, &c);
  const double inv = 1.0 / (double)n;
  out[j] = {c * inv, -s * inv};
}

hipError_t launch_phase_table(const Plan& P, int axis, double tau, void* out, hipStream_t s) {
  const int n = P.n[axis];
  hipLaunchKernelGGL(phase_table_kernel, dim3((n + 255) / 256), dim3(256), 0, s, reinterpret_cast<cx<double>*>(out),
                     P.k2[axis], n, P.p.hbar_m, tau);
  return hipGetLastError();
}

// ------------------------------------------------------- adaptive step
// State (doubles): [0..2] step sizes dt_n at slot n mod 3; [6..7] kick factor
// dt_n / hbar at 6 + n mod 2; from kAdaptScalars on, three groups of
// kVmaxBuckets running max |V| values: the kick pass of step n records into
// group n mod 3 (group 2 also holds the initial potential's).
// Drift tables: adapt_tab[p][axis] for steps of parity p, adapt_tab[2][axis]
// for the opening half drift.
struct AdaptArgs {
  double* st;
  cx<double>* tab;
  const double* k2[3];
  int n[3];
  int dim;
  int nmax;
  double hbar, dt_max, courant, dtk;
  int64_t step;
  int last_next;
  double* dt_out;
};

// Time-step rule: dt = min(dt_max, c_f * dt_kinetic, c_f * 2 pi hbar / max|V|).
__device__ __forceinline__ double adapt_rule(const AdaptArgs& a, double vmax) {
  double dt = fmin(a.dt_max, a.courant * a.dtk);
  if (vmax > 0.0) dt = fmin(dt, a.courant * 6.283185307179586476925286766559 * a.hbar / vmax);
  return dt;
}

__device__ __forceinline__ cx<double> drift_factor(const AdaptArgs& a, int axis, int j, double tau) {
  const double arg = a.hbar * a.k2[axis][j] * tau * 0.5;
  double sn, cs;
  sincos(arg, &sn, &cs);
  const double inv = 1.0 / (double)a.n[axis];
  return {cs * inv, -sn * inv};
}

__device__ __forceinline__ double bucket_max(const double* b) {
  double m = 0.0;
  for (int i = 0; i < kVmaxBuckets; ++i) m = fmax(m, b[i]);
  return m;
}

__global__ void adapt_kernel(AdaptArgs a) {
  const int axis = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  double* S = a.st;
  double* buckets = S + kAdaptScalars;
  const bool lead_block = blockIdx.x == 0 && blockIdx.y == 0;
  const bool lead = lead_block && threadIdx.x == 0;
  if (a.step < 0) {
    const double d0 = adapt_rule(a, bucket_max(buckets + 2 * kVmaxBuckets));  // steps 0 and 1
    if (j < a.n[axis]) {
      a.tab[(size_t)(2 * 3 + axis) * a.nmax + j] = drift_factor(a, axis, j, 0.5 * d0);
      a.tab[(size_t)(0 * 3 + axis) * a.nmax + j] = drift_factor(a, axis, j, a.last_next ? 0.5 * d0 : d0);
    }
    if (lead) {
      S[0] = d0;
      S[1] = d0;
      S[6] = d0 / a.hbar;
    }
    // groups 0 and 1 were cleared with the state; group 2 is read above
    return;
  }
  const int64_t n = a.step;
  const double d1 = S[(n + 1) % 3];                                     // step n + 1
  const double d2 = adapt_rule(a, bucket_max(buckets + (n % 3) * kVmaxBuckets));  // step n + 2
  const int p = (int)((n + 1) % 2);
  if (j < a.n[axis])
    a.tab[(size_t)(p * 3 + axis) * a.nmax + j] = drift_factor(a, axis, j, a.last_next ? 0.5 * d1 : 0.5 * (d1 + d2));
  if (lead_block && threadIdx.x < kVmaxBuckets) buckets[((n + 1) % 3) * kVmaxBuckets + threadIdx.x] = 0.0;
  if (lead) {
    if (a.dt_out) a.dt_out[n] = S[n % 3];
    S[(n + 2) % 3] = d2;
    S[6 + p] = d1 / a.hbar;
  }
}

__global__ void adapt_clear_kernel(double* st, int len) {
  for (int i = threadIdx.x; i < len; i += blockDim.x) st[i] = 0.0;
}

hipError_t launch_adapt_clear(const Plan& P, hipStream_t s) {
  hipLaunchKernelGGL(adapt_clear_kernel, dim3(1), dim3(256), 0, s, P.adapt, kAdaptScalars + 3 * kVmaxBuckets);
  return hipGetLastError();
}

hipError_t launch_adapt(const Plan& P, int64_t step, int last_next, double dt_max, double courant, double dtk,
                        double* dt_out, hipStream_t s) {
  AdaptArgs a;
  a.st = P.adapt;
  a.tab = reinterpret_cast<cx<double>*>(P.adapt_tab);
  for (int d = 0; d < 3; ++d) {
    a.k2[d] = P.k2[d];
    a.n[d] = P.n[d];
  }
  a.dim = P.dim;
  a.nmax = P.nmax;
  a.hbar = P.p.hbar_m;
  a.dt_max = dt_max;
  a.courant = courant;
  a.dtk = dtk;
  a.step = step;
  a.last_next = last_next;
  a.dt_out = dt_out;
  hipLaunchKernelGGL(adapt_kernel, dim3((unsigned)((P.nmax + 255) / 256), (unsigned)P.dim), dim3(256), 0, s, a);
  return hipGetLastError();
}

// Mean density m_tot * sum_g |psi_g|^2 / N of every field, FP64, in two
// launches: kFieldMeanParts workgroups per field sum consecutive chunks of it
// (enough workgroups to stream the ensemble at full bandwidth), then one
// thread per field adds its partial sums in a fixed order.
template <class T>
__global__ void __launch_bounds__(256) field_mean_parts_kernel(const void* psi, const void* psi_cl, int64_t n_real,
                                                               int64_t ncell, int64_t chunk, int nb, double* parts) {
  __shared__ double red[4];
  const int64_t f = blockIdx.x / nb;  // block f * nb + b sums chunk b of field f
  const int64_t b = blockIdx.x % nb;
  const cx<T>* fp = f < n_real ? reinterpret_cast<const cx<T>*>(psi) + f * ncell : reinterpret_cast<const cx<T>*>(psi_cl);
  const int64_t g0 = b * chunk;
  const int64_t g1 = g0 + chunk < ncell ? g0 + chunk : ncell;
  double s = 0.0;
#pragma unroll 4
  for (int64_t g = g0 + threadIdx.x; g < g1; g += 256) s += (double)abs2(fp[g]);
  s = block_sum(s, red);
  if (threadIdx.x == 0) parts[blockIdx.x] = s;
}

__global__ void field_mean_finish_kernel(const double* parts, int nb, int64_t nfield, int64_t ncell, double m_tot,
                                         double* out) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nfield) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += parts[f * nb + b];
  out[f] = m_tot * s / (double)ncell;
}

hipError_t launch_field_mean(const Plan& P, const void* psi, const void* psi_cl, int64_t nfield, double* out,
                             hipStream_t s) {
  if (nfield <= 0) return hipSuccess;
  // chunks of at least 16 elements per thread, at most kFieldMeanParts per field;
  // the plan's partial-sum buffer holds nfield * kFieldMeanParts doubles
  int64_t nb = (P.ncell + 4095) / 4096;
  if (nb > kFieldMeanParts) nb = kFieldMeanParts;
  if (nb < 1) nb = 1;
  const int64_t chunk = (P.ncell + nb - 1) / nb;
  if ((size_t)(nfield * nb) > P.partial_len) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(nfield * nb));
  if (P.fp32)
    hipLaunchKernelGGL(field_mean_parts_kernel<float>, grid, dim3(256), 0, s, psi, psi_cl, (int64_t)P.p.n_real,
                       P.ncell, chunk, (int)nb, P.partial);
  else
    hipLaunchKernelGGL(field_mean_parts_kernel<double>, grid, dim3(256), 0, s, psi, psi_cl, (int64_t)P.p.n_real,
                       P.ncell, chunk, (int)nb, P.partial);
  hipLaunchKernelGGL(field_mean_finish_kernel, dim3((unsigned)((nfield + 255) / 256)), dim3(256), 0, s, P.partial,
                     (int)nb, nfield, P.ncell, P.p.m_tot, out);
  return hipGetLastError();
}

}  // namespace tw
