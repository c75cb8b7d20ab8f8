// Strided-axis passes in the LDS-tile organisation (body in pass_cols.hpp).
#include "common.hpp"
#include "fft.hpp"
#include "internal.hpp"
#include "pass_common.hpp"
#include "pass_cols.hpp"

namespace tw {

template <class T, int N, int MODE>
__global__ void __launch_bounds__((ColsCfg<T, N>::THREADS)) cols_kernel(PassArgs a) {
  cols_body<T, N, MODE>(a, blockIdx.x, gridDim.x, pair_slot(a));
}

template <class T, int N>
static hipError_t launch_cols_tn(int mode, const PassArgs& a, hipStream_t s, int ny) {
  using Cfg = ColsCfg<T, N>;
  const int64_t npencils = a.ncell / N;
  dim3 grid((unsigned)((npencils + Cfg::C - 1) / Cfg::C), (unsigned)ny);
  dim3 block(Cfg::THREADS);
  auto go = [&](auto kern) -> hipError_t {
    if constexpr (Cfg::LDS > 64 * 1024) {
      hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void*>(kern), Cfg::LDS);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, grid, block, Cfg::LDS, s, a);
    return hipGetLastError();
  };
  switch (mode) {
    case PASS_DRIFT: return go(cols_kernel<T, N, PASS_DRIFT>);
    case PASS_DRIFT_RHO: return go(cols_kernel<T, N, PASS_DRIFT_RHO>);
    case PASS_ZFWD: return go(cols_kernel<T, N, PASS_ZFWD>);
    case PASS_ZPOISSON: return go(cols_kernel<T, N, PASS_ZPOISSON>);
    case PASS_ZINV: return go(cols_kernel<T, N, PASS_ZINV>);
    case PASS_KICK_DRIFT: return go(cols_kernel<T, N, PASS_KICK_DRIFT>);
    case PASS_RHO: return go(cols_kernel<T, N, PASS_RHO>);
    case PASS_KIN_SUM: return go(cols_kernel<T, N, PASS_KIN_SUM>);
    case PASS_POT_SUM: return go(cols_kernel<T, N, PASS_POT_SUM>);
    default: return hipErrorInvalidValue;
  }
}

template <class T>
static hipError_t launch_cols_t(int mode, const PassArgs& a, hipStream_t s, int ny) {
  switch (a.n[a.axis]) {
#define TW_CASE(L) \
  case L: return launch_cols_tn<T, L>(mode, a, s, ny);
    TW_PASS_LENGTHS(TW_CASE)
#undef TW_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pass_cols(const Plan& P, int mode, const PassArgs& a, hipStream_t s, int ny) {
  if (ny <= 0) return hipSuccess;
  return P.fp32 ? launch_cols_t<float>(mode, a, s, ny) : launch_cols_t<double>(mode, a, s, ny);
}

int cols_pencils_per_group(int n, bool fp32) {
  auto pick = [&](auto tag) -> int {
    using T = decltype(tag);
    switch (n) {
#define TW_CASE(L) \
  case L: return ColsCfg<T, L>::C;
      TW_PASS_LENGTHS(TW_CASE)
#undef TW_CASE
      default: return 0;
    }
  };
  return fp32 ? pick(float{}) : pick(double{});
}

}  // namespace tw
