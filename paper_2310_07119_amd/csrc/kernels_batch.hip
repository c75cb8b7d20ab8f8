// Grouped pass kernels for batches of ensembles with different grid sizes.
//
// One launch covers the same pass (mode, axis) of every size class in the
// batch: the 1D grid is the concatenation of each class's (pencil group, pair)
// blocks, and every block runs the pass body compiled for its class's length.
// All bodies used here run with 256 threads, so one launch shape serves every
// class; dynamic LDS is sized for the largest class.
#include "common.hpp"
#include "fft.hpp"
#include "internal.hpp"
#include "pass_cols.hpp"
#include "pass_common.hpp"
#include "pass_rows.hpp"

namespace tw {

// lengths the grouped kernels are compiled for
#define TW_BATCH_LENGTHS(X) X(16) X(24) X(32) X(48) X(64) X(96) X(128)

bool batch_length_supported(int n) {
  switch (n) {
#define TW_CASE(L) case L:
    TW_BATCH_LENGTHS(TW_CASE)
#undef TW_CASE
    return true;
    default: return false;
  }
}

// KIND: 0 row pass, 1 strided pass (interleaved pencils), 2 strided pass (LDS tiles)
template <class T, int N, int MODE, int KIND>
__device__ __forceinline__ void grouped_body(const PassArgs& a, unsigned bx, unsigned nbx, int64_t by) {
  if constexpr (KIND == 0) {
    static_assert(pass_threads<T, N, true>() == 256, "grouped row bodies run with 256 threads");
    pass_body<T, N, MODE, true>(a, bx, nbx, by);
  } else if constexpr (KIND == 1) {
    static_assert(pass_threads<T, N, false>() == 256, "grouped strided bodies run with 256 threads");
    pass_body<T, N, MODE, false>(a, bx, nbx, by);
  } else {
    static_assert(ColsCfg<T, N>::THREADS == 256, "grouped tile bodies run with 256 threads");
    cols_body<T, N, MODE>(a, bx, nbx, by);
  }
}

template <class T, int MODE, int KIND>
__global__ void __launch_bounds__(256) grouped_kernel(GroupArgs g) {
  const unsigned b = blockIdx.x;
  int c = 0;
  while (c + 1 < g.nclass && b >= g.start[c + 1]) ++c;
  const unsigned local = b - g.start[c];
  const unsigned nbx = g.groups[c];
  const unsigned bx = local % nbx;
  const int64_t by = local / nbx;
  const PassArgs& a = g.a[c];
  switch (a.n[a.axis]) {
#define TW_CASE(L)                                   \
  case L:                                            \
    grouped_body<T, L, MODE, KIND>(a, bx, nbx, by); \
    break;
    TW_BATCH_LENGTHS(TW_CASE)
#undef TW_CASE
    default: break;
  }
}

// LDS of a pencil body per pass mode (the drifting modes may hold two
// buffers per pencil; the FP64 kick pass and the transform-only modes one)
template <class T, int N, bool ROWS>
constexpr size_t pencil_lds_bytes(int mode) {
  return mode == PASS_KICK_DRIFT     ? pass_lds_bytes<T, N, ROWS, PASS_KICK_DRIFT>()
         : pass_mode_drifts(mode) ? pass_lds_bytes<T, N, ROWS, PASS_DRIFT>()
                                  : pass_lds_bytes<T, N, ROWS, PASS_ZFWD>();
}

template <class T, int N, int KIND>
constexpr size_t grouped_lds_bytes(int mode) {
  if constexpr (KIND == 0) return pencil_lds_bytes<T, N, true>(mode);
  else if constexpr (KIND == 1) return pencil_lds_bytes<T, N, false>(mode);
  else return ColsCfg<T, N>::LDS;
}

template <class T, int KIND>
size_t grouped_lds_for(int n, int mode) {
  switch (n) {
#define TW_CASE(L) \
  case L: return grouped_lds_bytes<T, L, KIND>(mode);
    TW_BATCH_LENGTHS(TW_CASE)
#undef TW_CASE
    default: return 0;
  }
}

template <class T, int N, int KIND>
int grouped_groups_n() {
  if constexpr (KIND == 0) return pencils_per_group<T, N, true>();
  else if constexpr (KIND == 1) return pencils_per_group<T, N, false>();
  else return ColsCfg<T, N>::C;
}

template <class T, int KIND>
int grouped_pencils_for(int n) {
  switch (n) {
#define TW_CASE(L) \
  case L: return grouped_groups_n<T, L, KIND>();
    TW_BATCH_LENGTHS(TW_CASE)
#undef TW_CASE
    default: return 0;
  }
}

template <class T, int KIND>
static hipError_t launch_grouped_tk(int mode, GroupArgs& g, hipStream_t s) {
  size_t lds = 0;
  uint32_t start = 0;
  for (int c = 0; c < g.nclass; ++c) {
    const PassArgs& a = g.a[c];
    const int n = a.n[a.axis];
    const int pc = grouped_pencils_for<T, KIND>(n);
    const size_t l = grouped_lds_for<T, KIND>(n, mode);
    if (pc <= 0 || l == 0) return hipErrorInvalidValue;
    if (l > lds) lds = l;
    const int64_t npencils = a.ncell / n;
    const int64_t npairs = (a.nfield + 1) / 2 - a.pair0;
    g.groups[c] = (uint32_t)((npencils + pc - 1) / pc);
    g.start[c] = start;
    start += g.groups[c] * (uint32_t)(npairs > 0 ? npairs : 0);
  }
  g.start[g.nclass] = start;
  if (start == 0) return hipSuccess;
  auto go = [&](auto kern) -> hipError_t {
    if (lds > 64 * 1024) {
      hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void*>(kern), lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(start), dim3(256), lds, s, g);
    return hipGetLastError();
  };
  switch (mode) {
    case PASS_DRIFT: return go(grouped_kernel<T, PASS_DRIFT, KIND>);
    case PASS_DRIFT_RHO: return go(grouped_kernel<T, PASS_DRIFT_RHO, KIND>);
    case PASS_ZFWD: return go(grouped_kernel<T, PASS_ZFWD, KIND>);
    case PASS_ZPOISSON: return go(grouped_kernel<T, PASS_ZPOISSON, KIND>);
    case PASS_ZINV: return go(grouped_kernel<T, PASS_ZINV, KIND>);
    case PASS_KICK_DRIFT: return go(grouped_kernel<T, PASS_KICK_DRIFT, KIND>);
    default: return hipErrorInvalidValue;
  }
}

// Launch `mode` along the axis stored in g.a[*] (the same for every class) for
// all classes at once. Row passes (stride 1) use the row body; strided passes
// use the organisation `variant` (0 interleaved, 1 LDS tiles).
hipError_t launch_grouped(bool fp32, int mode, GroupArgs& g, int variant, hipStream_t s) {
  if (g.nclass <= 0) return hipSuccess;
  const bool rows = g.a[0].stride == 1;
  const int kind = rows ? 0 : (variant == 1 ? 2 : 1);
  if (fp32) {
    if (kind == 0) return launch_grouped_tk<float, 0>(mode, g, s);
    if (kind == 1) return launch_grouped_tk<float, 1>(mode, g, s);
    return launch_grouped_tk<float, 2>(mode, g, s);
  }
  if (kind == 0) return launch_grouped_tk<double, 0>(mode, g, s);
  if (kind == 1) return launch_grouped_tk<double, 1>(mode, g, s);
  return launch_grouped_tk<double, 2>(mode, g, s);
}

}  // namespace tw
