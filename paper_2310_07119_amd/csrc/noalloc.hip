// tw_moments_static: the moment reductions of tw_moments without a plan and
// without any allocation. Their partial sums live in a fixed device array of
// this file instead of a plan's workspace.
#include <cmath>
#include <mutex>

#include "common.hpp"
#include "internal.hpp"

namespace tw {
namespace {

// Partial sums of the moment reductions: one double per (realization,
// wavefront of 64 cells), three per wavefront for Q and the two deviations,
// one per realization and three totals. 32 MiB; every GPU the library runs
// on holds its own copy until the process ends.
constexpr int64_t kStaticScratchDoubles = int64_t(1) << 22;
__device__ __align__(256) double scratch[kStaticScratchDoubles];

// Device address of `scratch` on each device, looked up once per device with
// that device current. Host code passes these addresses, never the array's
// name (a host-side stand-in, not a device address).
constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};

int scratch_on_current_device(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return report_error(TW_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return report_error(TW_EUNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return report_error(TW_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch[dev] = static_cast<double*>(p);
  }
  *out = g_scratch[dev];
  return TW_OK;
}

}  // namespace
}  // namespace tw

using namespace tw;

extern "C" int tw_moments_static(const tw_problem* pr, const void* psi, const void* psi_cl,
                                 const tw_moments_out* out, void* stream) {
  if (!pr || !out) return report_error(TW_EINVAL, "NULL problem or output struct");
  if (pr->dim < 1 || pr->dim > 3) return report_error(TW_EINVAL, "dim must be 1, 2 or 3 (got %d)", pr->dim);
  if (pr->reserved != 0) return report_error(TW_EINVAL, "reserved field must be 0");
  if (pr->precision != TW_FP64 && pr->precision != TW_FP32_SPLIT)
    return report_error(TW_EINVAL, "unknown precision %d", pr->precision);
  int64_t ncell = 1;
  double dv = 1.0;
  for (int d = 0; d < 3; ++d) {
    if (d < pr->dim) {
      if (pr->n[d] < 1) return report_error(TW_EINVAL, "n[%d] must be positive", d);
      if (!(pr->box[d] > 0.0) || !std::isfinite(pr->box[d])) return report_error(TW_EINVAL, "box[%d] must be > 0", d);
      ncell *= pr->n[d];
      dv *= pr->box[d] / pr->n[d];
    } else if (pr->n[d] != 1) {
      return report_error(TW_EINVAL, "n[%d] must be 1 for an unused axis", d);
    }
  }
  if (!(pr->m_tot > 0.0) || !std::isfinite(pr->m_tot)) return report_error(TW_EINVAL, "m_tot must be > 0");
  if (!(pr->n_tot > 0.0)) return report_error(TW_EINVAL, "n_tot must be > 0");
  if (pr->n_real < 1) return report_error(TW_EINVAL, "n_real must be >= 1");
  if (out->energy || out->mode_occ || out->var_amp || out->var_phase || out->decoherence)
    return report_error(TW_EUNSUPPORTED,
                        "tw_moments_static computes no energies, mode occupations or amplitude/phase spreads "
                        "(they need a plan's spectral scratch): set those outputs to NULL");
  const size_t elem = pr->precision == TW_FP32_SPLIT ? 8 : 16;
  if (!psi) return report_error(TW_EINVAL, "psi is NULL");
  if (reinterpret_cast<uintptr_t>(psi) % elem != 0)
    return report_error(TW_ELAYOUT, "psi is not aligned to the %zu-byte complex element", elem);
  if (psi_cl && reinterpret_cast<uintptr_t>(psi_cl) % elem != 0)
    return report_error(TW_ELAYOUT, "psi_classical is not aligned to the %zu-byte complex element", elem);
  const int64_t need = moments_partial_doubles(pr->n_real, ncell);
  if (need > kStaticScratchDoubles)
    return report_error(TW_EUNSUPPORTED,
                        "tw_moments_static: n_real * ceil(N/64) + 3 ceil(N/64) + n_real + 3 = %lld partial sums "
                        "exceed its fixed scratch of %lld doubles (32 MiB); use tw_moments with a plan",
                        (long long)need, (long long)kStaticScratchDoubles);
  double* partial = nullptr;
  if (int rc = scratch_on_current_device(&partial)) return rc;
  const MomGeom G{pr->n_real, ncell, pr->m_tot, dv, pr->n_tot, pr->precision == TW_FP32_SPLIT};
  const hipError_t e =
      launch_moments_geom(G, partial, psi, psi_cl, out, nullptr, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return report_error(TW_EHIP, "tw_moments_static launch: %s", hipGetErrorString(e));
  return TW_OK;
}
