// C ABI: plan management, argument validation and the launch sequences of
// tw_sample / tw_step / tw_moments (declared in include/tw.h).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "common.hpp"
#include "fft.hpp"
#include "internal.hpp"

namespace tw {

hipError_t ensure_dynamic_lds(const void* kern, size_t bytes) {
  static std::mutex mu;
  static std::unordered_map<const void*, size_t> granted;
  std::lock_guard<std::mutex> lock(mu);
  auto it = granted.find(kern);
  if (it != granted.end() && it->second >= bytes) return hipSuccess;
  const hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) granted[kern] = bytes;
  return e;
}

namespace {
thread_local std::string g_error;
}  // namespace

int report_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

namespace {

#define fail report_error

#define TW_HIP(expr)                                                                 \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) return fail(TW_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

// ----------------------------------------------------------- kernel timing
struct ProfRec {
  int kind;
  hipEvent_t a, b;
};
struct Prof {
  std::vector<ProfRec> recs;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
};

const char* const kKindNames[KIND_COUNT] = {
    "pass_drift", "pass_drift_rho", "pass_zfwd", "pass_zpoisson", "pass_zinv", "pass_kick_drift",
    "pass_rho", "pass_kin_sum", "pass_pot_sum", "step1d_resident", "sample", "moments",
    "tables", "field_mean", "energy_finalize", "mode_occ",
    "pass_slab_drift", "pass_slab_drift_rho", "pass_slab_poisson", "pass_slab_kick_drift"};

// Run launcher f; when profiling, bracket it with events on stream s.
template <class F>
hipError_t timed(Plan& P, int kind, hipStream_t s, F&& f) {
  if (!P.profiling) return f();
  Prof* pr = static_cast<Prof*>(P.prof);
  std::pair<hipEvent_t, hipEvent_t> ev;
  if (!pr->pool.empty()) {
    ev = pr->pool.back();
    pr->pool.pop_back();
  } else {
    hipError_t e = hipEventCreate(&ev.first);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&ev.second);
    if (e != hipSuccess) return e;
  }
  hipError_t e = hipEventRecord(ev.first, s);
  if (e != hipSuccess) return e;
  e = f();
  hipError_t e2 = hipEventRecord(ev.second, s);
  pr->recs.push_back({kind, ev.first, ev.second});
  return e != hipSuccess ? e : e2;
}

int64_t axis_stride(const Plan& P, int axis) {
  if (axis == 0) return 1;
  if (axis == 1) return P.n[0];
  return (int64_t)P.n[0] * P.n[1];
}

void free_plan(Plan* P) {
  if (!P) return;
  for (int d = 0; d < 3; ++d) {
    if (P->twd[d]) (void)hipFree(P->twd[d]);
    if (P->k2[d]) (void)hipFree(P->k2[d]);
  }
  if (P->phase) (void)hipFree(P->phase);
  if (P->z) (void)hipFree(P->z);
  if (P->psi_alt) (void)hipFree(P->psi_alt);
  if (P->side) (void)hipStreamDestroy(P->side);
  if (P->ev_fork) (void)hipEventDestroy(P->ev_fork);
  if (P->ev_join) (void)hipEventDestroy(P->ev_join);
  if (P->rho_mean) (void)hipFree(P->rho_mean);
  if (P->partial) (void)hipFree(P->partial);
  if (P->scratch_small) (void)hipFree(P->scratch_small);
  if (P->adapt) (void)hipFree(P->adapt);
  if (P->adapt_tab) (void)hipFree(P->adapt_tab);
  if (P->prof) {
    Prof* pr = static_cast<Prof*>(P->prof);
    for (auto& r : pr->recs) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (auto& r : pr->pool) {
      (void)hipEventDestroy(r.first);
      (void)hipEventDestroy(r.second);
    }
    delete pr;
  }
  delete P;
}

int check_ptr(const Plan& P, const void* p, const char* name, bool nullable) {
  if (!p) return nullable ? TW_OK : fail(TW_EINVAL, "%s is NULL", name);
  if (reinterpret_cast<uintptr_t>(p) % P.elem != 0)
    return fail(TW_ELAYOUT, "%s is not aligned to the %zu-byte complex element", name, P.elem);
  return TW_OK;
}

// groups (workgroups along x) of a pass along `axis`
int pass_groups(const Plan& P, int axis) {
  const int c = pass_pencils_per_group(P.n[axis], P.fp32, axis == 0, P.cols_variant);
  const int64_t np = P.ncell / P.n[axis];
  return (int)((np + c - 1) / c);
}

// Largest number of pass workgroups along any axis over both strided-pass
// organisations: the per-group energy partials are laid out with this stride.
int64_t partial_gmax(const Plan& P) {
  int64_t gmax = 1;
  if (!P.z) return gmax;
  for (int v = 0; v < 2; ++v) {
    Plan Q = P;
    Q.cols_variant = v;
    for (int d = 0; d < P.dim; ++d) gmax = std::max<int64_t>(gmax, pass_groups(Q, d));
  }
  return gmax;
}

PassArgs base_args(const Plan& P, void* psi, void* psi_cl, int64_t nfield) {
  PassArgs a;
  std::memset(&a, 0, sizeof(a));
  a.psi = psi;
  a.psi_cl = psi_cl;
  a.z = P.z;
  a.n_real = P.p.n_real;
  a.nfield = nfield;
  a.ncell = P.ncell;
  for (int d = 0; d < 3; ++d) {
    a.n[d] = P.n[d];
    a.k2[d] = P.k2[d];
  }
  a.green = -4.0 * M_PI * P.p.G / (double)P.ncell;
  a.m_tot = P.p.m_tot;
  a.variant = P.cols_variant;
  return a;
}

// One pass over pairs [pair0, pair0 + npairs) (npairs < 0: every pair).
hipError_t pass(Plan& P, PassArgs a, int mode, int axis, const void* phase, hipStream_t s, int64_t pair0 = 0,
                int64_t npairs = -1) {
  a.axis = axis;
  a.stride = axis_stride(P, axis);
  a.twd = P.twd[axis];
  a.phase = phase;
  a.pair0 = pair0;
  a.rev = (int32_t)(P.pass_seq++ & 1);
  if (npairs < 0) npairs = (a.nfield + 1) / 2 - pair0;
  return timed(P, mode, s, [&] { return launch_pass(P, mode, a, s, (int)npairs); });
}

// Pairs advanced together through all steps. Chunks small enough to stay in
// the 256 MB Infinity Cache were measured slower on MI355X (the passes are
// latency-bound and lose more to smaller grids than they gain from the cache),
// so by default the whole ensemble is one chunk.
int64_t default_chunk_pairs(const Plan& P) { return P.npairs; }

}  // namespace
}  // namespace tw

namespace tw {
namespace {

// Device-chosen step sizes (tw_step_adaptive).
struct Adapt {
  double dt_max, courant, dtk;
  double* dt_out;
};

// Test particles advanced with the fields (tw_step_tracers).
struct Tracers {
  double* tr;
  int64_t ntracer;
};

// Kinetic bound on the step (footnote on the time step of Sec. "Numerical
// implementation"): the phase gradient must not alias, dt < 4 pi /
// (hbar k_max dk) with k_max = pi/dx and dk = 2 pi/L, per axis.
double kinetic_dt_bound(const Plan& P) {
  double b = INFINITY;
  for (int d = 0; d < P.dim; ++d) {
    const double L = P.p.box[d], dx = L / P.n[d];
    b = std::min(b, 4.0 * M_PI / (P.p.hbar_m * (M_PI / dx) * (2.0 * M_PI / L)));
  }
  return b;
}

// The launch sequence of tw_step / tw_step_adaptive on stream s (arguments
// already validated). With `ad`, the kick factor and the drift tables of every
// step come from device memory, written by launch_adapt after each kick pass.
// With prepare = false the tables and density means are taken as already
// built (by an earlier call with prepare = true on a stream this one waits
// for); [pair_lo, pair_hi) limits the pairs advanced (pair_hi < 0: all).
int enqueue_step(Plan& P, void* psi, void* psi_cl, int64_t nsteps, double dt, hipStream_t s,
                 const Adapt* ad = nullptr, const Tracers* tc = nullptr, bool prepare = true, int64_t pair_lo = 0,
                 int64_t pair_hi = -1) {
  const int64_t nfield = P.p.n_real + (psi_cl ? 1 : 0);
  const double h = 0.5 * dt;
  // drift tables: slot (axis, 0) = half step, (axis, 1) = full step
  auto phase_slot = [&](int axis, int full) -> void* {
    return reinterpret_cast<char*>(P.phase) + sizeof(double) * 2 * (size_t)P.nmax * (2 * axis + full);
  };
  auto adapt_slot = [&](int set, int axis) -> void* {
    return reinterpret_cast<char*>(P.adapt_tab) + sizeof(double) * 2 * (size_t)P.nmax * (3 * set + axis);
  };
  // drift factors of the opening half drift, and of step st (merged, or the closing half)
  auto ph_open = [&](int axis) -> const void* { return ad ? adapt_slot(2, axis) : phase_slot(axis, 0); };
  auto ph_step = [&](int axis, int64_t st, bool last) -> const void* {
    return ad ? adapt_slot((int)(st % 2), axis) : phase_slot(axis, last ? 0 : 1);
  };
  if (!ad && prepare) {
    for (int d = 0; d < P.dim; ++d) {
      TW_HIP(timed(P, KIND_TABLES, s, [&] { return launch_phase_table(P, d, h, phase_slot(d, 0), s); }));
      TW_HIP(timed(P, KIND_TABLES, s, [&] { return launch_phase_table(P, d, dt, phase_slot(d, 1), s); }));
    }
  }
  if (P.fp32 && prepare)
    TW_HIP(timed(P, KIND_MEAN, s, [&] { return launch_field_mean(P, psi, psi_cl, nfield, P.rho_mean, s); }));
  const double kick = dt / P.p.hbar_m;

  if (P.dim == 1 && ad) {
    // device-chosen steps: one launch per step, max |V| buckets and step
    // sizes exactly as for D >= 2 (steps 0 and 1 from the fields on entry,
    // step n + 2 from the potential inside step n)
    TW_HIP(timed(P, KIND_TABLES, s, [&] { return launch_adapt_clear(P, s); }));
    TW_HIP(timed(P, KIND_STEP1D, s, [&] {
      return launch_step1d_adapt(P, psi, psi_cl, nfield, -1, nullptr, nullptr, nullptr,
                                 P.adapt + kAdaptScalars + 2 * kVmaxBuckets, s);
    }));
    TW_HIP(timed(P, KIND_TABLES, s, [&] {
      return launch_adapt(P, -1, nsteps == 1, ad->dt_max, ad->courant, ad->dtk, ad->dt_out, s);
    }));
    for (int64_t st = 0; st < nsteps; ++st) {
      TW_HIP(timed(P, KIND_STEP1D, s, [&] {
        return launch_step1d_adapt(P, psi, psi_cl, nfield, st, ph_open(0), ph_step(0, st, st + 1 == nsteps),
                                   P.adapt + 6 + st % 2, P.adapt + kAdaptScalars + (st % 3) * kVmaxBuckets, s);
      }));
      TW_HIP(timed(P, KIND_TABLES, s, [&] {
        return launch_adapt(P, st, st + 2 == nsteps, ad->dt_max, ad->courant, ad->dtk, ad->dt_out, s);
      }));
    }
    return TW_OK;
  }
  if (P.dim == 1) {
    TW_HIP(timed(P, KIND_STEP1D, s, [&] {
      return launch_step1d(P, psi, psi_cl, nfield, nsteps, phase_slot(0, 0), phase_slot(0, 1), kick, s);
    }));
    return TW_OK;
  }

  PassArgs a = base_args(P, psi, psi_cl, nfield);
  a.kick = kick;
  a.rho_mean = P.fp32 ? P.rho_mean : nullptr;
  const int D = P.dim;
  const int64_t npairs = (nfield + 1) / 2;
  const int64_t chunk = ad ? npairs : (P.chunk_pairs > 0 ? P.chunk_pairs : default_chunk_pairs(P));
  const int64_t plo = pair_lo, phi = pair_hi < 0 ? npairs : std::min<int64_t>(pair_hi, npairs);
  if (ad) {
    // max |V| of the initial fields (the potential passes of the energy), then
    // the sizes of steps 0 and 1 and their drift tables
    TW_HIP(timed(P, KIND_TABLES, s, [&] { return launch_adapt_clear(P, s); }));
    PassArgs b = a;
    b.vmax = P.adapt + kAdaptScalars + 2 * kVmaxBuckets;
    b.partial = P.partial;
    TW_HIP(pass(P, b, PASS_RHO, 0, nullptr, s));
    for (int d = 1; d < D - 1; ++d) TW_HIP(pass(P, b, PASS_ZFWD, d, nullptr, s));
    TW_HIP(pass(P, b, PASS_ZPOISSON, D - 1, nullptr, s));
    for (int d = D - 2; d >= 1; --d) TW_HIP(pass(P, b, PASS_ZINV, d, nullptr, s));
    TW_HIP(pass(P, b, PASS_POT_SUM, 0, nullptr, s));
    TW_HIP(timed(P, KIND_TABLES, s, [&] {
      return launch_adapt(P, -1, nsteps == 1, ad->dt_max, ad->courant, ad->dtk, ad->dt_out, s);
    }));
  }
  // kick pass of step st: the kick factor and max |V| slot of the adaptive
  // state; with test particles it also leaves the potentials in the scratch
  auto kick_args = [&](PassArgs& b, int64_t st) {
    if (tc) b.store_v = 1;
    if (!ad) return;
    b.kick_dev = P.adapt + 6 + st % 2;
    b.vmax = P.adapt + kAdaptScalars + (st % 3) * kVmaxBuckets;
  };
  // particles of every field after the kick pass whose storage order is perm
  auto push = [&](const int (&perm)[3]) -> hipError_t {
    if (!tc) return hipSuccess;
    return timed(P, KIND_MODES, s, [&] { return launch_tracers(P, tc->tr, nfield, tc->ntracer, perm, dt, s); });
  };
  auto after_kick = [&](int64_t st) -> hipError_t {
    if (!ad) return hipSuccess;
    return timed(P, KIND_TABLES, s, [&] {
      return launch_adapt(P, st, st + 2 == nsteps, ad->dt_max, ad->courant, ad->dtk, ad->dt_out, s);
    });
  };
  if (D == 2 && P.transpose2d) {
    // Alternating storage: the field passes read whole rows along physical axis
    // `o0` of fields stored o0-contiguous; the kick pass writes its output
    // transposed into the other buffer of a pair (the caller's fields, the
    // plan's second field buffer), so the next field pass again reads rows
    // along the other axis. The density transform stays in the layout of the
    // fields, and the Poisson pass runs along its strided axis in place. Only
    // the opening half drift reads fields along a strided axis. Each step moves
    // the fields once between the buffers; the closing drift puts them back
    // into the caller's buffer, x-contiguous.
    char* alt = static_cast<char*>(P.psi_alt);
    void* buf[2][2] = {{psi, psi_cl}, {alt, alt + P.elem * (size_t)P.p.n_real * (size_t)P.ncell}};
    for (int64_t c0 = plo; c0 < phi; c0 += chunk) {
      const int64_t nc = std::min<int64_t>(chunk, phi - c0);
      int cur = 0;  // buffer holding the fields
      // pass along physical axis `ax` over data stored `contig`-contiguous
      auto go = [&](int mode, int contig, int ax, const void* phase, int t_psi, int64_t kick_step = -1) {
        PassArgs b = a;
        if (kick_step >= 0) kick_args(b, kick_step);
        const int other = 1 - contig;
        b.n[0] = P.n[contig];
        b.n[1] = P.n[other];
        b.n[2] = 1;
        b.k2[0] = P.k2[contig];
        b.k2[1] = P.k2[other];
        b.axis = ax == contig ? 0 : 1;
        b.stride = ax == contig ? 1 : P.n[contig];
        b.twd = P.twd[ax];
        b.phase = phase;
        b.pair0 = c0;
        b.psi = buf[cur][0];
        b.psi_cl = buf[cur][1];
        b.t_psi = t_psi;
        b.psi_t = buf[1 - cur][0];
        b.psi_cl_t = buf[1 - cur][1];
        b.rev = (int32_t)(P.pass_seq++ & 1);
        hipError_t e = timed(P, mode, s, [&] { return launch_pass(P, mode, b, s, (int)nc); });
        if (t_psi) cur = 1 - cur;
        return e;
      };
      int o0 = 0, o1 = 1;  // fields start x-contiguous
      TW_HIP(go(PASS_DRIFT, 0, 1, ph_open(1), 0));
      TW_HIP(go(PASS_DRIFT_RHO, o0, o0, ph_open(o0), 0));
      for (int64_t st = 0; st < nsteps; ++st) {
        const bool last = (st + 1 == nsteps);
        TW_HIP(go(PASS_ZPOISSON, o0, o1, nullptr, 0));
        // kick and drift along o0; fields move to the other buffer, o1-contiguous
        TW_HIP(go(PASS_KICK_DRIFT, o0, o0, ph_step(o0, st, last), 1, st));
        TW_HIP(push({o0, o1, 2}));
        TW_HIP(after_kick(st));
        if (!last) {
          TW_HIP(go(PASS_DRIFT_RHO, o1, o1, ph_step(o1, st, false), 0));
          std::swap(o0, o1);
        } else {
          // closing half drift along o1; transposed back to x-contiguous when o1 is y
          TW_HIP(go(PASS_DRIFT, o1, o1, ph_step(o1, st, true), o1 != 0 ? 1 : 0));
        }
      }
      if (cur != 0) return fail(TW_EINVAL, "internal: alternating-storage schedule ended in the plan's buffer");
    }
    return TW_OK;
  }
  if (D == 3 && P.slab3d) {
    // xy-plane schedule: three HBM passes per step. Steps alternate between
    // kind B (density transformed along x, y by the plane pass; Poisson along
    // z by z-pencils; plane pass: inverse along x, y, kick, drift x, y) and
    // kind A (z-pencil drift + density transform along z; plane Poisson;
    // z-pencil inverse, kick, drift z). A merged drift is split between the
    // kick pass of one step and the density pass of the next.
    for (int64_t c0 = plo; c0 < phi; c0 += chunk) {
      const int64_t nc = std::min<int64_t>(chunk, phi - c0);
      auto zpass = [&](int mode, const void* phase, int64_t kick_step = -1) -> hipError_t {
        PassArgs b = a;
        if (kick_step >= 0) kick_args(b, kick_step);
        return pass(P, b, mode, 2, phase, s, c0, nc);
      };
      auto plane = [&](int mode, const void* phx, const void* phy, int64_t kick_step = -1) -> hipError_t {
        PassArgs b = a;
        if (kick_step >= 0) kick_args(b, kick_step);
        b.axis = 0;
        b.stride = 1;
        b.twd = P.twd[0];
        b.phase = phx;
        b.phase2 = phy;
        b.pair0 = c0;
        b.rev = (int32_t)(P.pass_seq++ & 1);
        return timed(P, KIND_SLAB + mode, s, [&] { return launch_slab(P, mode, b, s, (int)nc); });
      };
      TW_HIP(zpass(PASS_DRIFT, ph_open(2)));
      TW_HIP(plane(SLAB_DRIFT_RHO, ph_open(0), ph_open(1)));
      for (int64_t st = 0; st < nsteps; ++st) {
        const bool last = (st + 1 == nsteps);
        if (st % 2 == 0) {
          TW_HIP(zpass(PASS_ZPOISSON, nullptr));
          TW_HIP(plane(SLAB_KICK_DRIFT, ph_step(0, st, last), ph_step(1, st, last), st));
          TW_HIP(push({0, 1, 2}));
          TW_HIP(after_kick(st));
          if (!last) TW_HIP(zpass(PASS_DRIFT_RHO, ph_step(2, st, false)));
          else TW_HIP(zpass(PASS_DRIFT, ph_step(2, st, true)));
        } else {
          TW_HIP(plane(SLAB_POISSON, nullptr, nullptr));
          TW_HIP(zpass(PASS_KICK_DRIFT, ph_step(2, st, last), st));
          TW_HIP(push({0, 1, 2}));
          TW_HIP(after_kick(st));
          if (!last) TW_HIP(plane(SLAB_DRIFT_RHO, ph_step(0, st, false), ph_step(1, st, false)));
          else TW_HIP(plane(SLAB_DRIFT, ph_step(0, st, true), ph_step(1, st, true)));
        }
      }
    }
    return TW_OK;
  }
  // Realizations are independent: each chunk of pairs runs every step before
  // the next chunk starts.
  for (int64_t c0 = plo; c0 < phi; c0 += chunk) {
    const int64_t nc = std::min<int64_t>(chunk, phi - c0);
    auto run = [&](int mode, int axis, const void* phase) { return pass(P, a, mode, axis, phase, s, c0, nc); };
    int o[3] = {0, 1, 2};
    // opening half drift: every axis but o[0] plain, o[0] fused with the density transform
    for (int i = D - 1; i >= 1; --i) TW_HIP(run(PASS_DRIFT, o[i], ph_open(o[i])));
    TW_HIP(run(PASS_DRIFT_RHO, o[0], ph_open(o[0])));
    for (int64_t st = 0; st < nsteps; ++st) {
      const bool last = (st + 1 == nsteps);
      // rest of the forward transform of rho, Green's function, inverse (all but o[0])
      for (int i = 1; i < D - 1; ++i) TW_HIP(run(PASS_ZFWD, o[i], nullptr));
      TW_HIP(run(PASS_ZPOISSON, o[D - 1], nullptr));
      for (int i = D - 2; i >= 1; --i) TW_HIP(run(PASS_ZINV, o[i], nullptr));
      // last inverse along o[0] -> V, kick, drift along o[0]
      {
        PassArgs b = a;
        kick_args(b, st);
        TW_HIP(pass(P, b, PASS_KICK_DRIFT, o[0], ph_step(o[0], st, last), s, c0, nc));
      }
      TW_HIP(push({0, 1, 2}));
      TW_HIP(after_kick(st));
      if (!last) {
        for (int i = 1; i < D - 1; ++i) TW_HIP(run(PASS_DRIFT, o[i], ph_step(o[i], st, false)));
        TW_HIP(run(PASS_DRIFT_RHO, o[D - 1], ph_step(o[D - 1], st, false)));
        // reverse the axis order so the density transform just made is the first one
        int r[3] = {0, 0, 0};
        for (int i = 0; i < D; ++i) r[i] = o[D - 1 - i];
        for (int i = 0; i < D; ++i) o[i] = r[i];
      } else {
        for (int i = 1; i < D; ++i) TW_HIP(run(PASS_DRIFT, o[i], ph_step(o[i], st, true)));
      }
    }
  }
  return TW_OK;
}


}  // namespace
}  // namespace tw

using namespace tw;

extern "C" {

const char* tw_last_error(void) { return g_error.c_str(); }

int tw_plan_create(const tw_problem* pr, tw_plan* out) {
  if (!pr || !out) return fail(TW_EINVAL, "NULL problem or output pointer");
  *out = nullptr;
  if (pr->dim < 1 || pr->dim > 3) return fail(TW_EINVAL, "dim must be 1, 2 or 3 (got %d)", pr->dim);
  if (pr->reserved != 0) return fail(TW_EINVAL, "reserved field must be 0");
  if (pr->precision != TW_FP64 && pr->precision != TW_FP32_SPLIT)
    return fail(TW_EINVAL, "unknown precision %d", pr->precision);
  for (int d = 0; d < 3; ++d) {
    if (d < pr->dim) {
      if (pr->n[d] < 1) return fail(TW_EINVAL, "n[%d] must be positive", d);
      if (!(pr->box[d] > 0.0) || !std::isfinite(pr->box[d])) return fail(TW_EINVAL, "box[%d] must be > 0", d);
      const bool ok = pr->dim == 1 ? step1d_length_supported(pr->n[d]) : pass_length_supported(pr->n[d]);
      if (!ok) return fail(TW_EUNSUPPORTED, "n[%d]=%d outside the supported lengths", d, pr->n[d]);
    } else if (pr->n[d] != 1) {
      return fail(TW_EINVAL, "n[%d] must be 1 for an unused axis", d);
    }
  }
  if (!(pr->hbar_m > 0.0) || !std::isfinite(pr->hbar_m)) return fail(TW_EINVAL, "hbar_m must be > 0");
  if (!(pr->G >= 0.0) || !std::isfinite(pr->G)) return fail(TW_EINVAL, "G must be >= 0 and finite");
  if (!(pr->m_tot > 0.0) || !std::isfinite(pr->m_tot)) return fail(TW_EINVAL, "m_tot must be > 0");
  if (!(pr->n_tot > 0.0)) return fail(TW_EINVAL, "n_tot must be > 0");
  if (pr->n_real < 1) return fail(TW_EINVAL, "n_real must be >= 1");

  Plan* P = new (std::nothrow) Plan();
  if (!P) return fail(TW_ENOMEM, "host allocation failed");
  std::memset(static_cast<void*>(P), 0, sizeof(Plan));
  P->p = *pr;
  P->dim = pr->dim;
  P->ncell = 1;
  P->nmax = 1;
  double dv = 1.0, vol = 1.0;
  for (int d = 0; d < 3; ++d) {
    P->n[d] = d < pr->dim ? pr->n[d] : 1;
    P->ncell *= P->n[d];
    if (P->n[d] > P->nmax) P->nmax = P->n[d];
    if (d < pr->dim) {
      dv = dv * (pr->box[d] / pr->n[d]);
      vol = vol * pr->box[d];
    }
  }
  if (P->ncell > (int64_t)INT32_MAX) {  // the pass kernels index cells of a field with 32-bit integers
    delete P;
    return fail(TW_EINVAL, "a field may hold at most 2^31 - 1 cells");
  }
  P->dV = dv;
  P->volume = vol;
  P->fp32 = pr->precision == TW_FP32_SPLIT;
  P->elem = P->fp32 ? 8 : 16;
  P->nfield = pr->n_real + 1;
  P->npairs = (P->nfield + 1) / 2;
  P->chunk_pairs = 0;  // 0: default_chunk_pairs
  if (const char* env = getenv("TW_CHUNK_PAIRS")) P->chunk_pairs = atoll(env);
  P->split_streams = 0;
  if (const char* env = getenv("TW_STREAMS")) P->split_streams = atoi(env) >= 2;
  P->transpose2d = pr->dim == 2 ? 1 : 0;  // 2D: alternating storage, every pass reads rows
  if (const char* env = getenv("TW_TRANSPOSE")) P->transpose2d = pr->dim == 2 && atoi(env) != 0;
  // strided-pass organisation: tuning cache if it has this shape, else the
  // usual winner (LDS tiles for FP32, interleaved pencils for FP64)
  P->cols_variant = P->fp32 ? 1 : 0;
  if (hipGetDevice(&P->device) != hipSuccess) {
    free_plan(P);
    return fail(TW_EHIP, "no HIP device");
  }
  // D = 3 with square xy-planes that fit one workgroup's LDS: the plane schedule
  P->slab_ok = 0;
  if (pr->dim == 3 && P->n[0] == P->n[1]) {
    const size_t need = slab_lds_bytes(P->n[0], P->fp32);
    int maxlds = 0;
    if (need > 0 &&
        hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, P->device) == hipSuccess &&
        (size_t)maxlds >= need)
      P->slab_ok = 1;
  }
  P->slab3d = P->slab_ok;
  if (const char* env = getenv("TW_SLAB")) {  // explicit override (tests, experiments)
    P->slab3d = P->slab_ok && atoi(env) != 0;
    P->slab_tuned = 1;
  }

#define ALLOC(ptr, bytes)                                                               \
  do {                                                                                  \
    if (hipMalloc(reinterpret_cast<void**>(&(ptr)), (bytes)) != hipSuccess) {            \
      free_plan(P);                                                                     \
      (void)hipGetLastError();                                                          \
      return fail(TW_ENOMEM, "device allocation of %zu bytes failed", (size_t)(bytes)); \
    }                                                                                   \
  } while (0)

  // twiddle and wavenumber tables per axis
  for (int d = 0; d < 3; ++d) {
    const int n = P->n[d];
    std::vector<double> k2(n);
    for (int j = 0; j < n; ++j) {
      const int jj = (j < (n + 1) / 2) ? j : j - n;  // FFT order; Nyquist as -n/2
      const double k = 2.0 * M_PI * (double)jj / (d < pr->dim ? pr->box[d] : 1.0);
      k2[j] = d < pr->dim ? k * k : 0.0;
    }
    ALLOC(P->k2[d], sizeof(double) * n);
    if (hipMemcpy(P->k2[d], k2.data(), sizeof(double) * n, hipMemcpyHostToDevice) != hipSuccess) {
      free_plan(P);
      return fail(TW_EHIP, "table upload failed");
    }
    std::vector<double> tw2(2 * n);
    for (int e = 0; e < n; ++e) {
      const long double ang = -2.0L * 3.141592653589793238462643383279502884L * (long double)e / (long double)n;
      tw2[2 * e] = (double)cosl(ang);
      tw2[2 * e + 1] = (double)sinl(ang);
    }
    if (P->fp32) {
      // FP32 twiddles as shear pairs (fft.hpp): entry e holds (tan(phi/2),
      // sin phi) of the angle -2 pi e / n reduced to |phi| <= pi/2, by a half
      // turn (a sign flip the kernels read off the index) and/or a whole turn
      std::vector<float> tf(2 * n);
      const long double two_pi = 6.283185307179586476925286766559005768L;
      for (int e = 0; e < n; ++e) {
        long double phi = -two_pi * (long double)e / (long double)n;
        if (twiddle_flip(e, n)) phi += 0.5L * two_pi;
        else if (4 * e >= 3 * n) phi += two_pi;
        tf[2 * e] = (float)tanl(0.5L * phi);
        tf[2 * e + 1] = (float)sinl(phi);
      }
      ALLOC(P->twd[d], sizeof(float) * 2 * n);
      if (hipMemcpy(P->twd[d], tf.data(), sizeof(float) * 2 * n, hipMemcpyHostToDevice) != hipSuccess) {
        free_plan(P);
        return fail(TW_EHIP, "table upload failed");
      }
    } else {
      ALLOC(P->twd[d], sizeof(double) * 2 * n);
      if (hipMemcpy(P->twd[d], tw2.data(), sizeof(double) * 2 * n, hipMemcpyHostToDevice) != hipSuccess) {
        free_plan(P);
        return fail(TW_EHIP, "table upload failed");
      }
    }
  }
  ALLOC(P->phase, sizeof(double) * 2 * 3 * 2 * P->nmax);
  // spectral scratch: one complex field per pair of realizations (diagnostics
  // need it in 1D too, where n >= 16)
  const bool need_z = pr->dim >= 2 || pass_length_supported(P->n[0]);
  if (need_z) ALLOC(P->z, P->elem * (size_t)P->npairs * (size_t)P->ncell);
  if (P->transpose2d) {
    // second field buffer for the alternating-storage schedule; a device too
    // small for it runs the strided-pass schedule instead
    const size_t fb = P->elem * (size_t)P->nfield * (size_t)P->ncell;
    if (hipMalloc(&P->psi_alt, fb) != hipSuccess) {
      (void)hipGetLastError();
      P->psi_alt = nullptr;
      P->transpose2d = 0;
    }
  }
  ALLOC(P->rho_mean, sizeof(double) * P->nfield);
  if (pr->dim >= 2) {
    const int v = tune_cache_lookup(tune_key(*P));
    if (v >= 0) {
      P->cols_variant = v;
      P->tuned = 1;
    }
    if (P->slab_ok && !getenv("TW_SLAB")) {
      const int sv = tune_cache_lookup(tune_key(*P) + "|slab");
      if (sv >= 0) {
        P->slab3d = sv;
        P->slab_tuned = 1;
      }
    }
  }
  if (const char* env = getenv("TW_COLS_VARIANT")) {  // explicit override (tests, experiments)
    const int v = atoi(env);
    if (v == 0 || v == 1) {
      P->cols_variant = v;
      P->tuned = 1;
    }
  }
  int64_t gmax = 1;
  if (need_z)
    for (int v = 0; v < 2; ++v) {  // partial sums sized for either organisation
      const int keep = P->cols_variant;
      P->cols_variant = v;
      for (int d = 0; d < pr->dim; ++d) gmax = std::max<int64_t>(gmax, pass_groups(*P, d));
      P->cols_variant = keep;
    }
  const int64_t nwaves = (P->ncell + 63) / 64;
  const int64_t energy_part = 4 * P->nfield * gmax + P->nfield;
  const int64_t mom_part = pr->n_real * nwaves + 3 * nwaves + pr->n_real + 8 + 2 * nwaves;
  P->partial_len = (size_t)std::max<int64_t>(energy_part + mom_part, P->nfield * kFieldMeanParts);
  ALLOC(P->partial, sizeof(double) * P->partial_len);
  ALLOC(P->scratch_small, sizeof(double) * 64);
  ALLOC(P->adapt, sizeof(double) * (kAdaptScalars + 3 * kVmaxBuckets));
  ALLOC(P->adapt_tab, sizeof(double) * 2 * 3 * 3 * (size_t)P->nmax);
#undef ALLOC
  *out = reinterpret_cast<tw_plan>(P);
  return TW_OK;
}

int tw_plan_destroy(tw_plan plan) {
  if (!plan) return TW_OK;
  Plan* P = reinterpret_cast<Plan*>(plan);
  (void)hipDeviceSynchronize();
  free_plan(P);
  return TW_OK;
}

int tw_sample(tw_plan plan, const void* psi_cl, uint64_t seed, int64_t real_offset, void* psi, void* stream) {
  if (!plan) return fail(TW_EINVAL, "NULL plan");
  Plan& P = *reinterpret_cast<Plan*>(plan);
  if (!psi_cl) return fail(TW_EINVAL, "psi_cl is NULL");
  if (reinterpret_cast<uintptr_t>(psi_cl) % 16 != 0) return fail(TW_ELAYOUT, "psi_cl is not 16-byte aligned");
  if (int rc = check_ptr(P, psi, "psi", false)) return rc;
  if (real_offset < 0) return fail(TW_EINVAL, "real_offset must be >= 0");
  if (P.p.n_real > 65535) return fail(TW_EUNSUPPORTED, "tw_sample supports at most 65535 realizations per call");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  TW_HIP(timed(P, KIND_SAMPLE, s, [&] { return launch_sample(P, psi_cl, seed, real_offset, psi, s); }));
  return TW_OK;
}

int tw_step(tw_plan plan, void* psi, void* psi_cl, int64_t nsteps, double dt, void* stream) {
  if (!plan) return fail(TW_EINVAL, "NULL plan");
  Plan& P = *reinterpret_cast<Plan*>(plan);
  if (int rc = check_ptr(P, psi, "psi", false)) return rc;
  if (int rc = check_ptr(P, psi_cl, "psi_classical", true)) return rc;
  if (nsteps < 0) return fail(TW_EINVAL, "nsteps must be >= 0");
  if (!std::isfinite(dt)) return fail(TW_EINVAL, "dt must be finite");
  if (nsteps == 0) return TW_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (P.split_streams && P.dim >= 2 && P.npairs >= 2 && hipStreamIsCapturing(s, &cap) == hipSuccess &&
      cap == hipStreamCaptureStatusNone) {
    // two halves of the pairs on two streams: their passes overlap, so one
    // half's strided Poisson pass runs beside the other half's row passes
    if (!P.side) {
      TW_HIP(hipStreamCreateWithFlags(&P.side, hipStreamNonBlocking));
      TW_HIP(hipEventCreateWithFlags(&P.ev_fork, hipEventDisableTiming));
      TW_HIP(hipEventCreateWithFlags(&P.ev_join, hipEventDisableTiming));
    }
    const int64_t nfield = P.p.n_real + (psi_cl ? 1 : 0);
    const int64_t half = ((nfield + 1) / 2) / 2;
    if (int rc = enqueue_step(P, psi, psi_cl, nsteps, dt, s, nullptr, nullptr, true, 0, 0)) return rc;
    TW_HIP(hipEventRecord(P.ev_fork, s));
    TW_HIP(hipStreamWaitEvent(P.side, P.ev_fork, 0));
    if (int rc = enqueue_step(P, psi, psi_cl, nsteps, dt, P.side, nullptr, nullptr, false, half, -1)) return rc;
    if (int rc = enqueue_step(P, psi, psi_cl, nsteps, dt, s, nullptr, nullptr, false, 0, half)) return rc;
    TW_HIP(hipEventRecord(P.ev_join, P.side));
    TW_HIP(hipStreamWaitEvent(s, P.ev_join, 0));
    return TW_OK;
  }
  return enqueue_step(P, psi, psi_cl, nsteps, dt, s);
}

int tw_step_tracers(tw_plan plan, void* psi, void* psi_cl, int64_t nsteps, double dt, double* tracers,
                    int64_t ntracer, void* stream) {
  if (!plan) return fail(TW_EINVAL, "NULL plan");
  Plan& P = *reinterpret_cast<Plan*>(plan);
  if (int rc = check_ptr(P, psi, "psi", false)) return rc;
  if (int rc = check_ptr(P, psi_cl, "psi_classical", true)) return rc;
  if (nsteps < 0) return fail(TW_EINVAL, "nsteps must be >= 0");
  if (!std::isfinite(dt)) return fail(TW_EINVAL, "dt must be finite");
  if (!tracers || ntracer < 1) return fail(TW_EINVAL, "tracers must be a device array with ntracer >= 1");
  if (reinterpret_cast<uintptr_t>(tracers) % 8 != 0) return fail(TW_ELAYOUT, "tracers must be 8-byte aligned");
  if (P.dim < 2 || !P.z) return fail(TW_EUNSUPPORTED, "test particles need D >= 2 (all axes >= 16 points)");
  if (P.chunk_pairs > 0 && P.chunk_pairs < P.npairs)
    return fail(TW_EUNSUPPORTED, "test particles need the whole ensemble in one chunk (TW_CHUNK_PAIRS)");
  if (nsteps == 0) return TW_OK;
  Tracers tc{tracers, ntracer};
  return enqueue_step(P, psi, psi_cl, nsteps, dt, reinterpret_cast<hipStream_t>(stream), nullptr, &tc);
}

int tw_tracer_spread(tw_plan plan, const double* tracers, int64_t ntracer, double* out, void* stream) {
  if (!plan) return fail(TW_EINVAL, "NULL plan");
  Plan& P = *reinterpret_cast<Plan*>(plan);
  if (!tracers || !out || ntracer < 1) return fail(TW_EINVAL, "bad tracer spread arguments");
  if (reinterpret_cast<uintptr_t>(tracers) % 8 != 0 || reinterpret_cast<uintptr_t>(out) % 8 != 0)
    return fail(TW_ELAYOUT, "tracers and out must be 8-byte aligned");
  TW_HIP(launch_tracer_spread(P, tracers, ntracer, out, reinterpret_cast<hipStream_t>(stream)));
  return TW_OK;
}

int tw_step_adaptive(tw_plan plan, void* psi, void* psi_cl, int64_t nsteps, double dt_max, double courant,
                     double* dt_out, void* stream) {
  if (!plan) return fail(TW_EINVAL, "NULL plan");
  Plan& P = *reinterpret_cast<Plan*>(plan);
  if (int rc = check_ptr(P, psi, "psi", false)) return rc;
  if (int rc = check_ptr(P, psi_cl, "psi_classical", true)) return rc;
  if (nsteps < 0) return fail(TW_EINVAL, "nsteps must be >= 0");
  if (!(dt_max > 0.0) || !std::isfinite(dt_max)) return fail(TW_EINVAL, "dt_max must be positive and finite");
  if (!(courant > 0.0) || !(courant <= 1.0)) return fail(TW_EINVAL, "courant must be in (0, 1]");
  if (reinterpret_cast<uintptr_t>(dt_out) % 8 != 0) return fail(TW_ELAYOUT, "dt_out must be 8-byte aligned");
  if (!P.adapt || (P.dim >= 2 && !P.z)) return fail(TW_EUNSUPPORTED, "adaptive steps need all axes >= 16 points for D >= 2");
  if (P.chunk_pairs > 0 && P.chunk_pairs < P.npairs)
    return fail(TW_EUNSUPPORTED, "adaptive steps need the whole ensemble in one chunk (TW_CHUNK_PAIRS)");
  if (nsteps == 0) return TW_OK;
  Adapt ad{dt_max, courant, kinetic_dt_bound(P), dt_out};
  return enqueue_step(P, psi, psi_cl, nsteps, dt_max, reinterpret_cast<hipStream_t>(stream), &ad);
}

int tw_moments(tw_plan plan, const void* psi, const void* psi_cl, const tw_moments_out* out, void* stream) {
  if (!plan) return fail(TW_EINVAL, "NULL plan");
  if (!out) return fail(TW_EINVAL, "NULL output struct");
  Plan& P = *reinterpret_cast<Plan*>(plan);
  if (int rc = check_ptr(P, psi, "psi", false)) return rc;
  if (int rc = check_ptr(P, psi_cl, "psi_classical", true)) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  double* energy_dev = nullptr;
  if (out->energy) {
    if (!P.z) return fail(TW_EUNSUPPORTED, "energy needs grid lengths >= 16");
    const int64_t nfield = P.p.n_real + (psi_cl ? 1 : 0);
    void* psi_m = const_cast<void*>(psi);
    void* cl_m = const_cast<void*>(psi_cl);
    PassArgs a = base_args(P, psi_m, cl_m, nfield);
    int ng[4] = {1, 1, 1, 1};
    for (int d = 0; d < P.dim; ++d) ng[d] = pass_groups(P, d);
    const int64_t gmax = partial_gmax(P);
    ng[3] = ng[0];
    const int64_t gstride = P.nfield * gmax;
    energy_dev = P.partial + 4 * gstride;
    if (P.fp32) {
      TW_HIP(timed(P, KIND_MEAN, s, [&] { return launch_field_mean(P, psi, psi_cl, nfield, P.rho_mean, s); }));
      a.rho_mean = P.rho_mean;
    }
    for (int d = 0; d < P.dim; ++d) {
      PassArgs b = a;
      b.partial = P.partial + d * gstride;
      TW_HIP(pass(P, b, PASS_KIN_SUM, d, nullptr, s));
    }
    TW_HIP(pass(P, a, PASS_RHO, 0, nullptr, s));
    for (int d = 1; d < P.dim - 1; ++d) TW_HIP(pass(P, a, PASS_ZFWD, d, nullptr, s));
    if (P.dim >= 2) TW_HIP(pass(P, a, PASS_ZPOISSON, P.dim - 1, nullptr, s));
    for (int d = P.dim - 2; d >= 1; --d) TW_HIP(pass(P, a, PASS_ZINV, d, nullptr, s));
    {
      PassArgs b = a;
      b.partial = P.partial + 3 * gstride;
      b.pot_green = P.dim == 1 ? 1 : 0;
      TW_HIP(pass(P, b, PASS_POT_SUM, 0, nullptr, s));
    }
    TW_HIP(timed(P, KIND_ENERGY, s,
                 [&] { return launch_energy_finalize(P, P.partial, gstride, nfield, ng, energy_dev, s); }));
    TW_HIP(hipMemcpyAsync(out->energy, energy_dev, sizeof(double) * P.p.n_real, hipMemcpyDeviceToDevice, s));
  }
  if (out->mode_occ) {
    if (!P.z) return fail(TW_EUNSUPPORTED, "mode occupations need grid lengths >= 16");
    // realizations only: slots p hold realization 2p (round 0) or 2p+1 (round 1)
    PassArgs a = base_args(P, const_cast<void*>(psi), nullptr, P.p.n_real);
    const int64_t nslots = (P.p.n_real + 1) / 2;
    for (int k = 0; k < 2; ++k) {
      TW_HIP(timed(P, KIND_MODES, s, [&] { return launch_gather_round(P, psi, nslots, k, s); }));
      for (int d = 0; d < P.dim; ++d) TW_HIP(pass(P, a, PASS_ZFWD, d, nullptr, s));
      TW_HIP(timed(P, KIND_MODES, s, [&] { return launch_mode_occ(P, nslots, k, out->mode_occ, s); }));
    }
  }
  if (out->var_amp || out->var_phase || out->decoherence) {
    // after the moment reductions' own region
    const int64_t nwaves = (P.ncell + 63) / 64;
    double* scratch = P.partial + 4 * P.nfield * partial_gmax(P) + P.nfield + P.p.n_real * nwaves + 3 * nwaves +
                      P.p.n_real + 8;
    TW_HIP(timed(P, KIND_MODES, s, [&] {
      return launch_decoherence(P, psi, out->var_amp, out->var_phase, out->decoherence, scratch, s);
    }));
  }
  Plan Q = P;
  // the moment reductions use the region after the energy partials
  Q.partial = P.partial + 4 * P.nfield * partial_gmax(P) + P.nfield;
  TW_HIP(timed(P, KIND_MOMENTS, s, [&] { return launch_moments(Q, psi, psi_cl, out, energy_dev, s); }));
  return TW_OK;
}

int tw_plan_autotune(tw_plan plan, int32_t* variant_out, void* stream) {
  if (!plan) return fail(TW_EINVAL, "NULL plan");
  Plan& P = *reinterpret_cast<Plan*>(plan);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const bool need_slab = P.slab_ok && !P.slab_tuned;
  if ((P.dim == 1 || P.tuned) && !need_slab) {  // no strided passes, or already chosen (cache / override / earlier call)
    P.tuned = 1;
    if (variant_out) *variant_out = P.cols_variant;
    return TW_OK;
  }
  const bool need_cols = !(P.dim == 1 || P.tuned);
  // Under the 2D alternating schedule only the Poisson pass is strided and it
  // touches only the pair scratch: time it on the plan's own scratch at full
  // size. Otherwise time every strided pass on a scratch ensemble of up to 32
  // pairs (enough workgroups to fill the device).
  const bool z_only = P.dim == 2 && P.transpose2d;
  const int64_t npt = z_only ? P.npairs : std::min<int64_t>(P.npairs, 32);
  const int64_t nf = 2 * npt;
  void* tmp = nullptr;
  if (!z_only && hipMalloc(&tmp, (size_t)nf * P.ncell * P.elem) != hipSuccess) {
    (void)hipGetLastError();
    return fail(TW_ENOMEM, "autotune scratch allocation failed");
  }
  struct Free {
    void* p;
    ~Free() {
      if (p) (void)hipFree(p);
    }
  } guard{tmp};
  if (tmp) TW_HIP(hipMemsetAsync(tmp, 0, (size_t)nf * P.ncell * P.elem, s));
  TW_HIP(hipMemsetAsync(P.z, 0, (size_t)npt * P.ncell * P.elem, s));
  auto phase_slot = [&](int axis, int full) -> void* {
    return reinterpret_cast<char*>(P.phase) + sizeof(double) * 2 * (size_t)P.nmax * (2 * axis + full);
  };
  for (int d = 0; d < P.dim; ++d) {
    TW_HIP(launch_phase_table(P, d, 5e-5, phase_slot(d, 0), s));
    TW_HIP(launch_phase_table(P, d, 1e-4, phase_slot(d, 1), s));
  }
  Plan Q = P;
  Q.p.n_real = nf;
  Q.profiling = false;
  PassArgs a = base_args(Q, tmp, nullptr, nf);
  a.kick = 1e-4;
  hipEvent_t e0, e1;
  TW_HIP(hipEventCreate(&e0));
  TW_HIP(hipEventCreate(&e1));
  double us[2] = {0.0, 0.0};
  // the strided passes a step runs: all five kinds, or with the 2D
  // alternating-storage schedule only the Poisson pass
  const int modes[5] = {PASS_ZPOISSON, PASS_DRIFT_RHO, PASS_KICK_DRIFT, PASS_DRIFT, PASS_ZFWD};
  const int nmodes = z_only ? 1 : 5;
  int rc = TW_OK;
  for (int v = 0; v < 2 && rc == TW_OK && need_cols; ++v) {
    Q.cols_variant = v;
    a.variant = v;
    for (int rep = 0; rep < 4 && rc == TW_OK; ++rep) {  // rep 0 warms up
      if (hipEventRecord(e0, s) != hipSuccess) rc = fail(TW_EHIP, "event record failed");
      for (int d = 1; d < P.dim && rc == TW_OK; ++d)
        for (int m = 0; m < nmodes && rc == TW_OK; ++m) {
          hipError_t e = pass(Q, a, modes[m], d, phase_slot(d, 1), s, 0, npt);
          if (e != hipSuccess) rc = fail(TW_EHIP, "autotune pass: %s", hipGetErrorString(e));
        }
      float ms = 0.f;
      if (rc == TW_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                          hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = fail(TW_EHIP, "event timing failed");
      if (rep > 0) us[v] += 1e3 * ms / 3.0;
    }
  }
  if (rc == TW_OK && need_cols) {
    P.cols_variant = us[1] < us[0] ? 1 : 0;
    P.tuned = 1;
    tune_cache_store(tune_key(P), P.cols_variant, us);
  }
  // D = 3: the xy-plane schedule against the pencil schedule, two whole steps
  // of the scratch ensemble each (at most as many fields as the plan holds:
  // the density means and partial sums are sized for those)
  if (rc == TW_OK && need_slab && tmp) {
    int64_t nps = npt;
    if (2 * nps > P.nfield) nps -= 1;
    if (nps >= 1) {
      Plan S = P;
      S.p.n_real = 2 * nps;
      S.profiling = false;
      S.chunk_pairs = 0;
      double su[2] = {0.0, 0.0};
      for (int v = 0; v < 2 && rc == TW_OK; ++v) {
        S.slab3d = v;
        for (int rep = 0; rep < 3 && rc == TW_OK; ++rep) {  // rep 0 warms up
          if (hipEventRecord(e0, s) != hipSuccess) rc = fail(TW_EHIP, "event record failed");
          if (rc == TW_OK) rc = enqueue_step(S, tmp, nullptr, 2, 1e-4, s);
          float ms = 0.f;
          if (rc == TW_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                              hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            rc = fail(TW_EHIP, "event timing failed");
          if (rep > 0) su[v] += 1e3 * ms / 2.0;
        }
      }
      if (rc == TW_OK) {
        P.slab3d = su[1] < su[0] ? 1 : 0;
        P.slab_tuned = 1;
        tune_cache_store(tune_key(P) + "|slab", P.slab3d, su);
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != TW_OK) return rc;
  P.tuned = 1;
  if (variant_out) *variant_out = P.cols_variant;
  return TW_OK;
}

int tw_plan_set_profiling(tw_plan plan, int32_t enable) {
  if (!plan) return fail(TW_EINVAL, "NULL plan");
  Plan& P = *reinterpret_cast<Plan*>(plan);
  if (enable && !P.prof) P.prof = new (std::nothrow) Prof();
  if (enable && !P.prof) return fail(TW_ENOMEM, "host allocation failed");
  P.profiling = enable != 0;
  return TW_OK;
}

int tw_plan_get_profile(tw_plan plan, int32_t n_kinds, int64_t* launches, double* total_ms) {
  if (!plan) return fail(TW_EINVAL, "NULL plan");
  if (n_kinds < 0 || (n_kinds > 0 && (!launches || !total_ms))) return fail(TW_EINVAL, "bad output arrays");
  Plan& P = *reinterpret_cast<Plan*>(plan);
  for (int k = 0; k < n_kinds; ++k) {
    launches[k] = 0;
    total_ms[k] = 0.0;
  }
  if (!P.prof) return TW_OK;
  Prof* pr = static_cast<Prof*>(P.prof);
  int rc = TW_OK;
  for (auto& r : pr->recs) {
    if (rc == TW_OK) {
      float ms = 0.f;
      hipError_t e = hipEventSynchronize(r.b);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
      if (e != hipSuccess) rc = fail(TW_EHIP, "event timing failed: %s", hipGetErrorString(e));
      else if (r.kind >= 0 && r.kind < n_kinds) {
        launches[r.kind] += 1;
        total_ms[r.kind] += ms;
      }
    }
    pr->pool.push_back({r.a, r.b});
  }
  pr->recs.clear();
  return rc;
}

const char* tw_kernel_kind_name(int32_t kind) {
  if (kind < 0 || kind >= KIND_COUNT) return "";
  return kKindNames[kind];
}

}  // extern "C"

// ===================================================================== batches
// Ensembles of several grid sizes advanced together: every pass of a step is
// one grouped launch over all size classes, and a whole tw_batch_step call
// (tables, density means, all steps) is captured once into a hipGraph and
// replayed while the arguments stay the same.
namespace tw {
namespace {

struct Batch {
  int count = 0;
  Plan* plans[kMaxClasses] = {nullptr, nullptr, nullptr, nullptr};
  bool fp32 = false;
  int dim = 0;
  int variant = 0;  // strided-pass organisation of the grouped launches
  int mode = 0;     // 0: one grouped launch per pass; 1: one kernel chain per class, run as parallel graph branches
  int tuned = 0;
  hipStream_t cap = nullptr;
  hipStream_t br[kMaxClasses] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kMaxClasses] = {nullptr, nullptr, nullptr, nullptr};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t key_nsteps = -1;
  double key_dt = 0.0;
  void* key_psi[kMaxClasses] = {nullptr, nullptr, nullptr, nullptr};
  void* key_cl[kMaxClasses] = {nullptr, nullptr, nullptr, nullptr};
};

void free_batch(Batch* B) {
  if (!B) return;
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  if (B->cap) (void)hipStreamDestroy(B->cap);
  for (int c = 0; c < kMaxClasses; ++c) {
    if (B->br[c]) (void)hipStreamDestroy(B->br[c]);
    if (B->join[c]) (void)hipEventDestroy(B->join[c]);
  }
  if (B->fork) (void)hipEventDestroy(B->fork);
  for (int c = 0; c < B->count; ++c) free_plan(B->plans[c]);
  delete B;
}

std::string batch_key(const Batch& B) {
  std::string k = tune_key(*B.plans[0]);
  k = k.substr(0, k.find('|')) + "|batch";
  for (int c = 0; c < B.count; ++c) {
    char buf[96];
    snprintf(buf, sizeof(buf), "|%dx%dx%d:%lld", B.plans[c]->n[0], B.plans[c]->n[1], B.plans[c]->n[2],
             (long long)B.plans[c]->npairs);
    k += buf;
  }
  return k + (B.fp32 ? "|fp32" : "|fp64");
}

void* phase_slot_of(const Plan& P, int axis, int full) {
  return reinterpret_cast<char*>(P.phase) + sizeof(double) * 2 * (size_t)P.nmax * (2 * axis + full);
}

// One grouped pass over pairs [0, npairs_c) of every class c.
hipError_t grouped(Batch& B, const PassArgs* base, int mode, int axis, int full, hipStream_t s,
                   const int64_t* npairs = nullptr) {
  GroupArgs g;
  std::memset(&g, 0, sizeof(g));
  g.nclass = B.count;
  for (int c = 0; c < B.count; ++c) {
    const Plan& P = *B.plans[c];
    PassArgs a = base[c];
    a.axis = axis;
    a.stride = axis_stride(P, axis);
    a.twd = P.twd[axis];
    a.phase = full >= 0 ? phase_slot_of(P, axis, full) : nullptr;
    a.pair0 = 0;
    if (npairs) a.nfield = std::min<int64_t>(a.nfield, 2 * npairs[c]);
    a.variant = B.variant;
    g.a[c] = a;
  }
  return launch_grouped(B.fp32, mode, g, B.variant, s);
}

// The launch sequence of tw_step for every class at once (all classes share
// the dimension, so they share the pass sequence and axis order).
int enqueue_batch(Batch& B, void* const* psi, void* const* psi_cl, int64_t nsteps, double dt, hipStream_t s) {
  PassArgs base[kMaxClasses];
  const double h = 0.5 * dt;
  for (int c = 0; c < B.count; ++c) {
    Plan& P = *B.plans[c];
    const int64_t nfield = P.p.n_real + (psi_cl && psi_cl[c] ? 1 : 0);
    for (int d = 0; d < P.dim; ++d) {
      TW_HIP(launch_phase_table(P, d, h, phase_slot_of(P, d, 0), s));
      TW_HIP(launch_phase_table(P, d, dt, phase_slot_of(P, d, 1), s));
    }
    if (P.fp32) TW_HIP(launch_field_mean(P, psi[c], psi_cl ? psi_cl[c] : nullptr, nfield, P.rho_mean, s));
    base[c] = base_args(P, psi[c], psi_cl ? psi_cl[c] : nullptr, nfield);
    base[c].kick = dt / P.p.hbar_m;
    base[c].rho_mean = P.fp32 ? P.rho_mean : nullptr;
  }
  const int D = B.dim;
  int o[3] = {0, 1, 2};
  for (int i = D - 1; i >= 1; --i) TW_HIP(grouped(B, base, PASS_DRIFT, o[i], 0, s));
  TW_HIP(grouped(B, base, PASS_DRIFT_RHO, o[0], 0, s));
  for (int64_t st = 0; st < nsteps; ++st) {
    const bool last = (st + 1 == nsteps);
    for (int i = 1; i < D - 1; ++i) TW_HIP(grouped(B, base, PASS_ZFWD, o[i], -1, s));
    TW_HIP(grouped(B, base, PASS_ZPOISSON, o[D - 1], -1, s));
    for (int i = D - 2; i >= 1; --i) TW_HIP(grouped(B, base, PASS_ZINV, o[i], -1, s));
    TW_HIP(grouped(B, base, PASS_KICK_DRIFT, o[0], last ? 0 : 1, s));
    if (!last) {
      for (int i = 1; i < D - 1; ++i) TW_HIP(grouped(B, base, PASS_DRIFT, o[i], 1, s));
      TW_HIP(grouped(B, base, PASS_DRIFT_RHO, o[D - 1], 1, s));
      int r[3] = {0, 0, 0};
      for (int i = 0; i < D; ++i) r[i] = o[D - 1 - i];
      for (int i = 0; i < D; ++i) o[i] = r[i];
    } else {
      for (int i = 1; i < D; ++i) TW_HIP(grouped(B, base, PASS_DRIFT, o[i], 0, s));
    }
  }
  return TW_OK;
}

// Each class runs its own tw_step sequence (its own plan's strided-pass
// organisation) on a stream of its own; forked from and joined back into s.
int enqueue_batch_branches(Batch& B, void* const* psi, void* const* psi_cl, int64_t nsteps, double dt,
                           hipStream_t s) {
  TW_HIP(hipEventRecord(B.fork, s));
  for (int c = 0; c < B.count; ++c) {
    TW_HIP(hipStreamWaitEvent(B.br[c], B.fork, 0));
    const int rc = enqueue_step(*B.plans[c], psi[c], psi_cl ? psi_cl[c] : nullptr, nsteps, dt, B.br[c]);
    if (rc != TW_OK) return rc;
    TW_HIP(hipEventRecord(B.join[c], B.br[c]));
    TW_HIP(hipStreamWaitEvent(s, B.join[c], 0));
  }
  return TW_OK;
}

int enqueue_batch_mode(Batch& B, void* const* psi, void* const* psi_cl, int64_t nsteps, double dt, hipStream_t s) {
  return B.mode == 1 ? enqueue_batch_branches(B, psi, psi_cl, nsteps, dt, s) : enqueue_batch(B, psi, psi_cl, nsteps, dt, s);
}

}  // namespace
}  // namespace tw

extern "C" {

int tw_batch_create(const tw_problem* problems, int32_t count, tw_batch* out) {
  if (!problems || !out) return fail(TW_EINVAL, "NULL problems or output pointer");
  *out = nullptr;
  if (count < 1 || count > kMaxClasses) return fail(TW_EINVAL, "count must be 1..%d", kMaxClasses);
  for (int c = 0; c < count; ++c) {
    const tw_problem& p = problems[c];
    if (p.dim != problems[0].dim || p.precision != problems[0].precision)
      return fail(TW_EINVAL, "all classes of a batch need the same dim and precision");
    if (p.dim < 2) return fail(TW_EUNSUPPORTED, "batches are for D = 2 or 3 (1D plans run resident already)");
    for (int d = 0; d < p.dim; ++d)
      if (!batch_length_supported(p.n[d]))
        return fail(TW_EUNSUPPORTED, "class %d: n[%d]=%d outside the batched lengths (16..128)", c, d, p.n[d]);
  }
  Batch* B = new (std::nothrow) Batch();
  if (!B) return fail(TW_ENOMEM, "host allocation failed");
  for (int c = 0; c < count; ++c) {
    tw_plan pl = nullptr;
    const int rc = tw_plan_create(&problems[c], &pl);
    if (rc != TW_OK) {
      free_batch(B);
      return rc;
    }
    B->plans[c] = reinterpret_cast<Plan*>(pl);
    B->count = c + 1;
  }
  B->fp32 = problems[0].precision == TW_FP32_SPLIT;
  B->dim = problems[0].dim;
  B->variant = B->fp32 ? 1 : 0;
  const int v = tune_cache_lookup(batch_key(*B));
  if (v >= 0) {
    B->variant = v;
    B->tuned = 1;
  }
  if (const char* env = getenv("TW_COLS_VARIANT")) {
    const int ev = atoi(env);
    if (ev == 0 || ev == 1) {
      B->variant = ev;
      B->tuned = 1;
    }
  }
  const int m = tune_cache_lookup(batch_key(*B) + "|mode");
  if (m >= 0) B->mode = m;
  if (const char* env = getenv("TW_BATCH_MODE")) {
    const int em = atoi(env);
    if (em == 0 || em == 1) B->mode = em;
  }
  bool ok = hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&B->fork, hipEventDisableTiming) == hipSuccess;
  for (int c = 0; c < count && ok; ++c)
    ok = hipStreamCreateWithFlags(&B->br[c], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&B->join[c], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    free_batch(B);
    return fail(TW_EHIP, "stream or event creation failed");
  }
  *out = reinterpret_cast<tw_batch>(B);
  return TW_OK;
}

int tw_batch_plan(tw_batch batch, int32_t index, tw_plan* out) {
  if (!batch || !out) return fail(TW_EINVAL, "NULL batch or output pointer");
  Batch& B = *reinterpret_cast<Batch*>(batch);
  if (index < 0 || index >= B.count) return fail(TW_EINVAL, "class index %d out of range", index);
  *out = reinterpret_cast<tw_plan>(B.plans[index]);
  return TW_OK;
}

int tw_batch_destroy(tw_batch batch) {
  if (!batch) return TW_OK;
  (void)hipDeviceSynchronize();
  free_batch(reinterpret_cast<Batch*>(batch));
  return TW_OK;
}

int tw_batch_autotune(tw_batch batch, int32_t* variant_out, int32_t* mode_out, void* stream) {
  if (!batch) return fail(TW_EINVAL, "NULL batch");
  Batch& B = *reinterpret_cast<Batch*>(batch);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (B.tuned) {
    if (variant_out) *variant_out = B.variant;
    if (mode_out) *mode_out = B.mode;
    return TW_OK;
  }
  // scratch: up to 8 pairs of every class
  void* tmp[kMaxClasses] = {nullptr, nullptr, nullptr, nullptr};
  int64_t npt[kMaxClasses];
  PassArgs base[kMaxClasses];
  int rc = TW_OK;
  for (int c = 0; c < B.count && rc == TW_OK; ++c) {
    Plan& P = *B.plans[c];
    npt[c] = std::min<int64_t>(P.npairs, 8);
    const size_t bytes = (size_t)(2 * npt[c]) * P.ncell * P.elem;
    if (hipMalloc(&tmp[c], bytes) != hipSuccess) {
      (void)hipGetLastError();
      rc = fail(TW_ENOMEM, "autotune scratch allocation failed");
      break;
    }
    if (hipMemsetAsync(tmp[c], 0, bytes, s) != hipSuccess || hipMemsetAsync(P.z, 0, npt[c] * P.ncell * P.elem, s) != hipSuccess)
      rc = fail(TW_EHIP, "scratch clear failed");
    for (int d = 0; d < P.dim && rc == TW_OK; ++d)
      if (launch_phase_table(P, d, 1e-4, phase_slot_of(P, d, 1), s) != hipSuccess) rc = fail(TW_EHIP, "tables");
    Plan Q = P;
    Q.p.n_real = 2 * npt[c];
    base[c] = base_args(Q, tmp[c], nullptr, 2 * npt[c]);
    base[c].n_real = 2 * npt[c];
    base[c].kick = 1e-4;
  }
  double us[2] = {0.0, 0.0};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (rc == TW_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    rc = fail(TW_EHIP, "event creation failed");
  const int modes[5] = {PASS_DRIFT_RHO, PASS_ZPOISSON, PASS_KICK_DRIFT, PASS_DRIFT, PASS_ZFWD};
  const int nmodes = 5;  // batches run the in-place schedule
  const int keep = B.variant;
  for (int v = 0; v < 2 && rc == TW_OK; ++v) {
    B.variant = v;
    for (int rep = 0; rep < 4 && rc == TW_OK; ++rep) {
      if (hipEventRecord(e0, s) != hipSuccess) rc = fail(TW_EHIP, "event record failed");
      for (int d = 1; d < B.dim && rc == TW_OK; ++d)
        for (int m = 0; m < nmodes && rc == TW_OK; ++m) {
          hipError_t e = grouped(B, base, modes[m], d, 1, s, npt);
          if (e != hipSuccess) rc = fail(TW_EHIP, "autotune pass: %s", hipGetErrorString(e));
        }
      float ms = 0.f;
      if (rc == TW_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                          hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = fail(TW_EHIP, "event timing failed");
      if (rep > 0) us[v] += 1e3 * ms / 3.0;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(s);
  for (int c = 0; c < B.count; ++c)
    if (tmp[c]) (void)hipFree(tmp[c]);
  if (rc != TW_OK) {
    B.variant = keep;
    return rc;
  }
  B.variant = us[1] < us[0] ? 1 : 0;
  tune_cache_store(batch_key(B), B.variant, us);
  // per-class organisation for the branch mode, then both modes timed on
  // full-size scratch ensembles (2 steps each after one warm-up)
  for (int c = 0; c < B.count; ++c) {
    const int rc2 = tw_plan_autotune(reinterpret_cast<tw_plan>(B.plans[c]), nullptr, stream);
    if (rc2 != TW_OK) return rc2;
  }
  {
    void* full[kMaxClasses] = {nullptr, nullptr, nullptr, nullptr};
    int rc3 = TW_OK;
    for (int c = 0; c < B.count && rc3 == TW_OK; ++c) {
      const Plan& P = *B.plans[c];
      const size_t bytes = (size_t)P.p.n_real * P.ncell * P.elem;
      if (hipMalloc(&full[c], bytes) != hipSuccess) {
        (void)hipGetLastError();
        rc3 = fail(TW_ENOMEM, "autotune scratch allocation failed");
      } else if (hipMemsetAsync(full[c], 0, bytes, s) != hipSuccess) {
        rc3 = fail(TW_EHIP, "scratch clear failed");
      }
    }
    double mus[2] = {0.0, 0.0};
    hipEvent_t f0 = nullptr, f1 = nullptr;
    if (rc3 == TW_OK && (hipEventCreate(&f0) != hipSuccess || hipEventCreate(&f1) != hipSuccess))
      rc3 = fail(TW_EHIP, "event creation failed");
    for (int m = 0; m < 2 && rc3 == TW_OK; ++m) {
      B.mode = m;
      for (int rep = 0; rep < 2 && rc3 == TW_OK; ++rep) {
        if (hipEventRecord(f0, s) != hipSuccess) rc3 = fail(TW_EHIP, "event record failed");
        if (rc3 == TW_OK) rc3 = enqueue_batch_mode(B, full, nullptr, 2, 1e-4, s);
        float ms = 0.f;
        if (rc3 == TW_OK && (hipEventRecord(f1, s) != hipSuccess || hipEventSynchronize(f1) != hipSuccess ||
                             hipEventElapsedTime(&ms, f0, f1) != hipSuccess))
          rc3 = fail(TW_EHIP, "event timing failed");
        if (rep > 0) mus[m] = 1e3 * ms;
      }
    }
    if (f0) (void)hipEventDestroy(f0);
    if (f1) (void)hipEventDestroy(f1);
    (void)hipStreamSynchronize(s);
    for (int c = 0; c < B.count; ++c)
      if (full[c]) (void)hipFree(full[c]);
    if (rc3 != TW_OK) return rc3;
    B.mode = mus[1] < mus[0] ? 1 : 0;
    tune_cache_store(batch_key(B) + "|mode", B.mode, mus);
  }
  B.tuned = 1;
  if (B.exec) {  // a captured graph used the previous choice
    (void)hipDeviceSynchronize();
    (void)hipGraphExecDestroy(B.exec);
    (void)hipGraphDestroy(B.graph);
    B.exec = nullptr;
    B.graph = nullptr;
    B.key_nsteps = -1;
  }
  if (variant_out) *variant_out = B.variant;
  if (mode_out) *mode_out = B.mode;
  return TW_OK;
}

int tw_batch_step(tw_batch batch, void* const* psi, void* const* psi_classical, int64_t nsteps, double dt,
                  void* stream) {
  if (!batch) return fail(TW_EINVAL, "NULL batch");
  Batch& B = *reinterpret_cast<Batch*>(batch);
  if (!psi) return fail(TW_EINVAL, "psi array is NULL");
  for (int c = 0; c < B.count; ++c) {
    if (int rc = check_ptr(*B.plans[c], psi[c], "psi[c]", false)) return rc;
    if (psi_classical)
      if (int rc = check_ptr(*B.plans[c], psi_classical[c], "psi_classical[c]", true)) return rc;
  }
  if (nsteps < 0) return fail(TW_EINVAL, "nsteps must be >= 0");
  if (!std::isfinite(dt)) return fail(TW_EINVAL, "dt must be finite");
  if (nsteps == 0) return TW_OK;
  bool same = B.exec && B.key_nsteps == nsteps && B.key_dt == dt;
  for (int c = 0; c < B.count && same; ++c)
    same = B.key_psi[c] == psi[c] && B.key_cl[c] == (psi_classical ? psi_classical[c] : nullptr);
  if (!same) {
    if (B.exec) TW_HIP(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));  // old graph may be in flight
    if (B.exec) (void)hipGraphExecDestroy(B.exec);
    if (B.graph) (void)hipGraphDestroy(B.graph);
    B.exec = nullptr;
    B.graph = nullptr;
    B.key_nsteps = -1;
    TW_HIP(hipStreamBeginCapture(B.cap, hipStreamCaptureModeRelaxed));
    const int rc = enqueue_batch_mode(B, psi, psi_classical, nsteps, dt, B.cap);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(B.cap, &g);
    if (rc != TW_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (ec != hipSuccess) return fail(TW_EHIP, "graph capture failed: %s", hipGetErrorString(ec));
    B.graph = g;
    TW_HIP(hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0));
    B.key_nsteps = nsteps;
    B.key_dt = dt;
    for (int c = 0; c < B.count; ++c) {
      B.key_psi[c] = psi[c];
      B.key_cl[c] = psi_classical ? psi_classical[c] : nullptr;
    }
  }
  TW_HIP(hipGraphLaunch(B.exec, reinterpret_cast<hipStream_t>(stream)));
  return TW_OK;
}

}  // extern "C"
