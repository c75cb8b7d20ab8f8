// Host-side plan structure and the launchers each kernel translation unit exports.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "tw.h"

namespace tw {

// Arguments of one pencil pass over the ensemble (see kernels_step.hip).
constexpr int kVmaxBuckets = 64;     // atomic-max slots per recorded maximum
constexpr int kAdaptScalars = 16;    // adaptive-step state before the max|V| buckets
constexpr int kFieldMeanParts = 64;  // partial sums per field of the mean-density reduction

struct PassArgs {
  void* psi;               // [n_real][N] fields (plan precision)
  void* psi_cl;            // extra classical field or nullptr
  void* z;                 // [npairs][N] spectral density / potential scratch
  int64_t n_real;
  int64_t nfield;          // n_real + (psi_cl != nullptr)
  int64_t ncell;           // N = n0 n1 n2
  int64_t stride;          // element stride of the pass axis
  int32_t axis;            // 0, 1, 2
  int32_t n[3];
  const void* twd;         // W_n^e table of the pass length, plan precision
  const void* phase;       // cx<double>[n_axis] drift factor exp(-i hbar k^2 tau/2)/n_axis
  const double* k2[3];     // per-axis k^2 tables (FFT order)
  double green;            // -4 pi G / N   (Poisson factor; 1/N of the inverse folded in)
  double kick;             // dt / hbar
  double m_tot;
  const double* rho_mean;  // [nfield] density mean subtracted before the transform, or nullptr
  double* partial;         // reduction output for diagnostic passes
  int32_t pot_green;       // PASS_POT_SUM: apply G(k) along the axis before the inverse (D = 1)
  int32_t variant;         // strided passes: 0 = pencil-interleaved, 1 = LDS tiles (see kernels_cols.hip)
  int64_t pair0;           // first pair of this launch (blockIdx.y + pair0)
  int32_t t_psi;           // row passes: store the fields transposed (element j of pencil p at j * npencils + p)
  void* psi_t;             // destination of transposed field stores (never the buffer being read)
  void* psi_cl_t;          // ... its classical-field slot
  const double* kick_dev;  // PASS_KICK_DRIFT: kick factor dt/hbar read from device memory (overrides kick)
  double* vmax;            // PASS_KICK_DRIFT / PASS_POT_SUM: running max |V|, kVmaxBuckets slots (atomic max on the bits)
  int32_t store_v;         // PASS_KICK_DRIFT: write the real-space potentials V_A + i V_B back into the pair scratch
  const void* phase2;      // plane passes (D = 3): drift factors along y (phase: along x)
  int32_t rev;             // pair slots taken in reverse launch order (the last slot first)
};

// Passes over whole xy-planes of a D = 3 grid held in LDS (kernels_slab.hip).
enum SlabMode : int {
  SLAB_DRIFT = 0,       // psi <- drift along x, then along y
  SLAB_DRIFT_RHO = 1,   // drift x, y; z <- FFT_xy(rho_A - mean_A + i (rho_B - mean_B))
  SLAB_POISSON = 2,     // z <- IFFT_xy(G(k) FFT_xy z)   (z already transformed along z)
  SLAB_KICK_DRIFT = 3,  // V_A + i V_B <- IFFT_xy z; psi <- kick; drift x, y
  SLAB_NMODES = 4
};

enum PassMode : int {
  PASS_DRIFT = 0,       // psi <- IFFT_a(phase * FFT_a psi)
  PASS_DRIFT_RHO = 1,   // drift, then z <- FFT_a(rho_A - mean_A + i (rho_B - mean_B))
  PASS_ZFWD = 2,        // z <- FFT_a z
  PASS_ZPOISSON = 3,    // z <- IFFT_a(G(k) FFT_a z)
  PASS_ZINV = 4,        // z <- IFFT_a z
  PASS_KICK_DRIFT = 5,  // V_A + i V_B <- IFFT_a z; psi <- kick; drift
  PASS_RHO = 6,         // z <- FFT_a(rho_A - mean_A + i (rho_B - mean_B))   (diagnostics)
  PASS_KIN_SUM = 7,     // partial[f][group] <- sum k_a^2 |FFT_a psi|^2     (diagnostics)
  PASS_POT_SUM = 8,     // V <- IFFT_a z; partial[f][group] <- sum V |psi|^2 (diagnostics)
  PASS_NMODES = 9
};

struct Plan {
  tw_problem p;
  int dim;
  int n[3];
  int64_t ncell;
  int64_t nfield;   // n_real + 1 (slot for the classical field)
  int64_t npairs;   // ceil(nfield / 2)
  double dV;
  double volume;
  bool fp32;
  size_t elem;      // bytes per complex element
  int device;
  // device tables
  void* twd[3];          // per axis, plan precision
  double* k2[3];         // per axis
  void* phase;           // cx<double>[3][2][nmax]: axis, (half, full)
  int nmax;
  // workspace
  void* z;               // [npairs][N] complex scratch (D >= 2)
  void* psi_alt;         // [nfield][N] second field buffer (2D alternating storage)
  double* rho_mean;      // [nfield]
  double* partial;       // reductions
  size_t partial_len;    // doubles
  double* scratch_small; // [64] misc device scalars
  double* adapt;         // adaptive-step state: dt ring [3], kick factors [2], then 3 x kVmaxBuckets max|V| slots
  void* adapt_tab;       // cx<double>[3][3][nmax]: drift tables of the adaptive schedule
  int64_t chunk_pairs;   // pairs advanced through all steps together (cache residency)
  int transpose2d;       // 2D steps use the alternating-storage row schedule
  int split_streams;     // tw_step runs two halves of the pairs on two streams
  hipStream_t side;      // the second stream (created on first use, default priority)
  hipEvent_t ev_fork, ev_join;
  int32_t slab3d;        // D = 3 steps use the xy-plane passes (3 HBM passes per step instead of 6)
  int32_t slab_ok;       // the plane kernels exist for this grid and fit the device's LDS
  int32_t slab_tuned;    // slab3d came from a measurement, the tuning cache or TW_SLAB
  int32_t cols_variant;  // kernel organisation of strided passes (autotuned, see tune.cpp)
  int32_t tuned;         // cols_variant came from a measurement or the tuning cache
  // Passes enqueued on this plan so far. Consecutive passes walk the pairs in
  // opposite orders, so that a pass starts on the pairs the previous one
  // touched last, which are still in the 256 MB Infinity Cache (bit-identical
  // results; measured on MI355X at 512^2 with 256 realizations: FP64 step
  // -3.8%, FP32 -2.5%).
  uint32_t pass_seq;
  // kernel timing (tw_plan_set_profiling)
  bool profiling;
  void* prof;            // opaque event record (api.hip)
};

enum KernelKind : int {
  KIND_STEP1D = PASS_NMODES,  // 9
  KIND_SAMPLE = 10,
  KIND_MOMENTS = 11,
  KIND_TABLES = 12,
  KIND_MEAN = 13,
  KIND_ENERGY = 14,
  KIND_MODES = 15,  // mode occupations and the amplitude/phase spread
  KIND_SLAB = 16,   // KIND_SLAB + SlabMode: the xy-plane passes
  KIND_COUNT = KIND_SLAB + SLAB_NMODES
};

// Opt kernel `kern` into `bytes` of dynamic LDS (needed above 64 KiB) before
// its first launch with that size; remembered per kernel, so every
// instantiation and every pass mode is set up once (thread-safe).
hipError_t ensure_dynamic_lds(const void* kern, size_t bytes);

// Launchers (return hipError_t of the launch).
hipError_t launch_pass(const Plan& P, int mode, const PassArgs& a, hipStream_t s, int npairs_or_fields);
hipError_t launch_pass_cols(const Plan& P, int mode, const PassArgs& a, hipStream_t s, int npairs);
// xy-plane pass over n[2] planes of pairs [pair0, pair0 + npairs); needs n[0] == n[1]
hipError_t launch_slab(const Plan& P, int mode, const PassArgs& a, hipStream_t s, int npairs);
// LDS bytes of the plane kernels for an n x n plane, 0 if none is compiled for n
size_t slab_lds_bytes(int n, bool fp32);
int cols_pencils_per_group(int n, bool fp32);
hipError_t launch_step1d(const Plan& P, void* psi, void* psi_cl, int64_t nfield, int64_t nsteps,
                         const void* phase_half, const void* phase_full, double kick, hipStream_t s);
// D = 1 with device-chosen steps: one step (or, with step < 0, the initial
// potential only) of every field per launch; records max |V| into vmax.
hipError_t launch_step1d_adapt(const Plan& P, void* psi, void* psi_cl, int64_t nfield, int64_t step,
                               const void* ph_open, const void* ph_step, const double* kick_dev, double* vmax,
                               hipStream_t s);
hipError_t launch_phase_table(const Plan& P, int axis, double tau, void* out, hipStream_t s);
// Adaptive time step: after the kick pass of step `step` (or, with step = -1,
// after the initial potential), choose the size of step + 2 (steps 0 and 1)
// from the recorded max |V|, log dt_out[step], and build the drift tables of
// step + 1 (merged half drifts, or the closing half drift if last_next).
hipError_t launch_adapt(const Plan& P, int64_t step, int last_next, double dt_max, double courant, double dtk,
                        double* dt_out, hipStream_t s);
hipError_t launch_adapt_clear(const Plan& P, hipStream_t s);
// Test particles: one leapfrog step of every field's particles in the
// potential the kick pass left in the pair scratch (stored with physical axis
// perm[0] fastest, then perm[1], perm[2]).
hipError_t launch_tracers(const Plan& P, double* tr, int64_t nfield, int64_t ntracer, const int perm[3], double dt,
                          hipStream_t s);
hipError_t launch_tracer_spread(const Plan& P, const double* tr, int64_t ntracer, double* out, hipStream_t s);
hipError_t launch_field_mean(const Plan& P, const void* psi, const void* psi_cl, int64_t nfield,
                             double* out_mean, hipStream_t s);
hipError_t launch_sample(const Plan& P, const void* psi_cl, uint64_t seed, int64_t real_offset,
                         void* psi, hipStream_t s);
hipError_t launch_energy_finalize(const Plan& P, const double* partial, int64_t gstride, int64_t nfield,
                                  const int ng[4], double* out, hipStream_t s);
hipError_t launch_gather_round(const Plan& P, const void* psi, int64_t nslots, int k, hipStream_t s);
hipError_t launch_decoherence(const Plan& P, const void* psi, double* var_amp, double* var_phase, double* integrals,
                              double* scratch, hipStream_t s);
hipError_t launch_mode_occ(const Plan& P, int64_t nslots, int accumulate, double* occ, hipStream_t s);
hipError_t launch_moments(const Plan& P, const void* psi, const void* psi_cl, const tw_moments_out* out,
                          const double* energy_dev, hipStream_t s);
// The moment reductions of launch_moments on an explicit geometry and partial-sum
// buffer of moments_partial_doubles(n_real, ncell) doubles.
struct MomGeom {
  int64_t n_real, ncell;
  double m_tot, dV, n_tot;
  bool fp32;
};
int64_t moments_partial_doubles(int64_t n_real, int64_t ncell);
hipError_t launch_moments_geom(const MomGeom& G, double* partial, const void* psi, const void* psi_cl,
                               const tw_moments_out* out, const double* energy_dev, hipStream_t s);
// Error reporting shared by the entry points: stores the message returned by
// tw_last_error and returns `code`.
int report_error(int code, const char* fmt, ...);

// Grouped launch over the size classes of a batch (kernels_batch.hip).
constexpr int kMaxClasses = 4;
struct GroupArgs {
  PassArgs a[kMaxClasses];
  uint32_t groups[kMaxClasses];     // x-blocks per pair of class c
  uint32_t start[kMaxClasses + 1];  // first block of class c (filled by the launcher)
  int32_t nclass;
};
hipError_t launch_grouped(bool fp32, int mode, GroupArgs& g, int variant, hipStream_t s);
bool batch_length_supported(int n);

// Autotuner cache (tune.hip).
std::string tune_key(const Plan& P);
int tune_cache_lookup(const std::string& key);
void tune_cache_store(const std::string& key, int variant, const double us[2]);

// Supported transform lengths and the pencils a pass workgroup holds.
bool pass_length_supported(int n);
int pass_pencils_per_group(int n, bool fp32, bool rows, int variant);
bool step1d_length_supported(int n);

}  // namespace tw
