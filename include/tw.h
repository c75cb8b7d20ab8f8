/*
 * tw.h - C ABI of the MI355X truncated-Wigner Schrodinger-Poisson ensemble library.
 *
 * The method (arXiv 2310.07119, Sec. "Truncated Wigner approximation"): an
 * ensemble of independent classical fields psi'_i is drawn from the Wigner
 * function of a coherent state (Sec. "Initial conditions generation",
 * Eq. (sample)), each field is advanced by the pseudo-spectral symplectic
 * leapfrog of Sec. "Integrating the equations of motion" for the normalised
 * Schrodinger-Poisson system of Eq. (mft_normed)
 *     i d_t psi' = (-hbar/2 lap + V/hbar) psi',   lap V = 4 pi G M_tot |psi'|^2,
 * and quantum expectation values are ensemble averages of Weyl symbols
 * (Sec. "Evaluating operators", Eq. (Q)).
 *
 * Conventions shared by every call
 *  - All functions are plain C, thread-compatible (one plan per thread or
 *    external locking), return a tw_status and never print. On failure
 *    tw_last_error() returns a message for the calling thread.
 *  - Array arguments are DEVICE pointers owned by the caller; the library never
 *    frees them. They must be contiguous and aligned to the complex element
 *    (16 bytes for complex128, 8 bytes for complex64), else TW_ELAYOUT.
 *  - Field layout: row-major [realization][z][y][x], x fastest, complex values
 *    interleaved (re, im). A TW_FP64 plan stores complex128; a TW_FP32_SPLIT
 *    plan stores complex64 fields (FP32 transforms, FP64 phase arguments,
 *    FP64 Poisson zero mode and FP64 diagnostics).
 *  - Fields are the normalised psi' of Eq. (mft_normed): sum_g |psi'_g|^2 dV = 1,
 *    mass density rho = m_tot |psi'|^2.
 *  - `stream` is a hipStream_t passed as void* (NULL = legacy default stream);
 *    every device call is enqueued on it and the call returns without waiting.
 *    Device faults surface as TW_EHIP on a later call.
 *  - A plan's workspace (spectral scratch, second field buffer, step tables,
 *    adaptive-step state, reduction partials) is shared by all its calls:
 *    calls on one plan must be ordered, e.g. issued on one stream. Different
 *    plans are independent.
 */
#ifndef TW_H
#define TW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TW_OK = 0,
  TW_EINVAL = -1,        /* bad argument value (NULL plan, n<1, dt not finite, ...) */
  TW_EUNSUPPORTED = -2,  /* valid but not implemented (grid size, dimension) */
  TW_ELAYOUT = -3,       /* misaligned pointer */
  TW_EHIP = -4,          /* HIP runtime error (launch failure, earlier device fault) */
  TW_ENOMEM = -5         /* device workspace allocation failed */
} tw_status;

typedef enum { TW_FP64 = 0, TW_FP32_SPLIT = 1 } tw_precision;

/* Problem statement: grid x_g = g dx, g in {0..n-1}^D (Sec. "Initial conditions
 * generation"); physical parameters of Eq. (mft_normed); n_tot is the
 * sampling particle number n^s_tot that sets the noise amplitude only
 * (Sec. "Estimating the breaktime"). */
typedef struct {
  int32_t dim;        /* D in {1,2,3} */
  int32_t n[3];       /* points per axis, x first; unused axes must be 1.
                         Supported: 16, 24, 32, 48, 64, 96, 128, 192, 256,
                         384, 512, 1024 (D=1 also 8) */
  double box[3];      /* box length per axis, > 0 (unused axes ignored) */
  double hbar_m;      /* hbar/m > 0 */
  double G;           /* Newton constant >= 0 (0 = free Schrodinger equation) */
  double m_tot;       /* total mass M_tot > 0 */
  double n_tot;       /* sampling particle number > 0 (may be +inf: no noise) */
  int64_t n_real;     /* number of realizations N_s >= 1 */
  int32_t precision;  /* tw_precision */
  int32_t reserved;   /* must be 0 */
} tw_problem;

typedef struct tw_plan_s* tw_plan;

/* Create a plan: validates the problem, builds twiddle and wavenumber tables
 * and allocates the device workspace (about half a field per realization for
 * D >= 2; for D = 2 also a second buffer of n_real + 1 fields, used by the
 * alternating-storage step schedule, which is skipped if that allocation
 * fails or TW_TRANSPOSE=0 is set in the environment). Synchronous. Uses the
 * current HIP device. */
int tw_plan_create(const tw_problem* problem, tw_plan* out);

/* Release the plan and its workspace. Waits for the device. NULL is a no-op. */
int tw_plan_destroy(tw_plan plan);

/* Wigner sampling (Eq. (sample)). For every realization r in [0, n_real) and
 * cell g: psi[r][g] = psi_cl[g] + (z1 + i z2) * 0.5 / sqrt(n_tot dV), with
 * (z1, z2) standard normal from Philox4x64-10 at counter (g, real_offset + r,
 * 0, 0), key (seed, 0x5457), mapped by the Box-Muller transform written as a
 * fixed sequence of correctly rounded double operations (series logarithm and
 * sine/cosine after exact range reduction, no fused multiply-add).
 *   psi_cl : device, [N] complex128 (always FP64), the coherent field.
 *   psi    : device, [n_real][N] complex128 (TW_FP64) or complex64
 *            (TW_FP32_SPLIT: the FP64 sample rounded to nearest).
 * Results are bit-reproducible from (seed, real_offset + r, g). */
int tw_sample(tw_plan plan, const void* psi_cl, uint64_t seed, int64_t real_offset,
              void* psi, void* stream);

/* Advance every field by nsteps leapfrog steps of size dt (Sec. "Integrating
 * the equations of motion"): half drift exp(-i hbar |k|^2 dt/4) in Fourier
 * space, potential V_k = -4 pi G rho_k / |k|^2 (zero mode removed) from the
 * drifted field's own density, kick exp(-i dt V / hbar), half drift.
 * Adjacent half drifts inside one call are merged; the state on return is
 * exactly that after nsteps complete steps. In D = 2 the fields alternate
 * between the caller's buffer and the plan's second buffer, transposed, while
 * the call runs (every pass then reads whole rows); on return they are back in
 * the caller's buffer in the usual layout.
 *   psi           : device, [n_real][N] fields in the plan's precision, in place.
 *   psi_classical : device, [N] one extra field in the plan's precision that is
 *                   evolved alongside (the noise-free classical run), or NULL.
 * nsteps >= 0; dt finite (negative dt runs backwards). TW_CHUNK_PAIRS=k in the
 * environment (read by tw_plan_create) advances k pairs of fields through all
 * steps before the next k (a cache-residency option; every pair per launch is
 * the default and was faster at every k measured). */
int tw_step(tw_plan plan, void* psi, void* psi_classical, int64_t nsteps, double dt,
            void* stream);

/* tw_step with step sizes chosen on the device (the time-step rule of Sec.
 * "Integrating the equations of motion" and its footnote on the kinetic
 * bound). Every step n has one size dt_n for all fields:
 *   dt = min(dt_max, courant * dt_K, courant * 2 pi hbar / max|V|),
 *   dt_K = min over axes of 4 pi / (hbar k_max dk), k_max = pi/dx, dk = 2 pi/L,
 * with max|V| over every cell of every field (realizations and the classical
 * field). Steps 0 and 1 use the potential of the fields on entry; step n + 2
 * uses the potential evaluated inside step n (the kick pass records its
 * maximum, and the merged half drifts between steps n and n + 1 need dt_{n+1}
 * before step n's potential exists). No host synchronisation: a small kernel
 * after each kick pass turns the recorded maximum into the next step size and
 * drift tables.
 *   dt_max  : > 0, upper bound on every step (also the step when nothing else binds).
 *   courant : c_f in (0, 1].
 *   dt_out  : device, [nsteps] doubles receiving dt_n (the elapsed time is their
 *             sum), or NULL; 8-byte aligned (else TW_ELAYOUT).
 * D = 1 runs one launch per step (each field inside one workgroup) instead
 * of tw_step's single resident launch, so that max|V| can cross the ensemble
 * between steps. D >= 2 needs every axis >= 16 points (TW_EUNSUPPORTED
 * otherwise). Other arguments as tw_step. */
int tw_step_adaptive(tw_plan plan, void* psi, void* psi_classical, int64_t nsteps, double dt_max,
                     double courant, double* dt_out, void* stream);

/* tw_step with test particles (Sec. "Modeling decoherence"): every field
 * carries ntracer particles that move in that field's own potential,
 * dr/dt = v, dv/dt = -grad V(r), advanced in the same splitting as the field:
 * r += v dt/2; v -= dt grad V(r) with the potential of the field's kick;
 * r += v dt/2. grad V is the fourth-order central difference on the grid
 * interpolated linearly (cloud-in-cell) to the particle. Positions are kept
 * unwrapped (the periodic box is used only to locate the cell).
 *   tracers : device, [nfield][ntracer][2 D] doubles, nfield = n_real (+1 with
 *             psi_classical, whose particles come last): r_0..r_{D-1},
 *             v_0..v_{D-1}; updated in place. 8-byte aligned.
 * D >= 2 only. Other arguments as tw_step. */
int tw_step_tracers(tw_plan plan, void* psi, void* psi_classical, int64_t nsteps, double dt,
                    double* tracers, int64_t ntracer, void* stream);

/* Spread of the test particles over the realizations (the first n_real
 * entries of `tracers`): out[i][k] = plug-in variance of coordinate k of
 * particle i (k < D positions, then D velocities); the per-axis uncertainty
 * product is sqrt(out[i][d] * out[i][D + d]).
 *   tracers : device, [>= n_real][ntracer][2 D] doubles.
 *   out     : device, [ntracer][2 D] doubles.
 * Both 8-byte aligned (else TW_ELAYOUT); NULL or ntracer < 1 gives TW_EINVAL. */
int tw_tracer_spread(tw_plan plan, const double* tracers, int64_t ntracer, double* out, void* stream);

/* Outputs of tw_moments. Every pointer is a caller-owned device array and may
 * be NULL to skip that output. */
typedef struct {
  void* mean_psi;     /* [N] complex128: <psi'>_g */
  double* mean_abs2;  /* [N] <|psi'|^2>_g, Weyl (symmetric) ordering */
  double* mean_rho;   /* [N] <rho>_g = m_tot <|psi'|^2>_g */
  double* var_rho;    /* [N] <(rho - <rho>)^2>_g, plug-in 1/N_s estimator */
  double* mode_occ;   /* [N] <|a_j|^2> per Fourier mode j (same index layout as the
                         grid, j in FFT order), a_j = F[alpha]_j / sqrt(N) with
                         alpha_g = sqrt(n_tot dV) psi'_g (unitary DFT, occupation
                         units; Sec. "Quantum description"): at sampling time
                         <|a_j|^2> = |a_cl,j|^2 + 1/2. Averages realizations only */
  double* var_amp;    /* [N] <(A - <A>)^2>_g of the amplitude A = |psi'| */
  double* var_phase;  /* [N] <dphi^2>_g, dphi = arg(psi' conj<psi'>) in (-pi, pi] */
  double* decoherence;/* [2]: Var A~ = sum_g dV <psi^dag psi> <dA^2>/<A>, Var phi~ =
                         sum_g dV <psi^dag psi> <dphi^2>/(pi/sqrt 3) (Sec. "Large
                         quantum corrections", Eqs. (varA), (varPhi)), with the
                         normal-ordered <psi^dag psi> = <|psi'|^2> - 1/(2 n_tot dV) */
  double* norm;       /* [n_real] sum_g |psi'|^2 dV per realization */
  double* energy;     /* [n_real] m_tot [ (hbar^2/2) int|grad psi'|^2 + (1/2) int V|psi'|^2 ] */
  double* scalars;    /* [8]: Q_raw, Q_sym, dev_rho_L1, dev_psi_L2, energy_mean,
                         norm_mean, nonfinite_count, energy_classical */
} tw_moments_out;

/* Ensemble moments (Sec. "Evaluating operators"; Eq. (Q)):
 *   Q_raw = sum_g dV (<|psi'|^2> - |<psi'>|^2);  Q_sym = Q_raw - N/(2 n_tot);
 *   dev_rho_L1 = sum_g dV |<rho> - rho_cl| / m_tot;  dev_psi_L2 = sum_g dV |<psi'> - psi'_cl|^2
 * (the two deviations need psi_classical, else they are 0); nonfinite_count
 * counts realizations holding a NaN or Inf. All sums are FP64. energy and
 * scalars[4], scalars[7] are computed only when `energy` is non-NULL (they need
 * one spectral transform and one Poisson solve per realization); mode_occ needs
 * one full D-dim forward transform per realization. Both use the plan's
 * spectral scratch and return TW_EUNSUPPORTED for plans with an axis shorter
 * than 16 points.
 *   psi           : device, [n_real][N] in the plan's precision.
 *   psi_classical : device, [N] in the plan's precision, or NULL. */
int tw_moments(tw_plan plan, const void* psi, const void* psi_classical,
               const tw_moments_out* out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the moment
 * reductions of tw_moments without a plan. Computes mean_psi, mean_abs2,
 * mean_rho, var_rho, norm and scalars exactly as tw_moments does (same
 * kernels; scalars[4] and scalars[7] are 0, as tw_moments gives them without
 * energies). Allocates nothing: its partial sums live in a fixed 32 MiB device
 * array of the library, one per GPU, held until the process ends, so
 *   n_real * ceil(N/64) + 3 * ceil(N/64) + n_real + 3 <= 4194304
 * (e.g. 512^2 with 256 realizations, 128^3 with 64) or TW_EUNSUPPORTED before
 * any launch. energy, mode_occ, var_amp, var_phase and decoherence must be
 * NULL (TW_EUNSUPPORTED: they need a plan's spectral scratch). Every call on a
 * GPU uses that GPU's one array: calls that overlap on one GPU (two streams,
 * two threads) race and must be ordered by the caller; the array keeps the
 * last call's partial sums, none of which a call reads before writing it.
 *   p             : the problem (grid, box, m_tot, n_tot, n_real, precision),
 *                   validated as by tw_plan_create except the FFT lengths.
 *   psi, psi_classical, out, stream : as tw_moments. */
int tw_moments_static(const tw_problem* p, const void* psi, const void* psi_classical,
                      const tw_moments_out* out, void* stream);

/* Autotune the kernel organisation of the passes along strided axes (y, z).
 * Returns at once if the plan's choice is already settled (tuning cache entry,
 * TW_COLS_VARIANT override, or an earlier call). Optional: TW_STREAMS=2 in the
 * environment makes tw_step run two halves of the pairs on two streams (+1-2%
 * on the 2D workload; off by default because overlapping kernels make
 * per-kernel timings meaningless). Otherwise it times both
 * available organisations on the strided passes a step runs: all of them on a
 * scratch ensemble of this plan's shape (up to 32 pairs of realizations,
 * allocated and freed here), or, under the D = 2 alternating-storage schedule,
 * only the Poisson pass on the plan's own spectral scratch at full size (its
 * contents are overwritten; no field is touched). It keeps the faster
 * for this plan and records it in the tuning cache ($TW_TUNE_CACHE, else
 * $XDG_CACHE_HOME or $HOME/.cache, file twa_mi355x_tune.json), which later
 * tw_plan_create calls with the same device, grid, precision and ensemble
 * size read. Synchronous. *variant_out (may be NULL) receives the choice
 * (0 = pencils interleaved across wavefronts, 1 = LDS tiles). Results do not
 * depend on the choice beyond rounding. The environment variable
 * TW_COLS_VARIANT=0|1, read by tw_plan_create, forces a choice instead. */
int tw_plan_autotune(tw_plan plan, int32_t* variant_out, void* stream);

/* ------------------------------------------------------------------ batches
 * Ensembles of different grid sizes advanced together (the same method per
 * size class). Every pass of a step is ONE launch covering all classes, and a
 * whole tw_batch_step call is captured once into a HIP graph and replayed with
 * a single graph launch while (nsteps, dt, field pointers) stay the same. */
typedef struct tw_batch_s* tw_batch;

/* problems[0..count-1], 1 <= count <= 4: one size class each, all with the same
 * dim (2 or 3) and precision; grid lengths 16, 24, 32, 48, 64, 96 or 128.
 * Creates one plan per class (owned by the batch). Synchronous. */
int tw_batch_create(const tw_problem* problems, int32_t count, tw_batch* out);

/* The plan of class `index`, owned by the batch (valid until tw_batch_destroy);
 * use it with tw_sample and tw_moments. Do not destroy it. */
int tw_batch_plan(tw_batch batch, int32_t index, tw_plan* out);

/* Tune the batch on scratch buffers (allocated and freed here): the
 * strided-pass organisation of the grouped launches (timed on up to 8 pairs
 * per class), each class plan (tw_plan_autotune), and the batching mode, timed
 * on full-size scratch ensembles: 0 = one grouped launch per pass for all
 * classes, 1 = one kernel chain per class, the chains running as parallel
 * branches of the graph. Choices are cached under a key listing every class
 * (TW_BATCH_MODE=0|1 and TW_COLS_VARIANT=0|1 force them instead). Synchronous.
 * *variant_out and *mode_out (either may be NULL) receive the choices. */
int tw_batch_autotune(tw_batch batch, int32_t* variant_out, int32_t* mode_out, void* stream);

/* tw_step for every class: psi[c] (and psi_classical[c] if the array is
 * non-NULL; entries may be NULL) are class c's fields. Captures the launch
 * sequence into a graph on first use with these arguments (the capture runs on
 * streams owned by the batch), then launches the graph on `stream`. Results
 * equal those of tw_step on the class plans with the same strided-pass
 * organisation. */
int tw_batch_step(tw_batch batch, void* const* psi, void* const* psi_classical, int64_t nsteps, double dt,
                  void* stream);

/* Waits for the device, releases graphs, plans and workspace. NULL is a no-op. */
int tw_batch_destroy(tw_batch batch);

/* Kernel timing for measurement tools (not needed for the method itself).
 * When enabled, every kernel launched by tw_sample / tw_step / tw_moments on
 * this plan is bracketed by two HIP events recorded on the launch stream.
 * Kernel kinds are numbered 0 .. TW_NUM_KERNEL_KINDS-1 (tw_kernel_kind_name). */
#define TW_NUM_KERNEL_KINDS 16
int tw_plan_set_profiling(tw_plan plan, int32_t enable);

/* Waits for the recorded events, writes for each kind k < n_kinds the number
 * of launches[k] and their summed device time total_ms[k] since the last call,
 * then clears the record. Host arrays of n_kinds elements owned by the caller. */
int tw_plan_get_profile(tw_plan plan, int32_t n_kinds, int64_t* launches, double* total_ms);

/* Static name of kernel kind k ("" outside the range). */
const char* tw_kernel_kind_name(int32_t kind);

/* ------------------------------------------------------- learned surrogate
 * A Fourier neural operator (Li et al., 2020; not part of the paper) that maps
 * fields derived from the classical run to the ensemble moments the method
 * produces. Its dense contractions (pointwise layers, truncated DFTs, weight
 * gradients) run on BF16 matrix cores with FP32 accumulation; mode mixing,
 * GELU, biases and reductions run in FP32/FP64.
 *
 * Layout: inputs x [B][H][W][c_in], outputs y [B][H][W][c_out], FP32, channel
 * last. Parameters are one flat FP32 buffer, in order: lift_w [c_in][width],
 * lift_b [width]; for each layer l: R_re, R_im [2 modes_y][modes_x][width][width]
 * (modes ky in {0..modes_y-1, H-modes_y..H-1}, kx in {0..modes_x-1}),
 * W [width][width], b [width]; q1_w [width][proj], q1_b [proj];
 * q2_w [proj][c_out], q2_b [c_out]. Gradients use the same layout. */
typedef struct {
  int32_t H, W;         /* grid */
  int32_t c_in;         /* input channels */
  int32_t width;        /* hidden channels */
  int32_t modes_x;      /* kept kx = 0..modes_x-1 (modes_x <= W/2) */
  int32_t modes_y;      /* kept ky: modes_y lowest non-negative and negative (2 modes_y <= H) */
  int32_t layers;       /* Fourier layers, 1..8 */
  int32_t proj;         /* hidden width of the projection */
  int32_t c_out;        /* output channels */
} tw_fno_config;
typedef struct tw_fno_s* tw_fno;

/* Number of FP32 parameters of the configuration. */
int64_t tw_fno_param_count(const tw_fno_config* config);

/* Allocate the tables and the activation workspace for up to max_batch fields
 * (max_batch * H <= 65535). Synchronous. */
int tw_fno_create(const tw_fno_config* config, int32_t max_batch, tw_fno* out);
int tw_fno_destroy(tw_fno fno);

/* Deterministic initialisation from `seed` (counter hash): weights uniform in
 * +-1/sqrt(fan_in), spectral weights uniform in (0, 1/width^2), biases 0. */
int tw_fno_init_params(tw_fno fno, uint64_t seed, float* params, void* stream);

/* y = network(x) for `batch` fields; keeps the activations in the workspace
 * for a following tw_fno_backward with the same params and x. */
int tw_fno_forward(tw_fno fno, const float* params, const float* x, int32_t batch, float* y, void* stream);

/* grads (overwritten) = d(sum dy * y)/d(params) for the last tw_fno_forward. */
int tw_fno_backward(tw_fno fno, const float* params, const float* x, int32_t batch, const float* dy, float* grads,
                    void* stream);

/* loss[0] = mean((y - t)^2) over n values (FP64 sums in a fixed order), dy =
 * 2 (y - t) / n (dy and loss may be NULL). Device pointers. The partial sums
 * live in a small fixed device array of the library: calls that overlap on one
 * GPU (two streams, two threads) race and must be ordered by the caller. */
int tw_fno_mse(const float* y, const float* t, int64_t n, float* dy, float* loss, void* stream);

/* One bias-corrected Adam step (Kingma and Ba) over n parameters; step >= 1. */
int tw_fno_adam(float* params, const float* grads, float* m, float* v, int64_t n, float lr, float b1, float b2,
                float eps, int64_t step, void* stream);

/* Message of the last tw_fno_* failure on the calling thread. */
const char* tw_fno_last_error(void);

/* Message describing the last failure on the calling thread ("" if none). */
const char* tw_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TW_H */
