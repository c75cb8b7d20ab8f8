// Ensemble moments (Sec. "Evaluating operators": <Omega> ~ (1/N_s) sum_i Omega_W[psi_i];
// Eq. (Q) for the quantumness). One pass over the ensemble, one thread per cell,
// realizations read in turn so every load is coalesced along x; all sums FP64.
// Second moments are accumulated about the first realization's value (shifted
// sums), which keeps the variance free of cancellation when the noise is small.
#include "common.hpp"
#include "internal.hpp"

namespace tw {

struct MomArgs {
  const void* psi;
  const void* psi_cl;
  int64_t n_real;
  int64_t ncell;
  double m_tot;
  double dV;
  cx<double>* mean_psi;
  double* mean_abs2;
  double* mean_rho;
  double* var_rho;
  double* wave_norm;  // [n_real][nwaves]
  double* wave_q;     // [3][nwaves]: Q, dev_rho, dev_psi
  int64_t nwaves;
};

__device__ __forceinline__ double wave_sum(double x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

template <class T>
__global__ void __launch_bounds__(256) moments_cell_kernel(MomArgs a) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = g < a.ncell;
  const int64_t wave = g >> 6;
  const int lane = threadIdx.x & 63;
  const cx<T>* psi = reinterpret_cast<const cx<T>*>(a.psi);

  cx<double> c0 = {0.0, 0.0};
  double k0 = 0.0;
  double s_a2 = 0.0, sd_a2 = 0.0, sdd_a2 = 0.0, sdd = 0.0;
  cx<double> sd = {0.0, 0.0};
  for (int64_t r = 0; r < a.n_real; ++r) {
    cx<double> v = {0.0, 0.0};
    if (active) {
      const cx<T> w = psi[r * a.ncell + g];
      v = {(double)w.re, (double)w.im};
    }
    const double a2 = v.re * v.re + v.im * v.im;
    if (r == 0) {
      c0 = v;
      k0 = a2;
    }
    s_a2 += a2;
    const double da = a2 - k0;
    sd_a2 += da;
    sdd_a2 += da * da;
    const cx<double> d = v - c0;
    sd = sd + d;
    sdd += d.re * d.re + d.im * d.im;
    const double wn = wave_sum(a2);
    if (lane == 0 && wave < a.nwaves) a.wave_norm[r * a.nwaves + wave] = wn;
  }
  const double inv = 1.0 / (double)a.n_real;
  const cx<double> m1 = {c0.re + sd.re * inv, c0.im + sd.im * inv};
  const double m2 = s_a2 * inv;
  const double mda = sd_a2 * inv;
  const double var_a2 = sdd_a2 * inv - mda * mda;
  const double var_psi = sdd * inv - (sd.re * sd.re + sd.im * sd.im) * inv * inv;
  double q = 0.0, dr = 0.0, dp = 0.0;
  if (active) {
    if (a.mean_psi) a.mean_psi[g] = m1;
    if (a.mean_abs2) a.mean_abs2[g] = m2;
    if (a.mean_rho) a.mean_rho[g] = a.m_tot * m2;
    if (a.var_rho) a.var_rho[g] = a.m_tot * a.m_tot * var_a2;
    q = var_psi * a.dV;
    if (a.psi_cl) {
      const cx<T> w = reinterpret_cast<const cx<T>*>(a.psi_cl)[g];
      const cx<double> cl = {(double)w.re, (double)w.im};
      dr = fabs(m2 - (cl.re * cl.re + cl.im * cl.im)) * a.dV;
      const cx<double> e = m1 - cl;
      dp = (e.re * e.re + e.im * e.im) * a.dV;
    }
  }
  q = wave_sum(q);
  dr = wave_sum(dr);
  dp = wave_sum(dp);
  if (lane == 0 && wave < a.nwaves) {
    a.wave_q[wave] = q;
    a.wave_q[a.nwaves + wave] = dr;
    a.wave_q[2 * a.nwaves + wave] = dp;
  }
}

// Sum `len` doubles at src + b*len for block b; result * scale to dst[b].
__global__ void __launch_bounds__(256) row_sum_kernel(const double* __restrict__ src, int64_t len, double scale,
                                                      double* __restrict__ dst) {
  __shared__ double red[4];
  const int64_t b = blockIdx.x;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < len; i += blockDim.x) s += src[b * len + i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) dst[b] = (red[0] + red[1] + red[2] + red[3]) * scale;
}

// scalars: [0] Q_raw [1] Q_sym [2] dev_rho_L1 [3] dev_psi_L2 [4] energy mean
// [5] norm mean [6] nonfinite count [7] classical energy
__global__ void __launch_bounds__(256) scalars_kernel(const double* __restrict__ qsum /*[3]*/,
                                                      const double* __restrict__ norms, const double* __restrict__ energy,
                                                      int64_t n_real, double vacuum, int have_cl, int have_energy,
                                                      double* __restrict__ out) {
  __shared__ double red[3][4];
  double sn = 0.0, se = 0.0, nf = 0.0;
  for (int64_t r = threadIdx.x; r < n_real; r += blockDim.x) {
    const double v = norms[r];
    if (isfinite(v)) sn += v;
    else nf += 1.0;
    if (have_energy) se += energy[r];
  }
  sn = wave_sum(sn);
  se = wave_sum(se);
  nf = wave_sum(nf);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = sn;
    red[1][threadIdx.x >> 6] = se;
    red[2][threadIdx.x >> 6] = nf;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double tn = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    const double te = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    const double tf = red[2][0] + red[2][1] + red[2][2] + red[2][3];
    out[0] = qsum[0];
    out[1] = qsum[0] - vacuum;
    out[2] = have_cl ? qsum[1] : 0.0;
    out[3] = have_cl ? qsum[2] : 0.0;
    out[4] = have_energy ? te / (double)n_real : 0.0;
    out[5] = (n_real - tf) > 0 ? tn / (double)(n_real - tf) : 0.0;
    out[6] = tf;
    out[7] = (have_energy && have_cl) ? energy[n_real] : 0.0;
  }
}

int64_t moments_partial_doubles(int64_t n_real, int64_t ncell) {
  const int64_t nwaves = (ncell + 63) / 64;
  return n_real * nwaves + 3 * nwaves + n_real + 3;
}

// Every slot of `partial` that a later kernel reads is written first in the
// same call (one per wavefront of cells and realization, then the row sums),
// so the buffer needs no clearing between calls.
hipError_t launch_moments_geom(const MomGeom& G, double* partial, const void* psi, const void* psi_cl,
                               const tw_moments_out* out, const double* energy_dev, hipStream_t s) {
  const int64_t nwaves = (G.ncell + 63) / 64;
  MomArgs a;
  a.psi = psi;
  a.psi_cl = psi_cl;
  a.n_real = G.n_real;
  a.ncell = G.ncell;
  a.m_tot = G.m_tot;
  a.dV = G.dV;
  a.mean_psi = reinterpret_cast<cx<double>*>(out->mean_psi);
  a.mean_abs2 = out->mean_abs2;
  a.mean_rho = out->mean_rho;
  a.var_rho = out->var_rho;
  a.wave_norm = partial;
  a.wave_q = partial + G.n_real * nwaves;
  a.nwaves = nwaves;
  double* norms = a.wave_q + 3 * nwaves;  // [n_real]
  double* qsum = norms + G.n_real;        // [3]
  dim3 grid((unsigned)((G.ncell + 255) / 256));
  if (G.fp32) hipLaunchKernelGGL(moments_cell_kernel<float>, grid, dim3(256), 0, s, a);
  else hipLaunchKernelGGL(moments_cell_kernel<double>, grid, dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(row_sum_kernel, dim3((unsigned)G.n_real), dim3(256), 0, s, a.wave_norm, nwaves, G.dV, norms);
  hipLaunchKernelGGL(row_sum_kernel, dim3(3), dim3(256), 0, s, a.wave_q, nwaves, 1.0, qsum);
  if (out->norm) {
    e = hipMemcpyAsync(out->norm, norms, sizeof(double) * G.n_real, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  if (out->scalars) {
    const double vacuum = (double)G.ncell / (2.0 * G.n_tot);
    hipLaunchKernelGGL(scalars_kernel, dim3(1), dim3(256), 0, s, qsum, norms, energy_dev, G.n_real, vacuum,
                       psi_cl ? 1 : 0, energy_dev ? 1 : 0, out->scalars);
  }
  return hipGetLastError();
}

hipError_t launch_moments(const Plan& P, const void* psi, const void* psi_cl, const tw_moments_out* out,
                          const double* energy_dev, hipStream_t s) {
  const MomGeom G{P.p.n_real, P.ncell, P.p.m_tot, P.dV, P.p.n_tot, P.fp32};
  return launch_moments_geom(G, P.partial, psi, psi_cl, out, energy_dev, s);
}

// Energy assembly: E_f = m_tot [ (hbar^2/2) dV sum_a KS_a / n_a + (1/2) dV PS ]
// with KS_a the per-axis sums sum k_a^2 |FFT_a psi|^2 over pencils and PS = sum V |psi|^2.
__global__ void __launch_bounds__(256) energy_kernel(const double* __restrict__ partial, int64_t gstride,
                                                     int64_t nfield, int ng0, int ng1, int ng2, int ngp, int dim,
                                                     int n0, int n1, int n2, double hbar, double m_tot, double dV,
                                                     double* __restrict__ out) {
  __shared__ double red[4];
  const int64_t f = blockIdx.x;
  const int ng[4] = {ng0, ng1, ng2, ngp};
  const int nn[3] = {n0, n1, n2};
  double total = 0.0;
  for (int slot = 0; slot < 4; ++slot) {
    if (slot < 3 && slot >= dim) continue;
    const double* src = partial + (int64_t)slot * gstride + f * ng[slot];
    double s = 0.0;
    for (int i = threadIdx.x; i < ng[slot]; i += blockDim.x) s += src[i];
    s = wave_sum(s);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    const double t = red[0] + red[1] + red[2] + red[3];
    if (slot < 3) total += 0.5 * hbar * hbar * dV * t / (double)nn[slot];
    else total += 0.5 * dV * t;
  }
  if (threadIdx.x == 0) out[f] = m_tot * total;
}

hipError_t launch_energy_finalize(const Plan& P, const double* partial, int64_t gstride, int64_t nfield,
                                  const int ng[4], double* out, hipStream_t s) {
  if (nfield <= 0) return hipSuccess;
  hipLaunchKernelGGL(energy_kernel, dim3((unsigned)nfield), dim3(256), 0, s, partial, gstride, nfield, ng[0], ng[1],
                     ng[2], ng[3], P.dim, P.n[0], P.n[1], P.n[2], P.p.hbar_m, P.p.m_tot, P.dV, out);
  return hipGetLastError();
}

// Mode occupations <|a_j|^2> (Sec. "Quantum description": the field is a sum
// of mode operators; a_j = F[alpha]_j / sqrt(N) with alpha = sqrt(n_tot dV) psi').
// Realizations are transformed in two rounds through the pair scratch: round k
// places realization 2p+k in slot p, the D-dim forward transform runs on every
// slot, and the squared moduli are added per mode in a fixed order.
template <class T>
__global__ void __launch_bounds__(256) gather_round_kernel(const void* __restrict__ psi, int64_t n_real,
                                                           int64_t ncell, int64_t nslots, int k, void* __restrict__ z) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nslots * ncell) return;
  const int64_t p = i / ncell, g = i - p * ncell;
  const int64_t r = 2 * p + k;
  const cx<T>* src = reinterpret_cast<const cx<T>*>(psi);
  reinterpret_cast<cx<T>*>(z)[i] = r < n_real ? src[r * ncell + g] : cx<T>{(T)0, (T)0};
}

template <class T>
__global__ void __launch_bounds__(256) mode_occ_kernel(const void* __restrict__ z, int64_t nslots, int64_t ncell,
                                                       double scale, int accumulate, double* __restrict__ occ) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ncell) return;
  const cx<T>* zz = reinterpret_cast<const cx<T>*>(z);
  double s = 0.0;
  for (int64_t p = 0; p < nslots; ++p) {
    const cx<T> v = zz[p * ncell + g];
    s += (double)v.re * (double)v.re + (double)v.im * (double)v.im;
  }
  occ[g] = (accumulate ? occ[g] : 0.0) + scale * s;
}

hipError_t launch_gather_round(const Plan& P, const void* psi, int64_t nslots, int k, hipStream_t s) {
  const int64_t total = nslots * P.ncell;
  if (total <= 0) return hipSuccess;
  dim3 grid((unsigned)((total + 255) / 256));
  if (P.fp32) hipLaunchKernelGGL(gather_round_kernel<float>, grid, dim3(256), 0, s, psi, P.p.n_real, P.ncell, nslots, k, P.z);
  else hipLaunchKernelGGL(gather_round_kernel<double>, grid, dim3(256), 0, s, psi, P.p.n_real, P.ncell, nslots, k, P.z);
  return hipGetLastError();
}

hipError_t launch_mode_occ(const Plan& P, int64_t nslots, int accumulate, double* occ, hipStream_t s) {
  // |a_j|^2 = n_tot dV |F[psi']_j|^2 / N, averaged over the realizations
  const double scale = P.p.n_tot * P.dV / ((double)P.ncell * (double)P.p.n_real);
  dim3 grid((unsigned)((P.ncell + 255) / 256));
  if (P.fp32) hipLaunchKernelGGL(mode_occ_kernel<float>, grid, dim3(256), 0, s, P.z, nslots, P.ncell, scale, accumulate, occ);
  else hipLaunchKernelGGL(mode_occ_kernel<double>, grid, dim3(256), 0, s, P.z, nslots, P.ncell, scale, accumulate, occ);
  return hipGetLastError();
}

// Amplitude and phase spread of the ensemble (Sec. "Large quantum
// corrections", Eqs. (varA) and (varPhi)): per cell the plug-in variances of
// A = |psi'| and of the phase deviation dphi = arg(psi' conj<psi'>) in
// (-pi, pi], weighted by the normal-ordered density <psi^dag psi> =
// <|psi'|^2> - 1/(2 n_tot dV) and integrated over the box:
//   Var A~   = sum_g dV <psi^dag psi> <dA^2> / <A>
//   Var phi~ = sum_g dV <psi^dag psi> <dphi^2> / (pi / sqrt 3).
// Two passes over the realizations per cell (means first, then deviations).
struct DecoArgs {
  const void* psi;
  int64_t n_real;
  int64_t ncell;
  double dV;
  double vac;  // 1 / (2 n_tot dV): Weyl minus normal ordering per cell
  double* var_amp;
  double* var_phase;
  double* wave_d;  // [2][nwaves]
  int64_t nwaves;
};

template <class T>
__global__ void __launch_bounds__(256) decoherence_kernel(DecoArgs a) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = g < a.ncell;
  const int64_t wave = g >> 6;
  const int lane = threadIdx.x & 63;
  const cx<T>* psi = reinterpret_cast<const cx<T>*>(a.psi);
  const double inv = 1.0 / (double)a.n_real;
  cx<double> s1 = {0.0, 0.0};
  double s2 = 0.0, sa = 0.0;
  if (active) {
    for (int64_t r = 0; r < a.n_real; ++r) {
      const cx<T> w = psi[r * a.ncell + g];
      const cx<double> v = {(double)w.re, (double)w.im};
      const double a2 = v.re * v.re + v.im * v.im;
      s1 = s1 + v;
      s2 += a2;
      sa += sqrt(a2);
    }
  }
  const cx<double> m1 = {s1.re * inv, s1.im * inv};
  const double ma = sa * inv;
  double va = 0.0, vp = 0.0;
  if (active) {
    for (int64_t r = 0; r < a.n_real; ++r) {
      const cx<T> w = psi[r * a.ncell + g];
      const cx<double> v = {(double)w.re, (double)w.im};
      const double da = sqrt(v.re * v.re + v.im * v.im) - ma;
      va += da * da;
      const cx<double> u = cmulc(v, m1);
      const double ph = atan2(u.im, u.re);
      vp += ph * ph;
    }
  }
  va *= inv;
  vp *= inv;
  double ia = 0.0, ip = 0.0;
  if (active) {
    if (a.var_amp) a.var_amp[g] = va;
    if (a.var_phase) a.var_phase[g] = vp;
    const double occ = s2 * inv - a.vac;
    ia = ma > 0.0 ? a.dV * occ * va / ma : 0.0;
    ip = a.dV * occ * vp / (3.14159265358979323846 / sqrt(3.0));
  }
  ia = wave_sum(ia);
  ip = wave_sum(ip);
  if (lane == 0 && wave < a.nwaves) {
    a.wave_d[wave] = ia;
    a.wave_d[a.nwaves + wave] = ip;
  }
}

hipError_t launch_decoherence(const Plan& P, const void* psi, double* var_amp, double* var_phase, double* integrals,
                              double* scratch, hipStream_t s) {
  const int64_t nwaves = (P.ncell + 63) / 64;
  DecoArgs a;
  a.psi = psi;
  a.n_real = P.p.n_real;
  a.ncell = P.ncell;
  a.dV = P.dV;
  a.vac = 1.0 / (2.0 * P.p.n_tot * P.dV);
  a.var_amp = var_amp;
  a.var_phase = var_phase;
  a.wave_d = scratch;
  a.nwaves = nwaves;
  dim3 grid((unsigned)((P.ncell + 255) / 256));
  if (P.fp32) hipLaunchKernelGGL(decoherence_kernel<float>, grid, dim3(256), 0, s, a);
  else hipLaunchKernelGGL(decoherence_kernel<double>, grid, dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !integrals) return e;
  hipLaunchKernelGGL(row_sum_kernel, dim3(2), dim3(256), 0, s, scratch, nwaves, 1.0, integrals);
  return hipGetLastError();
}

}  // namespace tw
