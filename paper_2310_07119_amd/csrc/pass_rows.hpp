// Body of one workgroup of a pencil pass (row passes, and the interleaved
// organisation of strided passes); kernels_step.hip wraps it in kernels and the
// batched launcher calls it for every size class.
#pragma once
#include "pass_common.hpp"

namespace tw {

// One workgroup of a pass: x-block bx of nbx, pair slot by (relative to a.pair0).
template <class T, int N, int MODE, bool ROWS>
__device__ __forceinline__ void pass_body(const PassArgs& a, unsigned bx, unsigned nbx, int64_t by) {
  constexpr int TPP = fft_threads(N);
  constexpr int R = N / TPP;
  constexpr int C = pencils_per_group<T, N, ROWS>();
  constexpr bool SW = ROWS;  // wavefront-local exchanges
  constexpr bool DUAL = pass_dual<T, N, ROWS, MODE>();  // the pair's two fields transformed in lockstep
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* lds_all = reinterpret_cast<cx<T>*>(smem_raw);
  double* red = reinterpret_cast<double*>(smem_raw + (size_t)C * fft_lds_stride(N) * sizeof(cx<T>) * (DUAL ? 2 : 1));

  const int tid = threadIdx.x;
  const int c = ROWS ? tid / TPP : tid % C;
  const int t = ROWS ? tid % TPP : tid / C;
  cx<T>* lds = lds_all + c * fft_lds_stride(N);
  cx<T>* ldsB = lds_all + (DUAL ? C + c : c) * fft_lds_stride(N);  // second buffer of the pencil slot
  const int64_t npencils = a.ncell / N;
  const unsigned grp = xcd_group_remap(bx, nbx);
  const int64_t p = (int64_t)grp * C + c;
  const bool active = p < npencils;
  const int64_t pp = active ? p : 0;
  // FP64 row passes (always along the contiguous axis: stride 1, checked by
  // the launchers) take the stride as a constant: the 64-bit address
  // arithmetic folds away, which brings the drift+density pass to three
  // wavefronts per SIMD (4% faster on MI355X). The FP32 row passes ran 9%
  // slower in the kick pass with it and keep the runtime stride.
  constexpr bool UNIT = ROWS && sizeof(T) == 8;
  const int64_t stride = UNIT ? 1 : a.stride;
  // (cell counts stay below 2^31: 32-bit index arithmetic)
  const uint32_t p32 = (uint32_t)pp, s32 = (uint32_t)stride;
  const int64_t base = UNIT ? pp * N : (int64_t)((p32 % s32) + (p32 / s32) * s32 * (uint32_t)N);
  const int64_t pair = a.pair0 + by;
  const int64_t fA = 2 * pair, fB = 2 * pair + 1;
  const bool hasB = fB < a.nfield;

  auto load = [&](const cx<T>* f, cx<T> (&v)[R]) {
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = active ? f[base + (int64_t)(t + TPP * m) * stride] : cx<T>{(T)0, (T)0};
  };
  auto store = [&](cx<T>* f, const cx<T> (&v)[R]) {
    if (active) {
#pragma unroll
      for (int m = 0; m < R; ++m) f[base + (int64_t)(t + TPP * m) * stride] = v[m];
    }
  };
  // Transposed store (row passes of the 2D alternating-storage schedule): the
  // C pencils of the workgroup go through their LDS buffers so that each
  // store instruction writes C contiguous elements of the transposed field.
  // The destination is always another buffer than the one this pass reads:
  // other workgroups may not have loaded their pencils yet.
  auto store_t = [&](cx<T>* f, const cx<T> (&v)[R]) {
    __syncthreads();  // every wavefront is done with its transform's LDS traffic
#pragma unroll
    for (int m = 0; m < R; ++m) lds[lds_pad(t + TPP * m)] = v[m];
    __syncthreads();
    const int cc = tid % C, jj = tid / C;
    const int64_t pc = (int64_t)grp * C + cc;
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int j = jj + TPP * m;
      const cx<T> w = lds_all[cc * fft_lds_stride(N) + lds_pad(j)];
      if (pc < npencils) f[(int64_t)j * npencils + pc] = w;
    }
    __syncthreads();
  };
  auto store_psi = [&](int64_t f, const cx<T> (&v)[R]) {
    if constexpr (ROWS) {
      if (a.t_psi) {
        store_t(field_ptr_t<T>(a, f), v);
        return;
      }
    }
    store(field_ptr<T>(a, f), v);
  };
  auto zero = [&](cx<T> (&v)[R]) {
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = cx<T>{(T)0, (T)0};
  };
  cx<T>* zp = reinterpret_cast<cx<T>*>(a.z) + pair * a.ncell;

  // Issue every global load of the pass before the first transform: the
  // exchanges carry fences that the compiler does not move loads across, so
  // loads placed later would each wait a full memory latency.
  cx<T> va[R], vb[R], zv[R];
  // FP64 drift+density pass: the wavefront issues its loads at raised
  // priority (measured 3.7% faster; the same in the kick pass, 4.5% slower)
  constexpr bool PRIO = MODE == PASS_DRIFT_RHO && sizeof(T) == 8;
  if constexpr (PRIO) __builtin_amdgcn_s_setprio(3);
  constexpr bool LOAD_PSI = MODE == PASS_DRIFT || MODE == PASS_DRIFT_RHO || MODE == PASS_RHO ||
                            MODE == PASS_KICK_DRIFT || MODE == PASS_KIN_SUM || MODE == PASS_POT_SUM;
  constexpr bool LOAD_Z = MODE == PASS_ZFWD || MODE == PASS_ZINV || MODE == PASS_ZPOISSON ||
                          MODE == PASS_KICK_DRIFT || MODE == PASS_POT_SUM;
  if constexpr (LOAD_Z) load(zp, zv);
  if constexpr (LOAD_PSI) {
    load(field_ptr<T>(a, fA), va);
    if (hasB) load(field_ptr<T>(a, fB), vb);
    else zero(vb);
  }
  TwiddleCache<T, N> tc;
  tc.load(reinterpret_cast<const cx<T>*>(a.twd), t);
  if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);

  auto drift = [&](cx<T> (&v)[R]) {
    fft_pencil<T, N, false, SW>(v, lds, t, tc);
    const cx<double>* __restrict__ ph = reinterpret_cast<const cx<double>*>(a.phase);
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = mul_d(v[m], ph[t + TPP * m]);
    fft_pencil<T, N, true, SW>(v, lds, t, tc);
  };
  // both fields of the pair (vb is zero when the pair has no second field)
  auto drift2 = [&](cx<T> (&x)[R], cx<T> (&y)[R]) {
    fft_pencil2<T, N, false, SW>(x, y, lds, ldsB, t, tc);
    const cx<double>* __restrict__ ph = reinterpret_cast<const cx<double>*>(a.phase);
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const cx<double> f = ph[t + TPP * m];
      x[m] = mul_d(x[m], f);
      y[m] = mul_d(y[m], f);
    }
    fft_pencil2<T, N, true, SW>(x, y, lds, ldsB, t, tc);
  };
  auto density = [&](const cx<T> (&v)[R], int64_t f, double (&rho)[R]) {
    const double mean = a.rho_mean ? a.rho_mean[f] : 0.0;
#pragma unroll
    for (int m = 0; m < R; ++m) rho[m] = a.m_tot * (double)abs2(v[m]) - mean;
  };

  // drift both fields of the pair and store them
  auto drift_store = [&]() {
    if constexpr (DUAL) {
      drift2(va, vb);
      store_psi(fA, va);
      if (hasB) store_psi(fB, vb);
    } else {
      drift(va);
      store_psi(fA, va);
      if (hasB) {
        drift(vb);
        store_psi(fB, vb);
      }
    }
  };

  if constexpr (MODE == PASS_DRIFT) {
    drift_store();
  } else if constexpr (MODE == PASS_DRIFT_RHO || MODE == PASS_RHO) {
    if constexpr (MODE == PASS_DRIFT_RHO) drift_store();
    double ra[R], rb[R];
    density(va, fA, ra);
    if (hasB) {
      density(vb, fB, rb);
    } else {
#pragma unroll
      for (int m = 0; m < R; ++m) rb[m] = 0.0;
    }
#pragma unroll
    for (int m = 0; m < R; ++m) zv[m] = {(T)ra[m], (T)rb[m]};
    fft_pencil<T, N, false, SW>(zv, lds, t, tc);
    store(zp, zv);
  } else if constexpr (MODE == PASS_ZFWD || MODE == PASS_ZINV || MODE == PASS_ZPOISSON) {
    if constexpr (MODE == PASS_ZINV) {
      fft_pencil<T, N, true, SW>(zv, lds, t, tc);
    } else {
      fft_pencil<T, N, false, SW>(zv, lds, t, tc);
    }
    if constexpr (MODE == PASS_ZPOISSON) {
      // grid coordinates of the pencil's first cell (cell counts stay below 2^31)
      const uint32_t b32 = (uint32_t)base, n0 = (uint32_t)a.n[0], n1 = (uint32_t)a.n[1];
      const uint32_t co[3] = {b32 % n0, (b32 / n0) % n1, b32 / (n0 * n1)};
      double k2o = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d)
        if (d != a.axis) k2o += a.k2[d][co[d]];
      const double* __restrict__ k2a = a.k2[a.axis];
#pragma unroll
      for (int m = 0; m < R; ++m) {
        zv[m] = mul_d(zv[m], green_factor<T>(k2o + k2a[t + TPP * m], a.green));
      }
      fft_pencil<T, N, true, SW>(zv, lds, t, tc);
    }
    store(zp, zv);
  } else if constexpr (MODE == PASS_KICK_DRIFT) {
    fft_pencil<T, N, true, SW>(zv, lds, t, tc);
    if (a.vmax) {
      double mx = 0.0;
#pragma unroll
      for (int m = 0; m < R; ++m) mx = fmax(mx, fmax(fabs((double)zv[m].re), hasB ? fabs((double)zv[m].im) : 0.0));
      mx = block_max(mx, red);
      if (tid == 0) record_max(a.vmax + ((bx + (unsigned)by) & (kVmaxBuckets - 1)), mx);
    }
    if (a.store_v) store(zp, zv);  // the potentials, for the test particles
    const double kick = a.kick_dev ? a.kick_dev[0] : a.kick;
    if constexpr (DUAL) {
      kick_values<T, R>(va, zv, false, kick);
      if (hasB) kick_values<T, R>(vb, zv, true, kick);
      drift_store();
    } else {  // one field at a time: kicking both first holds more registers
      kick_values<T, R>(va, zv, false, kick);
      drift(va);
      store_psi(fA, va);
      if (hasB) {
        kick_values<T, R>(vb, zv, true, kick);
        drift(vb);
        store_psi(fB, vb);
      }
    }
  } else if constexpr (MODE == PASS_KIN_SUM) {
    const double* __restrict__ k2a = a.k2[a.axis];
    for (int k = 0; k < 2; ++k) {
      if (k == 1 && !hasB) break;
      cx<T>* v = k == 0 ? va : vb;
      cx<T> w[R];
#pragma unroll
      for (int m = 0; m < R; ++m) w[m] = v[m];
      fft_pencil<T, N, false, SW>(w, lds, t, tc);
      double s = 0.0;
#pragma unroll
      for (int m = 0; m < R; ++m) s += k2a[t + TPP * m] * (double)abs2(w[m]);
      s = block_sum(s, red);
      if (tid == 0) a.partial[(2 * pair + k) * nbx + grp] = s;
    }
  } else if constexpr (MODE == PASS_POT_SUM) {
    if (a.pot_green) {
      const double* __restrict__ k2a = a.k2[a.axis];
#pragma unroll
      for (int m = 0; m < R; ++m) {
        zv[m] = mul_d(zv[m], green_factor<T>(k2a[t + TPP * m], a.green));
      }
    }
    fft_pencil<T, N, true, SW>(zv, lds, t, tc);
    if (a.vmax) {
      double mx = 0.0;
#pragma unroll
      for (int m = 0; m < R; ++m) mx = fmax(mx, fmax(fabs((double)zv[m].re), hasB ? fabs((double)zv[m].im) : 0.0));
      mx = block_max(mx, red);
      if (tid == 0) record_max(a.vmax + ((bx + (unsigned)by) & (kVmaxBuckets - 1)), mx);
    }
    for (int k = 0; k < 2; ++k) {
      if (k == 1 && !hasB) break;
      const cx<T>* v = k == 0 ? va : vb;
      double s = 0.0;
#pragma unroll
      for (int m = 0; m < R; ++m) s += (double)(k == 0 ? zv[m].re : zv[m].im) * (double)abs2(v[m]);
      s = block_sum(s, red);
      if (tid == 0) a.partial[(2 * pair + k) * nbx + grp] = s;
    }
  }
}

}  // namespace tw
