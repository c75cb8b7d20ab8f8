// Passes along a strided axis (y or z): the same per-pencil work as the row
// passes (drift, density transform, Poisson transforms, kick), organised so
// that global memory is touched in coalesced tiles and every FFT exchange stays
// inside one wavefront.
//
// A workgroup of 4 to 8 wavefronts owns C adjacent pencils (C >= 128 bytes of
// contiguous elements per row, one whole cache line). Each field is moved as a
// tile: every thread loads K elements row-by-row (consecutive lanes ->
// consecutive pencils, so a load instruction reads whole lines) into a padded LDS tile laid
// out pencil-major; after one workgroup barrier each wavefront reads whole
// pencils out of the tile in the FFT's natural layout, transforms them with
// wavefront-local exchanges inside that pencil's own slot, and writes them
// back; a second barrier and a coalesced tile store follow. The next tile's
// global loads are issued before the current tile's transforms so that memory
// latency overlaps the arithmetic.
#pragma once
#include "pass_common.hpp"

namespace tw {

template <class T, int N>
struct ColsCfg {
  static constexpr int TPP = fft_threads(N);
  static constexpr int R = N / TPP;
  static constexpr int PPW = 64 / TPP;                       // pencils per wavefront per round
  static constexpr int COAL = 128 / (int)(2 * sizeof(T));    // pencils per 128 contiguous bytes
  // at least 4 wavefronts; up to 8 so that one round covers the tile
  static constexpr int WAVES = (COAL / PPW) > 4 ? ((COAL / PPW) < 8 ? (COAL / PPW) : 8) : 4;
  static constexpr int THREADS = 64 * WAVES;
  static constexpr int C = COAL > WAVES * PPW ? COAL : WAVES * PPW;
  static constexpr int ROUNDS = C / (WAVES * PPW);
  static constexpr int LS = fft_lds_stride(N);
  static constexpr int K = C * N / THREADS;                  // tile elements per thread
  static constexpr int ROWSTEP = THREADS / C;
  static constexpr size_t LDS = (size_t)C * LS * 2 * sizeof(T) + 16 * sizeof(double);
  static_assert(THREADS % C == 0 && (C * N) % THREADS == 0, "tile shape");
};

__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// One workgroup of a strided pass: x-block bx of nbx, pair slot by (relative to a.pair0).
template <class T, int N, int MODE>
__device__ __forceinline__ void cols_body(const PassArgs& a, unsigned bx, unsigned nbx, int64_t by) {
  using Cfg = ColsCfg<T, N>;
  constexpr int TPP = Cfg::TPP, R = Cfg::R, C = Cfg::C, K = Cfg::K, LS = Cfg::LS;
  constexpr int ROUNDS = Cfg::ROUNDS, ROWSTEP = Cfg::ROWSTEP, PPW = Cfg::PPW;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* tile = reinterpret_cast<cx<T>*>(smem_raw);
  double* red = reinterpret_cast<double*>(smem_raw + (size_t)C * LS * sizeof(cx<T>));

  const int tid = threadIdx.x;
  const unsigned grp = xcd_group_remap(bx, nbx);
  const int64_t npencils = a.ncell / N;
  const int64_t stride = a.stride;
  const int64_t pair = a.pair0 + by;
  const int64_t fA = 2 * pair, fB = 2 * pair + 1;
  const bool hasB = fB < a.nfield;

  // tile-movement role: pencil cl of the tile, rows r0 + ROWSTEP k
  const int cl = tid % C;
  const int r0 = tid / C;
  const int64_t pl = (int64_t)grp * C + cl;
  const bool act_l = pl < npencils;
  const int64_t pll = act_l ? pl : 0;
  const uint32_t p32 = (uint32_t)pll, s32 = (uint32_t)stride;  // cell counts stay below 2^31
  const int64_t base_l = (int64_t)((p32 % s32) + (p32 / s32) * s32 * (uint32_t)N);
  // compute role: wavefront w, lane -> pencil slot and thread-in-pencil
  const int w = tid >> 6, lane = tid & 63;
  const int t = lane % TPP;

  auto gload = [&](const cx<T>* f, cx<T> (&st)[K]) {
#pragma unroll
    for (int k = 0; k < K; ++k)
      st[k] = act_l ? f[base_l + (int64_t)(r0 + ROWSTEP * k) * stride] : cx<T>{(T)0, (T)0};
  };
  auto tile_put = [&](const cx<T> (&st)[K]) {
#pragma unroll
    for (int k = 0; k < K; ++k) tile[cl * LS + lds_pad(r0 + ROWSTEP * k)] = st[k];
  };
  auto tile_store = [&](cx<T>* f) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const cx<T> v = tile[cl * LS + lds_pad(r0 + ROWSTEP * k)];
      if (act_l) f[base_l + (int64_t)(r0 + ROWSTEP * k) * stride] = v;
    }
  };
  auto slot = [&](int q) { return (q * Cfg::WAVES + w) * PPW + lane / TPP; };
  auto pencil_get = [&](int q, cx<T> (&v)[R]) {
    const cx<T>* src = tile + slot(q) * LS;
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = src[lds_pad(t + TPP * m)];
  };
  auto pencil_put = [&](int q, const cx<T> (&v)[R]) {
    cx<T>* dst = tile + slot(q) * LS;
#pragma unroll
    for (int m = 0; m < R; ++m) dst[lds_pad(t + TPP * m)] = v[m];
  };
  // pencil index (global) held by slot q, for k-space coordinates
  // (cell counts stay below 2^31: 32-bit arithmetic)
  auto pencil_base = [&](int q) -> uint32_t {
    const uint32_t p = grp * (uint32_t)C + (uint32_t)slot(q);
    const uint32_t pp = p < (uint32_t)npencils ? p : 0u;
    const uint32_t st = (uint32_t)stride;
    return (pp % st) + (pp / st) * st * (uint32_t)N;
  };

  TwiddleCache<T, N> tc;
  tc.load(reinterpret_cast<const cx<T>*>(a.twd), t);
  auto fwd = [&](int q, cx<T> (&v)[R]) { fft_pencil<T, N, false, true>(v, tile + slot(q) * LS, t, tc); };
  auto inv = [&](int q, cx<T> (&v)[R]) { fft_pencil<T, N, true, true>(v, tile + slot(q) * LS, t, tc); };
  auto drift = [&](int q, cx<T> (&v)[R]) {
    fwd(q, v);
    const cx<double>* __restrict__ ph = reinterpret_cast<const cx<double>*>(a.phase);
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = mul_d(v[m], ph[t + TPP * m]);
    inv(q, v);
  };
  cx<T>* zp = reinterpret_cast<cx<T>*>(a.z) + pair * a.ncell;
  cx<T> st[K];

  if constexpr (MODE == PASS_DRIFT || MODE == PASS_DRIFT_RHO || MODE == PASS_RHO) {
    T rho[2][ROUNDS][R];
    gload(field_ptr<T>(a, fA), st);
    for (int k = 0; k < 2; ++k) {
      const int64_t f = k == 0 ? fA : fB;
      if (k == 1 && !hasB) {
#pragma unroll
        for (int q = 0; q < ROUNDS; ++q)
#pragma unroll
          for (int m = 0; m < R; ++m) rho[1][q][m] = (T)0;
        break;
      }
      tile_put(st);
      lds_barrier();
      if (k == 0 && hasB) gload(field_ptr<T>(a, fB), st);
      const double mean = a.rho_mean ? a.rho_mean[f] : 0.0;
#pragma unroll
      for (int q = 0; q < ROUNDS; ++q) {
        cx<T> v[R];
        pencil_get(q, v);
        if constexpr (MODE != PASS_RHO) {
          drift(q, v);
          pencil_put(q, v);
        }
#pragma unroll
        for (int m = 0; m < R; ++m) rho[k][q][m] = (T)(a.m_tot * (double)abs2(v[m]) - mean);
      }
      lds_barrier();
      if constexpr (MODE != PASS_RHO) {
        tile_store(field_ptr<T>(a, f));
        lds_barrier();
      }
    }
    if constexpr (MODE != PASS_DRIFT) {
#pragma unroll
      for (int q = 0; q < ROUNDS; ++q) {
        cx<T> v[R];
#pragma unroll
        for (int m = 0; m < R; ++m) v[m] = {rho[0][q][m], rho[1][q][m]};
        fwd(q, v);
        pencil_put(q, v);
      }
      lds_barrier();
      tile_store(zp);
    }
  } else if constexpr (MODE == PASS_ZFWD || MODE == PASS_ZINV || MODE == PASS_ZPOISSON) {
    gload(zp, st);
    tile_put(st);
    lds_barrier();
    auto green = [&](int q, cx<T> (&v)[R]) {
      const uint32_t b = pencil_base(q), n0 = (uint32_t)a.n[0], n1 = (uint32_t)a.n[1];
      const uint32_t co[3] = {b % n0, (b / n0) % n1, b / (n0 * n1)};
      double k2o = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d)
        if (d != a.axis) k2o += a.k2[d][co[d]];
      const double* __restrict__ k2a = a.k2[a.axis];
#pragma unroll
      for (int m = 0; m < R; ++m) v[m] = mul_d(v[m], green_factor<T>(k2o + k2a[t + TPP * m], a.green));
    };
    if constexpr (ROUNDS % 2 == 0) {
      // a wavefront's pencils two at a time, transformed in lockstep (each
      // in its own tile slot, so no LDS beyond the tile)
#pragma unroll
      for (int q = 0; q < ROUNDS; q += 2) {
        cx<T> v0[R], v1[R];
        pencil_get(q, v0);
        pencil_get(q + 1, v1);
        cx<T>* l0 = tile + slot(q) * LS;
        cx<T>* l1 = tile + slot(q + 1) * LS;
        fft_pencil2<T, N, MODE == PASS_ZINV, true>(v0, v1, l0, l1, t, tc);
        if constexpr (MODE == PASS_ZPOISSON) {
          green(q, v0);
          green(q + 1, v1);
          fft_pencil2<T, N, true, true>(v0, v1, l0, l1, t, tc);
        }
        pencil_put(q, v0);
        pencil_put(q + 1, v1);
      }
    } else {
#pragma unroll
      for (int q = 0; q < ROUNDS; ++q) {
        cx<T> v[R];
        pencil_get(q, v);
        if constexpr (MODE == PASS_ZINV) {
          inv(q, v);
        } else {
          fwd(q, v);
        }
        if constexpr (MODE == PASS_ZPOISSON) {
          green(q, v);
          inv(q, v);
        }
        pencil_put(q, v);
      }
    }
    lds_barrier();
    tile_store(zp);
  } else if constexpr (MODE == PASS_KICK_DRIFT || MODE == PASS_POT_SUM) {
    cx<T> V[ROUNDS][R];
    gload(zp, st);
    tile_put(st);
    lds_barrier();
    gload(field_ptr<T>(a, fA), st);
#pragma unroll
    for (int q = 0; q < ROUNDS; ++q) {
      pencil_get(q, V[q]);
      if constexpr (MODE == PASS_POT_SUM) {
        if (a.pot_green) {
          const double* __restrict__ k2a = a.k2[a.axis];
#pragma unroll
          for (int m = 0; m < R; ++m) {
            V[q][m] = mul_d(V[q][m], green_factor<T>(k2a[t + TPP * m], a.green));
          }
        }
      }
      inv(q, V[q]);
    }
    if (a.vmax) {
      double mx = 0.0;
#pragma unroll
      for (int q = 0; q < ROUNDS; ++q)
#pragma unroll
        for (int m = 0; m < R; ++m)
          mx = fmax(mx, fmax(fabs((double)V[q][m].re), hasB ? fabs((double)V[q][m].im) : 0.0));
      mx = block_max(mx, red);
      if (tid == 0) record_max(a.vmax + ((bx + (unsigned)by) & (kVmaxBuckets - 1)), mx);
    }
    if (a.store_v) {  // the potentials, for the test particles
#pragma unroll
      for (int q = 0; q < ROUNDS; ++q) pencil_put(q, V[q]);
      lds_barrier();
      tile_store(zp);
    }
    const double kick = a.kick_dev ? a.kick_dev[0] : a.kick;
    for (int k = 0; k < 2; ++k) {
      const int64_t f = k == 0 ? fA : fB;
      if (k == 1 && !hasB) break;
      lds_barrier();
      tile_put(st);
      lds_barrier();
      if (k == 0 && hasB) gload(field_ptr<T>(a, fB), st);
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < ROUNDS; ++q) {
        cx<T> v[R];
        pencil_get(q, v);
        if constexpr (MODE == PASS_KICK_DRIFT) {
          kick_values<T, R>(v, V[q], k == 1, kick);
          drift(q, v);
          pencil_put(q, v);
        } else {
          const bool on = ((int64_t)grp * C + slot(q)) < npencils;
#pragma unroll
          for (int m = 0; m < R; ++m)
            s += on ? (double)(k == 0 ? V[q][m].re : V[q][m].im) * (double)abs2(v[m]) : 0.0;
        }
      }
      if constexpr (MODE == PASS_KICK_DRIFT) {
        lds_barrier();
        tile_store(field_ptr<T>(a, f));
      } else {
        s = block_sum(s, red);
        if (tid == 0) a.partial[f * nbx + grp] = s;
      }
    }
  } else if constexpr (MODE == PASS_KIN_SUM) {
    const double* __restrict__ k2a = a.k2[a.axis];
    gload(field_ptr<T>(a, fA), st);
    for (int k = 0; k < 2; ++k) {
      const int64_t f = k == 0 ? fA : fB;
      if (k == 1 && !hasB) break;
      if (k == 1) lds_barrier();
      tile_put(st);
      lds_barrier();
      if (k == 0 && hasB) gload(field_ptr<T>(a, fB), st);
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < ROUNDS; ++q) {
        cx<T> v[R];
        pencil_get(q, v);
        fwd(q, v);
        const bool on = ((int64_t)grp * C + slot(q)) < npencils;
#pragma unroll
        for (int m = 0; m < R; ++m) s += on ? k2a[t + TPP * m] * (double)abs2(v[m]) : 0.0;
      }
      s = block_sum(s, red);
      if (tid == 0) a.partial[f * nbx + grp] = s;
    }
  }
}

}  // namespace tw
