// Kernels of the Fourier-neural-operator surrogate: a strided batched GEMM on
// BF16 matrix cores (FP32 accumulate), spectral mode mixing, GELU, bias,
// reductions, MSE loss and Adam.
//
// GEMM: C[b] = beta C[b] + alpha A[b] B[b] with FP32 storage; both operands are
// rounded to BF16 (nearest, ties to even) as they are staged in LDS and
// multiplied with v_mfma_f32_16x16x32_bf16 (16x16 output block, K = 32 per
// instruction, FP32 accumulate). A workgroup of 4 wavefronts computes a 64x64
// tile; each wavefront owns a 32x32 quarter (2x2 MFMA blocks). Arbitrary
// element strides let the same kernel serve transposed operands, the DFT
// matrices of the spectral layers and split-K weight gradients.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdint.h>

#include "fno_internal.hpp"

namespace tw {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f32_to_bf16_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  const uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(r >> 16);
}

constexpr int GK = 32;        // K per stage (one MFMA)
constexpr int GLD = GK + 8;   // LDS row pitch in bf16 (16-byte pad)

// One workgroup of 4 wavefronts computes a TM x TN tile of C; each wavefront
// owns a 32 x 32 sub-tile (2 x 2 MFMA blocks of 16 x 16). TM x TN is 64 x 64,
// or 128 x 32 for the skinny products (N <= 32: the pointwise layers), where
// a square tile would leave half of its wavefronts on zero columns.
template <int TM, int TN>
__global__ void __launch_bounds__(256) gemm_bf16_kernel(GemmArgs g) {
  static_assert(TM * TN == 4096 && TM % 32 == 0 && TN % 32 == 0, "four 32x32 wavefront tiles");
  constexpr int WN = TN / 32;  // wavefronts along n
  constexpr int EA = TM * GK / 256, EB = TN * GK / 256;  // staged elements per thread
  __shared__ __align__(16) unsigned short As[TM * GLD];  // [m][k]
  __shared__ __align__(16) unsigned short Bs[TN * GLD];  // [n][k]  (B transposed)
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int64_t b = blockIdx.z;
  const int64_t m0 = (int64_t)blockIdx.y * TM, n0 = (int64_t)blockIdx.x * TN;
  const float* __restrict__ A = g.A + b * g.sAb;
  const float* __restrict__ B = g.B + b * g.sBb;
  float* __restrict__ C = g.C + b * g.sCb;
  const int wm = (w / WN) * 32, wn = (w % WN) * 32;

  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  // staging maps: the faster-moving index follows the operand's unit stride
  // when it has one
  const bool a_k_fast = g.sAk == 1;
  const bool b_n_fast = g.sBn == 1;
  for (int64_t k0 = 0; k0 < g.K; k0 += GK) {
    float va[EA], vb[EB];
#pragma unroll
    for (int e = 0; e < EA; ++e) {  // issue every load of the stage before converting
      const int idx = tid + 256 * e;
      const int mm = a_k_fast ? idx / GK : idx % TM;
      const int kk = a_k_fast ? idx % GK : idx / TM;
      const int64_t gm = m0 + mm, gk = k0 + kk;
      va[e] = (gm < g.M && gk < g.K) ? A[gm * g.sAm + gk * g.sAk] : 0.f;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int idx = tid + 256 * e;
      const int nn = b_n_fast ? idx % TN : idx / GK;
      const int kk = b_n_fast ? idx / TN : idx % GK;
      const int64_t gn = n0 + nn, gk = k0 + kk;
      vb[e] = (gn < g.N && gk < g.K) ? B[gk * g.sBk + gn * g.sBn] : 0.f;
    }
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int idx = tid + 256 * e;
      const int mm = a_k_fast ? idx / GK : idx % TM;
      const int kk = a_k_fast ? idx % GK : idx / TM;
      As[mm * GLD + kk] = f32_to_bf16_rne(va[e]);
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int idx = tid + 256 * e;
      const int nn = b_n_fast ? idx % TN : idx / GK;
      const int kk = b_n_fast ? idx / TN : idx % GK;
      Bs[nn * GLD + kk] = f32_to_bf16_rne(vb[e]);
    }
    __syncthreads();
    const int r = lane & 15, kq = (lane >> 4) * 8;
    bf16x8 af[2], bfr[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) af[i] = *reinterpret_cast<const bf16x8*>(&As[(wm + 16 * i + r) * GLD + kq]);
#pragma unroll
    for (int j = 0; j < 2; ++j) bfr[j] = *reinterpret_cast<const bf16x8*>(&Bs[(wn + 16 * j + r) * GLD + kq]);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  // output block (i, j): lane holds column (lane & 15), rows 4 (lane >> 4) + q
  const int col = lane & 15, rb = (lane >> 4) * 4;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t gm = m0 + wm + 16 * i + rb + q, gn = n0 + wn + 16 * j + col;
        if (gm < g.M && gn < g.N) {
          float* p = C + gm * g.sCm + gn * g.sCn;
          const float prev = g.beta != 0.f ? *p : 0.f;
          *p = g.beta * prev + g.alpha * acc[i][j][q];
        }
      }
}

hipError_t launch_gemm(const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
  if (g.batch > 65535) return hipErrorInvalidValue;
  if (g.N <= 32) {
    dim3 grid((unsigned)((g.N + 31) / 32), (unsigned)((g.M + 127) / 128), (unsigned)g.batch);
    hipLaunchKernelGGL((gemm_bf16_kernel<128, 32>), grid, dim3(256), 0, s, g);
  } else {
    dim3 grid((unsigned)((g.N + 63) / 64), (unsigned)((g.M + 63) / 64), (unsigned)g.batch);
    hipLaunchKernelGGL((gemm_bf16_kernel<64, 64>), grid, dim3(256), 0, s, g);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------- elementwise
__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// u[p, c] += s[p, c] (if s) + bias[c];  v = act ? GELU(u) : u (v may alias u when !act)
__global__ void bias_act_kernel(float* __restrict__ u, const float* __restrict__ s, const float* __restrict__ bias,
                                float* __restrict__ v, int64_t n, int C, int act) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float x = u[i] + (s ? s[i] : 0.f) + bias[i % C];
  u[i] = x;
  if (v) v[i] = act ? gelu_f(x) : x;
}

hipError_t launch_bias_act(float* u, const float* s, const float* bias, float* v, int64_t n, int C, int act,
                           hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(bias_act_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, u, s, bias, v, n, C, act);
  return hipGetLastError();
}

// d[i] = g[i] * GELU'(z[i])
__global__ void gelu_back_kernel(const float* __restrict__ g, const float* __restrict__ z, float* __restrict__ d,
                                 int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = g[i] * gelu_grad_f(z[i]);
}

hipError_t launch_gelu_back(const float* g, const float* z, float* d, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gelu_back_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, z, d, n);
  return hipGetLastError();
}

// out[c] (+)= sum over rows p < P of x[p, c]; one workgroup per column block,
// FP64 accumulation, fixed order (deterministic).
// Column sums of x[P][C] in two deterministic stages: block b sums rows
// [b*rows, (b+1)*rows) into parts[b][C] (threads laid out channel-fastest so a
// wavefront reads whole contiguous rows), then sum_parts adds the blocks.
__global__ void __launch_bounds__(256) colsum_parts_kernel(const float* __restrict__ x, int64_t P, int C, int TC,
                                                           int64_t rows, float* __restrict__ parts) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const int RL = 256 / TC;  // row lanes
  const int c0 = tid % TC, r0 = tid / TC;
  const int64_t rbeg = (int64_t)blockIdx.x * rows;
  const int64_t rend = rbeg + rows < P ? rbeg + rows : P;
  for (int cc = 0; cc < C; cc += TC) {
    const int c = cc + c0;
    double s = 0.0;
    if (r0 < RL && c < C) {
      for (int64_t r = rbeg + r0; r < rend; r += RL) s += (double)x[r * C + c];
    }
    red[tid] = s;
    __syncthreads();
    if (r0 == 0 && c < C) {
      double t = 0.0;
      for (int q = 0; q < RL; ++q) t += red[q * TC + c0];
      parts[(int64_t)blockIdx.x * C + c] = (float)t;
    }
    __syncthreads();
  }
}

hipError_t launch_colsum(const float* x, int64_t P, int C, float* out, int accumulate, float* parts,
                         int64_t parts_len, double* tmp, hipStream_t st) {
  if (P <= 0 || C <= 0) return hipErrorInvalidValue;
  int TC = 1;
  while (TC * 2 <= C && TC * 2 <= 64) TC *= 2;
  int64_t nblk = std::min<int64_t>(512, parts_len / C);
  nblk = std::min<int64_t>(nblk, (P + 255) / 256);
  if (nblk < 1) return hipErrorInvalidValue;
  const int64_t rows = (P + nblk - 1) / nblk;
  nblk = (P + rows - 1) / rows;
  hipLaunchKernelGGL(colsum_parts_kernel, dim3((unsigned)nblk), dim3(256), 0, st, x, P, C, TC, rows, parts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_sum_parts(parts, (int)nblk, C, out, accumulate, st, tmp);
}

// out[i] = sum_j parts[j * n + i]  (split-K reduction), out may accumulate
__global__ void sum_parts_kernel(const float* __restrict__ parts, int nparts, int64_t n, float* __restrict__ out,
                                 int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int j = 0; j < nparts; ++j) s += (double)parts[(int64_t)j * n + i];
  out[i] = (accumulate ? out[i] : 0.f) + (float)s;
}

// Two-level form for many partials: groups of 32 summed in parallel into
// FP64 sub-totals, then the sub-totals (fixed order, deterministic).
__global__ void sum_parts_group_kernel(const float* __restrict__ parts, int nparts, int64_t n, int group,
                                       double* __restrict__ tmp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int j0 = (int)blockIdx.y * group;
  const int j1 = min(nparts, j0 + group);
  double s = 0.0;
  for (int j = j0; j < j1; ++j) s += (double)parts[(int64_t)j * n + i];
  tmp[(int64_t)blockIdx.y * n + i] = s;
}

__global__ void sum_subtotals_kernel(const double* __restrict__ tmp, int ng, int64_t n, float* __restrict__ out,
                                     int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int g = 0; g < ng; ++g) s += tmp[(int64_t)g * n + i];
  out[i] = (accumulate ? out[i] : 0.f) + (float)s;
}

hipError_t launch_sum_parts(const float* parts, int nparts, int64_t n, float* out, int accumulate, hipStream_t st,
                            double* tmp) {
  if (n <= 0) return hipSuccess;
  const unsigned nb = (unsigned)((n + 255) / 256);
  if (tmp && nparts > 64) {
    constexpr int group = 32;
    const int ng = (nparts + group - 1) / group;
    hipLaunchKernelGGL(sum_parts_group_kernel, dim3(nb, (unsigned)ng), dim3(256), 0, st, parts, nparts, n, group, tmp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sum_subtotals_kernel, dim3(nb), dim3(256), 0, st, tmp, ng, n, out, accumulate);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(sum_parts_kernel, dim3(nb), dim3(256), 0, st, parts, nparts, n, out, accumulate);
  return hipGetLastError();
}

// -------------------------------------------------------- spectral mixing
// Forward: C[b,k,o] = sum_c B[b,k,c] R[k,c,o] over modes k (complex, FP32),
// with B and C laid out [b][mode][channel] in separate re/im planes.
__global__ void modemix_fwd_kernel(const float* __restrict__ br, const float* __restrict__ bi,
                                   const float* __restrict__ Rr, const float* __restrict__ Ri, float* __restrict__ cr,
                                   float* __restrict__ ci, int nb, int nmode, int C) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (b, k, o)
  const int64_t total = (int64_t)nb * nmode * C;
  if (i >= total) return;
  const int o = i % C;
  const int64_t bk = i / C;
  const int k = bk % nmode;
  float sr = 0.f, si = 0.f;
  const float* xr = br + bk * C;
  const float* xi = bi + bk * C;
  const float* wr = Rr + (int64_t)k * C * C + o;
  const float* wi = Ri + (int64_t)k * C * C + o;
  for (int c = 0; c < C; ++c) {
    const float a = xr[c], b = xi[c], p = wr[c * C], q = wi[c * C];
    sr += a * p - b * q;
    si += a * q + b * p;
  }
  cr[i] = sr;
  ci[i] = si;
}

// Backward: dB[b,k,c] = sum_o dC[b,k,o] conj(R[k,c,o]);
//           dR[k,c,o] = sum_b conj(B[b,k,c]) dC[b,k,o]  (FP64 sum over the batch)
__global__ void modemix_bwd_x_kernel(const float* __restrict__ dcr, const float* __restrict__ dci,
                                     const float* __restrict__ Rr, const float* __restrict__ Ri,
                                     float* __restrict__ dbr, float* __restrict__ dbi, int nb, int nmode, int C) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (b, k, c)
  const int64_t total = (int64_t)nb * nmode * C;
  if (i >= total) return;
  const int c = i % C;
  const int64_t bk = i / C;
  const int k = bk % nmode;
  float sr = 0.f, si = 0.f;
  const float* gr = dcr + bk * C;
  const float* gi = dci + bk * C;
  const float* wr = Rr + ((int64_t)k * C + c) * C;
  const float* wi = Ri + ((int64_t)k * C + c) * C;
  for (int o = 0; o < C; ++o) {
    const float a = gr[o], b = gi[o], p = wr[o], q = wi[o];
    sr += a * p + b * q;
    si += b * p - a * q;
  }
  dbr[i] = sr;
  dbi[i] = si;
}

__global__ void modemix_bwd_w_kernel(const float* __restrict__ br, const float* __restrict__ bi,
                                     const float* __restrict__ dcr, const float* __restrict__ dci,
                                     float* __restrict__ dRr, float* __restrict__ dRi, int nb, int nmode, int C) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (k, c, o)
  const int64_t total = (int64_t)nmode * C * C;
  if (i >= total) return;
  const int o = i % C;
  const int c = (i / C) % C;
  const int k = i / ((int64_t)C * C);
  double sr = 0.0, si = 0.0;
  for (int b = 0; b < nb; ++b) {
    const int64_t xb = ((int64_t)b * nmode + k) * C;
    const double a = br[xb + c], q = bi[xb + c], gr = dcr[xb + o], gi = dci[xb + o];
    sr += a * gr + q * gi;
    si += a * gi - q * gr;
  }
  dRr[i] = (float)sr;
  dRi[i] = (float)si;
}

hipError_t launch_modemix_fwd(const float* br, const float* bi, const float* Rr, const float* Ri, float* cr,
                              float* ci, int nb, int nmode, int C, hipStream_t st) {
  const int64_t total = (int64_t)nb * nmode * C;
  hipLaunchKernelGGL(modemix_fwd_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, br, bi, Rr, Ri, cr,
                     ci, nb, nmode, C);
  return hipGetLastError();
}

hipError_t launch_modemix_bwd(const float* br, const float* bi, const float* dcr, const float* dci, const float* Rr,
                              const float* Ri, float* dbr, float* dbi, float* dRr, float* dRi, int nb, int nmode,
                              int C, hipStream_t st) {
  int64_t total = (int64_t)nb * nmode * C;
  hipLaunchKernelGGL(modemix_bwd_x_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, dcr, dci, Rr, Ri,
                     dbr, dbi, nb, nmode, C);
  total = (int64_t)nmode * C * C;
  hipLaunchKernelGGL(modemix_bwd_w_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, br, bi, dcr, dci,
                     dRr, dRi, nb, nmode, C);
  return hipGetLastError();
}

// --------------------------------------------------------------- training
// loss = (1/n) sum (y - t)^2 (one workgroup, FP64, written to loss[0]); dy = 2 (y - t) / n
// Mean squared error and its gradient. One workgroup of 1024 threads so the
// loss is reduced in a fixed order without a workspace; four independent
// elements per thread per iteration keep enough loads in flight.
__global__ void __launch_bounds__(1024) mse_kernel(const float* __restrict__ y, const float* __restrict__ t, int64_t n,
                                                   float* __restrict__ dy, float* __restrict__ loss) {
  __shared__ double red[1024];
  const int tid = threadIdx.x;
  double s = 0.0;
  const double inv = 1.0 / (double)n;
  constexpr int U = 4;
  int64_t i = tid;
  for (; i + (U - 1) * 1024 < n; i += U * 1024) {
    float yv[U], tv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      yv[u] = y[i + u * 1024];
      tv[u] = t[i + u * 1024];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double d = (double)yv[u] - (double)tv[u];
      s += d * d;
      if (dy) dy[i + u * 1024] = (float)(2.0 * d * inv);
    }
  }
  for (; i < n; i += 1024) {
    const double d = (double)y[i] - (double)t[i];
    s += d * d;
    if (dy) dy[i] = (float)(2.0 * d * inv);
  }
  red[tid] = s;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (tid == 0 && loss) loss[0] = (float)(red[0] * inv);
}

hipError_t launch_mse(const float* y, const float* t, int64_t n, float* dy, float* loss, hipStream_t st) {
  hipLaunchKernelGGL(mse_kernel, dim3(1), dim3(1024), 0, st, y, t, n, dy, loss);
  return hipGetLastError();
}

// Adam (Kingma and Ba, 2015) with bias correction, FP32 state.
__global__ void adam_kernel(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

hipError_t launch_adam(float* th, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, int64_t step, hipStream_t st) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, th, g, m, v, n, lr, b1, b2,
                     eps, c1, c2);
  return hipGetLastError();
}

// Deterministic parameter initialisation from a counter hash (SplitMix64 of
// (seed, index)): weights uniform in (-s, s) with s = 1/sqrt(fan_in), spectral
// weights uniform in (0, 1/C^2), biases zero. Each tensor is one launch.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__global__ void init_kernel(float* __restrict__ p, int64_t n, uint64_t seed, float lo, float hi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t h = splitmix64(seed ^ splitmix64((uint64_t)i));
  const float u = (float)((h >> 40) + 0.5) * (1.f / 16777216.f);
  p[i] = lo + (hi - lo) * u;
}

hipError_t launch_init(float* p, int64_t n, uint64_t seed, float lo, float hi, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(init_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, seed, lo, hi);
  return hipGetLastError();
}

}  // namespace tw
