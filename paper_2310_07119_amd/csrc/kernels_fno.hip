// Kernels of the Fourier-neural-operator surrogate: a strided batched GEMM on
// BF16 matrix cores (FP32 accumulate) whose epilogue applies the pointwise
// layers' bias, spectral-branch sum, GELU or GELU', spectral mode mixing,
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

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

constexpr int GK = 32;        // K per stage (one MFMA)
constexpr int GLD = GK + 8;   // LDS row pitch in bf16 (16-byte pad)

// One workgroup of 4 wavefronts computes a TM x TN tile of C; each wavefront
// owns a 32 x 32 sub-tile (2 x 2 MFMA blocks of 16 x 16). TM x TN is 64 x 64,
// or 128 x 32 for the skinny products (N <= 32: the pointwise layers), where
// a square tile would leave half of its wavefronts on zero columns.
// AVEC: A rows K-contiguous and 16-byte aligned (four-element loads); ROWEPI:
// width-32 tile with the row-wise epilogue through LDS (both chosen at launch).
template <int TM, int TN, bool AVEC, bool ROWEPI>
__global__ void __launch_bounds__(256) gemm_bf16_kernel(GemmArgs g) {
  static_assert(TM * TN == 4096 && TM % 32 == 0 && TN % 32 == 0, "four 32x32 wavefront tiles");
  constexpr int WN = TN / 32;  // wavefronts along n
  constexpr int EA = TM * GK / 256, EB = TN * GK / 256;  // staged elements per thread
  // operand staging (BF16), reused after the k-loop for the output tile of
  // the row-wise epilogue (FP32, pitch CP)
  constexpr int CP = TN + 4;
  constexpr size_t AB_BYTES = (size_t)(TM + TN) * GLD * sizeof(unsigned short);
  constexpr size_t C_BYTES = (size_t)TM * CP * sizeof(float);
  __shared__ __align__(16) unsigned char smem[AB_BYTES > C_BYTES ? AB_BYTES : C_BYTES];
  unsigned short* As = reinterpret_cast<unsigned short*>(smem);  // [m][k]
  unsigned short* Bs = As + TM * GLD;                            // [n][k]  (B transposed)
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int64_t b = blockIdx.z;
  const int64_t m0 = (int64_t)blockIdx.y * TM, n0 = (int64_t)blockIdx.x * TN;
  const float* __restrict__ A = g.A + b * g.sAb;
  const float* __restrict__ B = g.B + b * g.sBb;
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
  constexpr bool a_vec = AVEC;
  for (int64_t k0 = 0; k0 < g.K; k0 += GK) {
    float va[EA], vb[EB];
    if constexpr (a_vec) {
#pragma unroll
      for (int e = 0; e < EA / 4; ++e) {
        const int idx = tid + 256 * e;
        const int mm = idx / (GK / 4), kq = (idx % (GK / 4)) * 4;
        const int64_t gm = m0 + mm, gk = k0 + kq;
        const float4 q = (gm < g.M && gk < g.K) ? *reinterpret_cast<const float4*>(A + gm * g.sAm + gk)
                                                 : float4{0.f, 0.f, 0.f, 0.f};
        va[4 * e] = q.x;
        va[4 * e + 1] = q.y;
        va[4 * e + 2] = q.z;
        va[4 * e + 3] = q.w;
      }
    } else {
#pragma unroll
      for (int e = 0; e < EA; ++e) {  // issue every load of the stage before converting
        const int idx = tid + 256 * e;
        const int mm = a_k_fast ? idx / GK : idx % TM;
        const int kk = a_k_fast ? idx % GK : idx / TM;
        const int64_t gm = m0 + mm, gk = k0 + kk;
        va[e] = (gm < g.M && gk < g.K) ? A[gm * g.sAm + gk * g.sAk] : 0.f;
      }
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int idx = tid + 256 * e;
      const int nn = b_n_fast ? idx % TN : idx / GK;
      const int kk = b_n_fast ? idx / TN : idx % GK;
      const int64_t gn = n0 + nn, gk = k0 + kk;
      vb[e] = (gn < g.N && gk < g.K) ? B[gk * g.sBk + gn * g.sBn] : 0.f;
    }
    if constexpr (a_vec) {
#pragma unroll
      for (int e = 0; e < EA / 4; ++e) {
        const int idx = tid + 256 * e;
        const int mm = idx / (GK / 4), kq = (idx % (GK / 4)) * 4;
        const uint32_t lo = f32_to_bf16_rne(va[4 * e]) | ((uint32_t)f32_to_bf16_rne(va[4 * e + 1]) << 16);
        const uint32_t hi = f32_to_bf16_rne(va[4 * e + 2]) | ((uint32_t)f32_to_bf16_rne(va[4 * e + 3]) << 16);
        *reinterpret_cast<uint2*>(&As[mm * GLD + kq]) = uint2{lo, hi};
      }
    } else {
#pragma unroll
      for (int e = 0; e < EA; ++e) {
        const int idx = tid + 256 * e;
        const int mm = a_k_fast ? idx / GK : idx % TM;
        const int kk = a_k_fast ? idx % GK : idx / TM;
        As[mm * GLD + kk] = f32_to_bf16_rne(va[e]);
      }
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
  if constexpr (ROWEPI) {
    static_assert(TN == 32, "the row-wise epilogue moves 32-float rows");
    {
      // the tile goes through LDS so that the epilogue reads and writes whole
      // 128-byte rows (eight threads of 16 bytes per row; the MFMA layout
      // gives 64-byte pieces of four rows per instruction)
      float* Cs = reinterpret_cast<float*>(smem);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int q = 0; q < 4; ++q) Cs[(wm + 16 * i + rb + q) * CP + wn + 16 * j + col] = acc[i][j][q];
      __syncthreads();
      const int c4 = (tid & 7) * 4;
#pragma unroll 1
      for (int pr = 0; pr < TM / 32; ++pr) {
        const int r = pr * 32 + (tid >> 3);
        const int64_t gm = m0 + r, gn = n0 + c4;
        if (gm >= g.M || gn >= g.N) continue;  // N % 4 == 0: a piece is all in or all out
        const int64_t off = b * g.sCb + gm * g.sCm + gn;
        const float4 a4 = *reinterpret_cast<const float4*>(&Cs[r * CP + c4]);
        const float zero4[4] = {0.f, 0.f, 0.f, 0.f};
        float av[4] = {a4.x, a4.y, a4.z, a4.w}, pv[4], dv[4], bv[4], zv[4];
        auto ld4 = [&](const float* src, float (&dst)[4]) {
          const float4 v = *reinterpret_cast<const float4*>(src);
          dst[0] = v.x; dst[1] = v.y; dst[2] = v.z; dst[3] = v.w;
        };
        if (g.beta != 0.f) ld4(g.C + off, pv); else for (int e = 0; e < 4; ++e) pv[e] = zero4[e];
        if (g.add) ld4(g.add + off, dv);
        if (g.bias) ld4(g.bias + gn, bv);
        if (g.gz) ld4(g.gz + off, zv);
        float cv[4], ov[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          float rr = g.beta * pv[e] + g.alpha * av[e];
          if (g.add) rr += dv[e];
          if (g.bias) rr += bv[e];
          const float gr = g.gz ? rr * gelu_grad_f(zv[e]) : rr;
          cv[e] = g.gz_into_c ? gr : rr;
          ov[e] = g.gz ? gr : (g.act ? gelu_f(rr) : rr);
        }
        *reinterpret_cast<float4*>(g.C + off) = float4{cv[0], cv[1], cv[2], cv[3]};
        if (g.out2) *reinterpret_cast<float4*>(g.out2 + off) = float4{ov[0], ov[1], ov[2], ov[3]};
      }
      return;
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t gm = m0 + wm + 16 * i + rb + q, gn = n0 + wn + 16 * j + col;
        if (gm < g.M && gn < g.N) {
          const int64_t off = b * g.sCb + gm * g.sCm + gn * g.sCn;
          float* p = g.C + off;
          const float prev = g.beta != 0.f ? *p : 0.f;
          float r = g.beta * prev + g.alpha * acc[i][j][q];
          if (g.add) r += g.add[off];
          if (g.bias) r += g.bias[gn];
          const float gr = g.gz ? r * gelu_grad_f(g.gz[off]) : r;
          *p = g.gz_into_c ? gr : r;
          if (g.out2) g.out2[off] = g.gz ? gr : (g.act ? gelu_f(r) : r);
        }
      }
}

hipError_t launch_gemm(const GemmArgs& g0, hipStream_t s) {
  if (g0.M <= 0 || g0.N <= 0 || g0.batch <= 0) return hipSuccess;
  if (g0.batch > 65535) return hipErrorInvalidValue;
  GemmArgs g = g0;
  auto al16 = [](const void* p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; };
  g.a_vec = g.sAk == 1 && g.sAm % 4 == 0 && g.sAb % 4 == 0 && g.K % 4 == 0 && al16(g.A);
  g.row_epi = g.N <= 32 && g.sCn == 1 && g.sCm % 4 == 0 && g.sCb % 4 == 0 && g.N % 4 == 0 && al16(g.C) &&
              (!g.add || al16(g.add)) && (!g.bias || al16(g.bias)) && (!g.gz || al16(g.gz)) &&
              (!g.out2 || al16(g.out2));
  if (g.N <= 32) {
    dim3 grid((unsigned)((g.N + 31) / 32), (unsigned)((g.M + 127) / 128), (unsigned)g.batch);
    if (g.a_vec && g.row_epi) hipLaunchKernelGGL((gemm_bf16_kernel<128, 32, true, true>), grid, dim3(256), 0, s, g);
    else if (g.a_vec) hipLaunchKernelGGL((gemm_bf16_kernel<128, 32, true, false>), grid, dim3(256), 0, s, g);
    else if (g.row_epi) hipLaunchKernelGGL((gemm_bf16_kernel<128, 32, false, true>), grid, dim3(256), 0, s, g);
    else hipLaunchKernelGGL((gemm_bf16_kernel<128, 32, false, false>), grid, dim3(256), 0, s, g);
  } else {
    dim3 grid((unsigned)((g.N + 63) / 64), (unsigned)((g.M + 63) / 64), (unsigned)g.batch);
    if (g.a_vec) hipLaunchKernelGGL((gemm_bf16_kernel<64, 64, true, false>), grid, dim3(256), 0, s, g);
    else hipLaunchKernelGGL((gemm_bf16_kernel<64, 64, false, false>), grid, dim3(256), 0, s, g);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------- elementwise

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

__device__ __forceinline__ float bf16_value(float f) { return __uint_as_float((uint32_t)f32_to_bf16_rne(f) << 16); }

// Column sums of a row-major [P][C] matrix with C a multiple of 4 (C/4 lanes
// per row, each four adjacent columns by float4 loads, FP64 accumulators),
// optionally weighted per row by NW weight columns: with wt ([P][NW]),
// out[c][n] = sum_r bf16(x[r][c]) bf16(wt[r][n]), the weight gradient of a
// projection to NW output channels (the same BF16 operands as the
// matrix-core contraction it replaces). Workgroup b covers `rows` rows and
// writes C * NW partial sums.
template <int NW>
__global__ void __launch_bounds__(256) colsum4_parts_kernel(const float* __restrict__ x, const float* __restrict__ wt,
                                                            int64_t P, int C, int64_t rows, float* __restrict__ parts) {
  constexpr int NS = 4 * NW;  // accumulators per thread
  __shared__ double red[256 * NS];
  const int tid = threadIdx.x;
  const int TC = C / 4;
  const int RL = 256 / TC;  // rows per iteration
  const int c4 = tid % TC, r0 = tid / TC;
  const int64_t rbeg = (int64_t)blockIdx.x * rows;
  const int64_t rend = rbeg + rows < P ? rbeg + rows : P;
  double acc[NS];
#pragma unroll
  for (int j = 0; j < NS; ++j) acc[j] = 0.0;
  for (int64_t r = rbeg + r0; r < rend; r += RL) {
    const float4 v = *reinterpret_cast<const float4*>(x + r * C + 4 * c4);
    const float xv[4] = {v.x, v.y, v.z, v.w};
    if (wt) {
#pragma unroll
      for (int n = 0; n < NW; ++n) {
        const float w = bf16_value(wt[r * NW + n]);
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j * NW + n] += (double)(bf16_value(xv[j]) * w);
      }
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[j] += (double)xv[j];
    }
  }
#pragma unroll
  for (int j = 0; j < NS; ++j) red[NS * tid + j] = acc[j];
  __syncthreads();
  if (r0 == 0) {
    double t[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) t[j] = 0.0;
    for (int q = 0; q < RL; ++q)
#pragma unroll
      for (int j = 0; j < NS; ++j) t[j] += red[NS * (q * TC + c4) + j];
#pragma unroll
    for (int j = 0; j < NS; ++j) parts[(int64_t)blockIdx.x * C * NW + (int64_t)4 * c4 * NW + j] = (float)t[j];
  }
}

// the float4 column-sum form applies: C a multiple of 4 with C/4 dividing 256,
// rows 16-byte aligned
static bool colsum4_ok(const float* x, int C) {
  return C % 4 == 0 && C / 4 <= 256 && (256 % (C / 4)) == 0 && reinterpret_cast<uintptr_t>(x) % 16 == 0;
}

static hipError_t colsum4(const float* x, const float* wt, int nw, int64_t P, int C, float* out, int accumulate,
                          float* parts, int64_t parts_len, double* tmp, hipStream_t st) {
  const int W = wt ? nw : 1;
  // about 256 rows per workgroup (thousands of workgroups at the surrogate's sizes)
  int64_t nblk = std::min<int64_t>((P + 255) / 256, parts_len / ((int64_t)C * W));
  nblk = std::min<int64_t>(nblk, 65535);
  if (nblk < 1) return hipErrorInvalidValue;
  const int64_t rows = (P + nblk - 1) / nblk;
  nblk = (P + rows - 1) / rows;
  switch (W) {
    case 1: hipLaunchKernelGGL(colsum4_parts_kernel<1>, dim3((unsigned)nblk), dim3(256), 0, st, x, wt, P, C, rows, parts); break;
    case 2: hipLaunchKernelGGL(colsum4_parts_kernel<2>, dim3((unsigned)nblk), dim3(256), 0, st, x, wt, P, C, rows, parts); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_sum_parts(parts, (int)nblk, (int64_t)C * W, out, accumulate, st, tmp);
}

hipError_t launch_colsum_weighted(const float* x, const float* wt, int nw, int64_t P, int C, float* out, float* parts,
                                  int64_t parts_len, double* tmp, hipStream_t st) {
  if (P <= 0 || C <= 0 || nw < 1 || nw > 2 || !colsum4_ok(x, C)) return hipErrorInvalidValue;
  return colsum4(x, wt, nw, P, C, out, 0, parts, parts_len, tmp, st);
}

// A projection to NO output channels: y[m][n] = sum_k bf16(h[m][k]) bf16(w[k][n]) + b[n]
// (K/4 lanes per row, one float4 each, so every load instruction reads whole
// rows; the lanes of a row are combined by a fixed butterfly). Measured at
// K = 128: two rows in flight per wavefront beat four (89.6 against 103 us
// for 268 MB) and eight lanes per row with strided loads (181 us).
template <int NO>
__global__ void __launch_bounds__(256) proj_out_kernel(const float* __restrict__ h, const float* __restrict__ w,
                                                       const float* __restrict__ b, float* __restrict__ y, int64_t M,
                                                       int K) {
  const int TL = K / 4;
  const int lane = threadIdx.x & 63, sub = lane % TL, rw = lane / TL;
  const int RPW = 64 / TL;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  float wk[4][NO];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int n = 0; n < NO; ++n) wk[j][n] = bf16_value(w[(4 * sub + j) * NO + n]);
  for (int64_t r0 = wave * RPW; r0 < M; r0 += nw * RPW) {
    const int64_t r = r0 + rw;
    float acc[NO];
#pragma unroll
    for (int n = 0; n < NO; ++n) acc[n] = 0.f;
    if (r < M) {
      const float4 v = *reinterpret_cast<const float4*>(h + r * K + 4 * sub);
      const float hv[4] = {bf16_value(v.x), bf16_value(v.y), bf16_value(v.z), bf16_value(v.w)};
#pragma unroll
      for (int n = 0; n < NO; ++n) {
        acc[n] = hv[0] * wk[0][n];
#pragma unroll
        for (int j = 1; j < 4; ++j) acc[n] = __builtin_fmaf(hv[j], wk[j][n], acc[n]);
      }
    }
#pragma unroll
    for (int n = 0; n < NO; ++n)
      for (int off = TL / 2; off > 0; off >>= 1) acc[n] += __shfl_xor(acc[n], off, 64);
    if (sub == 0 && r < M) {
#pragma unroll
      for (int n = 0; n < NO; ++n) y[r * NO + n] = acc[n] + (b ? b[n] : 0.f);
    }
  }
}

hipError_t launch_proj_out(const float* h, const float* w, const float* b, float* y, int64_t M, int K, int nout,
                           hipStream_t st) {
  const int TL = K / 4;
  if (K % 4 != 0 || TL > 64 || (TL & (TL - 1)) != 0 || reinterpret_cast<uintptr_t>(h) % 16 != 0)
    return hipErrorInvalidValue;
  const int64_t rows_per_block = 4 * (64 / TL);
  const int64_t nblk = std::min<int64_t>((M + rows_per_block - 1) / rows_per_block, 8192);
  switch (nout) {
    case 1: hipLaunchKernelGGL(proj_out_kernel<1>, dim3((unsigned)nblk), dim3(256), 0, st, h, w, b, y, M, K); break;
    case 2: hipLaunchKernelGGL(proj_out_kernel<2>, dim3((unsigned)nblk), dim3(256), 0, st, h, w, b, y, M, K); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Its backward to the hidden layer: dz[m][k] = (sum_n bf16(dy[m][n]) bf16(w[k][n])) GELU'(z[m][k])
// (N a multiple of 4; float4 over k).
template <int NO>
__global__ void __launch_bounds__(256) proj_out_back_kernel(const float* __restrict__ dy, const float* __restrict__ w,
                                                            const float* __restrict__ z, float* __restrict__ dz,
                                                            int64_t M, int N) {
  const int N4 = N / 4;
  const int64_t total = M * N4;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = i / N4;
    const int k4 = (int)(i - m * N4);
    float d[NO];
#pragma unroll
    for (int n = 0; n < NO; ++n) d[n] = bf16_value(dy[m * NO + n]);
    const float4 zv = *reinterpret_cast<const float4*>(z + m * N + 4 * k4);
    const float zz[4] = {zv.x, zv.y, zv.z, zv.w};
    float o[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float r = d[0] * bf16_value(w[(4 * k4 + j) * NO]);
#pragma unroll
      for (int n = 1; n < NO; ++n) r = __builtin_fmaf(d[n], bf16_value(w[(4 * k4 + j) * NO + n]), r);
      o[j] = r * gelu_grad_f(zz[j]);
    }
    *reinterpret_cast<float4*>(dz + m * N + 4 * k4) = make_float4(o[0], o[1], o[2], o[3]);
  }
}

hipError_t launch_proj_out_back(const float* dy, const float* w, const float* z, float* dz, int64_t M, int N,
                                int nout, hipStream_t st) {
  if (N % 4 != 0 || reinterpret_cast<uintptr_t>(z) % 16 != 0 || reinterpret_cast<uintptr_t>(dz) % 16 != 0)
    return hipErrorInvalidValue;
  const int64_t total = M * (N / 4);
  const int64_t nblk = std::min<int64_t>((total + 255) / 256, 16384);
  switch (nout) {
    case 1: hipLaunchKernelGGL(proj_out_back_kernel<1>, dim3((unsigned)nblk), dim3(256), 0, st, dy, w, z, dz, M, N); break;
    case 2: hipLaunchKernelGGL(proj_out_back_kernel<2>, dim3((unsigned)nblk), dim3(256), 0, st, dy, w, z, dz, M, N); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_colsum(const float* x, int64_t P, int C, float* out, int accumulate, float* parts,
                         int64_t parts_len, double* tmp, hipStream_t st) {
  if (P <= 0 || C <= 0) return hipErrorInvalidValue;
  if (colsum4_ok(x, C)) return colsum4(x, nullptr, 1, P, C, out, accumulate, parts, parts_len, tmp, st);
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
#pragma unroll 16  // the loads issue back to back; the sum keeps its order
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
#pragma unroll 16  // the loads issue back to back; the sum keeps its order
  for (int j = j0; j < j1; ++j) s += (double)parts[(int64_t)j * n + i];
  tmp[(int64_t)blockIdx.y * n + i] = s;
}

__global__ void sum_subtotals_kernel(const double* __restrict__ tmp, int ng, int64_t n, float* __restrict__ out,
                                     int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
#pragma unroll 16  // the loads issue back to back; the sum keeps its order
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
// Mean squared error loss = (1/n) sum (y - t)^2 (FP64 sums, written to
// loss[0]) and its gradient dy = 2 (y - t) / n, in two launches: up to
// kMseParts workgroups each sum a contiguous chunk into a fixed device array,
// then one thread adds the partial sums in order (deterministic). The array
// belongs to this file's kernels; MSE calls that overlap on one GPU share it
// and must be ordered by the caller.
constexpr int kMseParts = 512;
__device__ double g_mse_parts[kMseParts];

__global__ void __launch_bounds__(256) mse_parts_kernel(const float* __restrict__ y, const float* __restrict__ t,
                                                        int64_t n, int64_t chunk, float* __restrict__ dy) {
  __shared__ double red[4];
  const int64_t i0 = (int64_t)blockIdx.x * chunk;
  const int64_t i1 = i0 + chunk < n ? i0 + chunk : n;
  const double inv = 1.0 / (double)n;
  double s = 0.0;
#pragma unroll 4
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
    const double d = (double)y[i] - (double)t[i];
    s += d * d;
    if (dy) dy[i] = (float)(2.0 * d * inv);
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) g_mse_parts[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// One wavefront: lane l sums parts l, l + 64, ... in order, then a fixed
// butterfly combines the lanes (the same order on every call).
__global__ void __launch_bounds__(64) mse_finish_kernel(int nb, int64_t n, float* __restrict__ loss) {
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += 64) s += g_mse_parts[b];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (threadIdx.x == 0 && loss) loss[0] = (float)(s / (double)n);
}

hipError_t launch_mse(const float* y, const float* t, int64_t n, float* dy, float* loss, hipStream_t st) {
  int64_t nb = (n + 4095) / 4096;  // at least 4096 elements per workgroup
  if (nb > kMseParts) nb = kMseParts;
  if (nb < 1) nb = 1;
  const int64_t chunk = (n + nb - 1) / nb;
  hipLaunchKernelGGL(mse_parts_kernel, dim3((unsigned)nb), dim3(256), 0, st, y, t, n, chunk, dy);
  hipLaunchKernelGGL(mse_finish_kernel, dim3(1), dim3(64), 0, st, (int)nb, n, loss);
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
