// Device helpers shared by the row-pass and strided-pass kernels.
#pragma once
#include "common.hpp"
#include "fft.hpp"
#include "internal.hpp"

namespace tw {

// Pencils per workgroup. Row passes (stride 1): 4 wavefronts, every pencil
// inside one wavefront, so the FFT exchanges are wavefront-local. Strided passes:
// C adjacent pencils with lane = c + C t, so each global access instruction
// covers C contiguous elements (64 bytes: 4 complex128 or 8 complex64); the
// exchanges are workgroup-wide. Neighbouring workgroups share cache lines and
// DRAM pages; the block remap below places them on the same XCD.
template <class T, int N, bool ROWS>
__host__ __device__ constexpr int pencils_per_group() {
  constexpr int TPP = fft_threads(N);
  if constexpr (ROWS) {
    return 4 * (64 / TPP);
  } else {
    int c = 256 / TPP;
    const int coal = 64 / (int)(2 * sizeof(T));
    if (c < coal) c = coal;
    while (c > 1 && c * TPP > 512) c /= 2;
    while (c > 1 && (long)c * fft_lds_stride(N) * 2 * (long)sizeof(T) > 96 * 1024) c /= 2;
    return c;
  }
}

// Workgroups are dispatched round-robin over the 8 XCDs (id mod 8), each with
// its own L2. Passes touch every row of the field in short segments (strided
// reads, transposed stores), so the blocks reading neighbouring segments of the
// same rows should share one XCD and run at about the same time: groups of G
// consecutive logical blocks are placed on one XCD, physical 8k + x ->
// logical 8G (k / G) + G x + (k mod G), with the largest G in {16, 8, 4, 2}
// that divides the grid into whole rounds (else the identity). Measured on
// MI355X for the 512^2 passes: groups of 8 beat pairs by 3-5%, groups of 16
// beat 8 by another 1% (FP64).
__device__ __forceinline__ unsigned xcd_group_remap(unsigned b, unsigned nb) {
  unsigned G = 16;
  while (G >= 2 && nb % (8 * G) != 0) G >>= 1;
  if (G < 2) return b;
  const unsigned k = b >> 3, x = b & 7;
  return (k / G) * (8 * G) + x * G + (k % G);
}
// Pair slot of this workgroup: grid rows in launch order, or reversed (a.rev).
__device__ __forceinline__ unsigned pair_slot(const PassArgs& a) {
  return a.rev ? gridDim.y - 1 - blockIdx.y : blockIdx.y;
}
template <class T, int N, bool ROWS>
__host__ __device__ constexpr int pass_threads() {
  return pencils_per_group<T, N, ROWS>() * fft_threads(N);
}
// The drifting passes transform the two fields of a pair in lockstep (two
// LDS buffers per pencil) where both buffers of every pencil fit in 80 KB per
// workgroup, so that two workgroups still share a CU; the other passes keep
// one buffer per pencil. Measured on MI355X at 512^2: FP32 drift+rho pass -9%,
// FP32 kick pass -2%, FP64 drift+rho pass -3.5%; the FP64 kick pass, already
// at two wavefronts per SIMD, ran 2.3% slower and keeps one transform at a time.
#ifndef TW_PASS_DUAL
#define TW_PASS_DUAL 1
#endif
__host__ __device__ constexpr bool pass_mode_drifts(int mode) {
  return mode == PASS_DRIFT || mode == PASS_DRIFT_RHO || mode == PASS_KICK_DRIFT;
}
template <class T, int N, bool ROWS, int MODE>
__host__ __device__ constexpr bool pass_dual() {
  return TW_PASS_DUAL && pass_mode_drifts(MODE) && !(sizeof(T) == 8 && MODE == PASS_KICK_DRIFT) &&
         (long)pencils_per_group<T, N, ROWS>() * fft_lds_stride(N) * 4 * (long)sizeof(T) <= 80 * 1024;
}
template <class T, int N, bool ROWS, int MODE>
__host__ __device__ constexpr size_t pass_lds_bytes() {
  return (size_t)pencils_per_group<T, N, ROWS>() * fft_lds_stride(N) * 2 * sizeof(T) *
             (pass_dual<T, N, ROWS, MODE>() ? 2 : 1) +
         16 * sizeof(double);
}

template <class T>
__device__ __forceinline__ cx<T>* field_ptr(const PassArgs& a, int64_t f) {
  return f < a.n_real ? reinterpret_cast<cx<T>*>(a.psi) + f * a.ncell : reinterpret_cast<cx<T>*>(a.psi_cl);
}

template <class T>
__device__ __forceinline__ cx<T>* field_ptr_t(const PassArgs& a, int64_t f) {
  return f < a.n_real ? reinterpret_cast<cx<T>*>(a.psi_t) + f * a.ncell : reinterpret_cast<cx<T>*>(a.psi_cl_t);
}

// Sum of `x` over the workgroup; result valid in thread 0. `red` holds one
// double per wave.
__device__ __forceinline__ double block_sum(double x, double* red) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = x;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; ++w) s += red[w];
  }
  return s;
}

// Max of `x` over the workgroup, result valid in thread 0 (same layout as block_sum).
__device__ __forceinline__ double block_max(double x, double* red) {
  for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off, 64));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = x;
  __syncthreads();
  double m = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; ++w) m = fmax(m, red[w]);
  }
  return m;
}

// Running maximum of non-negative doubles: their bit patterns order like
// unsigned integers, so an integer atomic max is exact and order-independent.
// Workgroups spread their updates over kVmaxBuckets addresses (one address
// for a whole pass serialises thousands of atomics); readers take the max of
// the buckets.
__device__ __forceinline__ void record_max(double* dst, double m) {
  atomicMax(reinterpret_cast<unsigned long long*>(dst), (unsigned long long)__double_as_longlong(m));
}

}  // namespace tw
