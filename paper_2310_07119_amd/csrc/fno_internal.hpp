// Internal interfaces of the FNO surrogate kernels (kernels_fno.hip) used by
// the host orchestration in fno.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tw {

// C[b] = beta C[b] + alpha A[b] B[b]; element (m, k) of A[b] is A[b*sAb + m*sAm + k*sAk], etc.
struct GemmArgs {
  const float* A;
  const float* B;
  float* C;
  int64_t M, N, K, batch;
  int64_t sAb, sAm, sAk;
  int64_t sBb, sBk, sBn;
  int64_t sCb, sCm, sCn;
  float alpha, beta;
  // Epilogue, applied to r = beta C + alpha A B (all optional): r += add[b, m, n]
  // (same strides as C) and r += bias[n]; with gz, g = r GELU'(gz[b, m, n])
  // replaces r in C if gz_into_c; out2[b, m, n] (strides of C) receives g
  // with gz, else GELU(r) if act, else r.
  const float* add;
  const float* bias;
  const float* gz;
  float* out2;
  int32_t act;
  int32_t gz_into_c;
  int32_t a_vec;    // set by launch_gemm: A staged with four-element loads
  int32_t row_epi;  // set by launch_gemm: width-32 tiles write the epilogue as whole rows through LDS
};

hipError_t launch_gemm(const GemmArgs& g, hipStream_t s);
hipError_t launch_colsum(const float* x, int64_t P, int C, float* out, int accumulate, float* parts,
                         int64_t parts_len, double* tmp, hipStream_t st);
// the output projection with one or two channels (forward, and backward to
// the hidden layer with GELU'), and the weighted column sums of its weight gradient
hipError_t launch_proj_out(const float* h, const float* w, const float* b, float* y, int64_t M, int K, int nout,
                           hipStream_t st);
hipError_t launch_proj_out_back(const float* dy, const float* w, const float* z, float* dz, int64_t M, int N,
                                int nout, hipStream_t st);
hipError_t launch_colsum_weighted(const float* x, const float* wt, int nw, int64_t P, int C, float* out, float* parts,
                                  int64_t parts_len, double* tmp, hipStream_t st);
hipError_t launch_sum_parts(const float* parts, int nparts, int64_t n, float* out, int accumulate, hipStream_t st,
                            double* tmp);  // tmp: [ceil(nparts/32)][n] FP64 sub-totals, or NULL
hipError_t launch_modemix_fwd(const float* br, const float* bi, const float* Rr, const float* Ri, float* cr,
                              float* ci, int nb, int nmode, int C, hipStream_t st);
hipError_t launch_modemix_bwd(const float* br, const float* bi, const float* dcr, const float* dci, const float* Rr,
                              const float* Ri, float* dbr, float* dbi, float* dRr, float* dRi, int nb, int nmode,
                              int C, hipStream_t st);
hipError_t launch_mse(const float* y, const float* t, int64_t n, float* dy, float* loss, hipStream_t st);
hipError_t launch_adam(float* th, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, int64_t step, hipStream_t st);
hipError_t launch_init(float* p, int64_t n, uint64_t seed, float lo, float hi, hipStream_t st);

}  // namespace tw
