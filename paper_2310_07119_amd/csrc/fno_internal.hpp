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
};

hipError_t launch_gemm(const GemmArgs& g, hipStream_t s);
hipError_t launch_bias_act(float* u, const float* s, const float* bias, float* v, int64_t n, int C, int act,
                           hipStream_t st);
hipError_t launch_gelu_back(const float* g, const float* z, float* d, int64_t n, hipStream_t st);
hipError_t launch_colsum(const float* x, int64_t P, int C, float* out, int accumulate, float* parts,
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
