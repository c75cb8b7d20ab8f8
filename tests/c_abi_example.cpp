// The C ABI used directly, without the Python binding: a small 2D ensemble is
// sampled, stepped (with its classical field) and reduced through tw.h and the
// HIP runtime only. Writes the coherent field, the final fields and the
// moment scalars to a binary file for tests/test_gpu_c_abi.py to check against
// the oracle.
//   usage: tw_c_example <output file>
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "tw.h"

#define CHECK_TW(call)                                                    \
  do {                                                                    \
    int rc_ = (call);                                                     \
    if (rc_ != TW_OK) {                                                   \
      fprintf(stderr, "%s failed (%d): %s\n", #call, rc_, tw_last_error()); \
      return 1;                                                           \
    }                                                                     \
  } while (0)
#define CHECK_HIP(call)                                                          \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess) {                                                      \
      fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));          \
      return 1;                                                                  \
    }                                                                            \
  } while (0)

int main(int argc, char** argv) {
  if (argc != 2) {
    fprintf(stderr, "usage: %s <output file>\n", argv[0]);
    return 2;
  }
  const int nx = 64, ny = 32, nreal = 3, nsteps = 6;
  const long ncell = (long)nx * ny;
  tw_problem p = {};
  p.dim = 2;
  p.n[0] = nx;
  p.n[1] = ny;
  p.n[2] = 1;
  p.box[0] = 1.0;
  p.box[1] = 0.5;
  p.box[2] = 1.0;
  p.hbar_m = 1.0;
  p.G = 1.0;
  p.m_tot = 20.0;
  p.n_tot = 1e5;
  p.n_real = nreal;
  p.precision = TW_FP64;
  tw_plan plan = nullptr;
  CHECK_TW(tw_plan_create(&p, &plan));

  // coherent field: a smooth positive density, normalised to sum |psi|^2 dV = 1
  double* cl = (double*)malloc(sizeof(double) * 2 * ncell);
  const double dv = (1.0 / nx) * (0.5 / ny);
  double norm = 0.0;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const double rho = 1.0 + 0.3 * cos(2.0 * M_PI * x / nx) + 0.2 * sin(2.0 * M_PI * y / ny);
      cl[2 * (y * nx + x)] = sqrt(rho);
      cl[2 * (y * nx + x) + 1] = 0.0;
      norm += rho * dv;
    }
  for (long g = 0; g < 2 * ncell; ++g) cl[g] /= sqrt(norm);

  void *d_cl, *d_psi, *d_cl_t;
  double *d_scal, *d_norm;
  CHECK_HIP(hipMalloc(&d_cl, sizeof(double) * 2 * ncell));
  CHECK_HIP(hipMalloc(&d_cl_t, sizeof(double) * 2 * ncell));
  CHECK_HIP(hipMalloc(&d_psi, sizeof(double) * 2 * ncell * nreal));
  CHECK_HIP(hipMalloc(&d_scal, sizeof(double) * 8));
  CHECK_HIP(hipMalloc(&d_norm, sizeof(double) * nreal));
  CHECK_HIP(hipMemcpy(d_cl, cl, sizeof(double) * 2 * ncell, hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(d_cl_t, cl, sizeof(double) * 2 * ncell, hipMemcpyHostToDevice));
  hipStream_t s;
  CHECK_HIP(hipStreamCreate(&s));

  CHECK_TW(tw_sample(plan, d_cl, 7, 0, d_psi, s));
  CHECK_TW(tw_step(plan, d_psi, d_cl_t, nsteps, 2e-4, s));
  tw_moments_out out = {};
  out.scalars = d_scal;
  out.norm = d_norm;
  CHECK_TW(tw_moments(plan, d_psi, d_cl_t, &out, s));
  CHECK_HIP(hipStreamSynchronize(s));

  double* psi = (double*)malloc(sizeof(double) * 2 * ncell * nreal);
  double* clt = (double*)malloc(sizeof(double) * 2 * ncell);
  double scal[8];
  CHECK_HIP(hipMemcpy(psi, d_psi, sizeof(double) * 2 * ncell * nreal, hipMemcpyDeviceToHost));
  CHECK_HIP(hipMemcpy(clt, d_cl_t, sizeof(double) * 2 * ncell, hipMemcpyDeviceToHost));
  CHECK_HIP(hipMemcpy(scal, d_scal, sizeof(scal), hipMemcpyDeviceToHost));

  FILE* f = fopen(argv[1], "wb");
  if (!f) {
    fprintf(stderr, "cannot open %s\n", argv[1]);
    return 1;
  }
  fwrite(cl, sizeof(double), 2 * ncell, f);
  fwrite(psi, sizeof(double), 2 * ncell * nreal, f);
  fwrite(clt, sizeof(double), 2 * ncell, f);
  fwrite(scal, sizeof(double), 8, f);
  fclose(f);
  printf("Q_raw %.17g norm_mean %.17g\n", scal[0], scal[5]);

  CHECK_TW(tw_plan_destroy(plan));
  hipFree(d_cl);
  hipFree(d_cl_t);
  hipFree(d_psi);
  hipFree(d_scal);
  hipFree(d_norm);
  hipStreamDestroy(s);
  free(cl);
  free(psi);
  free(clt);
  return 0;
}
