// Test particles for the decoherence model (Sec. "Modeling decoherence"):
// every field carries its own particles, which move in that field's own
// potential, dr/dt = v, dv/dt = -grad V(r). They follow the fields' splitting:
// half drift, kick with the potential of the field kick, half drift, in one
// launch after the kick pass (which leaves V_A + i V_B of every pair in the
// pair scratch, in its own storage order). The gradient is the fourth-order
// central difference on the grid, interpolated to the particle linearly
// (cloud-in-cell weights); positions are kept unwrapped and wrapped only to
// find the cell.
#include "common.hpp"
#include "internal.hpp"

namespace tw {

struct TracerArgs {
  const void* z;        // [npairs][N] potentials, V_A + i V_B
  double* tr;           // [nfield][ntracer][2 dim]: positions, then velocities
  int64_t nfield, ntracer;
  int64_t ncell;
  int dim;
  int n[3];             // physical axes
  double box[3];
  int64_t stride[3];    // element stride of each physical axis in the scratch
  double dt;
};

template <class T>
__device__ __forceinline__ double potential_at(const TracerArgs& a, int64_t pair, int comp, const int (&c)[3]) {
  int64_t off = 0;
  for (int d = 0; d < a.dim; ++d) off += (int64_t)c[d] * a.stride[d];
  const cx<T> v = reinterpret_cast<const cx<T>*>(a.z)[pair * a.ncell + off];
  return comp ? (double)v.im : (double)v.re;
}

template <class T>
__global__ void __launch_bounds__(256) tracer_kernel(TracerArgs a) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= a.nfield * a.ntracer) return;
  const int64_t f = idx / a.ntracer;
  const int64_t pair = f / 2;
  const int comp = (int)(f % 2);
  double* p = a.tr + idx * 2 * a.dim;
  const int D = a.dim;
  double r[3], v[3];
  for (int d = 0; d < D; ++d) {
    v[d] = p[D + d];
    r[d] = p[d] + 0.5 * a.dt * v[d];
  }
  // cell and weights of the wrapped midpoint position
  int base[3] = {0, 0, 0};
  double frac[3] = {0.0, 0.0, 0.0};
  for (int d = 0; d < D; ++d) {
    const double L = a.box[d];
    const double u = r[d] - L * floor(r[d] / L);
    const double sc = u / (L / (double)a.n[d]);
    const double i0 = floor(sc);
    base[d] = (int)i0;
    frac[d] = sc - i0;
  }
  double g[3] = {0.0, 0.0, 0.0};
  for (int corner = 0; corner < (1 << D); ++corner) {
    double w = 1.0;
    int c[3] = {0, 0, 0};
    for (int d = 0; d < D; ++d) {
      const int bit = (corner >> d) & 1;
      w *= bit ? frac[d] : 1.0 - frac[d];
      c[d] = (base[d] + bit) % a.n[d];
    }
    for (int d = 0; d < D; ++d) {
      int q[3] = {c[0], c[1], c[2]};
      auto at = [&](int s) {
        q[d] = ((c[d] + s) % a.n[d] + a.n[d]) % a.n[d];
        return potential_at<T>(a, pair, comp, q);
      };
      const double dx = a.box[d] / (double)a.n[d];
      const double gd = (-at(2) + 8.0 * at(1) - 8.0 * at(-1) + at(-2)) / (12.0 * dx);
      g[d] += w * gd;
    }
  }
  for (int d = 0; d < D; ++d) {
    v[d] -= a.dt * g[d];
    p[D + d] = v[d];
    p[d] = r[d] + 0.5 * a.dt * v[d];
  }
}

hipError_t launch_tracers(const Plan& P, double* tr, int64_t nfield, int64_t ntracer, const int perm[3], double dt,
                          hipStream_t s) {
  TracerArgs a;
  a.z = P.z;
  a.tr = tr;
  a.nfield = nfield;
  a.ntracer = ntracer;
  a.ncell = P.ncell;
  a.dim = P.dim;
  int64_t st = 1;
  for (int k = 0; k < 3; ++k) {
    a.n[k] = P.n[k];
    a.box[k] = k < P.dim ? P.p.box[k] : 1.0;
    a.stride[k] = 0;
  }
  for (int k = 0; k < P.dim; ++k) {  // storage order: perm[0] fastest
    a.stride[perm[k]] = st;
    st *= P.n[perm[k]];
  }
  a.dt = dt;
  const int64_t total = nfield * ntracer;
  if (total <= 0) return hipSuccess;
  dim3 grid((unsigned)((total + 255) / 256));
  if (P.fp32) hipLaunchKernelGGL(tracer_kernel<float>, grid, dim3(256), 0, s, a);
  else hipLaunchKernelGGL(tracer_kernel<double>, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

// Plug-in variances over the realizations of every particle coordinate:
// out[i][k] for k < 2 dim (positions, then velocities).
__global__ void __launch_bounds__(256) tracer_spread_kernel(const double* __restrict__ tr, int64_t n_real,
                                                            int64_t ntracer, int width, double* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ntracer * width) return;
  const int64_t i = idx / width;
  const int k = (int)(idx % width);
  double m = 0.0;
  for (int64_t r = 0; r < n_real; ++r) m += tr[(r * ntracer + i) * width + k];
  m /= (double)n_real;
  double v = 0.0;
  for (int64_t r = 0; r < n_real; ++r) {
    const double d = tr[(r * ntracer + i) * width + k] - m;
    v += d * d;
  }
  out[idx] = v / (double)n_real;
}

hipError_t launch_tracer_spread(const Plan& P, const double* tr, int64_t ntracer, double* out, hipStream_t s) {
  const int width = 2 * P.dim;
  const int64_t total = ntracer * width;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(tracer_spread_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, tr,
                     (int64_t)P.p.n_real, ntracer, width, out);
  return hipGetLastError();
}

}  // namespace tw
