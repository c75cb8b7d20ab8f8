// Wigner sampling of the initial ensemble (Sec. "Initial conditions generation",
// Eq. (sample)): psi_i(x_g) = psi_cl(x_g) + complex Gaussian noise.
//
// This translation unit is compiled with -ffp-contract=off and uses no library
// transcendental: every floating-point result is a fixed sequence of correctly
// rounded IEEE-754 double operations, so the draw is bit-reproducible from
// (seed, realization, cell) on any conforming implementation.
//
// Generator: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), counter
// (g, r, 0, 0), key (seed, 0x5457). Words 0 and 1 become uniforms
// u = (floor(x / 2^12) + 1/2) 2^-52 and feed the Box-Muller transform
// z1 = sqrt(-2 ln u1) cos(2 pi u2), z2 = sqrt(-2 ln u1) sin(2 pi u2), with
//   ln u  : u = m 2^e, m in [sqrt(1/2), sqrt(2)), s = (m-1)/(m+1),
//           ln m = 2 s sum_{k<=12} s^{2k}/(2k+1) (Horner from k = 12), ln u = e ln2 + ln m;
//   angle : t = 4 u2, q = floor(t), f = t - q, f > 1/2 -> (f - 1, q + 1), theta = f pi/2;
//           sin theta = theta prod-form Taylor series to theta^21, cos theta to theta^20
//           (each factor multiplies by the correctly rounded reciprocal of
//           (2k)(2k+1) or (2k-1)(2k)), rotated by q quarter turns.
#include "common.hpp"
#include "internal.hpp"

#pragma clang fp contract(off)

namespace tw {
namespace {

constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kM1 = 0xCA5A826395121157ull;
constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kW1 = 0xBB67AE8584CAA73Bull;
constexpr uint64_t kSampleTag = 0x5457ull;

struct u64x4 {
  uint64_t w[4];
};

__device__ __forceinline__ u64x4 philox4x64_10(u64x4 x, uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += kW0;
      k1 += kW1;
    }
    const uint64_t hi0 = __umul64hi(kM0, x.w[0]);
    const uint64_t lo0 = kM0 * x.w[0];
    const uint64_t hi1 = __umul64hi(kM1, x.w[2]);
    const uint64_t lo1 = kM1 * x.w[2];
    u64x4 y;
    y.w[0] = hi1 ^ x.w[1] ^ k0;
    y.w[1] = lo1;
    y.w[2] = hi0 ^ x.w[3] ^ k1;
    y.w[3] = lo0;
    x = y;
  }
  return x;
}

__device__ __forceinline__ double to_unit(uint64_t x) {
  return ((double)(x >> 12) + 0.5) * 0x1p-52;
}

__device__ double ln_unit(double u) {
  const double kLn2 = 0.6931471805599453;
  const double kSqrtHalf = 0.7071067811865476;
  int e;
  double m = frexp(u, &e);  // u = m 2^e, m in [1/2, 1)
  if (m < kSqrtHalf) {
    m = m * 2.0;
    e = e - 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double t = s * s;
  double p = 1.0 / 25.0;
  for (int k = 11; k >= 0; --k) p = p * t + 1.0 / (double)(2 * k + 1);
  const double lnm = (s + s) * p;
  return (double)e * kLn2 + lnm;
}

__device__ void cos_sin_turn(double u, double* c_out, double* s_out) {
  const double kHalfPi = 1.5707963267948966;
  const double t4 = 4.0 * u;
  double q = floor(t4);
  double f = t4 - q;
  if (f > 0.5) {
    f = f - 1.0;
    q = q + 1.0;
  }
  const double th = f * kHalfPi;
  const double th2 = th * th;
  double ps = 1.0, pc = 1.0;
#pragma unroll
  for (int k = 10; k >= 1; --k) {
    // times the correctly rounded reciprocal of the factorial ratio (a constant)
    ps = 1.0 - (ps * th2) * (1.0 / (double)((2 * k) * (2 * k + 1)));
    pc = 1.0 - (pc * th2) * (1.0 / (double)((2 * k - 1) * (2 * k)));
  }
  const double s = th * ps;
  const double c = pc;
  switch (((int)q) & 3) {
    case 0: *c_out = c; *s_out = s; break;
    case 1: *c_out = -s; *s_out = c; break;
    case 2: *c_out = -c; *s_out = -s; break;
    default: *c_out = s; *s_out = -c; break;
  }
}

template <class T>
__global__ void __launch_bounds__(256) sample_kernel(const cx<double>* __restrict__ psi_cl, cx<T>* __restrict__ psi,
                                                     int64_t ncell, uint64_t seed, int64_t real_offset, double sc) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = blockIdx.y;
  if (g >= ncell) return;
  u64x4 ctr;
  ctr.w[0] = (uint64_t)g;
  ctr.w[1] = (uint64_t)(real_offset + r);
  ctr.w[2] = 0;
  ctr.w[3] = 0;
  const u64x4 out = philox4x64_10(ctr, seed, kSampleTag);
  const double u1 = to_unit(out.w[0]);
  const double u2 = to_unit(out.w[1]);
  const double rad = sqrt(-2.0 * ln_unit(u1));
  double c, s;
  cos_sin_turn(u2, &c, &s);
  const double z1 = rad * c;
  const double z2 = rad * s;
  const cx<double> cl = psi_cl[g];
  const double re = cl.re + z1 * sc;
  const double im = cl.im + z2 * sc;
  psi[r * ncell + g] = cx<T>{(T)re, (T)im};
}

}  // namespace

hipError_t launch_sample(const Plan& P, const void* psi_cl, uint64_t seed, int64_t real_offset, void* psi,
                         hipStream_t s) {
  const double sc = 0.5 / sqrt(P.p.n_tot * P.dV);
  dim3 grid((unsigned)((P.ncell + 255) / 256), (unsigned)P.p.n_real);
  if (P.fp32)
    hipLaunchKernelGGL(sample_kernel<float>, grid, dim3(256), 0, s, reinterpret_cast<const cx<double>*>(psi_cl),
                       reinterpret_cast<cx<float>*>(psi), P.ncell, seed, real_offset, sc);
  else
    hipLaunchKernelGGL(sample_kernel<double>, grid, dim3(256), 0, s, reinterpret_cast<const cx<double>*>(psi_cl),
                       reinterpret_cast<cx<double>*>(psi), P.ncell, seed, real_offset, sc);
  return hipGetLastError();
}

}  // namespace tw
