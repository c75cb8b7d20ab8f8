// Fourier-neural-operator surrogate: host orchestration of the forward and
// hand-written backward passes (kernels in kernels_fno.hip) behind the
// tw_fno_* C ABI.
//
// Network (Li et al., 2020): lift (c_in -> C, pointwise), L Fourier layers
//   u_l = S_l(v_l) + v_l W_l + b_l,   v_{l+1} = GELU(u_l) (identity after the last)
// with S_l(v) = inverse DFT of R_l times the DFT of v restricted to the modes
// kx < mx (real half-spectrum) and ky in {0..my-1, H-my..H-1}, then a
// projection C -> proj -> c_out with GELU in between. Every dense contraction
// (pointwise layers, the four truncated DFT stages, weight gradients) runs on
// the BF16 matrix-core GEMM; the pointwise GEMMs add the bias and the
// spectral branch and apply GELU (forward) or GELU' (backward) in their
// epilogue, in FP32; mode mixing runs in FP32, reductions in FP64. With one
// or two output channels the last projection's three contractions (dot
// products per position, their outer-product backward, weighted column sums)
// are streaming kernels on the same BF16-rounded operands.
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <utility>
#include <vector>

#include "fno_internal.hpp"
#include "internal.hpp"

namespace tw {
namespace {

thread_local std::string g_fno_error;

int ffail(int code, const char* msg) {
  g_fno_error = msg;
  return code;
}

#define FNO_HIP(expr)                                   \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return ffail(TW_EHIP, #expr); \
  } while (0)

struct Layout {  // offsets (floats) of every parameter tensor in the flat buffer
  int64_t lift_w, lift_b, q1_w, q1_b, q2_w, q2_b, total;
  int64_t Rre[8], Rim[8], W[8], b[8];
};

Layout make_layout(const tw_fno_config& c) {
  Layout L;
  const int64_t C = c.width, nm = 2LL * c.modes_y * c.modes_x;
  int64_t o = 0;
  L.lift_w = o; o += (int64_t)c.c_in * C;
  L.lift_b = o; o += C;
  for (int l = 0; l < c.layers; ++l) {
    L.Rre[l] = o; o += nm * C * C;
    L.Rim[l] = o; o += nm * C * C;
    L.W[l] = o; o += C * C;
    L.b[l] = o; o += C;
  }
  L.q1_w = o; o += C * c.proj;
  L.q1_b = o; o += c.proj;
  L.q2_w = o; o += (int64_t)c.proj * c.c_out;
  L.q2_b = o; o += c.c_out;
  L.total = o;
  return L;
}

struct Fno {
  tw_fno_config cfg;
  Layout L;
  int max_batch;
  // DFT matrices (FP32, rounded to BF16 where the GEMM reads them)
  float *f1_re, *f1_im;   // [W][mx]
  float *e2_re, *e2_im;   // [2my][H]
  float *e4_re, *e4_im;   // [H][2my]
  float *g5_re, *g5_im;   // [mx][W]
  // activations saved by the forward (for max_batch fields)
  float* v;      // [L+1][P][C]
  float* u;      // [L][P][C]
  float* bsav;   // [L][2][B][2my][mx][C]  (re, im)
  float* z1;     // [P][proj]
  float* h;      // [P][proj]
  // temporaries
  float *s, *t1, *t2;                 // [P][C]
  float *a_re, *a_im, *d_re, *d_im;   // [B][H][mx][C]
  float *c_re, *c_im, *bb_re, *bb_im; // [B][2my][mx][C]
  float* dz;     // [P][proj]
  float* parts;  // split-K partials
  int64_t parts_len;
  double* parts2;  // FP64 sub-totals of groups of 32 partials
  void* block;   // single allocation
};

int64_t positions(const Fno& F, int batch) { return (int64_t)batch * F.cfg.H * F.cfg.W; }

// Epilogue of a GEMM (GemmArgs): bias and added matrix, a second output with
// GELU, or a GELU' factor (the fused pointwise layers).
struct Epi {
  const float* add = nullptr;
  const float* bias = nullptr;
  const float* gz = nullptr;
  float* out2 = nullptr;
  int act = 0;
  int gz_into_c = 0;
};

hipError_t gemm(hipStream_t s, int64_t M, int64_t N, int64_t K, float alpha, const float* A, int64_t sAm,
                int64_t sAk, const float* B, int64_t sBk, int64_t sBn, float beta, float* C, int64_t sCm,
                int64_t sCn, int64_t batch = 1, int64_t sAb = 0, int64_t sBb = 0, int64_t sCb = 0,
                const Epi& epi = Epi()) {
  GemmArgs g;
  std::memset(&g, 0, sizeof(g));
  g.add = epi.add; g.bias = epi.bias; g.gz = epi.gz; g.out2 = epi.out2;
  g.act = epi.act; g.gz_into_c = epi.gz_into_c;
  g.A = A; g.B = B; g.C = C;
  g.M = M; g.N = N; g.K = K; g.batch = batch;
  g.sAb = sAb; g.sAm = sAm; g.sAk = sAk;
  g.sBb = sBb; g.sBk = sBk; g.sBn = sBn;
  g.sCb = sCb; g.sCm = sCm; g.sCn = sCn;
  g.alpha = alpha; g.beta = beta;
  return launch_gemm(g, s);
}

// dW[M x N] = A^T B summed over P positions, A = [P][M] rows, B = [P][N] rows,
// split over K (positions) into partials that are then summed (FP64). The
// weight matrices are one or two tiles, so the split supplies the parallelism:
// chunks of 512 positions give ~1000 workgroups at 256^2 x 8 fields (chunks of
// 8192 left three quarters of the chip idle and made these the slowest GEMMs).
hipError_t weight_grad(Fno& F, hipStream_t s, int64_t P, int64_t M, int64_t N, const float* A, const float* B,
                       float* out) {
  int64_t chunk = std::gcd(P, (int64_t)512);
  int64_t nsplit = P / chunk;
  while (nsplit * M * N > F.parts_len || nsplit > 65535) {  // coarser split if the partial buffer is short
    chunk *= 2;
    if (P % chunk != 0) return hipErrorInvalidValue;
    nsplit = P / chunk;
  }
  hipError_t e = gemm(s, M, N, chunk, 1.f, A, 1, M, B, N, 1, 0.f, F.parts, N, 1, nsplit, chunk * M, chunk * N, M * N);
  if (e != hipSuccess) return e;
  return launch_sum_parts(F.parts, (int)nsplit, M * N, out, 0, s, F.parts2);
}

// S(v) -> out, saving the y-transformed input (bsav) for the backward.
int spectral_fwd(Fno& F, hipStream_t s, int batch, const float* v, const float* Rre, const float* Rim, float* bsav_re,
                 float* bsav_im, float* out) {
  const tw_fno_config& c = F.cfg;
  const int64_t H = c.H, W = c.W, C = c.width, mx = c.modes_x, K2 = 2LL * c.modes_y;
  const int64_t nby = (int64_t)batch * H;
  // stage 1 (along x), batched over (b, y): A[kx][c] = sum_x F1[x][kx] v[x][c]
  FNO_HIP(gemm(s, mx, C, W, 1.f, F.f1_re, 1, mx, v, C, 1, 0.f, F.a_re, C, 1, nby, 0, W * C, mx * C));
  FNO_HIP(gemm(s, mx, C, W, 1.f, F.f1_im, 1, mx, v, C, 1, 0.f, F.a_im, C, 1, nby, 0, W * C, mx * C));
  // stage 2 (along y), batched over b: B = E2 A (complex)
  const int64_t nc = mx * C;
  FNO_HIP(gemm(s, K2, nc, H, 1.f, F.e2_re, H, 1, F.a_re, nc, 1, 0.f, bsav_re, nc, 1, batch, 0, H * nc, K2 * nc));
  FNO_HIP(gemm(s, K2, nc, H, -1.f, F.e2_im, H, 1, F.a_im, nc, 1, 1.f, bsav_re, nc, 1, batch, 0, H * nc, K2 * nc));
  FNO_HIP(gemm(s, K2, nc, H, 1.f, F.e2_re, H, 1, F.a_im, nc, 1, 0.f, bsav_im, nc, 1, batch, 0, H * nc, K2 * nc));
  FNO_HIP(gemm(s, K2, nc, H, 1.f, F.e2_im, H, 1, F.a_re, nc, 1, 1.f, bsav_im, nc, 1, batch, 0, H * nc, K2 * nc));
  // stage 3: mode mixing
  FNO_HIP(launch_modemix_fwd(bsav_re, bsav_im, Rre, Rim, F.c_re, F.c_im, batch, (int)(K2 * mx), (int)C, s));
  // stage 4 (inverse along y): D = E4 Cm
  FNO_HIP(gemm(s, H, nc, K2, 1.f, F.e4_re, K2, 1, F.c_re, nc, 1, 0.f, F.d_re, nc, 1, batch, 0, K2 * nc, H * nc));
  FNO_HIP(gemm(s, H, nc, K2, -1.f, F.e4_im, K2, 1, F.c_im, nc, 1, 1.f, F.d_re, nc, 1, batch, 0, K2 * nc, H * nc));
  FNO_HIP(gemm(s, H, nc, K2, 1.f, F.e4_re, K2, 1, F.c_im, nc, 1, 0.f, F.d_im, nc, 1, batch, 0, K2 * nc, H * nc));
  FNO_HIP(gemm(s, H, nc, K2, 1.f, F.e4_im, K2, 1, F.c_re, nc, 1, 1.f, F.d_im, nc, 1, batch, 0, K2 * nc, H * nc));
  // stage 5 (inverse along x), batched over (b, y): s[x][o] = sum_kx G5[kx][x] D[kx][o]
  FNO_HIP(gemm(s, W, C, mx, 1.f, F.g5_re, 1, W, F.d_re, C, 1, 0.f, out, C, 1, nby, 0, mx * C, W * C));
  FNO_HIP(gemm(s, W, C, mx, 1.f, F.g5_im, 1, W, F.d_im, C, 1, 1.f, out, C, 1, nby, 0, mx * C, W * C));
  return TW_OK;
}

// Adjoint of S: ds -> dv_out (overwritten), dR (overwritten).
int spectral_bwd(Fno& F, hipStream_t s, int batch, const float* ds, const float* bsav_re, const float* bsav_im,
                 const float* Rre, const float* Rim, float* dRre, float* dRim, float* dv_out) {
  const tw_fno_config& c = F.cfg;
  const int64_t H = c.H, W = c.W, C = c.width, mx = c.modes_x, K2 = 2LL * c.modes_y;
  const int64_t nby = (int64_t)batch * H, nc = mx * C;
  // stage 5 adjoint: dD[kx][c] = sum_x G5[kx][x] ds[x][c]
  FNO_HIP(gemm(s, mx, C, W, 1.f, F.g5_re, W, 1, ds, C, 1, 0.f, F.d_re, C, 1, nby, 0, W * C, mx * C));
  FNO_HIP(gemm(s, mx, C, W, 1.f, F.g5_im, W, 1, ds, C, 1, 0.f, F.d_im, C, 1, nby, 0, W * C, mx * C));
  // stage 4 adjoint: dC = E4^H dD  (E4^T element (k, y) = e4[y][k])
  FNO_HIP(gemm(s, K2, nc, H, 1.f, F.e4_re, 1, K2, F.d_re, nc, 1, 0.f, F.c_re, nc, 1, batch, 0, H * nc, K2 * nc));
  FNO_HIP(gemm(s, K2, nc, H, 1.f, F.e4_im, 1, K2, F.d_im, nc, 1, 1.f, F.c_re, nc, 1, batch, 0, H * nc, K2 * nc));
  FNO_HIP(gemm(s, K2, nc, H, 1.f, F.e4_re, 1, K2, F.d_im, nc, 1, 0.f, F.c_im, nc, 1, batch, 0, H * nc, K2 * nc));
  FNO_HIP(gemm(s, K2, nc, H, -1.f, F.e4_im, 1, K2, F.d_re, nc, 1, 1.f, F.c_im, nc, 1, batch, 0, H * nc, K2 * nc));
  // stage 3 adjoint
  FNO_HIP(launch_modemix_bwd(bsav_re, bsav_im, F.c_re, F.c_im, Rre, Rim, F.bb_re, F.bb_im, dRre, dRim, batch,
                             (int)(K2 * mx), (int)C, s));
  // stage 2 adjoint: dA = E2^H dB  (E2^T element (y, k) = e2[k][y])
  FNO_HIP(gemm(s, H, nc, K2, 1.f, F.e2_re, 1, H, F.bb_re, nc, 1, 0.f, F.a_re, nc, 1, batch, 0, K2 * nc, H * nc));
  FNO_HIP(gemm(s, H, nc, K2, 1.f, F.e2_im, 1, H, F.bb_im, nc, 1, 1.f, F.a_re, nc, 1, batch, 0, K2 * nc, H * nc));
  FNO_HIP(gemm(s, H, nc, K2, 1.f, F.e2_re, 1, H, F.bb_im, nc, 1, 0.f, F.a_im, nc, 1, batch, 0, K2 * nc, H * nc));
  FNO_HIP(gemm(s, H, nc, K2, -1.f, F.e2_im, 1, H, F.bb_re, nc, 1, 1.f, F.a_im, nc, 1, batch, 0, K2 * nc, H * nc));
  // stage 1 adjoint: dv[x][c] = sum_kx F1[x][kx] dA_re[kx][c] + F1im[x][kx] dA_im[kx][c]
  FNO_HIP(gemm(s, W, C, mx, 1.f, F.f1_re, mx, 1, F.a_re, C, 1, 0.f, dv_out, C, 1, nby, 0, mx * C, W * C));
  FNO_HIP(gemm(s, W, C, mx, 1.f, F.f1_im, mx, 1, F.a_im, C, 1, 1.f, dv_out, C, 1, nby, 0, mx * C, W * C));
  return TW_OK;
}

void fno_free(Fno* F) {
  if (!F) return;
  if (F->block) (void)hipFree(F->block);
  delete F;
}

}  // namespace
}  // namespace tw

using namespace tw;

extern "C" {

const char* tw_fno_last_error(void) { return g_fno_error.c_str(); }

int64_t tw_fno_param_count(const tw_fno_config* c) {
  if (!c) return -1;
  return make_layout(*c).total;
}

int tw_fno_create(const tw_fno_config* cfg, int32_t max_batch, tw_fno* out) {
  if (!cfg || !out) return ffail(TW_EINVAL, "NULL config or output pointer");
  *out = nullptr;
  const tw_fno_config& c = *cfg;
  if (c.H < 2 || c.W < 2 || c.c_in < 1 || c.width < 1 || c.proj < 1 || c.c_out < 1 || c.layers < 1 ||
      c.layers > 8 || c.modes_x < 1 || c.modes_y < 1 || max_batch < 1)
    return ffail(TW_EINVAL, "bad FNO configuration");
  if (c.modes_x >= c.W / 2 + 1 || 2 * c.modes_y > c.H) return ffail(TW_EINVAL, "too many modes for the grid");
  if ((int64_t)max_batch * c.H > 65535) return ffail(TW_EUNSUPPORTED, "max_batch * H must be <= 65535");
  Fno* F = new (std::nothrow) Fno();
  if (!F) return ffail(TW_ENOMEM, "host allocation failed");
  std::memset(static_cast<void*>(F), 0, sizeof(Fno));
  F->cfg = c;
  F->L = make_layout(c);
  F->max_batch = max_batch;
  const int64_t H = c.H, W = c.W, C = c.width, mx = c.modes_x, K2 = 2LL * c.modes_y, Lyr = c.layers;
  const int64_t P = (int64_t)max_batch * H * W;
  const int64_t big = std::max<int64_t>(C, c.proj);
  F->parts_len = 1024 * big * big;
  struct Piece {
    float** p;
    int64_t n;
  } pieces[] = {
      {&F->f1_re, W * mx}, {&F->f1_im, W * mx}, {&F->e2_re, K2 * H}, {&F->e2_im, K2 * H},
      {&F->e4_re, H * K2}, {&F->e4_im, H * K2}, {&F->g5_re, mx * W}, {&F->g5_im, mx * W},
      {&F->v, (Lyr + 1) * P * C}, {&F->u, Lyr * P * C}, {&F->bsav, Lyr * 2 * max_batch * K2 * mx * C},
      {&F->z1, P * c.proj}, {&F->h, P * c.proj}, {&F->s, P * C}, {&F->t1, P * C}, {&F->t2, P * C},
      {&F->a_re, max_batch * H * mx * C}, {&F->a_im, max_batch * H * mx * C},
      {&F->d_re, max_batch * H * mx * C}, {&F->d_im, max_batch * H * mx * C},
      {&F->c_re, max_batch * K2 * mx * C}, {&F->c_im, max_batch * K2 * mx * C},
      {&F->bb_re, max_batch * K2 * mx * C}, {&F->bb_im, max_batch * K2 * mx * C},
      {&F->dz, P * std::max<int64_t>(c.proj, c.c_out)}, {&F->parts, F->parts_len},
      {reinterpret_cast<float**>(&F->parts2), F->parts_len / 8}};  // ceil(nsplit/32) M N doubles
  int64_t total = 0;
  for (auto& pc : pieces) total += (pc.n + 63) / 64 * 64;
  if (hipMalloc(&F->block, sizeof(float) * total) != hipSuccess) {
    (void)hipGetLastError();
    delete F;
    return ffail(TW_ENOMEM, "workspace allocation failed");
  }
  float* base = static_cast<float*>(F->block);
  for (auto& pc : pieces) {
    *pc.p = base;
    base += (pc.n + 63) / 64 * 64;
  }
  // DFT matrices (FP64 angles, stored FP32)
  std::vector<float> f1r(W * mx), f1i(W * mx), e2r(K2 * H), e2i(K2 * H), e4r(H * K2), e4i(H * K2), g5r(mx * W),
      g5i(mx * W);
  const double tp = 6.283185307179586476925286766559;
  for (int64_t x = 0; x < W; ++x)
    for (int64_t k = 0; k < mx; ++k) {
      const double a = tp * (double)((x * k) % W) / (double)W;
      f1r[x * mx + k] = (float)std::cos(a);
      f1i[x * mx + k] = (float)(-std::sin(a));
      const double wk = (k == 0 ? 1.0 : 2.0) / (double)(H * W);
      g5r[k * W + x] = (float)(wk * std::cos(a));
      g5i[k * W + x] = (float)(-wk * std::sin(a));
    }
  for (int64_t q = 0; q < K2; ++q) {
    const int64_t ky = q < c.modes_y ? q : H - K2 + q;
    for (int64_t y = 0; y < H; ++y) {
      const double a = tp * (double)((ky * y) % H) / (double)H;
      e2r[q * H + y] = (float)std::cos(a);
      e2i[q * H + y] = (float)(-std::sin(a));
      e4r[y * K2 + q] = (float)std::cos(a);
      e4i[y * K2 + q] = (float)std::sin(a);
    }
  }
  bool ok = true;
  auto up = [&](float* d, const std::vector<float>& h) {
    ok = ok && hipMemcpy(d, h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice) == hipSuccess;
  };
  up(F->f1_re, f1r); up(F->f1_im, f1i); up(F->e2_re, e2r); up(F->e2_im, e2i);
  up(F->e4_re, e4r); up(F->e4_im, e4i); up(F->g5_re, g5r); up(F->g5_im, g5i);
  if (!ok) {
    fno_free(F);
    return ffail(TW_EHIP, "table upload failed");
  }
  *out = reinterpret_cast<tw_fno>(F);
  return TW_OK;
}

int tw_fno_destroy(tw_fno f) {
  if (!f) return TW_OK;
  (void)hipDeviceSynchronize();
  fno_free(reinterpret_cast<Fno*>(f));
  return TW_OK;
}

int tw_fno_init_params(tw_fno f, uint64_t seed, float* params, void* stream) {
  if (!f || !params) return ffail(TW_EINVAL, "NULL handle or params");
  Fno& F = *reinterpret_cast<Fno*>(f);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const tw_fno_config& c = F.cfg;
  const Layout& L = F.L;
  const float C = (float)c.width;
  auto uni = [&](int64_t off, int64_t n, float lo, float hi, uint64_t tag) -> int {
    FNO_HIP(launch_init(params + off, n, seed * 0x100000001B3ull + tag, lo, hi, s));
    return TW_OK;
  };
  const int64_t nm = 2LL * c.modes_y * c.modes_x;
  int rc = uni(L.lift_w, (int64_t)c.c_in * c.width, -1.f / std::sqrt((float)c.c_in), 1.f / std::sqrt((float)c.c_in), 1);
  rc |= uni(L.lift_b, c.width, 0.f, 0.f, 2);
  for (int l = 0; l < c.layers; ++l) {
    rc |= uni(L.Rre[l], nm * c.width * c.width, 0.f, 1.f / (C * C), 10 + 4 * l);
    rc |= uni(L.Rim[l], nm * c.width * c.width, 0.f, 1.f / (C * C), 11 + 4 * l);
    rc |= uni(L.W[l], (int64_t)c.width * c.width, -1.f / std::sqrt(C), 1.f / std::sqrt(C), 12 + 4 * l);
    rc |= uni(L.b[l], c.width, 0.f, 0.f, 13 + 4 * l);
  }
  rc |= uni(L.q1_w, (int64_t)c.width * c.proj, -1.f / std::sqrt(C), 1.f / std::sqrt(C), 3);
  rc |= uni(L.q1_b, c.proj, 0.f, 0.f, 4);
  rc |= uni(L.q2_w, (int64_t)c.proj * c.c_out, -1.f / std::sqrt((float)c.proj), 1.f / std::sqrt((float)c.proj), 5);
  rc |= uni(L.q2_b, c.c_out, 0.f, 0.f, 6);
  return rc ? TW_EHIP : TW_OK;
}

int tw_fno_forward(tw_fno f, const float* params, const float* x, int32_t batch, float* y, void* stream) {
  if (!f || !params || !x || !y) return ffail(TW_EINVAL, "NULL argument");
  Fno& F = *reinterpret_cast<Fno*>(f);
  if (batch < 1 || batch > F.max_batch) return ffail(TW_EINVAL, "batch outside 1..max_batch");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const tw_fno_config& c = F.cfg;
  const Layout& L = F.L;
  const int64_t P = positions(F, batch), C = c.width, K2 = 2LL * c.modes_y, mx = c.modes_x;
  const int64_t PC = (int64_t)F.max_batch * c.H * c.W * C;  // per-layer stride of saved activations
  const int64_t bstride = (int64_t)F.max_batch * K2 * mx * C;
  // every pointwise layer is one GEMM whose epilogue adds the bias (and the
  // spectral branch) and writes the activation
  float* v0 = F.v;
  Epi lift;
  lift.bias = params + L.lift_b;
  FNO_HIP(gemm(s, P, C, c.c_in, 1.f, x, c.c_in, 1, params + L.lift_w, C, 1, 0.f, v0, C, 1, 1, 0, 0, 0, lift));
  for (int l = 0; l < c.layers; ++l) {
    float* vl = F.v + l * PC;
    float* vn = F.v + (l + 1) * PC;
    float* ul = F.u + l * PC;
    float* br = F.bsav + (2 * l) * bstride;
    float* bi = F.bsav + (2 * l + 1) * bstride;
    if (int rc = spectral_fwd(F, s, batch, vl, params + L.Rre[l], params + L.Rim[l], br, bi, F.s)) return rc;
    Epi e;  // u_l = S(v_l) + v_l W_l + b_l, v_{l+1} = GELU(u_l) (u_l after the last layer)
    e.add = F.s;
    e.bias = params + L.b[l];
    e.out2 = vn;
    e.act = l < c.layers - 1 ? 1 : 0;
    FNO_HIP(gemm(s, P, C, C, 1.f, vl, C, 1, params + L.W[l], C, 1, 0.f, ul, C, 1, 1, 0, 0, 0, e));
  }
  const float* vL = F.v + (int64_t)c.layers * PC;
  Epi e1;
  e1.bias = params + L.q1_b;
  e1.out2 = F.h;
  e1.act = 1;
  FNO_HIP(gemm(s, P, c.proj, C, 1.f, vL, C, 1, params + L.q1_w, c.proj, 1, 0.f, F.z1, c.proj, 1, 1, 0, 0, 0, e1));
  // one or two output channels: streaming dot products per position (a
  // matrix-core tile would compute 32 columns to keep one or two)
  if (c.c_out <= 2 && launch_proj_out(F.h, params + L.q2_w, params + L.q2_b, y, P, c.proj, c.c_out, s) == hipSuccess)
    return TW_OK;
  (void)hipGetLastError();
  Epi e2;
  e2.bias = params + L.q2_b;
  FNO_HIP(gemm(s, P, c.c_out, c.proj, 1.f, F.h, c.proj, 1, params + L.q2_w, c.c_out, 1, 0.f, y, c.c_out, 1, 1, 0, 0,
               0, e2));
  return TW_OK;
}

int tw_fno_backward(tw_fno f, const float* params, const float* x, int32_t batch, const float* dy, float* grads,
                    void* stream) {
  if (!f || !params || !x || !dy || !grads) return ffail(TW_EINVAL, "NULL argument");
  Fno& F = *reinterpret_cast<Fno*>(f);
  if (batch < 1 || batch > F.max_batch) return ffail(TW_EINVAL, "batch outside 1..max_batch");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const tw_fno_config& c = F.cfg;
  const Layout& L = F.L;
  const int64_t P = positions(F, batch), C = c.width, K2 = 2LL * c.modes_y, mx = c.modes_x;
  const int64_t PC = (int64_t)F.max_batch * c.H * c.W * C;
  const int64_t bstride = (int64_t)F.max_batch * K2 * mx * C;
  // projection 2 (one or two output channels: a weighted column sum and an
  // outer product with GELU' instead of matrix-core tiles of width 1 or 2)
  const bool one = c.c_out <= 2 && launch_colsum_weighted(F.h, dy, c.c_out, P, c.proj, grads + L.q2_w, F.parts,
                                                          F.parts_len, F.parts2, s) == hipSuccess;
  if (!one) {
    (void)hipGetLastError();
    FNO_HIP(weight_grad(F, s, P, c.proj, c.c_out, F.h, dy, grads + L.q2_w));
  }
  FNO_HIP(launch_colsum(dy, P, c.c_out, grads + L.q2_b, 0, F.parts, F.parts_len, F.parts2, s));
  if (!one || launch_proj_out_back(dy, params + L.q2_w, F.z1, F.dz, P, c.proj, c.c_out, s) != hipSuccess) {
    (void)hipGetLastError();
    Epi eg;  // dz = (dy q2_w^T) GELU'(z1)
    eg.gz = F.z1;
    eg.gz_into_c = 1;
    FNO_HIP(gemm(s, P, c.proj, c.c_out, 1.f, dy, c.c_out, 1, params + L.q2_w, 1, c.c_out, 0.f, F.dz, c.proj, 1, 1, 0,
                 0, 0, eg));
  }
  // projection 1
  const float* vL = F.v + (int64_t)c.layers * PC;
  FNO_HIP(weight_grad(F, s, P, C, c.proj, vL, F.dz, grads + L.q1_w));
  FNO_HIP(launch_colsum(F.dz, P, c.proj, grads + L.q1_b, 0, F.parts, F.parts_len, F.parts2, s));
  // dv: gradient of the layer input v_l; du: of u_l. No activation follows the
  // last layer (du = dv there); before every other layer's gradient, the
  // data-gradient GEMM of the layer above also writes du = dv GELU'(u) in its
  // epilogue, into the buffer the current du does not occupy (F.s, free in the
  // backward pass, and F.t2 in turn)
  float* dv = F.t1;
  float* du = F.t2;
  float* du_next = F.s;
  FNO_HIP(gemm(s, P, C, c.proj, 1.f, F.dz, c.proj, 1, params + L.q1_w, 1, c.proj, 0.f, dv, C, 1));
  FNO_HIP(hipMemcpyAsync(du, dv, sizeof(float) * P * C, hipMemcpyDeviceToDevice, s));
  for (int l = c.layers - 1; l >= 0; --l) {
    const float* vl = F.v + l * PC;
    FNO_HIP(weight_grad(F, s, P, C, C, vl, du, grads + L.W[l]));
    FNO_HIP(launch_colsum(du, P, (int)C, grads + L.b[l], 0, F.parts, F.parts_len, F.parts2, s));
    const float* br = F.bsav + (2 * l) * bstride;
    const float* bi = F.bsav + (2 * l + 1) * bstride;
    if (int rc = spectral_bwd(F, s, batch, du, br, bi, params + L.Rre[l], params + L.Rim[l], grads + L.Rre[l],
                              grads + L.Rim[l], dv))
      return rc;
    Epi eb;
    if (l > 0) {
      eb.gz = F.u + (l - 1) * PC;
      eb.out2 = du_next;
    }
    FNO_HIP(gemm(s, P, C, C, 1.f, du, C, 1, params + L.W[l], 1, C, 1.f, dv, C, 1, 1, 0, 0, 0, eb));
    std::swap(du, du_next);
  }
  FNO_HIP(weight_grad(F, s, P, c.c_in, C, x, dv, grads + L.lift_w));
  FNO_HIP(launch_colsum(dv, P, (int)C, grads + L.lift_b, 0, F.parts, F.parts_len, F.parts2, s));
  return TW_OK;
}

int tw_fno_mse(const float* y, const float* t, int64_t n, float* dy, float* loss, void* stream) {
  if (!y || !t || n < 1) return ffail(TW_EINVAL, "bad MSE arguments");
  FNO_HIP(launch_mse(y, t, n, dy, loss, reinterpret_cast<hipStream_t>(stream)));
  return TW_OK;
}

int tw_fno_adam(float* params, const float* grads, float* m, float* v, int64_t n, float lr, float b1, float b2,
                float eps, int64_t step, void* stream) {
  if (!params || !grads || !m || !v || n < 1 || step < 1) return ffail(TW_EINVAL, "bad Adam arguments");
  FNO_HIP(launch_adam(params, grads, m, v, n, lr, b1, b2, eps, step, reinterpret_cast<hipStream_t>(stream)));
  return TW_OK;
}

}  // extern "C"
