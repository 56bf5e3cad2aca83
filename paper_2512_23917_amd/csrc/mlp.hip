// Sketch-rank model: a 35 -> 128 -> 128 -> 1 perceptron with exact GELU that
// predicts log2 chi*(eps) of a bond from its previous spectrum, trained on
// the GPU with hand-written forward, backward (pinball loss, tau = 0.9) and
// Adam kernels.  FP32 parameters and arithmetic.
//
// Flat parameter layout: W1 (128 x 35, row-major), b1 (128), W2 (128 x 128),
// b2 (128), W3 (1 x 128), b3 (1).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/tci_c.h"
#include "common.hpp"
#include "runtime.hpp"

struct tci_sketch_model_s {
  float* params = nullptr;  // device, N_PARAMS
  float* m = nullptr;       // Adam first moment
  float* v = nullptr;       // Adam second moment
  int64_t step = 0;
  tci_allocator al{};       // allocator of the three buffers (the creating context's)
  uint32_t magic = 0x5C37C4u;
};

namespace tci {

constexpr int NI = 35, NH = 128;
constexpr int OFF_W1 = 0, OFF_B1 = NH * NI, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH, OFF_W3 = OFF_B2 + NH,
              OFF_B3 = OFF_W3 + NH, NPARAM = OFF_B3 + 1;
constexpr float TAU = 0.9f;

__device__ inline void philox_round_m(uint32_t c[4], const uint32_t k[2]) {
  const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
  const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
  const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k[0];
  const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k[1];
  c[1] = (uint32_t)p1;
  c[3] = (uint32_t)p0;
  c[0] = n0;
  c[2] = n2;
}

// He-uniform initialisation: uniform u_e = (x_e + 0.5) 2^-32 with x_e the e-th
// 32-bit output of Philox4x32-10 (key = seed, stream 7); W = (2u - 1) sqrt(6 / fan_in).
__global__ void mlp_init_kernel(float* p, uint64_t seed) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;  // index over weights only
  const int nw = NH * NI + NH * NH + NH;
  if (e >= nw) return;
  uint32_t c[4] = {(uint32_t)(e >> 2), 0u, 7u, 0u};
  uint32_t k[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int r = 0; r < 10; ++r) {
    philox_round_m(c, k);
    k[0] += 0x9E3779B9u;
    k[1] += 0xBB67AE85u;
  }
  const double u = ((double)c[e & 3] + 0.5) * 2.3283064365386963e-10;
  if (e < NH * NI) {
    p[OFF_W1 + e] = (float)((2.0 * u - 1.0) * sqrt(6.0 / NI));
  } else if (e < NH * NI + NH * NH) {
    p[OFF_W2 + (e - NH * NI)] = (float)((2.0 * u - 1.0) * sqrt(6.0 / NH));
  } else {
    p[OFF_W3 + (e - NH * NI - NH * NH)] = (float)((2.0 * u - 1.0) * sqrt(6.0 / NH));
  }
}

__device__ inline float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ inline float gelu_d(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.3989422804014327f;
}

// Forward of one sample per workgroup (128 threads); z1, z2 (n x 128) kept for backward.
__global__ __launch_bounds__(128) void mlp_forward_kernel(const float* __restrict__ p, const float* __restrict__ X,
                                                          int n, float* z1o, float* z2o, float* y) {
  __shared__ float x[NI], h1[NH], h2[NH], red[2];
  const int s = blockIdx.x, j = threadIdx.x;
  if (s >= n) return;
  if (j < NI) x[j] = X[(long long)s * NI + j];
  __syncthreads();
  float a = p[OFF_B1 + j];
  for (int i = 0; i < NI; ++i) a += p[OFF_W1 + j * NI + i] * x[i];
  if (z1o) z1o[(long long)s * NH + j] = a;
  h1[j] = gelu(a);
  __syncthreads();
  float b = p[OFF_B2 + j];
  for (int i = 0; i < NH; ++i) b += p[OFF_W2 + j * NH + i] * h1[i];
  if (z2o) z2o[(long long)s * NH + j] = b;
  h2[j] = gelu(b);
  float c = p[OFF_W3 + j] * h2[j];
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((j & 63) == 0) red[j >> 6] = c;
  __syncthreads();
  if (j == 0) y[s] = red[0] + red[1] + p[OFF_B3];
}

// Per-sample gradient of the mean pinball loss (one sample per workgroup),
// written to G[s][0..NPARAM); loss_s = rho(t - y) / n.
__global__ __launch_bounds__(128) void mlp_backward_kernel(const float* __restrict__ p, const float* __restrict__ X,
                                                           const float* __restrict__ T, int n, const float* z1,
                                                           const float* z2, const float* y, float* G, float* loss) {
  __shared__ float x[NI], h1[NH], gz2[NH];
  const int s = blockIdx.x, j = threadIdx.x;
  if (s >= n) return;
  float* g = G + (long long)s * NPARAM;
  if (j < NI) x[j] = X[(long long)s * NI + j];
  const float a1 = z1[(long long)s * NH + j];
  const float a2 = z2[(long long)s * NH + j];
  h1[j] = gelu(a1);
  const float u = T[s] - y[s];
  const float gy = (u < 0.f ? (1.f - TAU) : -TAU) / (float)n;
  if (j == 0) {
    loss[s] = fmaxf(TAU * u, (TAU - 1.f) * u) / (float)n;
    g[OFF_B3] = gy;
  }
  const float h2j = gelu(a2);
  g[OFF_W3 + j] = gy * h2j;
  const float gzj = gy * p[OFF_W3 + j] * gelu_d(a2);
  gz2[j] = gzj;
  g[OFF_B2 + j] = gzj;
  __syncthreads();
  for (int i = 0; i < NH; ++i) g[OFF_W2 + j * NH + i] = gzj * h1[i];
  // g_h1[j] = sum_r gz2[r] W2[r][j]
  float gh = 0.f;
  for (int r = 0; r < NH; ++r) gh += gz2[r] * p[OFF_W2 + r * NH + j];
  const float g1 = gh * gelu_d(a1);
  g[OFF_B1 + j] = g1;
  for (int i = 0; i < NI; ++i) g[OFF_W1 + j * NI + i] = g1 * x[i];
}

// grad[q] = sum_s G[s][q] (fixed order), loss_total = sum_s loss[s] (thread 0)
__global__ void mlp_reduce_kernel(const float* G, const float* loss, int n, float* grad, float* loss_total) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < NPARAM) {
    float acc = 0.f;
    for (int s = 0; s < n; ++s) acc += G[(long long)s * NPARAM + q];
    grad[q] = acc;
  }
  if (q == 0) {
    float l = 0.f;
    for (int s = 0; s < n; ++s) l += loss[s];
    *loss_total = l;
  }
}

__global__ void adam_kernel(float* p, float* m, float* v, const float* g, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= NPARAM) return;
  const float gq = g[q];
  const float mq = b1 * m[q] + (1.f - b1) * gq;
  const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
  m[q] = mq;
  v[q] = vq;
  p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

// Features of one bond per thread: [log2 chi_max / 11, d / 4, -log10 eps / 16,
// 32 clamped log10 quantiles of the previous spectrum s (descending, length len[b])].
__global__ void features_kernel(const double* s, long long ss, const int* len, int chi_max, int d, double eps,
                                float* X, int n) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  const double* sb = s + b * ss;
  const int L = len[b];
  float* x = X + (long long)b * NI;
  x[0] = (float)(log2((double)chi_max) / 11.0);
  x[1] = (float)(d / 4.0);
  x[2] = (float)(-log10(eps) / 16.0);
  for (int t = 0; t < 32; ++t) {
    const int j = L > 1 ? (int)floor((t + 0.5) / 32.0 * (L - 1)) : 0;
    double q = -1.0;
    if (L > 0 && sb[0] > 0.0 && sb[j] > 0.0) q = log10(sb[j] / sb[0]) / 16.0;
    x[3 + t] = (float)fmin(0.0, fmax(-1.0, q));
  }
}

static tci_status model_check(tci_sketch_model m) {
  if (!m || m->magic != 0x5C37C4u) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "invalid sketch model");
  return TCI_OK;
}

static tci_status grads_impl(tci_context ctx, tci_sketch_model m, const float* X, const float* T, int n, float* grad,
                             float* loss_dev) {
  hipStream_t s = ctx->stream;
  float* z1 = static_cast<float*>(ctx->arena.get(sizeof(float) * (size_t)n * NH));
  float* z2 = static_cast<float*>(ctx->arena.get(sizeof(float) * (size_t)n * NH));
  float* y = static_cast<float*>(ctx->arena.get(sizeof(float) * (size_t)n));
  float* G = static_cast<float*>(ctx->arena.get(sizeof(float) * (size_t)n * NPARAM));
  float* ls = static_cast<float*>(ctx->arena.get(sizeof(float) * (size_t)n));
  if (!z1 || !z2 || !y || !G || !ls) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "mlp workspace");
  hipLaunchKernelGGL(mlp_forward_kernel, dim3(n), dim3(NH), 0, s, m->params, X, n, z1, z2, y);
  hipLaunchKernelGGL(mlp_backward_kernel, dim3(n), dim3(NH), 0, s, m->params, X, T, n, z1, z2, y, G, ls);
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, s, G, ls, n, grad, loss_dev);
  TCI_CHECK_HIP(hipGetLastError());
  return TCI_OK;
}

int sketch_model_nparams() { return NPARAM; }

tci_status sketch_predict_dev(tci_context ctx, tci_sketch_model m, const float* X, int n, float* y) {
  TCI_TRY(model_check(m));
  if (n <= 0) return TCI_OK;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3(n), dim3(NH), 0, ctx->stream, m->params, X, n, (float*)nullptr,
                     (float*)nullptr, y);
  TCI_CHECK_HIP(hipGetLastError());
  return TCI_OK;
}

tci_status sketch_features_dev(tci_context ctx, const double* s, long long ss, const int* len, int chi_max, int d,
                               double eps, float* X, int n) {
  hipLaunchKernelGGL(features_kernel, dim3((n + 63) / 64), dim3(64), 0, ctx->stream, s, ss, len, chi_max, d, eps, X, n);
  TCI_CHECK_HIP(hipGetLastError());
  return TCI_OK;
}

}  // namespace tci

using namespace tci;

extern "C" {

tci_status tci_sketch_model_create(tci_context ctx, uint64_t seed, tci_sketch_model* out) try {
  if (!ctx || !out) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  TCI_CHECK_HIP(hipSetDevice(ctx->device));
  auto* m = new tci_sketch_model_s();
  const size_t bytes = sizeof(float) * NPARAM;
  m->al = ctx->al;
  m->params = static_cast<float*>(dev_alloc(m->al, bytes, ctx->stream));
  m->m = static_cast<float*>(dev_alloc(m->al, bytes, ctx->stream));
  m->v = static_cast<float*>(dev_alloc(m->al, bytes, ctx->stream));
  if (!m->params || !m->m || !m->v) {
    dev_free(m->al, m->params, bytes, ctx->stream);
    dev_free(m->al, m->m, bytes, ctx->stream);
    dev_free(m->al, m->v, bytes, ctx->stream);
    delete m;
    TCI_RET(TCI_ERR_OUT_OF_MEMORY, "model allocation");
  }
  TCI_CHECK_HIP(hipMemsetAsync(m->params, 0, bytes, ctx->stream));
  TCI_CHECK_HIP(hipMemsetAsync(m->m, 0, bytes, ctx->stream));
  TCI_CHECK_HIP(hipMemsetAsync(m->v, 0, bytes, ctx->stream));
  const int nw = NH * NI + NH * NH + NH;
  hipLaunchKernelGGL(mlp_init_kernel, dim3((nw + 255) / 256), dim3(256), 0, ctx->stream, m->params, seed);
  TCI_CHECK_HIP(hipGetLastError());
  TCI_CHECK_HIP(hipStreamSynchronize(ctx->stream));
  *out = m;
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_sketch_model_destroy(tci_context ctx, tci_sketch_model m) try {
  if (!m) return TCI_OK;
  if (ctx) (void)hipStreamSynchronize(ctx->stream);
  const size_t bytes = sizeof(float) * NPARAM;
  hipStream_t st = ctx ? ctx->stream : nullptr;
  dev_free(m->al, m->params, bytes, st);
  dev_free(m->al, m->m, bytes, st);
  dev_free(m->al, m->v, bytes, st);
  m->magic = 0;
  delete m;
  return TCI_OK;
} TCI_API_CATCH

int64_t tci_sketch_model_nparams(void) { return NPARAM; }

tci_status tci_sketch_model_get_params(tci_context ctx, tci_sketch_model m, float* host, int64_t n) try {
  if (!ctx || !host) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  TCI_TRY(model_check(m));
  if (n != NPARAM) TCI_RET(TCI_ERR_SHAPE, "parameter count");
  TCI_CHECK_HIP(hipMemcpyAsync(host, m->params, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, ctx->stream));
  TCI_CHECK_HIP(hipStreamSynchronize(ctx->stream));
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_sketch_model_set_params(tci_context ctx, tci_sketch_model m, const float* host, int64_t n) try {
  if (!ctx || !host) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  TCI_TRY(model_check(m));
  if (n != NPARAM) TCI_RET(TCI_ERR_SHAPE, "parameter count");
  TCI_CHECK_HIP(hipMemcpyAsync(m->params, host, sizeof(float) * NPARAM, hipMemcpyHostToDevice, ctx->stream));
  TCI_CHECK_HIP(hipStreamSynchronize(ctx->stream));
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_sketch_model_save(tci_context ctx, tci_sketch_model m, const char* path) try {
  if (!path) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null path");
  std::vector<float> h(NPARAM);
  TCI_TRY(tci_sketch_model_get_params(ctx, m, h.data(), NPARAM));
  FILE* f = std::fopen(path, "wb");
  if (!f) TCI_RET(TCI_ERR_INVALID_ARGUMENT, std::string("cannot open ") + path);
  const char magic[8] = {'T', 'C', 'I', 'S', 'K', 'M', '1', 0};
  const int32_t np = NPARAM;
  bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(&np, 4, 1, f) == 1 &&
            std::fwrite(h.data(), sizeof(float), NPARAM, f) == (size_t)NPARAM;
  std::fclose(f);
  if (!ok) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "short write");
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_sketch_model_load(tci_context ctx, const char* path, tci_sketch_model* out) try {
  if (!ctx || !path || !out) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  FILE* f = std::fopen(path, "rb");
  if (!f) TCI_RET(TCI_ERR_INVALID_ARGUMENT, std::string("cannot open ") + path);
  char magic[8];
  int32_t np = 0;
  std::vector<float> h(NPARAM);
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "TCISKM1", 7) == 0 &&
            std::fread(&np, 4, 1, f) == 1 && np == NPARAM &&
            std::fread(h.data(), sizeof(float), NPARAM, f) == (size_t)NPARAM;
  std::fclose(f);
  if (!ok) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "not a sketch-model file");
  TCI_TRY(tci_sketch_model_create(ctx, 0, out));
  return tci_sketch_model_set_params(ctx, *out, h.data(), NPARAM);
} TCI_API_CATCH

tci_status tci_sketch_predict(tci_context ctx, tci_sketch_model m, const float* X, int n, float* y) try {
  if (!ctx || (n > 0 && (!X || !y))) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  TCI_CHECK_HIP(hipSetDevice(ctx->device));
  return sketch_predict_dev(ctx, m, X, n, y);
} TCI_API_CATCH

tci_status tci_sketch_grads(tci_context ctx, tci_sketch_model m, const float* X, const float* T, int n, float* grad,
                            float* loss) try {
  if (!ctx || !X || !T || !grad || n < 1) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "bad arguments");
  TCI_TRY(model_check(m));
  TCI_CHECK_HIP(hipSetDevice(ctx->device));
  ctx->arena.reset();
  float* ld = static_cast<float*>(ctx->arena.get(sizeof(float)));
  if (!ld) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
  TCI_TRY(grads_impl(ctx, m, X, T, n, grad, ld));
  if (loss) {
    TCI_CHECK_HIP(hipMemcpyAsync(loss, ld, sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
    TCI_CHECK_HIP(hipStreamSynchronize(ctx->stream));
  }
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_sketch_train_step(tci_context ctx, tci_sketch_model m, const float* X, const float* T, int n, float lr,
                                 float* loss) try {
  if (!ctx || !X || !T || n < 1) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "bad arguments");
  TCI_TRY(model_check(m));
  TCI_CHECK_HIP(hipSetDevice(ctx->device));
  ctx->arena.reset();
  float* grad = static_cast<float*>(ctx->arena.get(sizeof(float) * NPARAM));
  float* ld = static_cast<float*>(ctx->arena.get(sizeof(float)));
  if (!grad || !ld) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
  TCI_TRY(grads_impl(ctx, m, X, T, n, grad, ld));
  m->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = (float)(1.0 - std::pow(0.9, (double)m->step));
  const float c2 = (float)(1.0 - std::pow(0.999, (double)m->step));
  hipLaunchKernelGGL(adam_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, ctx->stream, m->params, m->m, m->v, grad,
                     lr, b1, b2, 1e-8f, c1, c2);
  TCI_CHECK_HIP(hipGetLastError());
  if (loss) {
    TCI_CHECK_HIP(hipMemcpyAsync(loss, ld, sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
    TCI_CHECK_HIP(hipStreamSynchronize(ctx->stream));
  }
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_sketch_features(tci_context ctx, const double* s, int64_t ss, const int32_t* len, int n, int chi_max,
                               int d, double eps, float* X) try {
  if (!ctx || !s || !len || !X || n < 1 || chi_max < 1 || !(eps > 0.0)) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "bad arguments");
  TCI_CHECK_HIP(hipSetDevice(ctx->device));
  return sketch_features_dev(ctx, s, ss, len, chi_max, d, eps, X, n);
} TCI_API_CATCH

}  // extern "C"
