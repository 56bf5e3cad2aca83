// Grouped FP32 GEMM: many independent row-major products of different sizes
// in one launch, C_p = alpha_p A_p B_p + beta_p C_p.  The workgroups of all
// problems form one linear grid; problem p owns the tiles
// [tile0_p, tile0_p + tiles_p) and a workgroup finds its problem by binary
// search over tile0.  v_mfma_f32_16x16x4f32 with FP32 accumulation.
//
// The tile shape is a template parameter; grouped_gemm_f32() picks it with a
// small autotuner: on the first call for a given problem-size signature it
// times every candidate shape on a scratch output and remembers the fastest.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <string>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "grouped.hpp"
#include "prof.hpp"

namespace tci {

typedef float f4v __attribute__((ext_vector_type(4)));

template <int BM, int BN>
__global__ __launch_bounds__(256) void grouped_gemm_f32_kernel(const GroupProb* P, const int* tile0, int np,
                                                               long long c_shift) {
  constexpr int BK = 16;
  constexpr int IM = BM / 32, JN = BN / 32;
  __shared__ float As[BK][BM + 4];
  __shared__ float Bs[BK][BN + 4];
  const int t = blockIdx.x;
  int lo = 0, hi = np - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tile0[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  const GroupProb pr = P[lo];
  const int tnc = (pr.n + BN - 1) / BN;
  const int local = t - tile0[lo];
  const int m0 = (local / tnc) * BM, n0 = (local % tnc) * BN;
  const float* Ap = pr.a;
  const float* Bp = pr.b;
  float* Cp = pr.c + c_shift;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int lr = lane & 15, lq = lane >> 4;

  f4v acc[IM][JN];
#pragma unroll
  for (int i = 0; i < IM; ++i)
#pragma unroll
    for (int j = 0; j < JN; ++j) acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};

  for (int k0 = 0; k0 < pr.k; k0 += BK) {
    for (int e = tid; e < BM * BK; e += 256) {
      const int r = e / BK, kk = e % BK;
      const int gr = m0 + r, gk = k0 + kk;
      As[kk][r] = (gr < pr.m && gk < pr.k) ? Ap[(long long)gr * pr.lda + gk] : 0.f;
    }
    for (int e = tid; e < BK * BN; e += 256) {
      const int kk = e / BN, c = e % BN;
      const int gk = k0 + kk, gc = n0 + c;
      Bs[kk][c] = (gk < pr.k && gc < pr.n) ? Bp[(long long)gk * pr.ldb + gc] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kq = 0; kq < BK; kq += 4) {
      float a[IM], b[JN];
#pragma unroll
      for (int i = 0; i < IM; ++i) a[i] = As[kq + lq][wm * (BM / 2) + i * 16 + lr];
#pragma unroll
      for (int j = 0; j < JN; ++j) b[j] = Bs[kq + lq][wn * (BN / 2) + j * 16 + lr];
#pragma unroll
      for (int i = 0; i < IM; ++i)
#pragma unroll
        for (int j = 0; j < JN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < IM; ++i)
#pragma unroll
    for (int j = 0; j < JN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * (BM / 2) + i * 16 + 4 * lq + r;
        const int col = n0 + wn * (BN / 2) + j * 16 + lr;
        if (row < pr.m && col < pr.n) {
          float* c = Cp + (long long)row * pr.ldc + col;
          float v = pr.alpha * acc[i][j][r];
          if (pr.beta != 0.f) v += pr.beta * *c;
          *c = v;
        }
      }
}

namespace {

struct Shape {
  int bm, bn;
};
constexpr Shape kShapes[] = {{32, 32}, {64, 64}, {128, 64}};
constexpr int kNumShapes = 3;

template <int BM, int BN>
hipError_t launch_shape(const GroupProb* P, const int* tile0, int np, int ntiles, long long c_shift, hipStream_t s) {
  hipLaunchKernelGGL((grouped_gemm_f32_kernel<BM, BN>), dim3(ntiles), dim3(256), 0, s, P, tile0, np, c_shift);
  return hipGetLastError();
}

hipError_t launch_idx(int idx, const GroupProb* P, const int* tile0, int np, int ntiles, long long c_shift,
                      hipStream_t s) {
  switch (idx) {
    case 0: return launch_shape<32, 32>(P, tile0, np, ntiles, c_shift, s);
    case 1: return launch_shape<64, 64>(P, tile0, np, ntiles, c_shift, s);
    default: return launch_shape<128, 64>(P, tile0, np, ntiles, c_shift, s);
  }
}

int tiles_of(const GroupProb& p, int bm, int bn) {
  if (p.m <= 0 || p.n <= 0) return 0;
  return ((p.m + bm - 1) / bm) * ((p.n + bn - 1) / bn);
}

// Signature of a problem set: count and size histogram on a log2 scale.
std::vector<long long> signature(const std::vector<GroupProb>& probs) {
  std::vector<long long> h(3 * 12 + 1, 0);
  auto bucket = [](int x) {
    int b = 0;
    while ((1 << b) < x && b < 11) ++b;
    return b;
  };
  for (const auto& p : probs) {
    ++h[bucket(std::max(p.m, 1))];
    ++h[12 + bucket(std::max(p.n, 1))];
    ++h[24 + bucket(std::max(p.k, 1))];
  }
  h[36] = (long long)probs.size();
  return h;
}

std::mutex g_tune_mu;
std::map<std::pair<int, std::vector<long long>>, int> g_tuned;   // (device, signature) -> shape index

}  // namespace

// Cache file: one line per tuned signature, "device shape h0 .. h36".
void grouped_tune_load(const std::string& path, int device) {
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (;;) {
    int dev = 0, shape = 0;
    if (std::fscanf(f, "%d %d", &dev, &shape) != 2) break;
    std::vector<long long> h(3 * 12 + 1, 0);
    bool ok = true;
    for (auto& v : h) ok = ok && std::fscanf(f, "%lld", &v) == 1;
    if (!ok) break;
    if (dev == device && shape >= 0 && shape < kNumShapes) g_tuned[{dev, h}] = shape;
  }
  std::fclose(f);
}

bool grouped_tune_save(const std::string& path) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  FILE* f = std::fopen(path.c_str(), "w");
  if (!f) return false;
  for (const auto& kv : g_tuned) {
    std::fprintf(f, "%d %d", kv.first.first, kv.second);
    for (long long v : kv.first.second) std::fprintf(f, " %lld", v);
    std::fprintf(f, "\n");
  }
  return std::fclose(f) == 0;
}

int grouped_tuned_shape(int device, const std::vector<GroupProb>& probs) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find({device, signature(probs)});
  return it == g_tuned.end() ? -1 : it->second;
}

hipError_t grouped_prepare(int device, const std::vector<GroupProb>& probs, GroupProb* P_dev, int* tile0_dev,
                           long long scratch_shift, hipStream_t s, GroupedPlan& plan) {
  const int np = (int)probs.size();
  plan = GroupedPlan{};
  plan.np = np;
  plan.P_dev = P_dev;
  plan.t0_dev = tile0_dev;
  if (np == 0) return hipSuccess;
  // host staging stays alive until the stream is synchronised below
  std::vector<std::vector<int>> t0(kNumShapes, std::vector<int>(np));
  std::vector<int> tot(kNumShapes, 0);
  for (int idx = 0; idx < kNumShapes; ++idx)
    for (int p = 0; p < np; ++p) {
      t0[idx][p] = tot[idx];
      tot[idx] += tiles_of(probs[p], kShapes[idx].bm, kShapes[idx].bn);
    }
  hipError_t e = hipMemcpyAsync(P_dev, probs.data(), sizeof(GroupProb) * np, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  int best = grouped_tuned_shape(device, probs);
  if (best < 0) {
    // autotune: time each shape (second of two runs) on the scratch output
    float best_ms = 1e30f;
    best = 1;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return hipErrorUnknown;
    if (hipEventCreate(&e1) != hipSuccess) {
      hipEventDestroy(e0);
      return hipErrorUnknown;
    }
    for (int idx = 0; idx < kNumShapes && e == hipSuccess; ++idx) {
      if (tot[idx] == 0) break;
      e = hipMemcpyAsync(tile0_dev, t0[idx].data(), sizeof(int) * np, hipMemcpyHostToDevice, s);
      for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
        if ((e = hipEventRecord(e0, s)) != hipSuccess) break;
        if ((e = launch_idx(idx, P_dev, tile0_dev, np, tot[idx], scratch_shift, s)) != hipSuccess) break;
        e = hipEventRecord(e1, s);
      }
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (e != hipSuccess) break;
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      if (ms < best_ms) {
        best_ms = ms;
        best = idx;
      }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[{device, signature(probs)}] = best;
  }
  plan.shape = best;
  plan.ntiles = tot[best];
  for (const auto& p : probs) plan.flops += 2.0 * p.m * (double)p.n * p.k;
  e = hipMemcpyAsync(tile0_dev, t0[best].data(), sizeof(int) * np, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

hipError_t grouped_launch(const GroupedPlan& plan, hipStream_t s) {
  if (plan.np == 0 || plan.ntiles == 0) return hipSuccess;
  ProfScope ps(s, plan.flops, "f32_fp32_grouped");
  return launch_idx(plan.shape, plan.P_dev, plan.t0_dev, plan.np, plan.ntiles, 0, s);
}

hipError_t grouped_gemm_f32(int device, const std::vector<GroupProb>& probs, GroupProb* P_dev, int* tile0_dev,
                            long long scratch_shift, hipStream_t s, int* shape_out) {
  GroupedPlan plan;
  hipError_t e = grouped_prepare(device, probs, P_dev, tile0_dev, scratch_shift, s, plan);
  if (e != hipSuccess) return e;
  if (shape_out) *shape_out = plan.shape;
  e = grouped_launch(plan, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

void grouped_shape_dims(int idx, int* bm, int* bn) {
  idx = std::max(0, std::min(kNumShapes - 1, idx));
  *bm = kShapes[idx].bm;
  *bn = kShapes[idx].bn;
}

}  // namespace tci
