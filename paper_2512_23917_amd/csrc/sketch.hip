// Device kernels of the randomized truncated SVD:
//   * Gaussian sketch Omega from the Philox4x32-10 counter-based generator
//     (Salmon, Moraes, Dror, Shaw, SC'11) with the Box-Muller transform;
//   * residual norms of approximate singular triplets,
//     r_j = || (theta V)_j - s_j U_j ||_2;
//   * the sketch rank of each problem from a predicted log2 chi.
#include "common.hpp"
#include "sketch_kernels.hpp"

namespace tci {

__device__ inline void philox_round(uint32_t c[4], const uint32_t k[2]) {
  const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
  const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
  const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  const uint32_t n0 = hi1 ^ c[1] ^ k[0];
  const uint32_t n2 = hi0 ^ c[3] ^ k[1];
  c[0] = n0;
  c[1] = lo1;
  c[2] = n2;
  c[3] = lo0;
}

__device__ inline void philox10(uint64_t block, uint32_t stream, uint64_t seed, uint32_t out[4]) {
  uint32_t c[4] = {(uint32_t)block, (uint32_t)(block >> 32), stream, 0u};
  uint32_t k[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    philox_round(c, k);
    k[0] += 0x9E3779B9u;
    k[1] += 0xBB67AE85u;
  }
  out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

// Normal number z[t] of the stream: block t/4, Box-Muller on pairs (x0,x1), (x2,x3).
__device__ inline double philox_normal_at(uint64_t t, uint32_t stream, uint64_t seed) {
  uint32_t x[4];
  philox10(t >> 2, stream, seed, x);
  const int q = (int)(t & 3);
  const int pair = q >> 1;
  const double u1 = ((double)x[2 * pair] + 0.5) * 2.3283064365386963e-10;
  const double u2 = ((double)x[2 * pair + 1] + 0.5) * 2.3283064365386963e-10;
  const double r = sqrt(-2.0 * log(u1));
  const double ang = 6.283185307179586 * u2;
  return (q & 1) ? r * sin(ang) : r * cos(ang);
}

// Omega_b (n x ld, columns j < k_b filled, the rest zero); entry (i, j):
// real: z[i*k_b + j]; complex: (z[2t] + i z[2t+1]) / sqrt(2), t = i*k_b + j.
template <typename T>
__global__ void sketch_fill_kernel(T* om, long long ld, long long som, int n, const int* kb, int kdef,
                                   uint64_t seed, const uint32_t* streams) {
  const int b = blockIdx.y;
  const int k = kb ? kb[b] : kdef;
  const uint32_t stream = streams ? streams[b] : (uint32_t)b;
  T* o = om + b * som;
  for (long long idx = blockIdx.x * 256LL + threadIdx.x; idx < (long long)n * ld; idx += (long long)gridDim.x * 256) {
    const long long i = idx / ld, j = idx % ld;
    if (j >= k) {
      o[idx] = T{};
      continue;
    }
    const uint64_t t = (uint64_t)(i * k + j);
    if constexpr (sizeof(T) == 16) {
      o[idx] = cd{philox_normal_at(2 * t, stream, seed) * 0.7071067811865476,
                  philox_normal_at(2 * t + 1, stream, seed) * 0.7071067811865476};
    } else if constexpr (sizeof(T) == 8 && !std::is_same<T, double>::value) {
      o[idx] = cf{(float)(philox_normal_at(2 * t, stream, seed) * 0.7071067811865476),
                  (float)(philox_normal_at(2 * t + 1, stream, seed) * 0.7071067811865476)};
    } else {
      o[idx] = (T)philox_normal_at(t, stream, seed);
    }
  }
}

hipError_t sketch_fill(int dt, void* om, long long ld, long long som, int n, const int* kb, int kdef, uint64_t seed,
                       const uint32_t* streams, int batch, hipStream_t s) {
  dim3 grid((unsigned)std::max<long long>(1, std::min<long long>(4096, ((long long)n * ld + 255) / 256)), batch);
  switch (dt) {
    case C128: hipLaunchKernelGGL(sketch_fill_kernel<cd>, grid, dim3(256), 0, s, (cd*)om, ld, som, n, kb, kdef, seed, streams); break;
    case C64: hipLaunchKernelGGL(sketch_fill_kernel<cf>, grid, dim3(256), 0, s, (cf*)om, ld, som, n, kb, kdef, seed, streams); break;
    case F64: hipLaunchKernelGGL(sketch_fill_kernel<double>, grid, dim3(256), 0, s, (double*)om, ld, som, n, kb, kdef, seed, streams); break;
    case F32: hipLaunchKernelGGL(sketch_fill_kernel<float>, grid, dim3(256), 0, s, (float*)om, ld, som, n, kb, kdef, seed, streams); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Raw Philox blocks for testing against published vectors: out[4*i..] = philox(i + first).
__global__ void philox_blocks_kernel(uint64_t seed, uint32_t stream, uint64_t first, long long n, uint32_t* out) {
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= n) return;
  uint32_t x[4];
  philox10(first + (uint64_t)i, stream, seed, x);
  out[4 * i + 0] = x[0];
  out[4 * i + 1] = x[1];
  out[4 * i + 2] = x[2];
  out[4 * i + 3] = x[3];
}

hipError_t philox_blocks(uint64_t seed, uint32_t stream, uint64_t first, long long n, uint32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(philox_blocks_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, seed, stream, first, n, out);
  return hipGetLastError();
}

// r[b][j] = || P[:, j] - s[b][j] U[:, j] ||_2 for j < chi[b]  (P = theta V, m x ld)
template <typename T>
__global__ __launch_bounds__(64) void resid_kernel(const T* P, const T* U, long long ld, long long sPU, int m,
                                                   const double* sv, long long ss, const int* chi, double* r) {
  const int j = blockIdx.x, b = blockIdx.y;
  if (j >= chi[b]) return;
  const T* p = P + b * sPU;
  const T* u = U + b * sPU;
  const double sj = sv[b * ss + j];
  double acc = 0.0;
  for (int i = threadIdx.x; i < m; i += 64) {
    if constexpr (sizeof(T) == 16) {
      const cd a = p[(long long)i * ld + j], c = u[(long long)i * ld + j];
      const double dr = a.x - sj * c.x, di = a.y - sj * c.y;
      acc += dr * dr + di * di;
    } else {
      const double dv = (double)p[(long long)i * ld + j] - sj * (double)u[(long long)i * ld + j];
      acc += dv * dv;
    }
  }
  acc = wave_sum(acc);
  if (threadIdx.x == 0) r[b * ss + j] = sqrt(acc);
}

hipError_t residual_norms(int dt, const void* P, const void* U, long long ld, long long sPU, int m, int maxchi,
                          const double* sv, long long ss, const int* chi, double* r, int batch, hipStream_t s) {
  dim3 grid(maxchi, batch);
  if (dt == C128) hipLaunchKernelGGL(resid_kernel<cd>, grid, dim3(64), 0, s, (const cd*)P, (const cd*)U, ld, sPU, m, sv, ss, chi, r);
  else if (dt == F64) hipLaunchKernelGGL(resid_kernel<double>, grid, dim3(64), 0, s, (const double*)P, (const double*)U, ld, sPU, m, sv, ss, chi, r);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace tci
