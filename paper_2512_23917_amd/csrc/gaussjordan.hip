// Matrix inverse by Gauss-Jordan elimination with partial pivoting on the
// augmented matrix [A | I] (n x 2n, row-major, FP64 or complex FP64).
//
// Column k takes two launches:
//  * gj_pivot_kernel (one workgroup): the row p >= k of largest modulus in
//    column k (smallest index on ties), the swap of rows k and p, the scaling
//    of row k by 1 / pivot, and the multipliers f[i] = M[i, k] (f[k] = 0)
//    saved before the elimination overwrites the column;
//  * gj_eliminate_kernel: M[i, j] -= f[i] * M[k, j] for every row i and the
//    columns j >= k (columns left of k are already zero in row k).  Row k is
//    read, never written (f[k] = 0), so the launch has no intra-grid hazard.
// A zero (or NaN) pivot records its column + 1 in *status (the first one
// wins); the caller zeroes *status before and reads it once at the end.
#include "gaussjordan.hpp"

#include <algorithm>

namespace tci {

namespace {

constexpr int GJ_THREADS = 1024;
constexpr int GJ_ROWS = 16;   // rows per workgroup of the elimination

__device__ inline double modsq(double v) { return v * v; }
__device__ inline double modsq(cd v) { return v.x * v.x + v.y * v.y; }
__device__ inline double recip_of(double v, double) { return 1.0 / v; }
__device__ inline cd recip_of(cd v, double m2) { return cd{v.x / m2, -v.y / m2}; }
__device__ inline double mul(double a, double b) { return a * b; }
__device__ inline cd mul(cd a, cd b) { return a * b; }
__device__ inline double sub(double a, double b) { return a - b; }
__device__ inline cd sub(cd a, cd b) { return a - b; }
__device__ inline bool nonzero(double v) { return v != 0.0; }
__device__ inline bool nonzero(cd v) { return v.x != 0.0 || v.y != 0.0; }
template <typename T>
__device__ inline T zero_of();
template <>
__device__ inline double zero_of<double>() { return 0.0; }
template <>
__device__ inline cd zero_of<cd>() { return cd{0.0, 0.0}; }
template <typename T>
__device__ inline T one_of();
template <>
__device__ inline double one_of<double>() { return 1.0; }
template <>
__device__ inline cd one_of<cd>() { return cd{1.0, 0.0}; }

template <typename T>
__global__ void gj_init_kernel(const T* __restrict__ a, T* __restrict__ m, int n) {
  const long long total = 2LL * n * n;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < total; e += (long long)gridDim.x * 256) {
    const long long i = e / (2 * n), j = e % (2 * n);
    m[e] = j < n ? a[i * n + j] : (j - n == i ? one_of<T>() : zero_of<T>());
  }
}

template <typename T>
__global__ void __launch_bounds__(GJ_THREADS) gj_pivot_kernel(T* __restrict__ m, int n, int k, T* __restrict__ f,
                                                               int* __restrict__ status) {
  __shared__ double s_val[GJ_THREADS / 64];
  __shared__ int s_idx[GJ_THREADS / 64];
  __shared__ int s_p;
  __shared__ T s_piv;
  const long long ld = 2LL * n;
  const int tid = threadIdx.x;
  double best = -1.0;
  int bi = n;
  for (int i = k + tid; i < n; i += GJ_THREADS) {
    const double v = modsq(m[i * ld + k]);
    if (v > best) {   // rows visited in increasing order: keeps the first of equal values
      best = v;
      bi = i;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(best, off, 64);
    const int oi = __shfl_xor(bi, off, 64);
    if (ov > best || (ov == best && oi < bi)) {
      best = ov;
      bi = oi;
    }
  }
  if ((tid & 63) == 0) {
    s_val[tid >> 6] = best;
    s_idx[tid >> 6] = bi;
  }
  __syncthreads();
  if (tid == 0) {
    double bv = s_val[0];
    int bx = s_idx[0];
    for (int w = 1; w < GJ_THREADS / 64; ++w)
      if (s_val[w] > bv || (s_val[w] == bv && s_idx[w] < bx)) {
        bv = s_val[w];
        bx = s_idx[w];
      }
    if (bx >= n) bx = k;   // the whole column is NaN
    s_p = bx;
    s_piv = m[(long long)bx * ld + k];
    // one thread of the only workgroup, launches ordered on the stream: a plain store
    if (!(bv > 0.0) && *status == 0) *status = k + 1;
  }
  __syncthreads();
  const int p = s_p;
  if (p != k) {
    for (long long j = tid; j < ld; j += GJ_THREADS) {
      const T t = m[k * ld + j];
      m[k * ld + j] = m[p * ld + j];
      m[p * ld + j] = t;
    }
  }
  __syncthreads();
  const T piv = s_piv;
  const double m2 = modsq(piv);
  const T inv = m2 > 0.0 ? recip_of(piv, m2) : zero_of<T>();
  for (int i = tid; i < n; i += GJ_THREADS) f[i] = i == k ? zero_of<T>() : m[(long long)i * ld + k];
  __syncthreads();
  for (long long j = k + tid; j < ld; j += GJ_THREADS) m[k * ld + j] = mul(inv, m[k * ld + j]);
}

template <typename T>
__global__ void gj_eliminate_kernel(T* __restrict__ m, int n, int k, const T* __restrict__ f) {
  const long long ld = 2LL * n;
  const long long j = k + blockIdx.x * 256LL + threadIdx.x;
  if (j >= ld) return;
  const T pk = m[k * ld + j];
  const int i0 = blockIdx.y * GJ_ROWS;
  const int i1 = std::min(n, i0 + GJ_ROWS);
  for (int i = i0; i < i1; ++i) {
    const T fi = f[i];
    if (nonzero(fi)) m[(long long)i * ld + j] = sub(m[(long long)i * ld + j], mul(fi, pk));
  }
}

template <typename T>
hipError_t run(const void* a, int n, void* work, void* f, int* status, hipStream_t s) {
  T* m = static_cast<T*>(work);
  const long long total = 2LL * n * n;
  const unsigned g0 = (unsigned)std::max<long long>(1, std::min<long long>(8192, (total + 255) / 256));
  hipLaunchKernelGGL(gj_init_kernel<T>, dim3(g0), dim3(256), 0, s, static_cast<const T*>(a), m, n);
  for (int k = 0; k < n; ++k) {
    hipLaunchKernelGGL(gj_pivot_kernel<T>, dim3(1), dim3(GJ_THREADS), 0, s, m, n, k, static_cast<T*>(f), status);
    const long long cols = 2LL * n - k;
    const dim3 grid((unsigned)((cols + 255) / 256), (unsigned)((n + GJ_ROWS - 1) / GJ_ROWS));
    hipLaunchKernelGGL(gj_eliminate_kernel<T>, grid, dim3(256), 0, s, m, n, k, static_cast<const T*>(f));
  }
  return hipGetLastError();
}

}  // namespace

size_t gauss_jordan_work_bytes(int dt, int n) { return elem_bytes(dt) * (2ULL * n * n + n); }

hipError_t gauss_jordan_inverse(int dt, const void* a, int n, void* work, int* status, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  void* f = static_cast<char*>(work) + elem_bytes(dt) * 2ULL * n * n;
  switch (dt) {
    case F64: return run<double>(a, n, work, f, status, s);
    case C128: return run<cd>(a, n, work, f, status, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tci
