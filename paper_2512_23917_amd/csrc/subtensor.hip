// Sub-tensor movement and construction kernels: strided box copies (extract,
// shrink, expand, replace, concatenate, stack), constant fill, identity,
// partial trace, real and imaginary parts, and the identity shift used by the
// matrix exponential.
#include "subtensor.hpp"

#include <algorithm>
#include <type_traits>

namespace tci {

namespace {

struct b16 {
  unsigned long long lo, hi;
};

template <typename E>
__global__ void box_copy_kernel(const E* __restrict__ src, E* __restrict__ dst, BoxCopy c) {
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < c.total; e += (long long)gridDim.x * 256) {
    long long rem = e, so = c.soff, dof = c.doff;
    for (int b = c.order - 1; b >= 0; --b) {
      const long long i = rem % c.dims[b];
      rem /= c.dims[b];
      so += i * c.sstride[b];
      dof += i * c.dstride[b];
    }
    dst[dof] = src[so];
  }
}

unsigned grid_of(long long n) {
  return (unsigned)std::max<long long>(1, std::min<long long>(4096, (n + 255) / 256));
}

template <typename T>
__global__ void fill_kernel(T* x, long long n, T v) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) x[i] = v;
}

template <typename T>
__device__ inline void acc_add(double& r, double& im, const T& v);
template <>
__device__ inline void acc_add<float>(double& r, double&, const float& v) { r += v; }
template <>
__device__ inline void acc_add<double>(double& r, double&, const double& v) { r += v; }
template <>
__device__ inline void acc_add<cf>(double& r, double& im, const cf& v) { r += v.x; im += v.y; }
template <>
__device__ inline void acc_add<cd>(double& r, double& im, const cd& v) { r += v.x; im += v.y; }

template <typename T>
__device__ inline T make_val(double r, double im);
template <>
__device__ inline float make_val<float>(double r, double) { return (float)r; }
template <>
__device__ inline double make_val<double>(double r, double) { return r; }
template <>
__device__ inline cf make_val<cf>(double r, double im) { return cf{(float)r, (float)im}; }
template <>
__device__ inline cd make_val<cd>(double r, double im) { return cd{r, im}; }

// out[o] = sum over the traced multi-index t of in[base(o) + t . tstride]
template <typename T>
__global__ void trace_kernel(const T* __restrict__ in, T* __restrict__ out, TraceArgs a) {
  for (long long o = blockIdx.x * 256LL + threadIdx.x; o < a.nout; o += (long long)gridDim.x * 256) {
    long long rem = o, base = 0;
    for (int b = a.nkeep - 1; b >= 0; --b) {
      const long long i = rem % a.kdims[b];
      rem /= a.kdims[b];
      base += i * a.kstride[b];
    }
    double r = 0.0, im = 0.0;
    for (long long t = 0; t < a.ntr; ++t) {
      long long tr = t, off = base;
      for (int p = a.npair - 1; p >= 0; --p) {
        const long long i = tr % a.pdims[p];
        tr /= a.pdims[p];
        off += i * a.pstride[p];
      }
      acc_add<T>(r, im, in[off]);
    }
    out[o] = make_val<T>(r, im);
  }
}

template <typename T>
__global__ void add_diag_kernel(T* a, long long ld, int n, double v) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double r, im = 0.0;
  T x = a[(long long)i * ld + i];
  if constexpr (sizeof(T) == 4 || sizeof(T) == 8 && std::is_same<T, double>::value) {
    r = (double)x + v;
    a[(long long)i * ld + i] = make_val<T>(r, 0.0);
  } else {
    r = (double)x.x + v;
    im = (double)x.y;
    a[(long long)i * ld + i] = make_val<T>(r, im);
  }
}

template <typename C, typename R>
__global__ void part_kernel(const C* __restrict__ in, R* __restrict__ out, long long n, int imag) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    out[i] = imag ? in[i].y : in[i].x;
}

}  // namespace

hipError_t complex_part(int dt, const void* in, void* out, long long n, bool imag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned g = grid_of(n);
  switch (dt) {
    case C64:
      hipLaunchKernelGGL((part_kernel<cf, float>), dim3(g), dim3(256), 0, s, (const cf*)in, (float*)out, n, (int)imag);
      break;
    case C128:
      hipLaunchKernelGGL((part_kernel<cd, double>), dim3(g), dim3(256), 0, s, (const cd*)in, (double*)out, n,
                         (int)imag);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t box_copy(size_t elem, const void* src, void* dst, const BoxCopy& c, hipStream_t s) {
  if (c.total <= 0) return hipSuccess;
  if (c.order < 1 || c.order > SUB_MAX_ORDER) return hipErrorInvalidValue;
  const unsigned g = grid_of(c.total);
  switch (elem) {
    case 4: hipLaunchKernelGGL(box_copy_kernel<float>, dim3(g), dim3(256), 0, s, (const float*)src, (float*)dst, c); break;
    case 8:
      hipLaunchKernelGGL(box_copy_kernel<unsigned long long>, dim3(g), dim3(256), 0, s,
                         (const unsigned long long*)src, (unsigned long long*)dst, c);
      break;
    case 16: hipLaunchKernelGGL(box_copy_kernel<b16>, dim3(g), dim3(256), 0, s, (const b16*)src, (b16*)dst, c); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t fill_value(int dt, void* x, long long n, double vr, double vi, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned g = grid_of(n);
  switch (dt) {
    case F32: hipLaunchKernelGGL(fill_kernel<float>, dim3(g), dim3(256), 0, s, (float*)x, n, (float)vr); break;
    case F64: hipLaunchKernelGGL(fill_kernel<double>, dim3(g), dim3(256), 0, s, (double*)x, n, vr); break;
    case C64:
      hipLaunchKernelGGL(fill_kernel<cf>, dim3(g), dim3(256), 0, s, (cf*)x, n, cf{(float)vr, (float)vi});
      break;
    case C128: hipLaunchKernelGGL(fill_kernel<cd>, dim3(g), dim3(256), 0, s, (cd*)x, n, cd{vr, vi}); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t add_diag(int dt, void* a, long long ld, int n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned g = (unsigned)((n + 255) / 256);
  switch (dt) {
    case F32: hipLaunchKernelGGL(add_diag_kernel<float>, dim3(g), dim3(256), 0, s, (float*)a, ld, n, v); break;
    case F64: hipLaunchKernelGGL(add_diag_kernel<double>, dim3(g), dim3(256), 0, s, (double*)a, ld, n, v); break;
    case C64: hipLaunchKernelGGL(add_diag_kernel<cf>, dim3(g), dim3(256), 0, s, (cf*)a, ld, n, v); break;
    case C128: hipLaunchKernelGGL(add_diag_kernel<cd>, dim3(g), dim3(256), 0, s, (cd*)a, ld, n, v); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t partial_trace(int dt, const void* in, void* out, const TraceArgs& a, hipStream_t s) {
  if (a.nout <= 0) return hipSuccess;
  const unsigned g = grid_of(a.nout);
  switch (dt) {
    case F32: hipLaunchKernelGGL(trace_kernel<float>, dim3(g), dim3(256), 0, s, (const float*)in, (float*)out, a); break;
    case F64: hipLaunchKernelGGL(trace_kernel<double>, dim3(g), dim3(256), 0, s, (const double*)in, (double*)out, a); break;
    case C64: hipLaunchKernelGGL(trace_kernel<cf>, dim3(g), dim3(256), 0, s, (const cf*)in, (cf*)out, a); break;
    case C128: hipLaunchKernelGGL(trace_kernel<cd>, dim3(g), dim3(256), 0, s, (const cd*)in, (cd*)out, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace tci
