// Elementwise and vector kernels: dtype conversion, conjugation, scaling,
// linear combinations (TCI-spec appendix: convert, cplx_conj, scale,
// linear_combine), elementwise closeness (close), the Lanczos multi-dot /
// multi-axpy with FP64 accumulation, and the two-site MPO product W12.
#include <array>
#include <utility>

#include "common.hpp"
#include "vecops.hpp"

namespace tci {

template <typename T> struct VT;
template <> struct VT<double> { typedef double R; static constexpr bool c = false; };
template <> struct VT<float> { typedef float R; static constexpr bool c = false; };
template <> struct VT<cd> { typedef double R; static constexpr bool c = true; };
template <> struct VT<cf> { typedef float R; static constexpr bool c = true; };

__device__ inline void get2(const double* p, long long i, double& r, double& im) { r = p[i]; im = 0; }
__device__ inline void get2(const float* p, long long i, double& r, double& im) { r = p[i]; im = 0; }
__device__ inline void get2(const cd* p, long long i, double& r, double& im) { r = p[i].x; im = p[i].y; }
__device__ inline void get2(const cf* p, long long i, double& r, double& im) { r = p[i].x; im = p[i].y; }
__device__ inline void put2(double* p, long long i, double r, double) { p[i] = r; }
__device__ inline void put2(float* p, long long i, double r, double) { p[i] = (float)r; }
__device__ inline void put2(cd* p, long long i, double r, double im) { p[i] = cd{r, im}; }
__device__ inline void put2(cf* p, long long i, double r, double im) { p[i] = cf{(float)r, (float)im}; }

template <typename S, typename D>
__global__ void convert_kernel(const S* in, D* out, long long n) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    double r, im;
    get2(in, i, r, im);
    put2(out, i, r, im);
  }
}

static unsigned grid_for(long long n) { return (unsigned)std::max<long long>(1, std::min<long long>(4096, (n + 255) / 256)); }

template <typename S>
static hipError_t convert_from(const S* in, int dst, void* out, long long n, hipStream_t s) {
  switch (dst) {
    case F32: hipLaunchKernelGGL((convert_kernel<S, float>), dim3(grid_for(n)), dim3(256), 0, s, in, (float*)out, n); break;
    case F64: hipLaunchKernelGGL((convert_kernel<S, double>), dim3(grid_for(n)), dim3(256), 0, s, in, (double*)out, n); break;
    case C64: hipLaunchKernelGGL((convert_kernel<S, cf>), dim3(grid_for(n)), dim3(256), 0, s, in, (cf*)out, n); break;
    case C128: hipLaunchKernelGGL((convert_kernel<S, cd>), dim3(grid_for(n)), dim3(256), 0, s, in, (cd*)out, n); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t convert(int src, const void* in, int dst, void* out, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  switch (src) {
    case F32: return convert_from((const float*)in, dst, out, n, s);
    case F64: return convert_from((const double*)in, dst, out, n, s);
    case C64: return convert_from((const cf*)in, dst, out, n, s);
    case C128: return convert_from((const cd*)in, dst, out, n, s);
  }
  return hipErrorInvalidValue;
}

// out = conj(in) (plain copy for real types)
template <typename T>
__global__ void conj_kernel(const T* in, T* out, long long n) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    double r, im;
    get2(in, i, r, im);
    put2(out, i, r, -im);
  }
}

hipError_t conjugate(int dt, const void* in, void* out, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  switch (dt) {
    case F32: hipLaunchKernelGGL(conj_kernel<float>, dim3(grid_for(n)), dim3(256), 0, s, (const float*)in, (float*)out, n); break;
    case F64: hipLaunchKernelGGL(conj_kernel<double>, dim3(grid_for(n)), dim3(256), 0, s, (const double*)in, (double*)out, n); break;
    case C64: hipLaunchKernelGGL(conj_kernel<cf>, dim3(grid_for(n)), dim3(256), 0, s, (const cf*)in, (cf*)out, n); break;
    case C128: hipLaunchKernelGGL(conj_kernel<cd>, dim3(grid_for(n)), dim3(256), 0, s, (const cd*)in, (cd*)out, n); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// out = sum_q c_q in_q, c_q complex (re, im) in double, q < nin; in pointers
// and coefficients passed through a small device array.
template <typename T>
__global__ void lincomb_kernel(const LinCombArgs a, T* out, long long n) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    double ar = 0, ai = 0;
    for (int q = 0; q < a.nin; ++q) {
      double r, im;
      get2(reinterpret_cast<const T*>(a.in[q]), i, r, im);
      ar += a.cre[q] * r - a.cim[q] * im;
      ai += a.cre[q] * im + a.cim[q] * r;
    }
    put2(out, i, ar, ai);
  }
}

hipError_t linear_combine(int dt, const LinCombArgs& a, void* out, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  switch (dt) {
    case F32: hipLaunchKernelGGL(lincomb_kernel<float>, dim3(grid_for(n)), dim3(256), 0, s, a, (float*)out, n); break;
    case F64: hipLaunchKernelGGL(lincomb_kernel<double>, dim3(grid_for(n)), dim3(256), 0, s, a, (double*)out, n); break;
    case C64: hipLaunchKernelGGL(lincomb_kernel<cf>, dim3(grid_for(n)), dim3(256), 0, s, a, (cf*)out, n); break;
    case C128: hipLaunchKernelGGL(lincomb_kernel<cd>, dim3(grid_for(n)), dim3(256), 0, s, a, (cd*)out, n); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Per-block maximum of |a_i - b_i| (modulus for complex), final max over blocks.
template <typename T>
__global__ __launch_bounds__(256) void maxdiff_kernel(const T* a, const T* b, long long n, double* partial) {
  __shared__ double sh[256];
  double m = 0.0;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    double ar, ai, br, bi;
    get2(a, i, ar, ai);
    get2(b, i, br, bi);
    const double dr = ar - br, di = ai - bi;
    const double v = sqrt(dr * dr + di * di);
    m = (v > m || v != v) ? v : m;
  }
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      const double o = sh[threadIdx.x + off];
      if (o > sh[threadIdx.x] || o != o) sh[threadIdx.x] = o;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

hipError_t max_abs_diff(int dt, const void* a, const void* b, long long n, double* partial, int nparts,
                        hipStream_t s) {
  const unsigned g = (unsigned)std::max<long long>(1, std::min<long long>(nparts, (n + 255) / 256));
  switch (dt) {
    case F32: hipLaunchKernelGGL(maxdiff_kernel<float>, dim3(g), dim3(256), 0, s, (const float*)a, (const float*)b, n, partial); break;
    case F64: hipLaunchKernelGGL(maxdiff_kernel<double>, dim3(g), dim3(256), 0, s, (const double*)a, (const double*)b, n, partial); break;
    case C64: hipLaunchKernelGGL(maxdiff_kernel<cf>, dim3(g), dim3(256), 0, s, (const cf*)a, (const cf*)b, n, partial); break;
    case C128: hipLaunchKernelGGL(maxdiff_kernel<cd>, dim3(g), dim3(256), 0, s, (const cd*)a, (const cd*)b, n, partial); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Lanczos vector kernels on complex128 vectors of length n.
//   multidot: c_q = <v_q, w> = sum_i conj(v_q[i]) w[i], q < nv (basis rows of
//             length n, ld n), two-pass deterministic reduction;
//   multiaxpy: w[i] += sum_q c_q v_q[i]  (c given as (re, im) on the device).
// ---------------------------------------------------------------------------
constexpr int MD_BLOCKS = 1024;
constexpr int MD_MAXV = 32;
static_assert(MULTIDOT_PARTIAL_DOUBLES >= MD_BLOCKS * MD_MAXV * 2, "multidot partial buffer");

__device__ inline double wave_sum64(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Basis vectors are complex128, or complex64 for the complex64 operands
// (arithmetic in FP64 either way).
__device__ inline cd ldv(const cd* p) { return *p; }
__device__ inline cd ldv(const cf* p) {
  const cf v = *p;
  return cd{(double)v.x, (double)v.y};
}
// Two consecutive elements (p 16-byte aligned): one 16-byte load for complex64.
__device__ inline void ldv2(const cd* p, cd& a, cd& b) {
  a = p[0];
  b = p[1];
}
__device__ inline void ldv2(const cf* p, cd& a, cd& b) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  a = cd{(double)v.x, (double)v.y};
  b = cd{(double)v.z, (double)v.w};
}
// The sweeps below take element pairs (2i, 2i+1) when n is even, so that a
// complex64 basis vector is read with 16-byte loads; an odd n runs the
// single-element loop over all of it.

// NV is a compile-time bound on nv so that the accumulators stay in registers.
template <int NV, typename VT>
__global__ __launch_bounds__(256) void multidot_partial_kernel(const VT* V, int nv, const cd* w, long long n,
                                                               double* partial, const double* gate) {
  if (gate && *gate == 0.0) return;   // the pass is switched off on the device
  __shared__ double sh[4][2 * NV];
  double accr[NV], acci[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) { accr[q] = 0.0; acci[q] = 0.0; }
  const long long np2 = (n & 1) ? 0 : n / 2, stride = (long long)gridDim.x * 256;
  for (long long i2 = blockIdx.x * 256LL + threadIdx.x; i2 < np2; i2 += stride) {
    const cd x0 = w[2 * i2], x1 = w[2 * i2 + 1];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      if (q < nv) {
        cd v0, v1;
        ldv2(V + (long long)q * n + 2 * i2, v0, v1);
        accr[q] += (v0.x * x0.x + v0.y * x0.y) + (v1.x * x1.x + v1.y * x1.y);
        acci[q] += (v0.x * x0.y - v0.y * x0.x) + (v1.x * x1.y - v1.y * x1.x);
      }
    }
  }
  for (long long i = 2 * np2 + blockIdx.x * 256LL + threadIdx.x; i < n; i += stride) {
    const cd x = w[i];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      if (q < nv) {
        const cd v = ldv(V + (long long)q * n + i);
        accr[q] += v.x * x.x + v.y * x.y;
        acci[q] += v.x * x.y - v.y * x.x;
      }
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    if (q < nv) {
      const double r = wave_sum64(accr[q]), im = wave_sum64(acci[q]);
      if (lane == 0) { sh[wv][2 * q] = r; sh[wv][2 * q + 1] = im; }
    }
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < 2 * nv) {
    const double v = (sh[0][t] + sh[1][t]) + (sh[2][t] + sh[3][t]);
    partial[((long long)blockIdx.x * MD_MAXV + t / 2) * 2 + (t & 1)] = v;
  }
}

// One workgroup per coefficient q: fixed-order sums of the block partials.
__global__ __launch_bounds__(256) void multidot_final_kernel(const double* partial, int nparts, int nv, double* out,
                                                             const double* gate = nullptr) {
  if (gate && *gate == 0.0) return;
  __shared__ double sr[256], si[256];
  const int q = blockIdx.x, t = threadIdx.x;
  double ar = 0.0, ai = 0.0;
  for (int b = t; b < nparts; b += 256) {
    ar += partial[((long long)b * MD_MAXV + q) * 2 + 0];
    ai += partial[((long long)b * MD_MAXV + q) * 2 + 1];
  }
  sr[t] = ar;
  si[t] = ai;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) { sr[t] += sr[t + off]; si[t] += si[t + off]; }
    __syncthreads();
  }
  if (t == 0) { out[2 * q] = sr[0]; out[2 * q + 1] = si[0]; }
}

static unsigned md_grid(long long n) {
  return (unsigned)std::max<long long>(1, std::min<long long>(MD_BLOCKS, (n + 255) / 256));
}

// Launch tables with one instantiation per basis size (1..MD_MAXV), so that
// each kernel holds exactly the registers its basis needs.
template <typename VT>
using MdLaunch = void (*)(unsigned, hipStream_t, const VT*, int, const cd*, long long, double*, const double*);
template <int NV, typename VT>
void md_launch(unsigned g, hipStream_t s, const VT* V, int nv, const cd* w, long long n, double* partial,
               const double* gate) {
  hipLaunchKernelGGL((multidot_partial_kernel<NV, VT>), dim3(g), dim3(256), 0, s, V, nv, w, n, partial, gate);
}
template <typename VT, int... I>
constexpr std::array<MdLaunch<VT>, sizeof...(I)> md_make(std::integer_sequence<int, I...>) {
  return {&md_launch<I + 1, VT>...};
}
template <typename VT>
static const std::array<MdLaunch<VT>, MD_MAXV>& md_table() {
  static const auto t = md_make<VT>(std::make_integer_sequence<int, MD_MAXV>{});
  return t;
}

hipError_t multidot(const void* V, int nv, const void* w, long long n, double* partial, double* out,
                    hipStream_t s, int vdt, const double* gate) {
  if (nv <= 0) return hipSuccess;
  if (nv > MD_MAXV || (vdt != C128 && vdt != C64)) return hipErrorInvalidValue;
  const unsigned g = md_grid(n);
  const cd* wc = (const cd*)w;
  if (vdt == C64) md_table<cf>()[nv - 1](g, s, (const cf*)V, nv, wc, n, partial, gate);
  else md_table<cd>()[nv - 1](g, s, (const cd*)V, nv, wc, n, partial, gate);
  hipLaunchKernelGGL(multidot_final_kernel, dim3(nv), dim3(256), 0, s, partial, (int)g, nv, out, gate);
  return hipGetLastError();
}

// w = y (complex64 widened to complex128) and d = <v, w> in one sweep (block
// partials in the multidot layout, q = 0).
template <typename VT>
__global__ __launch_bounds__(256) void widen_dot_kernel(const cf* y, const VT* v, cd* w, long long n,
                                                       double* partial) {
  __shared__ double sh[4][2];
  double ar = 0.0, ai = 0.0;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    const cf yv = y[i];
    const cd x{(double)yv.x, (double)yv.y};
    w[i] = x;
    const cd vv = ldv(v + i);
    ar += vv.x * x.x + vv.y * x.y;
    ai += vv.x * x.y - vv.y * x.x;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  ar = wave_sum64(ar);
  ai = wave_sum64(ai);
  if (lane == 0) { sh[wv][0] = ar; sh[wv][1] = ai; }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < 2) partial[(long long)blockIdx.x * MD_MAXV * 2 + t] = (sh[0][t] + sh[1][t]) + (sh[2][t] + sh[3][t]);
}

hipError_t widen_multidot_c64(const void* y, const void* v, void* w, long long n, double* partial, double* out,
                              hipStream_t s, int vdt) {
  const unsigned g = md_grid(n);
  if (vdt == C64)
    hipLaunchKernelGGL(widen_dot_kernel<cf>, dim3(g), dim3(256), 0, s, (const cf*)y, (const cf*)v, (cd*)w, n, partial);
  else
    hipLaunchKernelGGL(widen_dot_kernel<cd>, dim3(g), dim3(256), 0, s, (const cf*)y, (const cd*)v, (cd*)w, n, partial);
  hipLaunchKernelGGL(multidot_final_kernel, dim3(1), dim3(256), 0, s, partial, (int)g, 1, out);
  return hipGetLastError();
}

// out (complex64) = x * (sr + i si) rounded
__global__ void scale_to_c64_kernel(const cd* x, double sr, double si, cf* out, long long n) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    const cd a = x[i];
    out[i] = cf{(float)(sr * a.x - si * a.y), (float)(sr * a.y + si * a.x)};
  }
}

hipError_t scale_to_c64(const void* x, double sr, double si, void* out, long long n, hipStream_t s) {
  hipLaunchKernelGGL(scale_to_c64_kernel, dim3(grid_for(n)), dim3(256), 0, s, (const cd*)x, sr, si, (cf*)out, n);
  return hipGetLastError();
}


// w += sign * sum_q c_q v_q; with nrm_part, block b also stores its part of ||w||^2.
template <int NV, typename VT>
__global__ __launch_bounds__(256) void multiaxpy_kernel(const VT* V, int nv, const double* c, double sign, cd* w,
                                                        long long n, double* nrm_part, const double* gate) {
  if (gate && *gate == 0.0) return;   // the pass is switched off on the device
  __shared__ double sh[4];
  double cr[NV], ci[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    cr[q] = q < nv ? sign * c[2 * q] : 0.0;
    ci[q] = q < nv ? sign * c[2 * q + 1] : 0.0;
  }
  double ss = 0.0;
  const long long np2 = (n & 1) ? 0 : n / 2, stride = (long long)gridDim.x * 256;
  for (long long i2 = blockIdx.x * 256LL + threadIdx.x; i2 < np2; i2 += stride) {
    cd a0 = w[2 * i2], a1 = w[2 * i2 + 1];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      if (q < nv) {
        cd v0, v1;
        ldv2(V + (long long)q * n + 2 * i2, v0, v1);
        a0.x += cr[q] * v0.x - ci[q] * v0.y;
        a0.y += cr[q] * v0.y + ci[q] * v0.x;
        a1.x += cr[q] * v1.x - ci[q] * v1.y;
        a1.y += cr[q] * v1.y + ci[q] * v1.x;
      }
    }
    w[2 * i2] = a0;
    w[2 * i2 + 1] = a1;
    ss += (a0.x * a0.x + a0.y * a0.y) + (a1.x * a1.x + a1.y * a1.y);
  }
  for (long long i = 2 * np2 + blockIdx.x * 256LL + threadIdx.x; i < n; i += stride) {
    cd acc = w[i];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      if (q < nv) {
        const cd v = ldv(V + (long long)q * n + i);
        acc.x += cr[q] * v.x - ci[q] * v.y;
        acc.y += cr[q] * v.y + ci[q] * v.x;
      }
    }
    w[i] = acc;
    ss += acc.x * acc.x + acc.y * acc.y;
  }
  if (nrm_part) {
    ss = wave_sum64(ss);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = ss;
    __syncthreads();
    if (threadIdx.x == 0) nrm_part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  }
}

__global__ __launch_bounds__(256) void sum_parts_kernel(const double* part, int nparts, double* out,
                                                        const double* gate) {
  if (gate && *gate == 0.0) return;
  __shared__ double sh[256];
  const int t = threadIdx.x;
  double a = 0.0;
  for (int b = t; b < nparts; b += 256) a += part[b];
  sh[t] = a;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) sh[t] += sh[t + off];
    __syncthreads();
  }
  if (t == 0) out[0] = sh[0];
}

template <typename VT>
using MaLaunch = void (*)(unsigned, hipStream_t, const VT*, int, const double*, double, cd*, long long, double*,
                          const double*);
template <int NV, typename VT>
void ma_launch(unsigned g, hipStream_t s, const VT* V, int nv, const double* c, double sign, cd* w, long long n,
               double* nrm_part, const double* gate) {
  hipLaunchKernelGGL((multiaxpy_kernel<NV, VT>), dim3(g), dim3(256), 0, s, V, nv, c, sign, w, n, nrm_part, gate);
}
template <typename VT, int... I>
constexpr std::array<MaLaunch<VT>, sizeof...(I)> ma_make(std::integer_sequence<int, I...>) {
  return {&ma_launch<I + 1, VT>...};
}
template <typename VT>
static const std::array<MaLaunch<VT>, MD_MAXV>& ma_table() {
  static const auto t = ma_make<VT>(std::make_integer_sequence<int, MD_MAXV>{});
  return t;
}

static hipError_t multiaxpy_launch(const void* V, int nv, const double* c, double sign, void* w, long long n,
                                   double* nrm_part, hipStream_t s, int vdt, const double* gate = nullptr) {
  if (vdt != C128 && vdt != C64) return hipErrorInvalidValue;
  const unsigned g = md_grid(n);
  cd* wc = (cd*)w;
  if (vdt == C64) ma_table<cf>()[nv - 1](g, s, (const cf*)V, nv, c, sign, wc, n, nrm_part, gate);
  else ma_table<cd>()[nv - 1](g, s, (const cd*)V, nv, c, sign, wc, n, nrm_part, gate);
  return hipGetLastError();
}

hipError_t multiaxpy(const void* V, int nv, const double* c, double sign, void* w, long long n, hipStream_t s,
                     int vdt) {
  if (nv <= 0) return hipSuccess;
  if (nv > MD_MAXV) return hipErrorInvalidValue;
  return multiaxpy_launch(V, nv, c, sign, w, n, nullptr, s, vdt);
}

// Fused sweep of one Lanczos step: w -= alpha v_{NV-1} + beta v_{NV-2} (the
// beta term for NV >= 2; alpha = *palpha, on the device), then
// d_q = <v_q, w> of the updated w for q < NV (block partials in the multidot
// layout).  Only the two recurrence vectors are held across the update; the
// others are streamed once for their dot.
template <int NV, typename VT>
__global__ __launch_bounds__(256) void three_term_dot_kernel(const VT* V, const double* palpha, const double* pbeta,
                                                             cd* w, long long n, double* partial) {
  __shared__ double sh[4][2 * NV];
  const double alpha = *palpha;
  const double beta = pbeta ? *pbeta : 0.0;
  double accr[NV], acci[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) { accr[q] = 0.0; acci[q] = 0.0; }
  const long long np2 = (n & 1) ? 0 : n / 2, stride = (long long)gridDim.x * 256;
  for (long long i2 = blockIdx.x * 256LL + threadIdx.x; i2 < np2; i2 += stride) {
    const long long i = 2 * i2;
    cd y0 = w[i], y1 = w[i + 1];
    cd vj0, vj1, vp0{0.0, 0.0}, vp1{0.0, 0.0};
    ldv2(V + (long long)(NV - 1) * n + i, vj0, vj1);
    y0.x -= alpha * vj0.x;
    y0.y -= alpha * vj0.y;
    y1.x -= alpha * vj1.x;
    y1.y -= alpha * vj1.y;
    if constexpr (NV >= 2) {
      ldv2(V + (long long)(NV - 2) * n + i, vp0, vp1);
      y0.x -= beta * vp0.x;
      y0.y -= beta * vp0.y;
      y1.x -= beta * vp1.x;
      y1.y -= beta * vp1.y;
    }
    w[i] = y0;
    w[i + 1] = y1;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      cd v0, v1;
      if (q == NV - 1) {
        v0 = vj0;
        v1 = vj1;
      } else if (q == NV - 2) {
        v0 = vp0;
        v1 = vp1;
      } else {
        ldv2(V + (long long)q * n + i, v0, v1);
      }
      accr[q] += (v0.x * y0.x + v0.y * y0.y) + (v1.x * y1.x + v1.y * y1.y);
      acci[q] += (v0.x * y0.y - v0.y * y0.x) + (v1.x * y1.y - v1.y * y1.x);
    }
  }
  for (long long i = 2 * np2 + blockIdx.x * 256LL + threadIdx.x; i < n; i += stride) {
    cd y = w[i];
    const cd vj = ldv(V + (long long)(NV - 1) * n + i);
    y.x -= alpha * vj.x;
    y.y -= alpha * vj.y;
    cd vp{0.0, 0.0};
    if constexpr (NV >= 2) {
      vp = ldv(V + (long long)(NV - 2) * n + i);
      y.x -= beta * vp.x;
      y.y -= beta * vp.y;
    }
    w[i] = y;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const cd v = q == NV - 1 ? vj : (q == NV - 2 ? vp : ldv(V + (long long)q * n + i));
      accr[q] += v.x * y.x + v.y * y.y;
      acci[q] += v.x * y.y - v.y * y.x;
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    const double r = wave_sum64(accr[q]), im = wave_sum64(acci[q]);
    if (lane == 0) { sh[wv][2 * q] = r; sh[wv][2 * q + 1] = im; }
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < 2 * NV) {
    const double vv = (sh[0][t] + sh[1][t]) + (sh[2][t] + sh[3][t]);
    partial[((long long)blockIdx.x * MD_MAXV + t / 2) * 2 + (t & 1)] = vv;
  }
}

template <typename VT>
using TtLaunch = void (*)(unsigned, hipStream_t, const VT*, const double*, const double*, cd*, long long, double*);
template <int NV, typename VT>
void tt_launch(unsigned g, hipStream_t s, const VT* V, const double* alpha, const double* beta, cd* w, long long n,
               double* partial) {
  hipLaunchKernelGGL((three_term_dot_kernel<NV, VT>), dim3(g), dim3(256), 0, s, V, alpha, beta, w, n, partial);
}
template <typename VT, int... I>
constexpr std::array<TtLaunch<VT>, sizeof...(I)> tt_make(std::integer_sequence<int, I...>) {
  return {&tt_launch<I + 1, VT>...};
}
template <typename VT>
static const std::array<TtLaunch<VT>, MD_MAXV>& tt_table() {
  static const auto t = tt_make<VT>(std::make_integer_sequence<int, MD_MAXV>{});
  return t;
}

hipError_t three_term_multidot(const void* V, int nv, const double* alpha, const double* beta, void* w, long long n,
                               double* partial, double* out, hipStream_t s, int vdt) {
  if (nv <= 0 || nv > MD_MAXV || (vdt != C128 && vdt != C64)) return hipErrorInvalidValue;
  const unsigned g = md_grid(n);
  if (vdt == C64) tt_table<cf>()[nv - 1](g, s, (const cf*)V, alpha, beta, (cd*)w, n, partial);
  else tt_table<cd>()[nv - 1](g, s, (const cd*)V, alpha, beta, (cd*)w, n, partial);
  hipLaunchKernelGGL(multidot_final_kernel, dim3(nv), dim3(256), 0, s, partial, (int)g, nv, out);
  return hipGetLastError();
}

hipError_t multiaxpy_norm2(const void* V, int nv, const double* c, double sign, void* w, long long n,
                           double* partial, double* out, hipStream_t s, int vdt, const double* gate) {
  if (nv <= 0 || nv > MD_MAXV) return hipErrorInvalidValue;
  hipError_t e = multiaxpy_launch(V, nv, c, sign, w, n, partial, s, vdt, gate);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(256), 0, s, partial, (int)md_grid(n), out, gate);
  return hipGetLastError();
}

// w = x * (sr + i si) (scaled copy, complex128)
__global__ void scale_copy_kernel(const cd* x, double sr, double si, cd* w, long long n) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    const cd v = x[i];
    w[i] = cd{sr * v.x - si * v.y, sr * v.y + si * v.x};
  }
}

// The same with the factor (ps[0] + i ps[1]) read on the device.
__global__ void scale_copy_dev_kernel(const cd* x, const double* ps, cd* w, long long n, const double* gate) {
  if (gate && *gate == 0.0) return;
  const double sr = ps[0], si = ps[1];
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    const cd v = x[i];
    w[i] = cd{sr * v.x - si * v.y, sr * v.y + si * v.x};
  }
}
__global__ void scale_to_c64_dev_kernel(const cd* x, const double* ps, cf* out, long long n, const double* gate) {
  if (gate && *gate == 0.0) return;
  const double sr = ps[0], si = ps[1];
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    const cd a = x[i];
    out[i] = cf{(float)(sr * a.x - si * a.y), (float)(sr * a.y + si * a.x)};
  }
}

hipError_t scale_copy_dev(const void* x, const double* ps, void* w, long long n, hipStream_t s,
                          const double* gate) {
  hipLaunchKernelGGL(scale_copy_dev_kernel, dim3(grid_for(n)), dim3(256), 0, s, (const cd*)x, ps, (cd*)w, n, gate);
  return hipGetLastError();
}

hipError_t scale_to_c64_dev(const void* x, const double* ps, void* out, long long n, hipStream_t s,
                            const double* gate) {
  hipLaunchKernelGGL(scale_to_c64_dev_kernel, dim3(grid_for(n)), dim3(256), 0, s, (const cd*)x, ps, (cf*)out, n,
                     gate);
  return hipGetLastError();
}

hipError_t scale_copy(const void* x, double sr, double si, void* w, long long n, hipStream_t s) {
  hipLaunchKernelGGL(scale_copy_kernel, dim3(grid_for(n)), dim3(256), 0, s, (const cd*)x, sr, si, (cd*)w, n);
  return hipGetLastError();
}

// Elementwise in-place scaling by a complex scalar for any dtype.
template <typename T>
__global__ void scale_kernel(T* x, long long n, double sr, double si) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    double r, im;
    get2(x, i, r, im);
    put2(x, i, sr * r - si * im, sr * im + si * r);
  }
}

hipError_t scale_inplace(int dt, void* x, long long n, double sr, double si, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  switch (dt) {
    case F32: hipLaunchKernelGGL(scale_kernel<float>, dim3(grid_for(n)), dim3(256), 0, s, (float*)x, n, sr, si); break;
    case F64: hipLaunchKernelGGL(scale_kernel<double>, dim3(grid_for(n)), dim3(256), 0, s, (double*)x, n, sr, si); break;
    case C64: hipLaunchKernelGGL(scale_kernel<cf>, dim3(grid_for(n)), dim3(256), 0, s, (cf*)x, n, sr, si); break;
    case C128: hipLaunchKernelGGL(scale_kernel<cd>, dim3(grid_for(n)), dim3(256), 0, s, (cd*)x, n, sr, si); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// W12[(w, s1', s2'), (s1, s2, w'')] = sum_{w'} W1[w,w',s1,s1'] W2[w',w'',s2,s2']
// (one thread per output element; W1, W2 of shape (wd, wd, d, d)).
template <typename T>
__global__ void w12_kernel(const T* W1, const T* W2, T* W12, int wd, int d) {
  const int K = wd * d * d;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= K * K) return;
  const int row = idx / K, col = idx % K;
  const int w = row / (d * d), s1p = (row / d) % d, s2p = row % d;
  const int s1 = col / (d * wd), s2 = (col / wd) % d, wpp = col % wd;
  double ar = 0, ai = 0;
  for (int wp = 0; wp < wd; ++wp) {
    double r1, i1, r2, i2;
    get2(W1, (((long long)w * wd + wp) * d + s1) * d + s1p, r1, i1);
    get2(W2, (((long long)wp * wd + wpp) * d + s2) * d + s2p, r2, i2);
    ar += r1 * r2 - i1 * i2;
    ai += r1 * i2 + i1 * r2;
  }
  put2(W12, idx, ar, ai);
}

hipError_t mpo_pair(int dt, const void* W1, const void* W2, void* W12, int wd, int d, hipStream_t s) {
  const int K = wd * d * d, n = K * K;
  switch (dt) {
    case F32: hipLaunchKernelGGL(w12_kernel<float>, dim3((n + 255) / 256), dim3(256), 0, s, (const float*)W1, (const float*)W2, (float*)W12, wd, d); break;
    case F64: hipLaunchKernelGGL(w12_kernel<double>, dim3((n + 255) / 256), dim3(256), 0, s, (const double*)W1, (const double*)W2, (double*)W12, wd, d); break;
    case C64: hipLaunchKernelGGL(w12_kernel<cf>, dim3((n + 255) / 256), dim3(256), 0, s, (const cf*)W1, (const cf*)W2, (cf*)W12, wd, d); break;
    case C128: hipLaunchKernelGGL(w12_kernel<cd>, dim3((n + 255) / 256), dim3(256), 0, s, (const cd*)W1, (const cd*)W2, (cd*)W12, wd, d); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Upper triangle of a k x k matrix (strict lower part zeroed), diagonal
// multiplied by mask (0 for dropped columns): R factor of Cholesky-QR.
template <typename T>
__global__ void triu_mask_kernel(T* R, long long ld, long long sR, int k, const double* mask, long long smask) {
  const int b = blockIdx.y;
  for (long long idx = blockIdx.x * 256LL + threadIdx.x; idx < (long long)k * k; idx += (long long)gridDim.x * 256) {
    const int r = (int)(idx / k), c = (int)(idx % k);
    T* p = R + b * sR + (long long)r * ld + c;
    if (r > c) put2(p, 0, 0.0, 0.0);
    else if (r == c) {
      double vr, vi;
      get2(p, 0, vr, vi);
      const double m = mask[b * smask + r];
      put2(p, 0, vr * m, vi * m);
    }
  }
}

hipError_t triu_mask(int dt, void* R, long long ld, long long sR, int k, const double* mask, long long smask,
                     int batch, hipStream_t s) {
  dim3 g(grid_for((long long)k * k), batch);
  switch (dt) {
    case F64: hipLaunchKernelGGL(triu_mask_kernel<double>, g, dim3(256), 0, s, (double*)R, ld, sR, k, mask, smask); break;
    case C128: hipLaunchKernelGGL(triu_mask_kernel<cd>, g, dim3(256), 0, s, (cd*)R, ld, sR, k, mask, smask); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Reverse the order of the first k columns of U (n x ld) and of lam (for
// ascending eigenvalue order).
template <typename T>
__global__ void reverse_cols_kernel(T* U, long long ld, int rows, int k) {
  const long long idx = blockIdx.x * 256LL + threadIdx.x;
  if (idx >= (long long)rows * (k / 2)) return;
  const int r = (int)(idx / (k / 2)), c = (int)(idx % (k / 2));
  T* row = U + (long long)r * ld;
  const T t = row[c];
  row[c] = row[k - 1 - c];
  row[k - 1 - c] = t;
}

hipError_t reverse_columns(int dt, void* U, long long ld, int rows, int k, hipStream_t s) {
  if (k < 2) return hipSuccess;
  const long long n = (long long)rows * (k / 2);
  const unsigned g = (unsigned)((n + 255) / 256);
  if (dt == C128) hipLaunchKernelGGL(reverse_cols_kernel<cd>, dim3(g), dim3(256), 0, s, (cd*)U, ld, rows, k);
  else if (dt == F64) hipLaunchKernelGGL(reverse_cols_kernel<double>, dim3(g), dim3(256), 0, s, (double*)U, ld, rows, k);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace tci

namespace tci {

// Kernel fill of zeros: safe inside captured HIP graphs (no memset nodes).
__global__ void zero_fill_kernel(unsigned int* p, long long nwords, unsigned char* tail, int ntail) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < nwords; i += (long long)gridDim.x * 256) p[i] = 0u;
  if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

hipError_t zero_fill(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  if (reinterpret_cast<uintptr_t>(p) % 4 != 0) return hipErrorInvalidValue;
  const long long nwords = (long long)(bytes / 4);
  const int ntail = (int)(bytes % 4);
  const unsigned g = (unsigned)std::max<long long>(1, std::min<long long>(2048, (nwords + 255) / 256));
  hipLaunchKernelGGL(zero_fill_kernel, dim3(g), dim3(256), 0, s, static_cast<unsigned int*>(p), nwords,
                     static_cast<unsigned char*>(p) + nwords * 4, ntail);
  return hipGetLastError();
}

__global__ void zero_fill_rows_kernel(unsigned char* p, long long words, long long stride) {
  unsigned int* q = reinterpret_cast<unsigned int*>(p + blockIdx.y * stride);
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < words; i += (long long)gridDim.x * 256) q[i] = 0u;
}

hipError_t zero_fill_rows(void* p, size_t bytes, size_t stride, int count, hipStream_t s) {
  if (bytes == 0 || count <= 0) return hipSuccess;
  if (reinterpret_cast<uintptr_t>(p) % 4 != 0 || bytes % 4 != 0 || stride % 4 != 0 || bytes > stride)
    return hipErrorInvalidValue;
  const long long words = (long long)(bytes / 4);
  const unsigned g = (unsigned)std::max<long long>(1, std::min<long long>(256, (words + 255) / 256));
  hipLaunchKernelGGL(zero_fill_rows_kernel, dim3(g, count), dim3(256), 0, s, static_cast<unsigned char*>(p), words,
                     (long long)stride);
  return hipGetLastError();
}

}  // namespace tci
