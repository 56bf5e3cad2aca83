// Sub-tensor movement and construction kernels (see subtensor.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace tci {

constexpr int SUB_MAX_ORDER = 9;   // bonds of a tensor, plus one inserted by stack

// dst[doff + sum_b i_b dstride_b] = src[soff + sum_b i_b sstride_b] for every
// index i of the box dims[0..order) (row-major walk, element strides).
struct BoxCopy {
  int order;
  long long dims[SUB_MAX_ORDER];
  long long sstride[SUB_MAX_ORDER];
  long long dstride[SUB_MAX_ORDER];
  long long soff, doff, total;
};
hipError_t box_copy(size_t elem_bytes, const void* src, void* dst, const BoxCopy& c, hipStream_t s);

// out[i] = Re in[i] (imag false) or Im in[i] (imag true); in is C64 or
// C128, out the matching real type.
hipError_t complex_part(int dtype, const void* in, void* out, long long n, bool imag, hipStream_t s);

hipError_t fill_value(int dtype, void* x, long long n, double vr, double vi, hipStream_t s);
// a[i, i] += v for i < n (real shift; row-major, leading dimension ld)
hipError_t add_diag(int dtype, void* a, long long ld, int n, double v, hipStream_t s);

// Partial trace: out[o] = sum_t in[base(o) + sum_p t_p pstride_p]; the kept
// bonds kdims/kstride (row-major over o), the traced pairs pdims/pstride
// (pstride_p = the sum of the strides of the two paired bonds).
struct TraceArgs {
  int nkeep, npair;
  long long kdims[SUB_MAX_ORDER], kstride[SUB_MAX_ORDER];
  long long pdims[SUB_MAX_ORDER], pstride[SUB_MAX_ORDER];
  long long nout, ntr;
};
hipError_t partial_trace(int dtype, const void* in, void* out, const TraceArgs& a, hipStream_t s);

}  // namespace tci
