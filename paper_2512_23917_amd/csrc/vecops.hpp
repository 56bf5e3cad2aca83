// Elementwise / vector kernels (see vecops.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace tci {

constexpr int LINCOMB_MAX = 16;
struct LinCombArgs {
  int nin;
  const void* in[LINCOMB_MAX];
  double cre[LINCOMB_MAX], cim[LINCOMB_MAX];
};

hipError_t convert(int src, const void* in, int dst, void* out, long long n, hipStream_t s);
hipError_t conjugate(int dt, const void* in, void* out, long long n, hipStream_t s);
hipError_t linear_combine(int dt, const LinCombArgs& a, void* out, long long n, hipStream_t s);
// partial: nparts doubles; the result is max over partial[0 .. min(nparts, blocks)-1]
hipError_t max_abs_diff(int dt, const void* a, const void* b, long long n, double* partial, int nparts,
                        hipStream_t s);
constexpr int MULTIDOT_PARTIAL_DOUBLES = 1024 * 32 * 2;
// V: nv basis vectors of length n, complex128 (vdt = C128) or complex64 (C64);
// w and the arithmetic are complex128.
// gate (optional, device): when *gate == 0 the launches do nothing (a pass
// that the device decided to skip), out keeps its contents.
hipError_t multidot(const void* V, int nv, const void* w, long long n, double* partial, double* out,
                    hipStream_t s, int vdt = C128, const double* gate = nullptr);
hipError_t multiaxpy(const void* V, int nv, const double* c, double sign, void* w, long long n, hipStream_t s,
                     int vdt = C128);
// Lanczos recurrence fused with the multidot of its result:
// w -= alpha v_{nv-1} + beta v_{nv-2} (alpha, beta: device doubles; beta
// null for zero, ignored for nv = 1), then out[2q], out[2q+1] = <v_q, w> for q < nv
// (partial: MULTIDOT_PARTIAL_DOUBLES doubles of workspace)
hipError_t three_term_multidot(const void* V, int nv, const double* alpha, const double* beta, void* w, long long n,
                               double* partial, double* out, hipStream_t s, int vdt = C128);
// multiaxpy, then out[0] = ||w||^2 (partial: MULTIDOT_PARTIAL_DOUBLES doubles of workspace)
hipError_t multiaxpy_norm2(const void* V, int nv, const double* c, double sign, void* w, long long n,
                           double* partial, double* out, hipStream_t s, int vdt = C128,
                           const double* gate = nullptr);
hipError_t scale_copy(const void* x, double sr, double si, void* w, long long n, hipStream_t s);
// w = x (ps[0] + i ps[1]) with the factor on the device (complex128 -> complex128 / complex64);
// nothing is written when gate is given and *gate == 0
hipError_t scale_copy_dev(const void* x, const double* ps, void* w, long long n, hipStream_t s,
                          const double* gate = nullptr);
hipError_t scale_to_c64_dev(const void* x, const double* ps, void* out, long long n, hipStream_t s,
                            const double* gate = nullptr);
// w (complex128) = y (complex64), then out[0], out[1] = <v, w> (partial:
// MULTIDOT_PARTIAL_DOUBLES doubles of workspace)
hipError_t widen_multidot_c64(const void* y, const void* v, void* w, long long n, double* partial, double* out,
                              hipStream_t s, int vdt = C128);
// out (complex64) = (sr + i si) x, x complex128
hipError_t scale_to_c64(const void* x, double sr, double si, void* out, long long n, hipStream_t s);

hipError_t scale_inplace(int dt, void* x, long long n, double sr, double si, hipStream_t s);
hipError_t mpo_pair(int dt, const void* W1, const void* W2, void* W12, int wd, int d, hipStream_t s);
hipError_t triu_mask(int dt, void* R, long long ld, long long sR, int k, const double* mask, long long smask,
                     int batch, hipStream_t s);
// Zero `bytes` bytes at p (4-byte aligned) with a kernel, usable under graph capture.
hipError_t zero_fill(void* p, size_t bytes, hipStream_t s);
// Zero the first `bytes` of each of `count` regions `stride` bytes apart
// (4-byte aligned sizes).
hipError_t zero_fill_rows(void* p, size_t bytes, size_t stride, int count, hipStream_t s);
hipError_t reverse_columns(int dt, void* U, long long ld, int rows, int k, hipStream_t s);

}  // namespace tci
