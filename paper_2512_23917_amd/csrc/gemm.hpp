// Batched matrix-core GEMM interface (see gemm.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace tci {

// C_b = alpha * diag(rs_b) op(A_b) op(B_b) diag(cs_b) + beta * C_b for b < batch.
// All matrices row-major; op(A) is m x k, op(B) is k x n, C is m x n.
// dims (optional, device): per-problem (m, n, k), each clamped to the launch maxima.
// rs / cs (optional, device, real double): per-problem row / column scales.
struct GemmArgs {
  int m, n, k;
  int opA, opB;
  const void* A; long long lda, sA;
  const void* B; long long ldb, sB;
  void* C; long long ldc, sC;
  double alpha_re, alpha_im, beta_re, beta_im;
  const int* dims;
  const double* rs; long long s_rs;
  const double* cs; long long s_cs;
  int batch;
  // > 0: only entries with col - row < lower_band are needed;
  // output tiles whose every entry has col - row >= lower_band are skipped
  // and left unchanged (Hermitian results read from the lower triangle).
  int lower_band;
  // Optional device scratch for the FP64 kernels.  A launch with too few
  // output tiles to occupy every compute unit cuts K into chunks whose raw
  // partial products go to kws (FP64, one M x N slab per chunk and problem);
  // a second pass sums the chunks in order and applies the scales, alpha and
  // beta.  Null = never split.  Set by the caller; ksplit is set by gemm().
  void* kws; size_t kws_bytes;
  int ksplit;
};

// Scratch that lets any FP64 launch split (see GemmArgs::kws).
constexpr size_t GEMM_SPLITK_WS_BYTES = (size_t)96 << 20;

inline GemmArgs gemm_args(int m, int n, int k, int opA, int opB, const void* A, long long lda,
                          const void* B, long long ldb, void* C, long long ldc) {
  GemmArgs a{};
  a.m = m; a.n = n; a.k = k; a.opA = opA; a.opB = opB;
  a.A = A; a.lda = lda; a.B = B; a.ldb = ldb; a.C = C; a.ldc = ldc;
  a.alpha_re = 1.0; a.beta_re = 0.0;
  a.batch = 1;
  return a;
}

// dtype: tci DType (F32, F64, C64, C128); prec: Precision (ignored for F64 / C128).
hipError_t gemm(int dtype, int prec, const GemmArgs& a, hipStream_t s);
hipError_t gemm_scale_c(int dtype, const GemmArgs& a, hipStream_t s);

}  // namespace tci
