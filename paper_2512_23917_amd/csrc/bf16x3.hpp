// Split-BF16x3 GEMM on pre-split operand planes (see bf16x3.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>

namespace tci {

struct PlaneGemmArgs {
  int m, n, k;              // logical sizes (k only for flop accounting)
  int Mp, Np, Kp;           // padded plane sizes (multiples of 128, 128, 32)
  const __bf16* Ap; long long sAp;   // planes of op(A): [P][Mp][Kp] per problem
  const __bf16* Bp; long long sBp;   // planes of op(B)^T: [P][Np][Kp] per problem
  void* C; long long ldc, sC;        // float / complex-float output, row-major
  double alpha_re, alpha_im, beta_re, beta_im;
  int batch;
};

int planes_of(int dtype);
int pad_rows(int r);
int pad_k(int k);
size_t planes_bytes(int dtype, int rows, int k);
hipError_t split_a(int dtype, int opA, const void* A, long long lda, long long sA, int M, int K, void* dst, int batch,
                   hipStream_t s);
hipError_t split_b(int dtype, int opB, const void* B, long long ldb, long long sB, int K, int N, void* dst, int batch,
                   hipStream_t s);
hipError_t gemm_planes(int dtype, const PlaneGemmArgs& a, hipStream_t s);
// X2[a][j][b] = sum_k W12[k][j] X1[a][k][b] (FP32) written into the planes of
// the row-major matrix X2' ((a, j / w) x ((j % w) chir + b)), Mp x Kp padded;
// kw = w d^2 must be 20 (w = 5, d = 2), else hipErrorInvalidValue.
hipError_t w12_to_planes(int dtype, const void* X1, const void* W12, int chil, int kw, int chir, int w, void* planes,
                         int Mp, int Kp, hipStream_t s);

}  // namespace tci
