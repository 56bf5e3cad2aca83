// One-sided Jacobi SVD of small matrices (see jacobi.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>

namespace tci {

// Largest smaller dimension handled by the Jacobi path.
constexpr int JACOBI_MAX_K = 64;

// Workspace elements per problem for an m x n problem (either orientation).
size_t jacobi_work_elems(int m, int n);

// Thin SVD of `batch` row-major rows x cols matrices (C128 or F64, problem b
// at A + b*sA, leading dimension lda), k = min(rows, cols) <= JACOBI_MAX_K:
// u (rows x k, stride su), vh (k x cols, stride svh), s (k, stride ss)
// descending; column gauge as tci_svd; sweeps[b] = sweeps used (-1 when
// not converged within 80).  work: batch * jacobi_work_elems elements.
hipError_t jacobi_svd(int dtype, const void* A, long long lda, long long sA, int rows, int cols, void* work,
                      void* u, long long su, void* vh, long long svh, double* s, long long ss, int* sweeps,
                      int batch, hipStream_t st);

}  // namespace tci
