// Matrix inverse by Gauss-Jordan elimination with partial pivoting (see
// gaussjordan.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace tci {

// Bytes of `work` for an n x n inverse of dtype dt (F64 or C128).
size_t gauss_jordan_work_bytes(int dtype, int n);

// a: n x n row-major (device).  On return the inverse is the right half of
// the n x 2n row-major matrix at `work` (leading dimension 2n, column offset
// n).  *status (device int, zeroed by the caller) becomes k + 1 when column k
// had no non-zero pivot (singular matrix).
hipError_t gauss_jordan_inverse(int dtype, const void* a, int n, void* work, int* status, hipStream_t s);

}  // namespace tci
