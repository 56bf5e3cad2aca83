// Kernels of the randomized truncated SVD (see sketch.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace tci {

// Omega_b: n x ld (row stride ld), columns j < k_b (kb device array, or kdef)
// drawn from Philox stream streams[b] (or b) with key `seed`; others zero.
hipError_t sketch_fill(int dt, void* om, long long ld, long long som, int n, const int* kb, int kdef, uint64_t seed,
                       const uint32_t* streams, int batch, hipStream_t s);
hipError_t philox_blocks(uint64_t seed, uint32_t stream, uint64_t first, long long n, uint32_t* out, hipStream_t s);
hipError_t residual_norms(int dt, const void* P, const void* U, long long ld, long long sPU, int m, int maxchi,
                          const double* sv, long long ss, const int* chi, double* r, int batch, hipStream_t s);

}  // namespace tci
