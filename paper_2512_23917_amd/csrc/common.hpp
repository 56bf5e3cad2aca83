// Shared device/host helpers for the MI355X (gfx950) two-site update library.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

namespace tci {

// Interleaved complex numbers, same layout as C99 complex / std::complex.
struct __align__(16) cd { double x, y; };
struct __align__(8) cf { float x, y; };

__host__ __device__ inline cd mk(double a, double b) { return cd{a, b}; }
__host__ __device__ inline cd operator+(cd a, cd b) { return {a.x + b.x, a.y + b.y}; }
__host__ __device__ inline cd operator-(cd a, cd b) { return {a.x - b.x, a.y - b.y}; }
__host__ __device__ inline cd operator*(cd a, cd b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__host__ __device__ inline cd operator*(double s, cd a) { return {s * a.x, s * a.y}; }
__host__ __device__ inline cd conjg(cd a) { return {a.x, -a.y}; }
__host__ __device__ inline double abs2(cd a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ inline cf operator+(cf a, cf b) { return {a.x + b.x, a.y + b.y}; }
__host__ __device__ inline cf operator*(cf a, cf b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }

// Element type tags.  The numeric values match the public tci_dtype enum.
enum DType : int { F32 = 0, F64 = 1, C64 = 2, C128 = 3 };
__host__ __device__ inline bool is_complex(int dt) { return dt == C64 || dt == C128; }
__host__ __device__ inline bool is_double(int dt) { return dt == F64 || dt == C128; }
__host__ __device__ inline size_t elem_bytes(int dt) {
  return dt == F32 ? 4 : (dt == F64 || dt == C64) ? 8 : 16;
}

// Matrix operand form: as stored, transposed, conjugate-transposed, conjugated.
enum Op : int { OP_N = 0, OP_T = 1, OP_C = 2, OP_R = 3 };

// Compute precision of a contraction.
enum Precision : int { PREC_FP64 = 0, PREC_FP32 = 1, PREC_BF16X3 = 2 };

// Wave-level reductions (wave64).
__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ inline float wave_sum(float v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-level sum for blockDim.x <= 1024 (all threads must call).
__device__ inline double block_sum(double v, double* scratch /* >= 16 doubles */) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < nw; ++i) t += scratch[i];
  __syncthreads();
  return t;
}

}  // namespace tci
