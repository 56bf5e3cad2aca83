// Kernels of the U(1) block-sparse update (see bsparse.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

namespace tci {

// Sector matrix src (r x c, row-major F32) -> zero-padded S x S FP64 slot.
struct PadDesc {
  const float* src;
  int r, c;
};
hipError_t pad_sectors(const PadDesc* desc, int nb, double* dst, int S, hipStream_t s);

// dst[i][j] = src[i][j] (mode 0), * scale[j] (mode 1) or * scale[i] (mode 2),
// FP64 -> F32, for i < rows, j < cols.
struct ScatDesc {
  const double* src;
  long long lds;
  int rows, cols;
  float* dst;
  long long ldd;
  const double* scale;
  int mode;
};
hipError_t scatter_blocks(const ScatDesc* desc, int nd, hipStream_t s);

}  // namespace tci
