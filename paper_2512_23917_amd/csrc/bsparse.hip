// Data-movement kernels of the U(1) block-sparse update: sector matrices
// padded into square FP64 batches, and kept factors scattered into the
// output blocks with an optional row or column scaling.  Both take a table of
// descriptors so that one launch serves every sector of every update.
#include <hip/hip_runtime.h>

#include "bsparse.hpp"
#include "common.hpp"

namespace tci {

__global__ __launch_bounds__(256) void pad_sectors_kernel(const PadDesc* desc, double* dst, int S) {
  const PadDesc d = desc[blockIdx.y];
  double* out = dst + (long long)blockIdx.y * S * S;
  const long long tot = (long long)S * S;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < tot; e += (long long)gridDim.x * 256) {
    const int i = (int)(e / S), j = (int)(e % S);
    out[e] = (i < d.r && j < d.c) ? (double)d.src[(long long)i * d.c + j] : 0.0;
  }
}

hipError_t pad_sectors(const PadDesc* desc, int nb, double* dst, int S, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  const long long tot = (long long)S * S;
  const unsigned gx = (unsigned)std::min<long long>(64, (tot + 255) / 256);
  hipLaunchKernelGGL(pad_sectors_kernel, dim3(gx, nb), dim3(256), 0, s, desc, dst, S);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void scatter_blocks_kernel(const ScatDesc* desc) {
  const ScatDesc d = desc[blockIdx.y];
  const long long tot = (long long)d.rows * d.cols;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < tot; e += (long long)gridDim.x * 256) {
    const int i = (int)(e / d.cols), j = (int)(e % d.cols);
    double v = d.src[(long long)i * d.lds + j];
    if (d.mode == 1) v *= d.scale[j];
    else if (d.mode == 2) v *= d.scale[i];
    d.dst[(long long)i * d.ldd + j] = (float)v;
  }
}

hipError_t scatter_blocks(const ScatDesc* desc, int nd, hipStream_t s) {
  if (nd <= 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_blocks_kernel, dim3(16, nd), dim3(256), 0, s, desc);
  return hipGetLastError();
}

}  // namespace tci
