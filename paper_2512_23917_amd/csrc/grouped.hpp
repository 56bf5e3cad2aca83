// Grouped FP32 GEMM with an autotuned tile shape (see grouped.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

namespace tci {

// One product C = alpha A B + beta C, all row-major, device pointers.
struct GroupProb {
  const float* a;
  const float* b;
  float* c;
  int m, n, k;
  int lda, ldb, ldc;
  float alpha, beta;
};

// P_dev / tile0_dev: device space for probs.size() entries.  While the tile
// shape of a new problem-size signature is tuned, the outputs are written at
// c + scratch_shift instead (scratch_shift in elements: a buffer as large as
// the outputs' span).  shape_out (optional): index of the tile shape used.
// Synchronises the stream before returning.
hipError_t grouped_gemm_f32(int device, const std::vector<GroupProb>& probs, GroupProb* P_dev, int* tile0_dev,
                            long long scratch_shift, hipStream_t s, int* shape_out);
int grouped_tuned_shape(int device, const std::vector<GroupProb>& probs);
// Tuned shapes of `device` from a cache file (missing file: nothing), and
// every tuned shape of the process into one (false when it cannot be written).
void grouped_tune_load(const std::string& path, int device);
bool grouped_tune_save(const std::string& path);

// The same in two halves: grouped_prepare uploads the tables, tunes the tile
// shape if needed and synchronises; grouped_launch only enqueues the kernel
// (so it can be recorded into a HIP graph; the tables are read at run time).
struct GroupedPlan {
  int shape = 1, ntiles = 0, np = 0;
  const GroupProb* P_dev = nullptr;
  const int* t0_dev = nullptr;
  double flops = 0.0;
};
hipError_t grouped_prepare(int device, const std::vector<GroupProb>& probs, GroupProb* P_dev, int* tile0_dev,
                           long long scratch_shift, hipStream_t s, GroupedPlan& plan);
hipError_t grouped_launch(const GroupedPlan& plan, hipStream_t s);
void grouped_shape_dims(int idx, int* bm, int* bn);

}  // namespace tci
