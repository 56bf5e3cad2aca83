// Optional per-launch timing of tagged kernels with HIP events (enabled by
// tci_profile_enable; used by the benchmark to time single kernels on the
// stream they run on).
#pragma once
#include <hip/hip_runtime.h>

namespace tci {

bool prof_on();
// Tag of the call site whose launches are being recorded (thread-local).
const char* prof_tag();
struct ProfTag {
  const char* prev;
  explicit ProfTag(const char* t);
  ~ProfTag();
};
// Record an event pair around one launch: call begin() before and end() after.
struct ProfScope {
  hipEvent_t a = nullptr, b = nullptr;
  hipStream_t s;
  double work;
  const char* tag;
  ProfScope(hipStream_t st, double w, const char* suffix);
  ~ProfScope();
};

}  // namespace tci
