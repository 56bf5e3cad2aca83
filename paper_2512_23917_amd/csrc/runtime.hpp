// Host runtime of the library: context, tensor handles, workspace arena,
// error reporting and the TCI_VERBOSE tracer.
#pragma once
#include <hip/hip_runtime.h>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <memory>
#include <string>
#include <vector>

#include "../../include/tci_c.h"
#include "common.hpp"

namespace tci {

constexpr int MAX_ORDER = 8;

// Per-thread message of the last failed call.
void set_error(const std::string& msg);

// Device memory through an allocator of tci_context_opts (hipMalloc /
// hipFree when its callbacks are NULL).  dev_alloc returns nullptr on failure.
void* dev_alloc(const tci_allocator& al, size_t bytes, hipStream_t s);
void dev_free(const tci_allocator& al, void* p, size_t bytes, hipStream_t s);

// Status of the exception being handled: every extern "C" entry point is a
// function-try-block ending in TCI_API_CATCH, so no C++ exception crosses the
// C ABI (std::bad_alloc -> TCI_ERR_OUT_OF_MEMORY, anything else ->
// TCI_ERR_INTERNAL, with the message in tci_last_error).
tci_status status_of_exception() noexcept;
#define TCI_API_CATCH \
  catch (...) { return ::tci::status_of_exception(); }

struct Chunk {
  void* ptr = nullptr;
  size_t cap = 0;
  size_t used = 0;
};

// Grow-only device arena.  Regions handed out during one API call stay valid
// until reset() at the start of the next call; all work is ordered on the
// context stream, so re-use by a later call is safe.
struct Arena {
  std::vector<Chunk> chunks;
  int device = 0;
  tci_allocator al{};            // the owning context's allocator
  const hipStream_t* stream = nullptr;   // the owning context's stream
  void reset() {
    for (auto& c : chunks) c.used = 0;
  }
  void* get(size_t bytes);
  void release();
  // bytes in use per chunk, and (address, capacity) per chunk, so that a
  // caller replaying a recorded sequence of allocations can restore the state
  std::vector<size_t> used_state() const {
    std::vector<size_t> u;
    for (const auto& c : chunks) u.push_back(c.used);
    return u;
  }
  void restore(const std::vector<size_t>& u) {
    for (size_t i = 0; i < chunks.size() && i < u.size(); ++i) chunks[i].used = u[i];
  }
  std::vector<long long> layout() const {
    std::vector<long long> l;
    for (const auto& c : chunks) {
      l.push_back((long long)(uintptr_t)c.ptr);
      l.push_back((long long)c.cap);
    }
    return l;
  }
};

}  // namespace tci

struct tci_context_s {
  int device = 0;
  hipStream_t stream = nullptr;
  int verbose = 0;
  int precision = TCI_PREC_FP32;  // mixed precision for F32 / C64 contractions
  int svd_mode = TCI_SVD_PLAIN;   // update composites called with params NULL
  tci_allocator al{};             // device allocator (NULL callbacks: hipMalloc / hipFree)
  std::string tune_path;          // grouped-GEMM tile cache file ("" = none)
  tci::Arena arena;
  // recorded HIP graphs of the block-sparse update (owned; see bsparse.cpp)
  std::shared_ptr<void> bs_graphs;
  // second stream (default priority) and an ordering event for work of one
  // call that overlaps the context stream's; created on first use, owned
  hipStream_t aux = nullptr;
  hipEvent_t aux_ev = nullptr;
  uint32_t magic = 0x7C1C0DE1u;
};

struct tci_tensor_s {
  int dtype = TCI_F64;
  int order = 0;
  int64_t shape[tci::MAX_ORDER] = {0};
  int32_t labels[tci::MAX_ORDER] = {0};
  int nlabels = 0;
  void* data = nullptr;
  size_t cap = 0;   // bytes of storage
  bool owns = false;
  tci_allocator al{};  // allocator of owned storage (copied from the creating context)
  bool empty = false;  // moved-from
};

namespace tci {

inline int64_t tsize(const tci_tensor_s* t) {
  int64_t n = 1;
  for (int i = 0; i < t->order; ++i) n *= t->shape[i];
  return n;
}
inline size_t tbytes(const tci_tensor_s* t) { return (size_t)tsize(t) * elem_bytes(t->dtype); }

// RAII-free status helpers.
#define TCI_CHECK_HIP(expr)                                                         \
  do {                                                                              \
    hipError_t _e = (expr);                                                         \
    if (_e != hipSuccess) {                                                         \
      ::tci::set_error(std::string("HIP error: ") + hipGetErrorString(_e) + " at " + \
                       __FILE__ + ":" + std::to_string(__LINE__));                  \
      return _e == hipErrorOutOfMemory ? TCI_ERR_OUT_OF_MEMORY : TCI_ERR_DEVICE;    \
    }                                                                               \
  } while (0)

#define TCI_RET(code, msg)      \
  do {                          \
    ::tci::set_error(msg);      \
    return (code);              \
  } while (0)

#define TCI_TRY(expr)                 \
  do {                                \
    tci_status _s = (expr);           \
    if (_s != TCI_OK) return _s;      \
  } while (0)

// Make `t` an owning (or adequately sized) tensor of the given shape/dtype.
tci_status ensure_shape(tci_context ctx, tci_tensor t, int dtype, int order, const int64_t* shape);

// Size of the fixed device scratch of tci_heff_matvec_noalloc (per device).
constexpr size_t HEFF_NOALLOC_SCRATCH_BYTES = size_t(64) << 20;

// Looks up, once per device, the device address of that scratch; call with
// `device` current (tci_create_context does).
tci_status noalloc_scratch_init(int device);

// Tracer for TCI_VERBOSE (Spec, environment variables).
struct Trace {
  tci_context ctx;
  const char* name;
  std::chrono::steady_clock::time_point t0;
  std::string info;
  Trace(tci_context c, const char* n, std::string i = "");
  ~Trace();
};

}  // namespace tci
