// Event-based kernel timing registry (see prof.hpp and tci_profile_* in tci_c.h).
#include "prof.hpp"

#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tci_c.h"
#include "runtime.hpp"

namespace tci {

namespace {
struct Rec {
  std::string tag;
  double work;
  hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
thread_local const char* tl_tag = "gemm";

hipEvent_t get_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

bool prof_on() { return g_on; }
const char* prof_tag() { return tl_tag; }
ProfTag::ProfTag(const char* t) : prev(tl_tag) { tl_tag = t; }
ProfTag::~ProfTag() { tl_tag = prev; }

ProfScope::ProfScope(hipStream_t st, double w, const char* suffix) : s(st), work(w), tag(suffix) {
  if (!g_on) return;
  std::lock_guard<std::mutex> lk(g_mu);
  a = get_event();
  b = get_event();
  if (a) (void)hipEventRecord(a, s);
}

ProfScope::~ProfScope() {
  if (!a || !b) return;
  (void)hipEventRecord(b, s);
  std::lock_guard<std::mutex> lk(g_mu);
  std::string t = std::string(tl_tag) + ":" + tag;
  g_recs.push_back(Rec{t, work, a, b});
}

}  // namespace tci

using namespace tci;

extern "C" {

tci_status tci_profile_enable(tci_context ctx, int enable) try {
  if (!ctx) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null context");
  (void)hipStreamSynchronize(ctx->stream);
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = enable != 0;
  for (auto& r : g_recs) {
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_profile_query(tci_context ctx, const char* tag, int64_t* count, double* total_ms, double* work) try {
  if (!ctx || !tag || !count || !total_ms || !work) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  (void)hipStreamSynchronize(ctx->stream);
  std::lock_guard<std::mutex> lk(g_mu);
  *count = 0;
  *total_ms = 0.0;
  *work = 0.0;
  for (auto& r : g_recs) {
    if (r.tag != tag) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
      (void)hipGetLastError();
      continue;
    }
    *count += 1;
    *total_ms += ms;
    *work += r.work;
  }
  return TCI_OK;
} TCI_API_CATCH

// Writes the distinct tags recorded so far, separated by '\n', into buf.
tci_status tci_profile_tags(tci_context ctx, char* buf, int cap) try {
  if (!ctx || !buf || cap <= 0) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  std::lock_guard<std::mutex> lk(g_mu);
  std::vector<std::string> seen;
  for (auto& r : g_recs) {
    bool have = false;
    for (auto& t : seen) have |= (t == r.tag);
    if (!have) seen.push_back(r.tag);
  }
  std::string out;
  for (auto& t : seen) out += t + "\n";
  std::strncpy(buf, out.c_str(), cap - 1);
  buf[cap - 1] = 0;
  return TCI_OK;
} TCI_API_CATCH

}  // extern "C"
