// C ABI of the two-site update library: context, tensors, TCI operations and
// the batched update composites.  Every numeric step launches this library's
// own HIP kernels (gemm.hip, eig.hip, linalg.hip, vecops.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/tci_c.h"
#include "common.hpp"
#include "eig.hpp"
#include "gemm.hpp"
#include "grouped.hpp"
#include "linalg.hpp"
#include "runtime.hpp"
#include "subtensor.hpp"
#include "tsvd.hpp"
#include "vecops.hpp"

namespace tci {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

tci_status status_of_exception() noexcept {
  tci_status code = TCI_ERR_INTERNAL;
  const char* msg = "internal error: unknown exception";
  std::string what;
  try {
    throw;
  } catch (const std::bad_alloc&) {
    code = TCI_ERR_OUT_OF_MEMORY;
    msg = "host memory allocation failed";
  } catch (const std::exception& e) {
    try {
      what = std::string("internal error: ") + e.what();
      msg = what.c_str();
    } catch (...) {
      msg = "internal error";
    }
  } catch (...) {
  }
  try {
    g_last_error = msg;
  } catch (...) {
    g_last_error.clear();
  }
  return code;
}

void* dev_alloc(const tci_allocator& al, size_t bytes, hipStream_t s) {
  if (al.alloc) return al.alloc(bytes, static_cast<void*>(s), al.user);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void dev_free(const tci_allocator& al, void* p, size_t bytes, hipStream_t s) {
  if (!p) return;
  if (al.free) al.free(p, bytes, static_cast<void*>(s), al.user);
  else (void)hipFree(p);
}

void* Arena::get(size_t bytes) {
  bytes = (bytes + 255) & ~size_t(255);
  if (bytes == 0) bytes = 256;
  for (auto& c : chunks) {
    if (c.cap - c.used >= bytes) {
      void* p = static_cast<char*>(c.ptr) + c.used;
      c.used += bytes;
      return p;
    }
  }
  Chunk c;
  c.cap = std::max(bytes, size_t(256) << 20);
  c.ptr = dev_alloc(al, c.cap, stream ? *stream : nullptr);
  if (!c.ptr) return nullptr;
  c.used = bytes;
  chunks.push_back(c);
  return c.ptr;
}

void Arena::release() {
  for (auto& c : chunks) dev_free(al, c.ptr, c.cap, stream ? *stream : nullptr);
  chunks.clear();
}

Trace::Trace(tci_context c, const char* n, std::string i) : ctx(c), name(n), info(std::move(i)) {
  if (ctx && ctx->verbose >= 2) t0 = std::chrono::steady_clock::now();
}
Trace::~Trace() {
  if (!ctx || ctx->verbose <= 0) return;
  if (ctx->verbose >= 2) {
    (void)hipStreamSynchronize(ctx->stream);
    const double us =
        std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
    fprintf(stderr, "TCI_VERBOSE: %s %s %.1f us\n", name, info.c_str(), us);
  } else {
    fprintf(stderr, "TCI_VERBOSE: %s %s\n", name, info.c_str());
  }
}

static std::string shape_str(const tci_tensor_s* t) {
  std::string s = "{";
  for (int i = 0; i < t->order; ++i) s += (i ? "," : "") + std::to_string(t->shape[i]);
  return s + "}";
}

static bool valid_dtype(int dt) { return dt >= TCI_F32 && dt <= TCI_C128; }

static tci_status alloc_storage(tci_context ctx, tci_tensor_s* t, size_t bytes) {
  if (t->owns && t->data && t->cap >= bytes) return TCI_OK;
  if (!t->owns && t->data) {
    if (t->cap >= bytes) return TCI_OK;
    TCI_RET(TCI_ERR_SHAPE, "borrowed output tensor too small");
  }
  if (t->owns && t->data) {
    (void)hipStreamSynchronize(ctx->stream);
    dev_free(t->al, t->data, t->cap, ctx->stream);
    t->data = nullptr;
    t->cap = 0;
  }
  const size_t want = std::max<size_t>(bytes, 16);
  void* p = dev_alloc(ctx->al, want, ctx->stream);
  if (!p) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "device allocation of " + std::to_string(want) + " bytes failed");
  t->data = p;
  t->cap = want;
  t->owns = true;
  t->al = ctx->al;
  return TCI_OK;
}

tci_status ensure_shape(tci_context ctx, tci_tensor t, int dtype, int order, const int64_t* shape) {
  if (!t) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null output tensor");
  int64_t n = 1;
  for (int i = 0; i < order; ++i) n *= shape[i];
  const size_t bytes = (size_t)n * elem_bytes(dtype);
  TCI_TRY(alloc_storage(ctx, t, bytes));
  t->dtype = dtype;
  t->order = order;
  for (int i = 0; i < order; ++i) t->shape[i] = shape[i];
  t->nlabels = 0;
  t->empty = false;
  return TCI_OK;
}

static tci_status check_ctx(tci_context ctx) {
  if (!ctx || ctx->magic != 0x7C1C0DE1u) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "invalid context");
  if (hipSetDevice(ctx->device) != hipSuccess) TCI_RET(TCI_ERR_DEVICE, "hipSetDevice failed");
  return TCI_OK;
}

static tci_status check_t(tci_tensor t, const char* what) {
  if (!t) TCI_RET(TCI_ERR_INVALID_ARGUMENT, std::string("null tensor: ") + what);
  if (t->empty) TCI_RET(TCI_ERR_INVALID_ARGUMENT, std::string("moved-from tensor: ") + what);
  return TCI_OK;
}

static int work_dtype(int dt) { return dt == C64 ? C128 : dt == F32 ? F64 : dt; }

static int prec_for(tci_context ctx, int dt) {
  return is_double(dt) ? PREC_FP64 : ctx->precision;
}

}  // namespace tci

using namespace tci;

extern "C" {

const char* tci_version(void) { return "1.0"; }
const char* tci_last_error(void) { return g_last_error.c_str(); }

void tci_update_params_default(tci_update_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->chi_min = 1;
  p->chi_max = INT64_MAX;
  p->direction = TCI_DIR_RIGHT;
  p->precision = TCI_PREC_FP64;
  p->svd_mode = TCI_SVD_PLAIN;
  p->power_iters = 2;
  p->cert_tol = 1e-7;
}

void tci_context_opts_default(tci_context_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = -1;
  o->svd_mode = TCI_SVD_PLAIN;
  o->verbosity = -1;
}

tci_status tci_create_context(tci_context* out, int device_id, void* hip_stream, const tci_context_opts* opts) try {
  if (!out) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "out is NULL");
  tci_context_opts o;
  tci_context_opts_default(&o);
  if (opts) o = *opts;
  if ((o.allocator.alloc == nullptr) != (o.allocator.free == nullptr))
    TCI_RET(TCI_ERR_INVALID_ARGUMENT, "allocator: set both alloc and free, or neither");
  if (o.precision != -1 && o.precision != TCI_PREC_FP32 && o.precision != TCI_PREC_BF16X3)
    TCI_RET(TCI_ERR_INVALID_ARGUMENT, "opts.precision must be -1, TCI_PREC_FP32 or TCI_PREC_BF16X3");
  if (o.svd_mode != TCI_SVD_PLAIN && o.svd_mode != TCI_SVD_RANDOMIZED)
    TCI_RET(TCI_ERR_INVALID_ARGUMENT, "opts.svd_mode must be TCI_SVD_PLAIN or TCI_SVD_RANDOMIZED");
  if (o.verbosity < -1 || o.verbosity > 2) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "opts.verbosity must be in [-1, 2]");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
    (void)hipGetLastError();
    TCI_RET(TCI_ERR_DEVICE, "no HIP device available");
  }
  if (device_id < 0 || device_id >= ndev) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "bad device id");
  TCI_CHECK_HIP(hipSetDevice(device_id));
  TCI_TRY(noalloc_scratch_init(device_id));
  auto* c = new tci_context_s();
  c->device = device_id;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->arena.device = device_id;
  c->al = o.allocator;
  c->arena.al = o.allocator;
  c->arena.stream = &c->stream;
  if (o.precision != -1) c->precision = o.precision;
  c->svd_mode = o.svd_mode;
  if (o.verbosity >= 0) c->verbose = o.verbosity;
  else if (const char* v = std::getenv("TCI_VERBOSE")) c->verbose = std::atoi(v);
  if (o.autotune_cache) {
    c->tune_path = o.autotune_cache;
    grouped_tune_load(c->tune_path, device_id);
  }
  *out = c;
  Trace tr(c, "create_context", "device=" + std::to_string(device_id));
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_destroy_context(tci_context ctx) try {
  TCI_TRY(check_ctx(ctx));
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->aux) {
    (void)hipStreamSynchronize(ctx->aux);
    (void)hipStreamDestroy(ctx->aux);
  }
  if (ctx->aux_ev) (void)hipEventDestroy(ctx->aux_ev);
  ctx->bs_graphs.reset();
  ctx->arena.release();
  tci_status st = TCI_OK;
  if (!ctx->tune_path.empty() && !grouped_tune_save(ctx->tune_path)) {
    set_error("could not write the autotune cache " + ctx->tune_path);
    st = TCI_ERR_INVALID_ARGUMENT;
  }
  ctx->magic = 0;
  delete ctx;
  return st;
} TCI_API_CATCH

tci_status tci_set_stream(tci_context ctx, void* hip_stream) try {
  TCI_TRY(check_ctx(ctx));
  (void)hipStreamSynchronize(ctx->stream);
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_set_precision(tci_context ctx, tci_precision prec) try {
  TCI_TRY(check_ctx(ctx));
  if (prec != TCI_PREC_FP32 && prec != TCI_PREC_BF16X3 && prec != TCI_PREC_FP64)
    TCI_RET(TCI_ERR_INVALID_ARGUMENT, "bad precision");
  ctx->precision = prec == TCI_PREC_FP64 ? TCI_PREC_FP32 : prec;
  return TCI_OK;
} TCI_API_CATCH

// ----------------------------------------------------------------- tensors
static tci_status make_tensor(tci_context ctx, tci_dtype dtype, int order, const int64_t* shape,
                              tci_tensor* out, bool zero) {
  TCI_TRY(check_ctx(ctx));
  if (!out) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "out is NULL");
  if (!valid_dtype(dtype)) TCI_RET(TCI_ERR_DTYPE, "bad dtype");
  if (order < 0 || order > MAX_ORDER || (order > 0 && !shape))
    TCI_RET(TCI_ERR_INVALID_ARGUMENT, "bad order/shape");
  for (int i = 0; i < order; ++i)
    if (shape[i] < 0) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "negative dimension");
  auto* t = new tci_tensor_s();
  tci_status st = ensure_shape(ctx, t, dtype, order, shape);
  if (st != TCI_OK) {
    delete t;
    return st;
  }
  if (zero && tbytes(t) > 0) {
    hipError_t e = hipMemsetAsync(t->data, 0, tbytes(t), ctx->stream);
    if (e != hipSuccess) {
      dev_free(t->al, t->data, t->cap, ctx->stream);
      delete t;
      TCI_CHECK_HIP(e);
    }
  }
  *out = t;
  return TCI_OK;
}

tci_status tci_allocate(tci_context ctx, tci_dtype dtype, int order, const int64_t* shape, tci_tensor* out) try {
  return make_tensor(ctx, dtype, order, shape, out, false);
} TCI_API_CATCH

tci_status tci_zeros(tci_context ctx, tci_dtype dtype, int order, const int64_t* shape, tci_tensor* out) try {
  return make_tensor(ctx, dtype, order, shape, out, true);
} TCI_API_CATCH

tci_status tci_wrap(tci_context ctx, tci_dtype dtype, int order, const int64_t* shape, void* dev_ptr,
                    tci_tensor* out) try {
  TCI_TRY(check_ctx(ctx));
  if (!out) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "out is NULL");
  if (!valid_dtype(dtype)) TCI_RET(TCI_ERR_DTYPE, "bad dtype");
  if (order < 0 || order > MAX_ORDER || (order > 0 && !shape))
    TCI_RET(TCI_ERR_INVALID_ARGUMENT, "bad order/shape");
  auto* t = new tci_tensor_s();
  t->dtype = dtype;
  t->order = order;
  for (int i = 0; i < order; ++i) {
    if (shape[i] < 0) {
      delete t;
      TCI_RET(TCI_ERR_INVALID_ARGUMENT, "negative dimension");
    }
    t->shape[i] = shape[i];
  }
  if (!dev_ptr && tsize(t) > 0) {
    delete t;
    TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null device pointer");
  }
  t->data = dev_ptr;
  t->cap = tbytes(t);
  t->owns = false;
  *out = t;
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_copy(tci_context ctx, tci_tensor in, tci_tensor* out) try {
  TCI_TRY(check_ctx(ctx));
  TCI_TRY(check_t(in, "in"));
  TCI_TRY(make_tensor(ctx, (tci_dtype)in->dtype, in->order, in->shape, out, false));
  if (tbytes(in) > 0)
    TCI_CHECK_HIP(hipMemcpyAsync((*out)->data, in->data, tbytes(in), hipMemcpyDeviceToDevice, ctx->stream));
  std::memcpy((*out)->labels, in->labels, sizeof(in->labels));
  (*out)->nlabels = in->nlabels;
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_move(tci_context ctx, tci_tensor* from, tci_tensor* out) try {
  TCI_TRY(check_ctx(ctx));
  if (!from || !*from || !out) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  auto* t = new tci_tensor_s(**from);
  tci_tensor_s* f = *from;
  f->data = nullptr;
  f->cap = 0;
  f->owns = false;
  f->order = 0;
  f->nlabels = 0;
  f->empty = true;
  *out = t;
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_destroy(tci_context ctx, tci_tensor t) try {
  if (!t) return TCI_OK;
  TCI_TRY(check_ctx(ctx));
  if (t->owns && t->data) {
    (void)hipStreamSynchronize(ctx->stream);
    dev_free(t->al, t->data, t->cap, ctx->stream);
  }
  delete t;
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_order(tci_context ctx, tci_tensor t, int* out) try {
  (void)ctx;
  if (!t || !out) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  *out = t->order;
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_shape(tci_context ctx, tci_tensor t, int64_t* shape_out, int cap) try {
  (void)ctx;
  if (!t || (!shape_out && cap > 0)) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  for (int i = 0; i < std::min(cap, t->order); ++i) shape_out[i] = t->shape[i];
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_size(tci_context ctx, tci_tensor t, int64_t* out) try {
  (void)ctx;
  if (!t || !out) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  *out = t->empty ? 0 : tsize(t);
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_size_bytes(tci_context ctx, tci_tensor t, int64_t* out) try {
  (void)ctx;
  if (!t || !out) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  *out = t->empty ? 0 : (int64_t)tbytes(t);
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_dtype_of(tci_context ctx, tci_tensor t, tci_dtype* out) try {
  (void)ctx;
  if (!t || !out) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  *out = (tci_dtype)t->dtype;
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_data_ptr(tci_context ctx, tci_tensor t, void** out) try {
  (void)ctx;
  if (!t || !out) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  *out = t->data;
  return TCI_OK;
} TCI_API_CATCH

static tci_status elem_offset(tci_tensor t, const int64_t* coors, size_t* off) {
  int64_t lin = 0;
  for (int i = 0; i < t->order; ++i) {
    if (coors[i] < 0 || coors[i] >= t->shape[i]) TCI_RET(TCI_ERR_SHAPE, "coordinate out of range");
    lin = lin * t->shape[i] + coors[i];
  }
  *off = (size_t)lin * elem_bytes(t->dtype);
  return TCI_OK;
}

tci_status tci_get_elem(tci_context ctx, tci_tensor t, const int64_t* coors, void* out) try {
  TCI_TRY(check_ctx(ctx));
  TCI_TRY(check_t(t, "t"));
  if (!out || (t->order > 0 && !coors)) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  size_t off = 0;
  TCI_TRY(elem_offset(t, coors, &off));
  TCI_CHECK_HIP(hipMemcpyAsync(out, static_cast<char*>(t->data) + off, elem_bytes(t->dtype),
                               hipMemcpyDeviceToHost, ctx->stream));
  TCI_CHECK_HIP(hipStreamSynchronize(ctx->stream));
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_set_elem(tci_context ctx, tci_tensor t, const int64_t* coors, const void* val) try {
  TCI_TRY(check_ctx(ctx));
  TCI_TRY(check_t(t, "t"));
  if (!val || (t->order > 0 && !coors)) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  size_t off = 0;
  TCI_TRY(elem_offset(t, coors, &off));
  TCI_CHECK_HIP(hipMemcpyAsync(static_cast<char*>(t->data) + off, val, elem_bytes(t->dtype),
                               hipMemcpyHostToDevice, ctx->stream));
  TCI_CHECK_HIP(hipStreamSynchronize(ctx->stream));
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_set_labels(tci_context ctx, tci_tensor t, const int32_t* labels, int n) try {
  (void)ctx;
  if (!t || n < 0 || n > MAX_ORDER || (n > 0 && !labels)) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "bad labels");
  if (n != t->order) TCI_RET(TCI_ERR_LABEL, "label count must equal the order");
  for (int i = 0; i < n; ++i) t->labels[i] = labels[i];
  t->nlabels = n;
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_get_labels(tci_context ctx, tci_tensor t, int32_t* labels, int cap) try {
  (void)ctx;
  if (!t || (cap > 0 && !labels)) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  for (int i = 0; i < std::min(cap, t->nlabels); ++i) labels[i] = t->labels[i];
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_from_host(tci_context ctx, tci_tensor t, const void* host, size_t bytes) try {
  TCI_TRY(check_ctx(ctx));
  TCI_TRY(check_t(t, "t"));
  if (bytes != tbytes(t)) TCI_RET(TCI_ERR_SHAPE, "byte count differs from size_bytes");
  if (bytes == 0) return TCI_OK;
  if (!host) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null host pointer");
  TCI_CHECK_HIP(hipMemcpyAsync(t->data, host, bytes, hipMemcpyHostToDevice, ctx->stream));
  TCI_CHECK_HIP(hipStreamSynchronize(ctx->stream));
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_to_host(tci_context ctx, tci_tensor t, void* host, size_t bytes) try {
  TCI_TRY(check_ctx(ctx));
  TCI_TRY(check_t(t, "t"));
  if (bytes != tbytes(t)) TCI_RET(TCI_ERR_SHAPE, "byte count differs from size_bytes");
  if (bytes == 0) return TCI_OK;
  if (!host) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null host pointer");
  TCI_CHECK_HIP(hipMemcpyAsync(host, t->data, bytes, hipMemcpyDeviceToHost, ctx->stream));
  TCI_CHECK_HIP(hipStreamSynchronize(ctx->stream));
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_convert(tci_context ctx, tci_tensor in, tci_dtype dtype, tci_tensor* out) try {
  TCI_TRY(check_ctx(ctx));
  TCI_TRY(check_t(in, "in"));
  if (!valid_dtype(dtype)) TCI_RET(TCI_ERR_DTYPE, "bad dtype");
  if (is_complex(in->dtype) && !is_complex(dtype))
    TCI_RET(TCI_ERR_DTYPE, "complex to real conversion is not defined");
  Trace tr(ctx, "convert", shape_str(in));
  TCI_TRY(make_tensor(ctx, dtype, in->order, in->shape, out, false));
  TCI_CHECK_HIP(tci::convert(in->dtype, in->data, dtype, (*out)->data, tsize(in), ctx->stream));
  return TCI_OK;
} TCI_API_CATCH

// ----------------------------------------------------------------- manipulation
tci_status tci_reshape(tci_context ctx, tci_tensor in, int order, const int64_t* shape, tci_tensor out) try {
  TCI_TRY(check_ctx(ctx));
  TCI_TRY(check_t(in, "in"));
  if (!out || order < 0 || order > MAX_ORDER || (order > 0 && !shape))
    TCI_RET(TCI_ERR_INVALID_ARGUMENT, "bad arguments");
  int64_t n = 1;
  for (int i = 0; i < order; ++i) n *= shape[i];
  if (n != tsize(in)) TCI_RET(TCI_ERR_SHAPE, "reshape must keep the number of elements");
  if (out == in) {
    in->order = order;
    for (int i = 0; i < order; ++i) in->shape[i] = shape[i];
    in->nlabels = 0;
    return TCI_OK;
  }
  TCI_TRY(ensure_shape(ctx, out, in->dtype, order, shape));
  if (tbytes(in) > 0)
    TCI_CHECK_HIP(hipMemcpyAsync(out->data, in->data, tbytes(in), hipMemcpyDeviceToDevice, ctx->stream));
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_transpose(tci_context ctx, tci_tensor in, const int32_t* perm, tci_tensor out) try {
  TCI_TRY(check_ctx(ctx));
  TCI_TRY(check_t(in, "in"));
  if (!out || (in->order > 0 && !perm)) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  bool seen[MAX_ORDER] = {false};
  for (int b = 0; b < in->order; ++b) {
    if (perm[b] < 0 || perm[b] >= in->order || seen[perm[b]]) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "bad permutation");
    seen[perm[b]] = true;
  }
  Trace tr(ctx, "transpose", shape_str(in));
  ctx->arena.reset();
  int64_t oshape[MAX_ORDER];
  long long ishape[MAX_ORDER];
  int p32[MAX_ORDER];
  for (int b = 0; b < in->order; ++b) {
    oshape[b] = in->shape[perm[b]];
    ishape[b] = in->shape[b];
    p32[b] = perm[b];
  }
  const size_t bytes = tbytes(in);
  void* src = in->data;
  if (out == in) {
    void* tmp = ctx->arena.get(bytes);
    if (!tmp) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
    if (bytes) TCI_CHECK_HIP(hipMemcpyAsync(tmp, in->data, bytes, hipMemcpyDeviceToDevice, ctx->stream));
    src = tmp;
  }
  const int dt = in->dtype, order = in->order;
  TCI_TRY(ensure_shape(ctx, out, dt, order, oshape));
  if (bytes) TCI_CHECK_HIP(tci::permute(dt, src, out->data, order, ishape, p32, ctx->stream));
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_cplx_conj(tci_context ctx, tci_tensor in, tci_tensor out) try {
  TCI_TRY(check_ctx(ctx));
  TCI_TRY(check_t(in, "in"));
  if (!out) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null output");
  if (out != in) TCI_TRY(ensure_shape(ctx, out, in->dtype, in->order, in->shape));
  TCI_CHECK_HIP(tci::conjugate(in->dtype, in->data, out->data, tsize(in), ctx->stream));
  return TCI_OK;
} TCI_API_CATCH

static void host_scalar(int dt, const void* s, double& r, double& i) {
  switch (dt) {
    case F32: r = *static_cast<const float*>(s); i = 0; break;
    case F64: r = *static_cast<const double*>(s); i = 0; break;
    case C64: r = static_cast<const float*>(s)[0]; i = static_cast<const float*>(s)[1]; break;
    default: r = static_cast<const double*>(s)[0]; i = static_cast<const double*>(s)[1]; break;
  }
}

tci_status tci_scale(tci_context ctx, tci_tensor inout, const void* s) try {
  TCI_TRY(check_ctx(ctx));
  TCI_TRY(check_t(inout, "inout"));
  if (!s) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null scalar");
  double r, i;
  host_scalar(inout->dtype, s, r, i);
  TCI_CHECK_HIP(tci::scale_inplace(inout->dtype, inout->data, tsize(inout), r, i, ctx->stream));
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_linear_combine(tci_context ctx, int n, const tci_tensor* ins, const void* coefs, tci_tensor out) try {
  TCI_TRY(check_ctx(ctx));
  if (n < 1 || n > LINCOMB_MAX || !ins || !out) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "bad arguments");
  for (int q = 0; q < n; ++q) {
    TCI_TRY(check_t(ins[q], "ins"));
    if (ins[q]->dtype != ins[0]->dtype) TCI_RET(TCI_ERR_DTYPE, "mixed dtypes");
    if (ins[q]->order != ins[0]->order) TCI_RET(TCI_ERR_SHAPE, "shapes differ");
    for (int b = 0; b < ins[0]->order; ++b)
      if (ins[q]->shape[b] != ins[0]->shape[b]) TCI_RET(TCI_ERR_SHAPE, "shapes differ");
  }
  const int dt = ins[0]->dtype;
  LinCombArgs a{};
  a.nin = n;
  const size_t es = elem_bytes(dt);
  for (int q = 0; q < n; ++q) {
    a.in[q] = ins[q]->data;
    if (coefs) host_scalar(dt, static_cast<const char*>(coefs) + q * es, a.cre[q], a.cim[q]);
    else { a.cre[q] = 1.0; a.cim[q] = 0.0; }
  }
  bool alias = false;
  for (int q = 0; q < n; ++q) alias |= (ins[q] == out);
  if (!alias) TCI_TRY(ensure_shape(ctx, out, dt, ins[0]->order, ins[0]->shape));
  // elementwise: out[i] depends on ins[*][i] only, so aliasing is safe
  TCI_CHECK_HIP(tci::linear_combine(dt, a, out->data, tsize(ins[0]), ctx->stream));
  return TCI_OK;
} TCI_API_CATCH

// ----------------------------------------------------------------- reductions
static tci_status norm2_dev(tci_context ctx, tci_tensor t, double* host_out) {
  double* dev = static_cast<double*>(ctx->arena.get(sizeof(double) * (SUMSQ_PARTIALS + 1)));
  if (!dev) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
  TCI_CHECK_HIP(sumsq_batched(t->dtype, t->data, tsize(t), 0, dev + SUMSQ_PARTIALS, dev, 1, ctx->stream));
  TCI_CHECK_HIP(hipMemcpyAsync(host_out, dev + SUMSQ_PARTIALS, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  TCI_CHECK_HIP(hipStreamSynchronize(ctx->stream));
  return TCI_OK;
}

tci_status tci_norm(tci_context ctx, tci_tensor t, double* out) try {
  TCI_TRY(check_ctx(ctx));
  TCI_TRY(check_t(t, "t"));
  if (!out) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null output");
  Trace tr(ctx, "norm", shape_str(t));
  ctx->arena.reset();
  double s2 = 0.0;
  TCI_TRY(norm2_dev(ctx, t, &s2));
  *out = std::sqrt(s2);
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_normalize(tci_context ctx, tci_tensor inout, double* old_norm) try {
  TCI_TRY(check_ctx(ctx));
  TCI_TRY(check_t(inout, "inout"));
  Trace tr(ctx, "normalize", shape_str(inout));
  ctx->arena.reset();
  double s2 = 0.0;
  TCI_TRY(norm2_dev(ctx, inout, &s2));
  const double nrm = std::sqrt(s2);
  if (old_norm) *old_norm = nrm;
  if (nrm > 0.0) TCI_CHECK_HIP(tci::scale_inplace(inout->dtype, inout->data, tsize(inout), 1.0 / nrm, 0.0, ctx->stream));
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_close(tci_context ctx, tci_tensor a, tci_tensor b, double eps, int* result) try {
  TCI_TRY(check_ctx(ctx));
  TCI_TRY(check_t(a, "a"));
  TCI_TRY(check_t(b, "b"));
  if (!result) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null result");
  if (a->dtype != b->dtype) TCI_RET(TCI_ERR_DTYPE, "dtypes differ");
  if (a->order != b->order) TCI_RET(TCI_ERR_SHAPE, "shapes differ");
  for (int i = 0; i < a->order; ++i)
    if (a->shape[i] != b->shape[i]) TCI_RET(TCI_ERR_SHAPE, "shapes differ");
  ctx->arena.reset();
  const int nparts = 256;
  double* part = static_cast<double*>(ctx->arena.get(sizeof(double) * nparts));
  if (!part) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
  const long long n = tsize(a);
  const int used = (int)std::max<long long>(1, std::min<long long>(nparts, (n + 255) / 256));
  TCI_CHECK_HIP(max_abs_diff(a->dtype, a->data, b->data, n, part, nparts, ctx->stream));
  std::vector<double> h(used);
  TCI_CHECK_HIP(hipMemcpyAsync(h.data(), part, sizeof(double) * used, hipMemcpyDeviceToHost, ctx->stream));
  TCI_CHECK_HIP(hipStreamSynchronize(ctx->stream));
  double m = 0.0;
  bool nan = false;
  for (double v : h) { if (v != v) nan = true; m = std::max(m, v); }
  *result = (!nan && m <= eps) ? 1 : 0;
  return TCI_OK;
} TCI_API_CATCH

// ----------------------------------------------------------------- contraction
static int find_lab(const int32_t* l, int n, int32_t x) {
  for (int i = 0; i < n; ++i)
    if (l[i] == x) return i;
  return -1;
}

tci_status tci_contract(tci_context ctx, tci_tensor a, const int32_t* la, int na, tci_tensor b,
                        const int32_t* lb, int nb, tci_tensor c, const int32_t* lc, int nc) try {
  TCI_TRY(check_ctx(ctx));
  TCI_TRY(check_t(a, "a"));
  TCI_TRY(check_t(b, "b"));
  if (!c) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null output");
  if (na != a->order || nb != b->order) TCI_RET(TCI_ERR_LABEL, "label count must equal the order");
  if (nc < 0 || nc > MAX_ORDER || (na && !la) || (nb && !lb) || (nc && !lc))
    TCI_RET(TCI_ERR_INVALID_ARGUMENT, "bad label arrays");
  if (a->dtype != b->dtype) TCI_RET(TCI_ERR_DTYPE, "operands have different dtypes");
  for (int i = 0; i < na; ++i) if (find_lab(la, i, la[i]) >= 0) TCI_RET(TCI_ERR_LABEL, "repeated label in a");
  for (int i = 0; i < nb; ++i) if (find_lab(lb, i, lb[i]) >= 0) TCI_RET(TCI_ERR_LABEL, "repeated label in b");
  for (int i = 0; i < nc; ++i) if (find_lab(lc, i, lc[i]) >= 0) TCI_RET(TCI_ERR_LABEL, "repeated label in c");
  int64_t cshape[MAX_ORDER];
  for (int i = 0; i < nc; ++i) {
    const int ia = find_lab(la, na, lc[i]), ib = find_lab(lb, nb, lc[i]);
    if ((ia >= 0) == (ib >= 0)) TCI_RET(TCI_ERR_LABEL, "label of c must appear in exactly one operand");
    cshape[i] = ia >= 0 ? a->shape[ia] : b->shape[ib];
  }
  for (int i = 0; i < na; ++i) {
    const int ib = find_lab(lb, nb, la[i]), ic = find_lab(lc, nc, la[i]);
    if (ib < 0 && ic < 0) TCI_RET(TCI_ERR_LABEL, "label of a in neither b nor c");
    if (ib >= 0 && b->shape[ib] != a->shape[i]) TCI_RET(TCI_ERR_SHAPE, "contracted dimensions differ");
  }
  for (int i = 0; i < nb; ++i) {
    if (find_lab(la, na, lb[i]) < 0 && find_lab(lc, nc, lb[i]) < 0)
      TCI_RET(TCI_ERR_LABEL, "label of b in neither a nor c");
  }
  Trace tr(ctx, "contract", shape_str(a) + "x" + shape_str(b));
  ctx->arena.reset();
  const int dt = a->dtype;
  const size_t es = elem_bytes(dt);
  // bond groups: I (free in a, a's order), S (summed, a's order), J (free in b, b's order)
  std::vector<int> I, S, J;
  for (int i = 0; i < na; ++i) (find_lab(lc, nc, la[i]) >= 0 ? I : S).push_back(i);
  for (int i = 0; i < nb; ++i) if (find_lab(lc, nc, lb[i]) >= 0) J.push_back(i);
  long long M = 1, N = 1, K = 1;
  for (int i : I) M *= a->shape[i];
  for (int i : S) K *= a->shape[i];
  for (int i : J) N *= b->shape[i];
  // operand A as M x K (op N) or K x M (op T) without moving data when possible
  std::vector<int> permA, permB;
  for (int i : I) permA.push_back(i);
  for (int i : S) permA.push_back(i);
  std::vector<int> Sb;  // positions in b of the summed labels, in S order
  for (int i : S) Sb.push_back(find_lab(lb, nb, la[i]));
  for (int i : Sb) permB.push_back(i);
  for (int i : J) permB.push_back(i);
  auto is_ident = [](const std::vector<int>& p) {
    for (size_t i = 0; i < p.size(); ++i) if (p[i] != (int)i) return false;
    return true;
  };
  // A^T form: a == [S..., I...]
  std::vector<int> permAt;
  for (int i : S) permAt.push_back(i);
  for (int i : I) permAt.push_back(i);
  std::vector<int> permBt;
  for (int i : J) permBt.push_back(i);
  for (int i : Sb) permBt.push_back(i);
  const void* Ap = a->data;
  const void* Bp = b->data;
  int opA = OP_N, opB = OP_N;
  long long lda = K, ldb = N;
  if (is_ident(permA)) {
    opA = OP_N; lda = K;
  } else if (is_ident(permAt)) {
    opA = OP_T; lda = M;
  } else {
    void* tmp = ctx->arena.get(tbytes(a));
    if (!tmp) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
    long long sh[MAX_ORDER]; int p[MAX_ORDER];
    for (int i = 0; i < na; ++i) { sh[i] = a->shape[i]; p[i] = permA[i]; }
    TCI_CHECK_HIP(tci::permute(dt, a->data, tmp, na, sh, p, ctx->stream));
    Ap = tmp; opA = OP_N; lda = K;
  }
  if (is_ident(permB)) {
    opB = OP_N; ldb = N;
  } else if (is_ident(permBt)) {
    opB = OP_T; ldb = K;
  } else {
    void* tmp = ctx->arena.get(tbytes(b));
    if (!tmp) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
    long long sh[MAX_ORDER]; int p[MAX_ORDER];
    for (int i = 0; i < nb; ++i) { sh[i] = b->shape[i]; p[i] = permB[i]; }
    TCI_CHECK_HIP(tci::permute(dt, b->data, tmp, nb, sh, p, ctx->stream));
    Bp = tmp; opB = OP_N; ldb = N;
  }
  // natural output order: I then J
  std::vector<int32_t> nat;
  for (int i : I) nat.push_back(la[i]);
  for (int i : J) nat.push_back(lb[i]);
  bool same = (int)nat.size() == nc;
  for (int i = 0; same && i < nc; ++i) same = (nat[i] == lc[i]);
  const bool alias = (c == a || c == b);
  void* Cp;
  if (same && !alias) {
    TCI_TRY(ensure_shape(ctx, c, dt, nc, cshape));
    Cp = c->data;
  } else {
    Cp = ctx->arena.get((size_t)M * N * es);
    if (!Cp) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
  }
  GemmArgs g = gemm_args((int)M, (int)N, (int)K, opA, opB, Ap, lda, Bp, ldb, Cp, N);
  if ((dt == C128 || dt == F64) && K >= 256) {
    // FP64 products with few output tiles split K (see gemm.hpp)
    g.kws = ctx->arena.get(GEMM_SPLITK_WS_BYTES);
    g.kws_bytes = g.kws ? GEMM_SPLITK_WS_BYTES : 0;
  }
  TCI_CHECK_HIP(gemm(dt, prec_for(ctx, dt), g, ctx->stream));
  if (!(same && !alias)) {
    // C has bonds nat; permute to lc
    long long sh[MAX_ORDER]; int p[MAX_ORDER];
    for (size_t i = 0; i < nat.size(); ++i) {
      const int ia = find_lab(la, na, nat[i]);
      sh[i] = ia >= 0 ? a->shape[ia] : b->shape[find_lab(lb, nb, nat[i])];
    }
    for (int i = 0; i < nc; ++i) p[i] = (int)(std::find(nat.begin(), nat.end(), lc[i]) - nat.begin());
    TCI_TRY(ensure_shape(ctx, c, dt, nc, cshape));
    if (nc > 0) TCI_CHECK_HIP(tci::permute(dt, Cp, c->data, nc, sh, p, ctx->stream));
    else TCI_CHECK_HIP(hipMemcpyAsync(c->data, Cp, es, hipMemcpyDeviceToDevice, ctx->stream));
  }
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_contract_str(tci_context ctx, tci_tensor a, const char* la, tci_tensor b, const char* lb,
                            tci_tensor c, const char* lc) try {
  if (!la || !lb || !lc) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null label string");
  int32_t A[MAX_ORDER + 1], B[MAX_ORDER + 1], C[MAX_ORDER + 1];
  const int na = (int)std::strlen(la), nb = (int)std::strlen(lb), nc = (int)std::strlen(lc);
  if (na > MAX_ORDER || nb > MAX_ORDER || nc > MAX_ORDER) TCI_RET(TCI_ERR_LABEL, "too many labels");
  for (int i = 0; i < na; ++i) A[i] = (unsigned char)la[i];
  for (int i = 0; i < nb; ++i) B[i] = (unsigned char)lb[i];
  for (int i = 0; i < nc; ++i) C[i] = (unsigned char)lc[i];
  return tci_contract(ctx, a, A, na, b, B, nb, c, C, nc);
} TCI_API_CATCH


// ---------------------------------------------------------------- sub-tensors
}  // extern "C"

namespace {

void row_major_strides(int order, const int64_t* shape, long long* st) {
  long long acc = 1;
  for (int b = order - 1; b >= 0; --b) {
    st[b] = acc;
    acc *= shape[b];
  }
}

// Source of an out-of-place operation: the input itself, or a copy of it in
// the arena when the output handle is the input handle (its storage may be
// reallocated by the output's shape change).
tci_status stable_source(tci_context ctx, tci_tensor in, tci_tensor out, const void*& src) {
  src = in->data;
  if (out != in) return TCI_OK;
  const size_t bytes = tbytes(in);
  void* tmp = ctx->arena.get(std::max<size_t>(bytes, 16));
  if (!tmp) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
  if (bytes) TCI_CHECK_HIP(hipMemcpyAsync(tmp, in->data, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  src = tmp;
  return TCI_OK;
}

// Copy the whole of src (shape sshape, order) into dst (shape dshape) at the
// offsets off[] (same order).
tci_status copy_box(tci_context ctx, int dt, const void* src, int order, const int64_t* sshape, void* dst,
                    const int64_t* dshape, const int64_t* off) {
  BoxCopy c{};
  c.order = order;
  long long ss[MAX_ORDER + 1], ds[MAX_ORDER + 1];
  row_major_strides(order, sshape, ss);
  row_major_strides(order, dshape, ds);
  c.total = 1;
  c.soff = 0;
  c.doff = 0;
  for (int b = 0; b < order; ++b) {
    c.dims[b] = sshape[b];
    c.sstride[b] = ss[b];
    c.dstride[b] = ds[b];
    c.doff += off[b] * ds[b];
    c.total *= sshape[b];
  }
  if (order == 0) {   // scalar
    c.order = 1;
    c.dims[0] = 1;
    c.sstride[0] = c.dstride[0] = 1;
  }
  TCI_CHECK_HIP(box_copy(elem_bytes(dt), src, dst, c, ctx->stream));
  return TCI_OK;
}

}  // namespace

extern "C" {

tci_status tci_fill(tci_context ctx, tci_dtype dtype, int order, const int64_t* shape, const void* value,
                    tci_tensor* out) try {
  if (!value) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null value");
  TCI_TRY(make_tensor(ctx, dtype, order, shape, out, false));
  double vr, vi;
  host_scalar(dtype, value, vr, vi);
  TCI_CHECK_HIP(fill_value(dtype, (*out)->data, tsize(*out), vr, vi, ctx->stream));
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_eye(tci_context ctx, tci_dtype dtype, int64_t n, tci_tensor* out) try {
  if (n < 0) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "negative dimension");
  const int64_t shape[2] = {n, n};
  TCI_TRY(make_tensor(ctx, dtype, 2, shape, out, true));
  TCI_CHECK_HIP(add_diag(dtype, (*out)->data, n, (int)n, 1.0, ctx->stream));
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_extract_sub(tci_context ctx, tci_tensor in, const int64_t* first, const int64_t* last,
                           tci_tensor out) try {
  TCI_TRY(check_ctx(ctx));
  TCI_TRY(check_t(in, "in"));
  if (!out || (in->order > 0 && (!first || !last))) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  const int order = in->order;
  int64_t oshape[MAX_ORDER];
  for (int b = 0; b < order; ++b) {
    if (first[b] < 0 || last[b] < first[b] || last[b] > in->shape[b])
      TCI_RET(TCI_ERR_INVALID_ARGUMENT, "range outside the bond");
    oshape[b] = last[b] - first[b];
  }
  Trace tr(ctx, "extract_sub", shape_str(in));
  ctx->arena.reset();
  const void* src;
  TCI_TRY(stable_source(ctx, in, out, src));
  const int dt = in->dtype;
  int64_t ishape[MAX_ORDER];
  for (int b = 0; b < order; ++b) ishape[b] = in->shape[b];
  TCI_TRY(ensure_shape(ctx, out, dt, order, oshape));
  BoxCopy c{};
  long long ss[MAX_ORDER + 1], ds[MAX_ORDER + 1];
  row_major_strides(order, ishape, ss);
  row_major_strides(order, oshape, ds);
  c.order = std::max(order, 1);
  c.dims[0] = 1;
  c.sstride[0] = c.dstride[0] = 1;
  c.total = 1;
  c.soff = c.doff = 0;
  for (int b = 0; b < order; ++b) {
    c.dims[b] = oshape[b];
    c.sstride[b] = ss[b];
    c.dstride[b] = ds[b];
    c.soff += first[b] * ss[b];
    c.total *= oshape[b];
  }
  TCI_CHECK_HIP(box_copy(elem_bytes(dt), src, out->data, c, ctx->stream));
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_shrink(tci_context ctx, tci_tensor in, int n, const int32_t* bonds, const int64_t* first,
                      const int64_t* last, tci_tensor out) try {
  TCI_TRY(check_ctx(ctx));
  TCI_TRY(check_t(in, "in"));
  if (n < 0 || (n > 0 && (!bonds || !first || !last))) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  int64_t f[MAX_ORDER], l[MAX_ORDER];
  bool seen[MAX_ORDER] = {false};
  for (int b = 0; b < in->order; ++b) {
    f[b] = 0;
    l[b] = in->shape[b];
  }
  for (int k = 0; k < n; ++k) {
    const int b = bonds[k];
    if (b < 0 || b >= in->order || seen[b]) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "bad bond index");
    seen[b] = true;
    f[b] = first[k];
    l[b] = last[k];
  }
  return tci_extract_sub(ctx, in, f, l, out);
} TCI_API_CATCH

tci_status tci_expand(tci_context ctx, tci_tensor in, int n, const int32_t* bonds, const int64_t* increments,
                      tci_tensor out) try {
  TCI_TRY(check_ctx(ctx));
  TCI_TRY(check_t(in, "in"));
  if (!out || n < 0 || (n > 0 && (!bonds || !increments))) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  const int order = in->order;
  int64_t ishape[MAX_ORDER], oshape[MAX_ORDER], zero[MAX_ORDER];
  bool seen[MAX_ORDER] = {false};
  for (int b = 0; b < order; ++b) {
    ishape[b] = oshape[b] = in->shape[b];
    zero[b] = 0;
  }
  for (int k = 0; k < n; ++k) {
    const int b = bonds[k];
    if (b < 0 || b >= order || seen[b] || increments[k] < 0) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "bad bond or increment");
    seen[b] = true;
    oshape[b] += increments[k];
  }
  Trace tr(ctx, "expand", shape_str(in));
  ctx->arena.reset();
  const void* src;
  TCI_TRY(stable_source(ctx, in, out, src));
  const int dt = in->dtype;
  TCI_TRY(ensure_shape(ctx, out, dt, order, oshape));
  if (tbytes(out)) TCI_CHECK_HIP(hipMemsetAsync(out->data, 0, tbytes(out), ctx->stream));
  return copy_box(ctx, dt, src, order, ishape, out->data, oshape, zero);
} TCI_API_CATCH

tci_status tci_replace_sub(tci_context ctx, tci_tensor in, tci_tensor sub, const int64_t* begin, tci_tensor out) try {
  TCI_TRY(check_ctx(ctx));
  TCI_TRY(check_t(in, "in"));
  TCI_TRY(check_t(sub, "sub"));
  if (!out || (in->order > 0 && !begin)) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  if (sub->order != in->order || sub->dtype != in->dtype) TCI_RET(TCI_ERR_SHAPE, "sub must match order and dtype");
  if (sub == out && out != in) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "out must not alias sub");
  const int order = in->order;
  int64_t ishape[MAX_ORDER], sshape[MAX_ORDER];
  for (int b = 0; b < order; ++b) {
    ishape[b] = in->shape[b];
    sshape[b] = sub->shape[b];
    if (begin[b] < 0 || begin[b] + sub->shape[b] > in->shape[b])
      TCI_RET(TCI_ERR_INVALID_ARGUMENT, "sub does not fit at begin");
  }
  Trace tr(ctx, "replace_sub", shape_str(in));
  if (out != in) {
    TCI_TRY(ensure_shape(ctx, out, in->dtype, order, ishape));
    if (tbytes(in)) TCI_CHECK_HIP(hipMemcpyAsync(out->data, in->data, tbytes(in), hipMemcpyDeviceToDevice, ctx->stream));
  }
  return copy_box(ctx, in->dtype, sub->data, order, sshape, out->data, ishape, begin);
} TCI_API_CATCH

tci_status tci_concatenate(tci_context ctx, int n, const tci_tensor* ins, int bond, tci_tensor out) try {
  TCI_TRY(check_ctx(ctx));
  if (n < 1 || !ins || !out) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "need at least one input and an output");
  for (int k = 0; k < n; ++k) {
    TCI_TRY(check_t(ins[k], "ins"));
    if (ins[k] == out) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "out must not alias an input");
  }
  const tci_tensor a = ins[0];
  const int order = a->order, dt = a->dtype;
  if (bond < 0 || bond >= order) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "bad bond index");
  int64_t oshape[MAX_ORDER];
  for (int b = 0; b < order; ++b) oshape[b] = a->shape[b];
  oshape[bond] = 0;
  for (int k = 0; k < n; ++k) {
    if (ins[k]->order != order || ins[k]->dtype != dt) TCI_RET(TCI_ERR_SHAPE, "inputs differ in order or dtype");
    for (int b = 0; b < order; ++b)
      if (b != bond && ins[k]->shape[b] != a->shape[b]) TCI_RET(TCI_ERR_SHAPE, "inputs differ off the bond");
    oshape[bond] += ins[k]->shape[bond];
  }
  Trace tr(ctx, "concatenate", shape_str(a));
  TCI_TRY(ensure_shape(ctx, out, dt, order, oshape));
  int64_t off[MAX_ORDER] = {0};
  for (int k = 0; k < n; ++k) {
    int64_t sshape[MAX_ORDER];
    for (int b = 0; b < order; ++b) sshape[b] = ins[k]->shape[b];
    TCI_TRY(copy_box(ctx, dt, ins[k]->data, order, sshape, out->data, oshape, off));
    off[bond] += sshape[bond];
  }
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_stack(tci_context ctx, int n, const tci_tensor* ins, int bond, tci_tensor out) try {
  TCI_TRY(check_ctx(ctx));
  if (n < 1 || !ins || !out) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "need at least one input and an output");
  for (int k = 0; k < n; ++k) {
    TCI_TRY(check_t(ins[k], "ins"));
    if (ins[k] == out) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "out must not alias an input");
  }
  const tci_tensor a = ins[0];
  const int order = a->order, dt = a->dtype;
  if (order + 1 > MAX_ORDER) TCI_RET(TCI_ERR_UNSUPPORTED, "result order above the maximum");
  if (bond < 0 || bond > order) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "bad bond index");
  for (int k = 0; k < n; ++k) {
    if (ins[k]->order != order || ins[k]->dtype != dt) TCI_RET(TCI_ERR_SHAPE, "inputs differ in order or dtype");
    for (int b = 0; b < order; ++b)
      if (ins[k]->shape[b] != a->shape[b]) TCI_RET(TCI_ERR_SHAPE, "inputs differ in shape");
  }
  // each input is viewed with a bond of dimension 1 inserted at `bond`
  int64_t oshape[MAX_ORDER], sshape[MAX_ORDER];
  for (int b = 0, c = 0; b <= order; ++b) {
    if (b == bond) {
      oshape[b] = n;
      sshape[b] = 1;
    } else {
      oshape[b] = a->shape[c];
      sshape[b] = a->shape[c];
      ++c;
    }
  }
  Trace tr(ctx, "stack", shape_str(a));
  TCI_TRY(ensure_shape(ctx, out, dt, order + 1, oshape));
  int64_t off[MAX_ORDER] = {0};
  for (int k = 0; k < n; ++k) {
    off[bond] = k;
    TCI_TRY(copy_box(ctx, dt, ins[k]->data, order + 1, sshape, out->data, oshape, off));
  }
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_trace(tci_context ctx, tci_tensor in, int npairs, const int32_t* pairs, tci_tensor out) try {
  TCI_TRY(check_ctx(ctx));
  TCI_TRY(check_t(in, "in"));
  if (!out || npairs < 0 || (npairs > 0 && !pairs)) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  const int order = in->order;
  bool used[MAX_ORDER] = {false};
  long long st[MAX_ORDER + 1];
  int64_t ishape[MAX_ORDER];
  for (int b = 0; b < order; ++b) ishape[b] = in->shape[b];
  row_major_strides(order, ishape, st);
  TraceArgs ta{};
  for (int p = 0; p < npairs; ++p) {
    const int x = pairs[2 * p], y = pairs[2 * p + 1];
    if (x < 0 || y < 0 || x >= order || y >= order || x == y || used[x] || used[y])
      TCI_RET(TCI_ERR_INVALID_ARGUMENT, "bad bond pair");
    if (in->shape[x] != in->shape[y]) TCI_RET(TCI_ERR_SHAPE, "paired bonds differ in dimension");
    used[x] = used[y] = true;
    ta.pdims[p] = in->shape[x];
    ta.pstride[p] = st[x] + st[y];
  }
  ta.npair = npairs;
  ta.ntr = 1;
  for (int p = 0; p < npairs; ++p) ta.ntr *= ta.pdims[p];
  int64_t oshape[MAX_ORDER];
  int nk = 0;
  ta.nout = 1;
  for (int b = 0; b < order; ++b) {
    if (used[b]) continue;
    oshape[nk] = in->shape[b];
    ta.kdims[nk] = in->shape[b];
    ta.kstride[nk] = st[b];
    ta.nout *= in->shape[b];
    ++nk;
  }
  ta.nkeep = nk;
  Trace tr(ctx, "trace", shape_str(in));
  ctx->arena.reset();
  const void* src;
  TCI_TRY(stable_source(ctx, in, out, src));
  const int dt = in->dtype;
  TCI_TRY(ensure_shape(ctx, out, dt, nk, oshape));
  TCI_CHECK_HIP(partial_trace(dt, src, out->data, ta, ctx->stream));
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_diag(tci_context ctx, tci_tensor in, tci_tensor out) try {
  TCI_TRY(check_ctx(ctx));
  TCI_TRY(check_t(in, "in"));
  if (!out) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  if (in->order != 1 && in->order != 2) TCI_RET(TCI_ERR_SHAPE, "diag needs a first- or second-order tensor");
  Trace tr(ctx, "diag", shape_str(in));
  ctx->arena.reset();
  const void* src;
  TCI_TRY(stable_source(ctx, in, out, src));
  const int dt = in->dtype;
  BoxCopy c{};
  c.order = 1;
  c.soff = c.doff = 0;
  if (in->order == 1) {   // vector -> diagonal matrix
    const int64_t n = in->shape[0];
    const int64_t shape[2] = {n, n};
    TCI_TRY(ensure_shape(ctx, out, dt, 2, shape));
    TCI_CHECK_HIP(fill_value(dt, out->data, (long long)n * n, 0.0, 0.0, ctx->stream));
    c.dims[0] = n;
    c.sstride[0] = 1;
    c.dstride[0] = n + 1;
    c.total = n;
  } else {                // matrix -> main diagonal, length min(d0, d1)
    const int64_t d1 = in->shape[1], n = std::min(in->shape[0], d1);
    TCI_TRY(ensure_shape(ctx, out, dt, 1, &n));
    c.dims[0] = n;
    c.sstride[0] = d1 + 1;
    c.dstride[0] = 1;
    c.total = n;
  }
  TCI_CHECK_HIP(box_copy(elem_bytes(dt), src, out->data, c, ctx->stream));
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_to_cplx(tci_context ctx, tci_tensor in, tci_tensor out) try {
  TCI_TRY(check_ctx(ctx));
  TCI_TRY(check_t(in, "in"));
  if (!out) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  Trace tr(ctx, "to_cplx", shape_str(in));
  ctx->arena.reset();
  const void* src;
  TCI_TRY(stable_source(ctx, in, out, src));
  const int dt = in->dtype, cdt = dt == F32 ? C64 : dt == F64 ? C128 : dt;
  int64_t shape[MAX_ORDER];
  for (int b = 0; b < in->order; ++b) shape[b] = in->shape[b];
  const long long n = tsize(in);
  TCI_TRY(ensure_shape(ctx, out, cdt, in->order, shape));
  TCI_CHECK_HIP(tci::convert(dt, src, cdt, out->data, n, ctx->stream));
  return TCI_OK;
} TCI_API_CATCH

namespace {
tci_status part_of(tci_context ctx, tci_tensor in, tci_tensor out, bool imag, const char* name) {
  TCI_TRY(check_ctx(ctx));
  TCI_TRY(check_t(in, "in"));
  if (!out) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  Trace tr(ctx, name, shape_str(in));
  ctx->arena.reset();
  const void* src;
  TCI_TRY(stable_source(ctx, in, out, src));
  const int dt = in->dtype, rdt = dt == C64 ? F32 : dt == C128 ? F64 : dt;
  int64_t shape[MAX_ORDER];
  for (int b = 0; b < in->order; ++b) shape[b] = in->shape[b];
  const long long n = tsize(in);
  TCI_TRY(ensure_shape(ctx, out, rdt, in->order, shape));
  if (is_complex(dt))
    TCI_CHECK_HIP(complex_part(dt, src, out->data, n, imag, ctx->stream));
  else if (imag)
    TCI_CHECK_HIP(fill_value(rdt, out->data, n, 0.0, 0.0, ctx->stream));
  else if (out->data != src && n > 0)
    TCI_CHECK_HIP(hipMemcpyAsync(out->data, src, (size_t)n * elem_bytes(dt), hipMemcpyDeviceToDevice, ctx->stream));
  return TCI_OK;
}
}  // namespace

tci_status tci_real(tci_context ctx, tci_tensor in, tci_tensor out) try { return part_of(ctx, in, out, false, "real"); } TCI_API_CATCH
tci_status tci_imag(tci_context ctx, tci_tensor in, tci_tensor out) try { return part_of(ctx, in, out, true, "imag"); } TCI_API_CATCH

// File layout: 8 bytes "TCIMI355", int32 format version (1), int32 dtype,
// int32 order, int32 zero, int64 shape[order], then the elements row-major in
// the host's (little-endian) byte order.
namespace {
constexpr char SAVE_MAGIC[8] = {'T', 'C', 'I', 'M', 'I', '3', '5', '5'};
constexpr int32_t SAVE_VERSION = 1;
}  // namespace

tci_status tci_save(tci_context ctx, tci_tensor t, const char* path) try {
  TCI_TRY(check_ctx(ctx));
  TCI_TRY(check_t(t, "t"));
  if (!path) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null path");
  Trace tr(ctx, "save", shape_str(t));
  std::vector<char> host(tbytes(t));
  if (!host.empty()) {
    TCI_CHECK_HIP(hipMemcpyAsync(host.data(), t->data, host.size(), hipMemcpyDeviceToHost, ctx->stream));
    TCI_CHECK_HIP(hipStreamSynchronize(ctx->stream));
  }
  FILE* f = std::fopen(path, "wb");
  if (!f) TCI_RET(TCI_ERR_INVALID_ARGUMENT, std::string("cannot open ") + path);
  const int32_t hdr[4] = {SAVE_VERSION, t->dtype, t->order, 0};
  bool ok = std::fwrite(SAVE_MAGIC, 1, 8, f) == 8 && std::fwrite(hdr, sizeof(int32_t), 4, f) == 4;
  if (ok && t->order > 0) ok = std::fwrite(t->shape, sizeof(int64_t), t->order, f) == (size_t)t->order;
  if (ok && !host.empty()) ok = std::fwrite(host.data(), 1, host.size(), f) == host.size();
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) TCI_RET(TCI_ERR_INVALID_ARGUMENT, std::string("short write to ") + path);
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_load(tci_context ctx, const char* path, tci_tensor* out) try {
  TCI_TRY(check_ctx(ctx));
  if (!path || !out) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  FILE* f = std::fopen(path, "rb");
  if (!f) TCI_RET(TCI_ERR_INVALID_ARGUMENT, std::string("cannot open ") + path);
  char magic[8];
  int32_t hdr[4];
  int64_t shape[MAX_ORDER];
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, SAVE_MAGIC, 8) == 0 &&
            std::fread(hdr, sizeof(int32_t), 4, f) == 4 && hdr[0] == SAVE_VERSION && valid_dtype(hdr[1]) &&
            hdr[2] >= 0 && hdr[2] <= MAX_ORDER;
  if (ok && hdr[2] > 0) ok = std::fread(shape, sizeof(int64_t), hdr[2], f) == (size_t)hdr[2];
  for (int b = 0; ok && b < hdr[2]; ++b) ok = shape[b] >= 0;
  if (!ok) {
    std::fclose(f);
    TCI_RET(TCI_ERR_INVALID_ARGUMENT, std::string("not a tensor file: ") + path);
  }
  long long n = 1;
  for (int b = 0; b < hdr[2]; ++b) n *= shape[b];
  std::vector<char> host((size_t)n * elem_bytes(hdr[1]));
  ok = host.empty() || std::fread(host.data(), 1, host.size(), f) == host.size();
  std::fclose(f);
  if (!ok) TCI_RET(TCI_ERR_INVALID_ARGUMENT, std::string("truncated tensor file: ") + path);
  TCI_TRY(make_tensor(ctx, (tci_dtype)hdr[1], hdr[2], shape, out, false));
  Trace tr(ctx, "load", shape_str(*out));
  if (!host.empty()) {
    TCI_CHECK_HIP(hipMemcpyAsync((*out)->data, host.data(), host.size(), hipMemcpyHostToDevice, ctx->stream));
    TCI_CHECK_HIP(hipStreamSynchronize(ctx->stream));
  }
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_show(tci_context ctx, tci_tensor t) try {
  TCI_TRY(check_ctx(ctx));
  TCI_TRY(check_t(t, "t"));
  static const char* names[] = {"F32", "F64", "C64", "C128"};
  std::vector<char> host(tbytes(t));
  if (!host.empty()) {
    TCI_CHECK_HIP(hipMemcpyAsync(host.data(), t->data, host.size(), hipMemcpyDeviceToHost, ctx->stream));
    TCI_CHECK_HIP(hipStreamSynchronize(ctx->stream));
  }
  std::printf("tensor %s shape %s\n", names[t->dtype], shape_str(t).c_str());
  const long long n = tsize(t);
  long long st[MAX_ORDER + 1];
  int64_t shp[MAX_ORDER];
  for (int b = 0; b < t->order; ++b) shp[b] = t->shape[b];
  row_major_strides(t->order, shp, st);
  for (long long e = 0; e < n; ++e) {
    std::printf("  (");
    for (int b = 0; b < t->order; ++b) std::printf(b ? ",%lld" : "%lld", (long long)((e / st[b]) % shp[b]));
    std::printf(") ");
    const char* p = host.data() + (size_t)e * elem_bytes(t->dtype);
    switch (t->dtype) {
      case F32: std::printf("%.9g\n", (double)*reinterpret_cast<const float*>(p)); break;
      case F64: std::printf("%.17g\n", *reinterpret_cast<const double*>(p)); break;
      case C64: {
        const float* c = reinterpret_cast<const float*>(p);
        std::printf("%.9g%+.9gj\n", (double)c[0], (double)c[1]);
        break;
      }
      default: {
        const double* c = reinterpret_cast<const double*>(p);
        std::printf("%.17g%+.17gj\n", c[0], c[1]);
      }
    }
  }
  std::fflush(stdout);
  return TCI_OK;
} TCI_API_CATCH

}  // extern "C"
