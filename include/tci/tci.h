// tci/tci.h -- C++17 interface of the MI355X two-site MPS update library, a
// header-only layer over the C ABI in tci_c.h.
//
// It follows the Tensor Computing Interface of arXiv:2512.23917 (the
// appendix that specifies TCI, "Spec" below): the type system (a tensor
// type, tci::tensor_traits and the alias templates over it, List / Pair /
// Map), and the core functions under their Spec names with in-place and
// out-of-place forms.  Every call forwards to the C ABI, so all tensor work
// runs in the library's HIP kernels on the context's stream; host data is
// touched only where the Spec passes host values (get_elem, set_elem,
// random, assign_from_range, to_range, save/load).
//
// Errors: a failing C call throws tci::error carrying the tci_status and the
// library's message.
//
// for_each / for_each_with_coors take a device functor and are available
// when this header is compiled by hipcc: the functor runs in a kernel that
// the including translation unit instantiates.
#ifndef TCI_TCI_H
#define TCI_TCI_H

#include <algorithm>
#include <complex>
#include <cstddef>
#include <cstdint>
#include <iterator>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../tci_c.h"

#if defined(__HIPCC__)
#include <hip/hip_complex.h>
#include <hip/hip_runtime.h>
#endif

namespace tci {

// ---------------------------------------------------------------- auxiliary types (Spec, type system)
template <typename T>
using List = std::vector<T>;
template <typename T, typename U>
using Pair = std::pair<T, U>;
template <typename T, typename U>
using Map = std::unordered_map<T, U>;

class error : public std::runtime_error {
 public:
  error(tci_status s, const std::string& what) : std::runtime_error(what), status(s) {}
  tci_status status;
};

namespace detail {
inline void check(tci_status s, const char* fn) {
  if (s != TCI_OK) throw error(s, std::string(fn) + ": " + tci_last_error());
}
template <typename E>
struct dtype_of;
template <>
struct dtype_of<float> { static constexpr tci_dtype value = TCI_F32; };
template <>
struct dtype_of<double> { static constexpr tci_dtype value = TCI_F64; };
template <>
struct dtype_of<std::complex<float>> { static constexpr tci_dtype value = TCI_C64; };
template <>
struct dtype_of<std::complex<double>> { static constexpr tci_dtype value = TCI_C128; };
template <typename E>
struct real_of { using type = E; };
template <typename R>
struct real_of<std::complex<R>> { using type = R; };
template <typename E>
struct cplx_of { using type = std::complex<E>; };
template <typename R>
struct cplx_of<std::complex<R>> { using type = std::complex<R>; };
}  // namespace detail

// ---------------------------------------------------------------- context
// Owns a tci_context on one HIP device, ordered on a borrowed stream.
class Context {
 public:
  Context() = default;
  // opts: the implementation-defined parameters of create_context
  // (allocator, precision, svd mode, autotune cache, verbosity); nullptr =
  // the defaults.
  explicit Context(int device, void* hip_stream = nullptr, const tci_context_opts* opts = nullptr)
      : stream_(hip_stream) {
    detail::check(tci_create_context(&h_, device, hip_stream, opts), "tci_create_context");
  }
  Context(const Context&) = delete;
  Context& operator=(const Context&) = delete;
  Context(Context&& o) noexcept : h_(o.h_), stream_(o.stream_) { o.h_ = nullptr; }
  Context& operator=(Context&& o) noexcept {
    if (this != &o) {
      reset();
      h_ = o.h_;
      stream_ = o.stream_;
      o.h_ = nullptr;
    }
    return *this;
  }
  ~Context() { reset(); }
  void reset() {
    if (h_) tci_destroy_context(h_);
    h_ = nullptr;
  }
  tci_context get() const { return h_; }
  // The HIP stream the context's work is ordered on (NULL: the null stream).
  void* stream() const { return stream_; }

 private:
  tci_context h_ = nullptr;
  void* stream_ = nullptr;
};

// ---------------------------------------------------------------- tensor
// Dense row-major tensor in device memory with element type E (float,
// double, std::complex<float>, std::complex<double>).  Move-only; a default
// constructed tensor is empty (Ten{} of the Spec).
template <typename E>
class Tensor {
  static_assert(std::is_same<E, float>::value || std::is_same<E, double>::value ||
                    std::is_same<E, std::complex<float>>::value || std::is_same<E, std::complex<double>>::value,
                "element type must be float, double, std::complex<float> or std::complex<double>");

 public:
  using elem_type = E;
  Tensor() = default;
  Tensor(tci_context ctx, tci_tensor h) : ctx_(ctx), h_(h) {}
  Tensor(const Tensor&) = delete;
  Tensor& operator=(const Tensor&) = delete;
  Tensor(Tensor&& o) noexcept : ctx_(o.ctx_), h_(o.h_) { o.ctx_ = nullptr, o.h_ = nullptr; }
  Tensor& operator=(Tensor&& o) noexcept {
    if (this != &o) {
      reset();
      ctx_ = o.ctx_;
      h_ = o.h_;
      o.ctx_ = nullptr, o.h_ = nullptr;
    }
    return *this;
  }
  ~Tensor() { reset(); }
  void reset() {
    if (h_) tci_destroy(ctx_, h_);
    h_ = nullptr;
    ctx_ = nullptr;
  }
  bool empty() const { return h_ == nullptr; }
  tci_tensor handle() const { return h_; }
  // Handle usable as an output: an empty tensor first gets an owning
  // order-0 allocation that the library resizes.
  tci_tensor out_handle(tci_context ctx) {
    if (!h_) {
      detail::check(tci_allocate(ctx, detail::dtype_of<E>::value, 0, nullptr, &h_), "tci_allocate");
      ctx_ = ctx;
    }
    return h_;
  }

 private:
  tci_context ctx_ = nullptr;
  tci_tensor h_ = nullptr;
};

// ---------------------------------------------------------------- traits (Spec, tensor_traits)
template <typename TenT>
struct tensor_traits;

template <typename E>
struct tensor_traits<Tensor<E>> {
  using ten_t = Tensor<E>;
  using order_t = int;
  using bond_dim_t = std::int64_t;
  using shape_t = List<bond_dim_t>;
  using bond_idx_t = int;
  using bond_label_t = std::int32_t;
  using ten_size_t = std::int64_t;
  using elem_t = E;
  using elem_coor_t = std::int64_t;
  using elem_coors_t = List<elem_coor_t>;
  using real_t = typename detail::real_of<E>::type;
  using real_ten_t = Tensor<real_t>;
  using cplx_t = typename detail::cplx_of<E>::type;
  using cplx_ten_t = Tensor<cplx_t>;
  using context_handle_t = Context;
};

template <typename TenT> using ten_t = typename tensor_traits<TenT>::ten_t;
template <typename TenT> using order_t = typename tensor_traits<TenT>::order_t;
template <typename TenT> using shape_t = typename tensor_traits<TenT>::shape_t;
template <typename TenT> using bond_dim_t = typename tensor_traits<TenT>::bond_dim_t;
template <typename TenT> using bond_idx_t = typename tensor_traits<TenT>::bond_idx_t;
template <typename TenT> using bond_label_t = typename tensor_traits<TenT>::bond_label_t;
template <typename TenT> using ten_size_t = typename tensor_traits<TenT>::ten_size_t;
template <typename TenT> using elem_t = typename tensor_traits<TenT>::elem_t;
template <typename TenT> using elem_coor_t = typename tensor_traits<TenT>::elem_coor_t;
template <typename TenT> using elem_coors_t = typename tensor_traits<TenT>::elem_coors_t;
template <typename TenT> using real_t = typename tensor_traits<TenT>::real_t;
template <typename TenT> using real_ten_t = typename tensor_traits<TenT>::real_ten_t;
template <typename TenT> using cplx_t = typename tensor_traits<TenT>::cplx_t;
template <typename TenT> using cplx_ten_t = typename tensor_traits<TenT>::cplx_ten_t;
template <typename TenT> using context_handle_t = typename tensor_traits<TenT>::context_handle_t;

namespace detail {
template <typename TenT>
inline tci_context C(context_handle_t<TenT>& ctx) { return ctx.get(); }
template <typename TenT>
constexpr tci_dtype DT = dtype_of<elem_t<TenT>>::value;
inline std::vector<std::int32_t> i32(const std::vector<int>& v) { return std::vector<std::int32_t>(v.begin(), v.end()); }
// out-of-place call on a fresh output tensor
template <typename OutT, typename F>
OutT fresh(Context& ctx, F&& f) {
  OutT out;
  f(out.out_handle(ctx.get()));
  return out;
}
}  // namespace detail

// General right eigendecomposition of the matricised tensor: w ascending by
// (real, imaginary) part, v {d_0..d_{k-1}, n} with unit-norm columns.
template <typename TenT>
void eig(context_handle_t<TenT>& ctx, const TenT& a, const order_t<TenT> num_of_bds_as_row, cplx_ten_t<TenT>& w,
         cplx_ten_t<TenT>& v) {
  detail::check(tci_eig(ctx.get(), a.handle(), num_of_bds_as_row, w.out_handle(ctx.get()), v.out_handle(ctx.get())),
                "tci_eig");
}
// Eigenvalues only.
template <typename TenT>
void eigvals(context_handle_t<TenT>& ctx, const TenT& a, const order_t<TenT> num_of_bds_as_row, cplx_ten_t<TenT>& w) {
  detail::check(tci_eigvals(ctx.get(), a.handle(), num_of_bds_as_row, w.out_handle(ctx.get())), "tci_eigvals");
}

// ---------------------------------------------------------------- miscellaneous (Spec)
inline std::string version() { return tci_version(); }

template <typename ContextHandleT>
void create_context(ContextHandleT& ctx, int device = 0, void* hip_stream = nullptr) {
  ctx = ContextHandleT(device, hip_stream);
}
template <typename ContextHandleT>
void destroy_context(ContextHandleT& ctx) {
  ctx.reset();
}

// ---------------------------------------------------------------- read-only queries (Spec)
template <typename TenT>
order_t<TenT> order(context_handle_t<TenT>& ctx, const TenT& a) {
  int r = 0;
  detail::check(tci_order(ctx.get(), a.handle(), &r), "tci_order");
  return r;
}
template <typename TenT>
shape_t<TenT> shape(context_handle_t<TenT>& ctx, const TenT& a) {
  const int r = order(ctx, a);
  shape_t<TenT> s(r);
  if (r) detail::check(tci_shape(ctx.get(), a.handle(), s.data(), r), "tci_shape");
  return s;
}
template <typename TenT>
ten_size_t<TenT> size(context_handle_t<TenT>& ctx, const TenT& a) {
  std::int64_t n = 0;
  detail::check(tci_size(ctx.get(), a.handle(), &n), "tci_size");
  return n;
}
template <typename TenT>
std::size_t size_bytes(context_handle_t<TenT>& ctx, const TenT& a) {
  std::int64_t n = 0;
  detail::check(tci_size_bytes(ctx.get(), a.handle(), &n), "tci_size_bytes");
  return static_cast<std::size_t>(n);
}
template <typename TenT>
elem_t<TenT> get_elem(context_handle_t<TenT>& ctx, const TenT& a, const elem_coors_t<TenT>& coors) {
  elem_t<TenT> v{};
  detail::check(tci_get_elem(ctx.get(), a.handle(), coors.data(), &v), "tci_get_elem");
  return v;
}

// ---------------------------------------------------------------- construction and destruction (Spec)
template <typename TenT>
TenT allocate(context_handle_t<TenT>& ctx, const shape_t<TenT>& shape) {
  tci_tensor h = nullptr;
  detail::check(tci_allocate(ctx.get(), detail::DT<TenT>, (int)shape.size(), shape.data(), &h), "tci_allocate");
  return TenT(ctx.get(), h);
}
template <typename TenT>
TenT zeros(context_handle_t<TenT>& ctx, const shape_t<TenT>& shape) {
  tci_tensor h = nullptr;
  detail::check(tci_zeros(ctx.get(), detail::DT<TenT>, (int)shape.size(), shape.data(), &h), "tci_zeros");
  return TenT(ctx.get(), h);
}
// Element at row-major position e is first[coors2idx(coors of e)].
template <typename TenT, typename RandomIt, typename Func>
TenT assign_from_range(context_handle_t<TenT>& ctx, const shape_t<TenT>& shape, RandomIt first, Func&& coors2idx) {
  std::int64_t n = 1;
  for (auto d : shape) n *= d;
  std::vector<elem_t<TenT>> host((std::size_t)n);
  elem_coors_t<TenT> c(shape.size(), 0);
  for (std::int64_t e = 0; e < n; ++e) {
    host[(std::size_t)e] = static_cast<elem_t<TenT>>(first[coors2idx(c)]);
    for (int b = (int)shape.size() - 1; b >= 0; --b) {
      if (++c[b] < shape[b]) break;
      c[b] = 0;
    }
  }
  TenT t = allocate<TenT>(ctx, shape);
  detail::check(tci_from_host(ctx.get(), t.handle(), host.data(), host.size() * sizeof(elem_t<TenT>)), "tci_from_host");
  return t;
}
// Elements drawn by gen() in row-major order.
template <typename TenT, typename RandNumGen>
TenT random(context_handle_t<TenT>& ctx, const shape_t<TenT>& shape, RandNumGen& gen) {
  std::int64_t n = 1;
  for (auto d : shape) n *= d;
  std::vector<elem_t<TenT>> host((std::size_t)n);
  for (auto& x : host) x = static_cast<elem_t<TenT>>(gen());
  TenT t = allocate<TenT>(ctx, shape);
  detail::check(tci_from_host(ctx.get(), t.handle(), host.data(), host.size() * sizeof(elem_t<TenT>)), "tci_from_host");
  return t;
}
template <typename TenT>
TenT eye(context_handle_t<TenT>& ctx, const bond_dim_t<TenT> n) {
  tci_tensor h = nullptr;
  detail::check(tci_eye(ctx.get(), detail::DT<TenT>, n, &h), "tci_eye");
  return TenT(ctx.get(), h);
}
template <typename TenT>
TenT fill(context_handle_t<TenT>& ctx, const shape_t<TenT>& shape, const elem_t<TenT> v) {
  tci_tensor h = nullptr;
  detail::check(tci_fill(ctx.get(), detail::DT<TenT>, (int)shape.size(), shape.data(), &v, &h), "tci_fill");
  return TenT(ctx.get(), h);
}
template <typename TenT>
TenT copy(context_handle_t<TenT>& ctx, const TenT& orig) {
  tci_tensor h = nullptr;
  detail::check(tci_copy(ctx.get(), orig.handle(), &h), "tci_copy");
  return TenT(ctx.get(), h);
}
template <typename TenT>
TenT move(context_handle_t<TenT>&, TenT& from) {
  return TenT(std::move(from));
}
template <typename TenT>
void clear(context_handle_t<TenT>&, TenT& a) {
  a.reset();
}

// ---------------------------------------------------------------- I/O (Spec)
template <typename TenT, typename Storage>
TenT load(context_handle_t<TenT>& ctx, Storage&& strg) {
  const std::string path(strg);
  tci_tensor h = nullptr;
  detail::check(tci_load(ctx.get(), path.c_str(), &h), "tci_load");
  TenT t(ctx.get(), h);
  tci_dtype dt;
  detail::check(tci_dtype_of(ctx.get(), h, &dt), "tci_dtype_of");
  if (dt != detail::DT<TenT>) throw error(TCI_ERR_DTYPE, "tci::load: file holds another element type");
  return t;
}
template <typename TenT, typename Storage>
void save(context_handle_t<TenT>& ctx, const TenT& a, Storage&& strg) {
  const std::string path(strg);
  detail::check(tci_save(ctx.get(), a.handle(), path.c_str()), "tci_save");
}

// ---------------------------------------------------------------- manipulation (Spec)
template <typename TenT>
void set_elem(context_handle_t<TenT>& ctx, TenT& a, const elem_coors_t<TenT>& coors, const elem_t<TenT> el) {
  detail::check(tci_set_elem(ctx.get(), a.handle(), coors.data(), &el), "tci_set_elem");
}
template <typename TenT>
void reshape(context_handle_t<TenT>& ctx, TenT& inout, const shape_t<TenT>& new_shape) {
  detail::check(tci_reshape(ctx.get(), inout.handle(), (int)new_shape.size(), new_shape.data(), inout.handle()),
                "tci_reshape");
}
template <typename TenT>
void reshape(context_handle_t<TenT>& ctx, const TenT& in, const shape_t<TenT>& new_shape, TenT& out) {
  detail::check(tci_reshape(ctx.get(), in.handle(), (int)new_shape.size(), new_shape.data(), out.out_handle(ctx.get())),
                "tci_reshape");
}
template <typename TenT>
void transpose(context_handle_t<TenT>& ctx, TenT& inout, const List<bond_idx_t<TenT>>& new_order) {
  const auto p = detail::i32(new_order);
  detail::check(tci_transpose(ctx.get(), inout.handle(), p.data(), inout.handle()), "tci_transpose");
}
template <typename TenT>
void transpose(context_handle_t<TenT>& ctx, const TenT& in, const List<bond_idx_t<TenT>>& new_order, TenT& out) {
  const auto p = detail::i32(new_order);
  detail::check(tci_transpose(ctx.get(), in.handle(), p.data(), out.out_handle(ctx.get())), "tci_transpose");
}
template <typename TenT>
void cplx_conj(context_handle_t<TenT>& ctx, TenT& inout) {
  detail::check(tci_cplx_conj(ctx.get(), inout.handle(), inout.handle()), "tci_cplx_conj");
}
template <typename TenT>
void cplx_conj(context_handle_t<TenT>& ctx, const TenT& in, TenT& out) {
  detail::check(tci_cplx_conj(ctx.get(), in.handle(), out.out_handle(ctx.get())), "tci_cplx_conj");
}
template <typename TenT>
cplx_ten_t<TenT> to_cplx(context_handle_t<TenT>& ctx, const TenT& in) {
  return detail::fresh<cplx_ten_t<TenT>>(ctx, [&](tci_tensor o) {
    detail::check(tci_to_cplx(ctx.get(), in.handle(), o), "tci_to_cplx");
  });
}
template <typename TenT>
real_ten_t<TenT> real(context_handle_t<TenT>& ctx, const TenT& in) {
  return detail::fresh<real_ten_t<TenT>>(ctx, [&](tci_tensor o) {
    detail::check(tci_real(ctx.get(), in.handle(), o), "tci_real");
  });
}
template <typename TenT>
real_ten_t<TenT> imag(context_handle_t<TenT>& ctx, const TenT& in) {
  return detail::fresh<real_ten_t<TenT>>(ctx, [&](tci_tensor o) {
    detail::check(tci_imag(ctx.get(), in.handle(), o), "tci_imag");
  });
}

namespace detail {
template <typename TenT>
void expand_impl(Context& ctx, const TenT& in, const Map<bond_idx_t<TenT>, bond_dim_t<TenT>>& m, tci_tensor out) {
  std::vector<std::int32_t> b;
  std::vector<std::int64_t> inc;
  for (const auto& kv : m) b.push_back(kv.first), inc.push_back(kv.second);
  check(tci_expand(ctx.get(), in.handle(), (int)b.size(), b.data(), inc.data(), out), "tci_expand");
}
template <typename TenT>
void shrink_impl(Context& ctx, const TenT& in,
                 const Map<bond_idx_t<TenT>, Pair<elem_coor_t<TenT>, elem_coor_t<TenT>>>& m, tci_tensor out) {
  std::vector<std::int32_t> b;
  std::vector<std::int64_t> f, l;
  for (const auto& kv : m) b.push_back(kv.first), f.push_back(kv.second.first), l.push_back(kv.second.second);
  check(tci_shrink(ctx.get(), in.handle(), (int)b.size(), b.data(), f.data(), l.data(), out), "tci_shrink");
}
template <typename TenT>
void extract_impl(Context& ctx, const TenT& in, const List<Pair<elem_coor_t<TenT>, elem_coor_t<TenT>>>& r,
                  tci_tensor out) {
  std::vector<std::int64_t> f, l;
  for (const auto& p : r) f.push_back(p.first), l.push_back(p.second);
  if ((int)r.size() != order(ctx, in)) throw error(TCI_ERR_INVALID_ARGUMENT, "tci::extract_sub: one range per bond");
  check(tci_extract_sub(ctx.get(), in.handle(), f.data(), l.data(), out), "tci_extract_sub");
}
template <typename TenT>
std::vector<tci_tensor> handles(const List<TenT>& ins) {
  std::vector<tci_tensor> h;
  for (const auto& t : ins) h.push_back(t.handle());
  return h;
}
}  // namespace detail

template <typename TenT>
void expand(context_handle_t<TenT>& ctx, TenT& inout, const Map<bond_idx_t<TenT>, bond_dim_t<TenT>>& m) {
  detail::expand_impl(ctx, inout, m, inout.handle());
}
template <typename TenT>
void expand(context_handle_t<TenT>& ctx, TenT& in, const Map<bond_idx_t<TenT>, bond_dim_t<TenT>>& m, TenT& out) {
  detail::expand_impl(ctx, in, m, out.out_handle(ctx.get()));
}
template <typename TenT>
void shrink(context_handle_t<TenT>& ctx, TenT& inout,
            const Map<bond_idx_t<TenT>, Pair<elem_coor_t<TenT>, elem_coor_t<TenT>>>& m) {
  detail::shrink_impl(ctx, inout, m, inout.handle());
}
template <typename TenT>
void shrink(context_handle_t<TenT>& ctx, const TenT& in,
            const Map<bond_idx_t<TenT>, Pair<elem_coor_t<TenT>, elem_coor_t<TenT>>>& m, TenT& out) {
  detail::shrink_impl(ctx, in, m, out.out_handle(ctx.get()));
}
template <typename TenT>
void extract_sub(context_handle_t<TenT>& ctx, TenT& inout, const List<Pair<elem_coor_t<TenT>, elem_coor_t<TenT>>>& r) {
  detail::extract_impl(ctx, inout, r, inout.handle());
}
template <typename TenT>
void extract_sub(context_handle_t<TenT>& ctx, const TenT& in, const List<Pair<elem_coor_t<TenT>, elem_coor_t<TenT>>>& r,
                 TenT& out) {
  detail::extract_impl(ctx, in, r, out.out_handle(ctx.get()));
}
template <typename TenT>
void replace_sub(context_handle_t<TenT>& ctx, TenT& inout, const TenT& sub, const elem_coors_t<TenT>& begin_pt) {
  detail::check(tci_replace_sub(ctx.get(), inout.handle(), sub.handle(), begin_pt.data(), inout.handle()),
                "tci_replace_sub");
}
template <typename TenT>
void replace_sub(context_handle_t<TenT>& ctx, const TenT& in, const TenT& sub, const elem_coors_t<TenT>& begin_pt,
                 TenT& out) {
  detail::check(tci_replace_sub(ctx.get(), in.handle(), sub.handle(), begin_pt.data(), out.out_handle(ctx.get())),
                "tci_replace_sub");
}
template <typename TenT>
TenT concatenate(context_handle_t<TenT>& ctx, const List<TenT>& ins, const bond_idx_t<TenT> concat_bdidx) {
  const auto h = detail::handles(ins);
  return detail::fresh<TenT>(ctx, [&](tci_tensor o) {
    detail::check(tci_concatenate(ctx.get(), (int)h.size(), h.data(), concat_bdidx, o), "tci_concatenate");
  });
}
template <typename TenT>
TenT stack(context_handle_t<TenT>& ctx, const List<TenT>& ins, const bond_idx_t<TenT> stack_bdidx) {
  const auto h = detail::handles(ins);
  return detail::fresh<TenT>(ctx, [&](tci_tensor o) {
    detail::check(tci_stack(ctx.get(), (int)h.size(), h.data(), stack_bdidx, o), "tci_stack");
  });
}
template <typename TenT>
void diag(context_handle_t<TenT>& ctx, TenT& inout) {
  detail::check(tci_diag(ctx.get(), inout.handle(), inout.handle()), "tci_diag");
}
template <typename TenT>
void diag(context_handle_t<TenT>& ctx, const TenT& in, TenT& out) {
  detail::check(tci_diag(ctx.get(), in.handle(), out.out_handle(ctx.get())), "tci_diag");
}

#if defined(__HIPCC__)
namespace detail {
constexpr int FOR_EACH_MAX_ORDER = 16;
struct Dims {
  long long d[FOR_EACH_MAX_ORDER];
};
template <typename Dev, typename F>
__global__ void for_each_kernel(Dev* p, long long n, F f) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    f(p[i]);
}
template <typename Dev, typename F>
__global__ void for_each_coors_kernel(Dev* p, long long n, int order, Dims dims, F f) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    long long c[FOR_EACH_MAX_ORDER];
    long long rem = i;
    for (int b = order - 1; b >= 0; --b) {
      c[b] = rem % dims.d[b];
      rem /= dims.d[b];
    }
    f(p[i], static_cast<const long long*>(c), order);
  }
}
// Device element type: HIP's own complex types share the layout of std::complex.
template <typename E>
struct dev_elem { using type = E; };
template <>
struct dev_elem<std::complex<float>> { using type = hipFloatComplex; };
template <>
struct dev_elem<std::complex<double>> { using type = hipDoubleComplex; };
template <typename TenT>
void* data_of(Context& ctx, const TenT& t) {
  void* p = nullptr;
  check(tci_data_ptr(ctx.get(), t.handle(), &p), "tci_data_ptr");
  return p;
}
inline void launch_check(const char* fn) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw error(TCI_ERR_DEVICE, std::string(fn) + ": " + hipGetErrorString(e));
}
inline unsigned grid_for(long long n) { return (unsigned)std::min<long long>(4096, (n + 255) / 256); }
}  // namespace detail

// Spec, manipulation: for_each.  f(elem&) is a __device__ functor applied to
// every element on the GPU, ordered on the context's stream.  Complex
// elements appear as hipFloatComplex / hipDoubleComplex.
template <typename TenT, typename Func>
void for_each(context_handle_t<TenT>& ctx, TenT& inout, Func&& f) {
  using Dev = typename detail::dev_elem<elem_t<TenT>>::type;
  const long long n = size(ctx, inout);
  if (n == 0) return;
  Dev* p = static_cast<Dev*>(detail::data_of(ctx, inout));
  hipLaunchKernelGGL((detail::for_each_kernel<Dev, std::decay_t<Func>>), dim3(detail::grid_for(n)), dim3(256), 0,
                     static_cast<hipStream_t>(ctx.stream()), p, n, f);
  detail::launch_check("tci::for_each");
}
// Spec, manipulation: for_each_with_coors.  f(elem&, const long long*
// coors, int order) on the GPU, coordinates row-major (at most 16 bonds),
// ordered on the context's stream.
template <typename TenT, typename Func>
void for_each_with_coors(context_handle_t<TenT>& ctx, TenT& inout, Func&& f) {
  using Dev = typename detail::dev_elem<elem_t<TenT>>::type;
  const auto shp = shape(ctx, inout);
  const long long n = size(ctx, inout);
  if (n == 0) return;
  if (shp.size() > (size_t)detail::FOR_EACH_MAX_ORDER)
    throw error(TCI_ERR_UNSUPPORTED, "tci::for_each_with_coors: more than 16 bonds");
  detail::Dims dims{};
  for (size_t b = 0; b < shp.size(); ++b) dims.d[b] = shp[b];
  Dev* p = static_cast<Dev*>(detail::data_of(ctx, inout));
  hipLaunchKernelGGL((detail::for_each_coors_kernel<Dev, std::decay_t<Func>>), dim3(detail::grid_for(n)), dim3(256),
                     0, static_cast<hipStream_t>(ctx.stream()), p, n, (int)shp.size(), dims, f);
  detail::launch_check("tci::for_each_with_coors");
}
#endif

// ---------------------------------------------------------------- linear algebra (Spec)
template <typename TenT>
real_t<TenT> norm(context_handle_t<TenT>& ctx, const TenT& a) {
  double r = 0.0;
  detail::check(tci_norm(ctx.get(), a.handle(), &r), "tci_norm");
  return static_cast<real_t<TenT>>(r);
}
template <typename TenT>
real_t<TenT> normalize(context_handle_t<TenT>& ctx, TenT& inout) {
  double r = 0.0;
  detail::check(tci_normalize(ctx.get(), inout.handle(), &r), "tci_normalize");
  return static_cast<real_t<TenT>>(r);
}
template <typename TenT>
real_t<TenT> normalize(context_handle_t<TenT>& ctx, const TenT& in, TenT& out) {
  out = copy(ctx, in);
  return normalize(ctx, out);
}
template <typename TenT>
void scale(context_handle_t<TenT>& ctx, TenT& inout, const elem_t<TenT> s) {
  detail::check(tci_scale(ctx.get(), inout.handle(), &s), "tci_scale");
}
template <typename TenT>
void scale(context_handle_t<TenT>& ctx, const TenT& in, const elem_t<TenT> s, TenT& out) {
  out = copy(ctx, in);
  scale(ctx, out, s);
}
template <typename TenT>
void trace(context_handle_t<TenT>& ctx, TenT& inout, const List<Pair<bond_idx_t<TenT>, bond_idx_t<TenT>>>& pairs) {
  std::vector<std::int32_t> p;
  for (const auto& q : pairs) p.push_back(q.first), p.push_back(q.second);
  detail::check(tci_trace(ctx.get(), inout.handle(), (int)pairs.size(), p.data(), inout.handle()), "tci_trace");
}
template <typename TenT>
void trace(context_handle_t<TenT>& ctx, const TenT& in, const List<Pair<bond_idx_t<TenT>, bond_idx_t<TenT>>>& pairs,
           TenT& out) {
  std::vector<std::int32_t> p;
  for (const auto& q : pairs) p.push_back(q.first), p.push_back(q.second);
  detail::check(tci_trace(ctx.get(), in.handle(), (int)pairs.size(), p.data(), out.out_handle(ctx.get())), "tci_trace");
}
template <typename TenT>
void exp(context_handle_t<TenT>& ctx, TenT& inout, const order_t<TenT> num_of_bds_as_row) {
  detail::check(tci_exp(ctx.get(), inout.handle(), num_of_bds_as_row, inout.handle()), "tci_exp");
}
template <typename TenT>
void exp(context_handle_t<TenT>& ctx, const TenT& in, const order_t<TenT> num_of_bds_as_row, TenT& out) {
  detail::check(tci_exp(ctx.get(), in.handle(), num_of_bds_as_row, out.out_handle(ctx.get())), "tci_exp");
}
template <typename TenT>
void inverse(context_handle_t<TenT>& ctx, TenT& inout, const order_t<TenT> num_of_bds_as_row) {
  detail::check(tci_inverse(ctx.get(), inout.handle(), num_of_bds_as_row, inout.handle()), "tci_inverse");
}
template <typename TenT>
void inverse(context_handle_t<TenT>& ctx, const TenT& in, const order_t<TenT> num_of_bds_as_row, TenT& out) {
  detail::check(tci_inverse(ctx.get(), in.handle(), num_of_bds_as_row, out.out_handle(ctx.get())), "tci_inverse");
}
template <typename TenT>
void contract(context_handle_t<TenT>& ctx, const TenT& a, const List<bond_label_t<TenT>>& bd_labs_a, const TenT& b,
              const List<bond_label_t<TenT>>& bd_labs_b, TenT& c, const List<bond_label_t<TenT>>& bd_labs_c) {
  tci_tensor ch = c.empty() ? c.out_handle(ctx.get()) : c.handle();
  detail::check(tci_contract(ctx.get(), a.handle(), bd_labs_a.data(), (int)bd_labs_a.size(), b.handle(),
                             bd_labs_b.data(), (int)bd_labs_b.size(), ch, bd_labs_c.data(), (int)bd_labs_c.size()),
                "tci_contract");
}
// String form: one character per label ("ijk").
template <typename TenT>
void contract(context_handle_t<TenT>& ctx, const TenT& a, const char* la, const TenT& b, const char* lb, TenT& c,
              const char* lc) {
  tci_tensor ch = c.empty() ? c.out_handle(ctx.get()) : c.handle();
  detail::check(tci_contract_str(ctx.get(), a.handle(), la, b.handle(), lb, ch, lc), "tci_contract_str");
}
template <typename TenT>
TenT linear_combine(context_handle_t<TenT>& ctx, const List<TenT>& ins) {
  const auto h = detail::handles(ins);
  return detail::fresh<TenT>(ctx, [&](tci_tensor o) {
    detail::check(tci_reshape(ctx.get(), h.at(0), order(ctx, ins[0]), shape(ctx, ins[0]).data(), o), "tci_reshape");
    detail::check(tci_linear_combine(ctx.get(), (int)h.size(), h.data(), nullptr, o), "tci_linear_combine");
  });
}
template <typename TenT>
TenT linear_combine(context_handle_t<TenT>& ctx, const List<TenT>& ins, const List<elem_t<TenT>>& coefs) {
  if (coefs.size() != ins.size()) throw error(TCI_ERR_INVALID_ARGUMENT, "tci::linear_combine: one coefficient per input");
  const auto h = detail::handles(ins);
  return detail::fresh<TenT>(ctx, [&](tci_tensor o) {
    detail::check(tci_reshape(ctx.get(), h.at(0), order(ctx, ins[0]), shape(ctx, ins[0]).data(), o), "tci_reshape");
    detail::check(tci_linear_combine(ctx.get(), (int)h.size(), h.data(), coefs.data(), o), "tci_linear_combine");
  });
}
template <typename TenT>
void svd(context_handle_t<TenT>& ctx, const TenT& a, const order_t<TenT> num_of_bds_as_row, TenT& u,
         real_ten_t<TenT>& s_diag, TenT& v_dag) {
  detail::check(tci_svd(ctx.get(), a.handle(), num_of_bds_as_row, u.out_handle(ctx.get()), s_diag.out_handle(ctx.get()),
                        v_dag.out_handle(ctx.get())),
                "tci_svd");
}
// Form (1): keep at most chi_max values, none below s_min.
template <typename TenT>
void trunc_svd(context_handle_t<TenT>& ctx, const TenT& a, const order_t<TenT> num_of_bds_as_row, TenT& u,
               real_ten_t<TenT>& s_diag, TenT& v_dag, real_t<TenT>& trunc_err, const bond_dim_t<TenT> chi_max,
               const real_t<TenT> s_min) {
  double e = 0.0;
  detail::check(tci_trunc_svd(ctx.get(), a.handle(), num_of_bds_as_row, u.out_handle(ctx.get()),
                              s_diag.out_handle(ctx.get()), v_dag.out_handle(ctx.get()), &e, 1, chi_max, 0.0, s_min),
                "tci_trunc_svd");
  trunc_err = static_cast<real_t<TenT>>(e);
}
// Form (2): at least chi_min, at most chi_max values, growing until the
// relative truncation error reaches target_trunc_err.
template <typename TenT>
void trunc_svd(context_handle_t<TenT>& ctx, const TenT& a, const order_t<TenT> num_of_bds_as_row, TenT& u,
               real_ten_t<TenT>& s_diag, TenT& v_dag, real_t<TenT>& trunc_err, const bond_dim_t<TenT> chi_min,
               const bond_dim_t<TenT> chi_max, const real_t<TenT> target_trunc_err, const real_t<TenT> s_min) {
  double e = 0.0;
  detail::check(tci_trunc_svd(ctx.get(), a.handle(), num_of_bds_as_row, u.out_handle(ctx.get()),
                              s_diag.out_handle(ctx.get()), v_dag.out_handle(ctx.get()), &e, chi_min, chi_max,
                              target_trunc_err, s_min),
                "tci_trunc_svd");
  trunc_err = static_cast<real_t<TenT>>(e);
}
template <typename TenT>
void qr(context_handle_t<TenT>& ctx, const TenT& a, const order_t<TenT> num_of_bds_as_row, TenT& q, TenT& r) {
  detail::check(tci_qr(ctx.get(), a.handle(), num_of_bds_as_row, q.out_handle(ctx.get()), r.out_handle(ctx.get())),
                "tci_qr");
}
template <typename TenT>
void lq(context_handle_t<TenT>& ctx, const TenT& a, const order_t<TenT> num_of_bds_as_row, TenT& l, TenT& q) {
  detail::check(tci_lq(ctx.get(), a.handle(), num_of_bds_as_row, l.out_handle(ctx.get()), q.out_handle(ctx.get())),
                "tci_lq");
}
// Hermitian eigensolve of the matricised tensor (rows = the first
// num_of_bds_as_row bonds): w ascending, v {d_0..d_{k-1}, n}.
template <typename TenT>
void eigh(context_handle_t<TenT>& ctx, const TenT& a, const order_t<TenT> num_of_bds_as_row, real_ten_t<TenT>& w,
          TenT& v) {
  detail::check(tci_eigh(ctx.get(), a.handle(), num_of_bds_as_row, w.out_handle(ctx.get()), v.out_handle(ctx.get())),
                "tci_eigh");
}
// Eigenvalues only, ascending.
template <typename TenT>
void eigvalsh(context_handle_t<TenT>& ctx, const TenT& a, const order_t<TenT> num_of_bds_as_row, real_ten_t<TenT>& w) {
  detail::check(tci_eigvalsh(ctx.get(), a.handle(), num_of_bds_as_row, w.out_handle(ctx.get())), "tci_eigvalsh");
}

// ---------------------------------------------------------------- miscellaneous (Spec)
// Element at row-major position e goes to first[coors2idx(coors of e)].
template <typename TenT, typename RandomIt, typename Func>
void to_range(context_handle_t<TenT>& ctx, const TenT& a, RandomIt first, Func&& coors2idx) {
  const auto shp = shape(ctx, a);
  const std::int64_t n = size(ctx, a);
  std::vector<elem_t<TenT>> host((std::size_t)n);
  if (n) detail::check(tci_to_host(ctx.get(), a.handle(), host.data(), host.size() * sizeof(elem_t<TenT>)), "tci_to_host");
  elem_coors_t<TenT> c(shp.size(), 0);
  for (std::int64_t e = 0; e < n; ++e) {
    first[coors2idx(c)] = host[(std::size_t)e];
    for (int b = (int)shp.size() - 1; b >= 0; --b) {
      if (++c[b] < shp[b]) break;
      c[b] = 0;
    }
  }
}
template <typename TenT>
void show(context_handle_t<TenT>& ctx, const TenT& a) {
  detail::check(tci_show(ctx.get(), a.handle()), "tci_show");
}
template <typename TenT>
bool close(context_handle_t<TenT>& ctx, const TenT& a, const TenT& b, const real_t<TenT> epsilon) {
  int r = 0;
  detail::check(tci_close(ctx.get(), a.handle(), b.handle(), (double)epsilon, &r), "tci_close");
  return r != 0;
}
// Element-type conversion between two tensors of this library (same or
// different contexts of one process).
template <typename Ten1T, typename Ten2T>
void convert(context_handle_t<Ten1T>& ctx1, const Ten1T& t1, context_handle_t<Ten2T>& ctx2, Ten2T& t2) {
  tci_tensor h = nullptr;
  detail::check(tci_convert(ctx1.get(), t1.handle(), detail::DT<Ten2T>, &h), "tci_convert");
  Ten2T tmp(ctx1.get(), h);
  const auto s = shape(ctx1, tmp);
  detail::check(tci_reshape(ctx2.get(), tmp.handle(), (int)s.size(), s.data(), t2.out_handle(ctx2.get())),
                "tci_reshape");
}

}  // namespace tci

#endif  // TCI_TCI_H
