// Exercise of the C++17 header tci/tci.h on the GPU: every function is
// called at least once and each check prints "CHECK <name> <residual>"
// (the Python test asserts the residuals); a thrown tci::error prints
// "FAIL <message>" and exits with status 1.
#include <tci/tci.h>

#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <utility>
#include <vector>

using Z = std::complex<double>;
using ZTen = tci::Tensor<Z>;
using DTen = tci::Tensor<double>;

namespace {

void report(const char* name, double r) { std::printf("CHECK %s %.3e\n", name, r); }

std::vector<Z> host(tci::Context& ctx, const ZTen& t) {
  std::vector<Z> v((size_t)tci::size(ctx, t));
  tci::to_range(ctx, t, v.begin(), [&](const tci::elem_coors_t<ZTen>& c) {
    const auto s = tci::shape(ctx, t);
    long long i = 0;
    for (size_t b = 0; b < c.size(); ++b) i = i * s[b] + c[b];
    return i;
  });
  return v;
}

// A List of move-only tensors (an initializer list would copy).
template <typename... T>
tci::List<ZTen> list_of(T&&... ts) {
  tci::List<ZTen> l;
  (l.push_back(std::move(ts)), ...);
  return l;
}

double maxdiff(const std::vector<Z>& a, const std::vector<Z>& b) {
  if (a.size() != b.size()) return 1e300;
  double m = 0;
  for (size_t i = 0; i < a.size(); ++i) m = std::max(m, std::abs(a[i] - b[i]));
  return m;
}

}  // namespace

int main(int argc, char** argv) {
  const std::string dir = argc > 1 ? argv[1] : ".";
  try {
    tci::Context ctx(0);
    std::printf("version %s\n", tci::version().c_str());
    std::mt19937_64 eng(7);
    std::normal_distribution<double> nd;
    auto gen = [&]() { return Z(nd(eng), nd(eng)); };

    // queries, construction, element access
    auto a = tci::random<ZTen>(ctx, {6, 2, 5}, gen);
    report("order", std::abs(tci::order(ctx, a) - 3));
    report("size_bytes", std::abs((double)tci::size_bytes(ctx, a) - 6 * 2 * 5 * 16));
    auto z = tci::zeros<ZTen>(ctx, {3, 4, 2});
    tci::set_elem(ctx, z, {2, 1, 0}, Z(1.5, -2));
    report("set_get_elem", std::abs(tci::get_elem(ctx, z, {2, 1, 0}) - Z(1.5, -2)));
    std::vector<Z> els{1, 2, 3, 4, 5, 6};
    auto r = tci::assign_from_range<ZTen>(ctx, {2, 3}, els.begin(),
                                          [](const tci::elem_coors_t<ZTen>& c) { return 3 * c[0] + c[1]; });
    report("assign_from_range", std::abs(tci::get_elem(ctx, r, {1, 1}) - Z(5)));
    auto f = tci::fill<ZTen>(ctx, {3, 2, 4}, Z(2));
    report("fill", std::abs(tci::get_elem(ctx, f, {0, 1, 3}) - Z(2)));
    auto e = tci::eye<ZTen>(ctx, 3);
    report("eye", std::abs(tci::get_elem(ctx, e, {1, 1}) - Z(1)) + std::abs(tci::get_elem(ctx, e, {1, 2})));
    auto c = tci::copy(ctx, a);
    report("copy", maxdiff(host(ctx, c), host(ctx, a)));
    auto m = tci::move(ctx, c);
    report("move", (c.empty() ? 0.0 : 1.0) + maxdiff(host(ctx, m), host(ctx, a)));
    tci::clear(ctx, m);
    report("clear", m.empty() ? 0.0 : 1.0);

    // I/O
    const std::string path = dir + "/hdr_check.ten";
    tci::save(ctx, a, path);
    auto l = tci::load<ZTen>(ctx, path);
    report("save_load", maxdiff(host(ctx, l), host(ctx, a)));

    // manipulation
    ZTen t;
    tci::transpose(ctx, a, {2, 0, 1}, t);
    report("transpose", std::abs(tci::get_elem(ctx, t, {4, 3, 1}) - tci::get_elem(ctx, a, {3, 1, 4})));
    ZTen rs;
    tci::reshape(ctx, a, {12, 5}, rs);
    report("reshape", std::abs(tci::get_elem(ctx, rs, {7, 2}) - tci::get_elem(ctx, a, {3, 1, 2})));
    ZTen cj;
    tci::cplx_conj(ctx, a, cj);
    report("cplx_conj", std::abs(tci::get_elem(ctx, cj, {1, 1, 1}) - std::conj(tci::get_elem(ctx, a, {1, 1, 1}))));
    auto re = tci::real(ctx, a);
    auto im = tci::imag(ctx, a);
    report("real_imag", std::abs(Z(tci::get_elem(ctx, re, {2, 0, 3}), tci::get_elem(ctx, im, {2, 0, 3})) -
                                 tci::get_elem(ctx, a, {2, 0, 3})));
    auto dreal = tci::real(ctx, a);
    auto zc = tci::to_cplx(ctx, dreal);
    report("to_cplx", std::abs(tci::get_elem(ctx, zc, {2, 0, 3}) - Z(tci::get_elem(ctx, dreal, {2, 0, 3}), 0)));
    ZTen ex;
    tci::expand(ctx, a, {{1, 2}, {0, 1}}, ex);
    auto exs = tci::shape(ctx, ex);
    report("expand", std::abs(exs[0] - 7) + std::abs(exs[1] - 4) + std::abs(tci::get_elem(ctx, ex, {6, 3, 0})) +
                         std::abs(tci::get_elem(ctx, ex, {5, 1, 4}) - tci::get_elem(ctx, a, {5, 1, 4})));
    ZTen sh;
    tci::shrink(ctx, a, {{0, {1, 4}}, {2, {2, 5}}}, sh);
    report("shrink", std::abs(tci::get_elem(ctx, sh, {0, 1, 0}) - tci::get_elem(ctx, a, {1, 1, 2})));
    ZTen sub;
    tci::extract_sub(ctx, a, {{2, 4}, {0, 2}, {1, 3}}, sub);
    report("extract_sub", std::abs(tci::get_elem(ctx, sub, {1, 1, 1}) - tci::get_elem(ctx, a, {3, 1, 2})));
    auto zz = tci::zeros<ZTen>(ctx, {6, 2, 5});
    tci::replace_sub(ctx, zz, sub, {3, 0, 2});
    report("replace_sub", std::abs(tci::get_elem(ctx, zz, {4, 1, 3}) - tci::get_elem(ctx, sub, {1, 1, 1})));
    tci::List<ZTen> parts;
    parts.push_back(tci::copy(ctx, a));
    parts.push_back(tci::copy(ctx, zz));
    auto cat = tci::concatenate(ctx, parts, 1);
    auto st = tci::stack(ctx, parts, 0);
    report("concatenate", std::abs(tci::shape(ctx, cat)[1] - 4) +
                              std::abs(tci::get_elem(ctx, cat, {4, 3, 3}) - tci::get_elem(ctx, zz, {4, 1, 3})));
    report("stack", std::abs(tci::get_elem(ctx, st, {1, 4, 1, 3}) - tci::get_elem(ctx, zz, {4, 1, 3})));
    auto dg = tci::eye<ZTen>(ctx, 4);
    tci::diag(ctx, dg);
    tci::diag(ctx, dg);
    report("diag", std::abs(tci::order(ctx, dg) - 2) + std::abs(tci::get_elem(ctx, dg, {3, 3}) - Z(1)));

    // device functors (the header compiled by hipcc)
    auto g = tci::copy(ctx, a);
    tci::for_each(ctx, g, [] __device__(hipDoubleComplex & x) {
      x.x *= 2.0;
      x.y *= 2.0;
    });
    if (hipDeviceSynchronize() != hipSuccess) throw tci::error(TCI_ERR_DEVICE, "synchronise after for_each");
    report("for_each", std::abs(tci::get_elem(ctx, g, {1, 0, 2}) - 2.0 * tci::get_elem(ctx, a, {1, 0, 2})));
    auto h = tci::zeros<ZTen>(ctx, {3, 4});
    tci::for_each_with_coors(ctx, h, [] __device__(hipDoubleComplex & x, const long long* cc, int) {
      x.x = (double)(10 * cc[0] + cc[1]);
      x.y = 0.0;
    });
    report("for_each_with_coors", std::abs(tci::get_elem(ctx, h, {2, 3}) - Z(23)));

    // linear algebra
    const double na = tci::norm(ctx, a);
    double ssq = 0;
    for (const auto& x : host(ctx, a)) ssq += std::norm(x);
    report("norm", std::abs(na - std::sqrt(ssq)) / na);
    auto nn = tci::copy(ctx, a);
    const double old = tci::normalize(ctx, nn);
    report("normalize", std::abs(old - na) / na + std::abs(tci::norm(ctx, nn) - 1.0));
    auto sc = tci::copy(ctx, a);
    tci::scale(ctx, sc, Z(0, 2));
    report("scale", std::abs(tci::get_elem(ctx, sc, {0, 1, 0}) - Z(0, 2) * tci::get_elem(ctx, a, {0, 1, 0})));
    auto tr = tci::random<ZTen>(ctx, {3, 4, 2, 4, 2}, gen);
    ZTen trout;
    tci::trace(ctx, tr, {{1, 3}, {2, 4}}, trout);
    Z want = 0;
    for (int j = 0; j < 4; ++j)
      for (int k = 0; k < 2; ++k) want += tci::get_elem(ctx, tr, {1, j, k, j, k});
    report("trace", std::abs(tci::get_elem(ctx, trout, {1}) - want));
    auto ee = tci::eye<ZTen>(ctx, 3);
    tci::exp(ctx, ee, 1);
    report("exp", std::abs(tci::get_elem(ctx, ee, {1, 1}) - std::exp(1.0)));
    auto sq = tci::random<ZTen>(ctx, {2, 3, 6}, gen);
    ZTen inv, prod;
    tci::inverse(ctx, sq, 2, inv);
    // the inverse keeps the input's shape: its rows are the 6 column indices of sq
    tci::reshape(ctx, inv, {6, 6});
    tci::contract(ctx, sq, {0, 1, 9}, inv, {9, 2}, prod, {0, 1, 2});
    report("inverse", std::abs(tci::get_elem(ctx, prod, {1, 2, 5}) - Z(1)) + std::abs(tci::get_elem(ctx, prod, {1, 2, 1})));
    ZTen u, vd, us;
    DTen s;
    tci::svd(ctx, a, 2, u, s, vd);
    tci::List<Z> sv;
    auto sz = tci::to_cplx(ctx, s);
    tci::diag(ctx, sz);
    tci::contract(ctx, u, "abk", sz, "kl", us, "abl");
    ZTen rec;
    tci::contract(ctx, us, "abl", vd, "lc", rec, "abc");
    report("svd", maxdiff(host(ctx, rec), host(ctx, a)) / na);
    ZTen tu, tv;
    DTen ts;
    double err = 0;
    tci::trunc_svd(ctx, a, 2, tu, ts, tv, err, 1, 3, 0.0, 0.0);
    report("trunc_svd", std::abs(tci::shape(ctx, ts)[0] - 3) + (err > 0 && err < 1 ? 0.0 : 1.0));
    ZTen q, rr, qr;
    tci::qr(ctx, a, 2, q, rr);
    tci::contract(ctx, q, "abk", rr, "kc", qr, "abc");
    report("qr", maxdiff(host(ctx, qr), host(ctx, a)) / na);
    ZTen ll, lqq, lq;
    auto w = tci::random<ZTen>(ctx, {3, 10}, gen);
    tci::lq(ctx, w, 1, ll, lqq);
    tci::contract(ctx, ll, "ak", lqq, "kc", lq, "ac");
    report("lq", maxdiff(host(ctx, lq), host(ctx, w)) / tci::norm(ctx, w));
    auto hm = tci::random<ZTen>(ctx, {8, 8}, gen);
    ZTen hc, herm;
    tci::transpose(ctx, hm, {1, 0}, hc);
    tci::cplx_conj(ctx, hc);
    herm = tci::linear_combine(ctx, list_of(tci::copy(ctx, hm), tci::copy(ctx, hc)));
    DTen ew, ew2;
    ZTen ev;
    tci::eigh(ctx, herm, 1, ew, ev);
    tci::eigvalsh(ctx, herm, 1, ew2);
    double tr_h = 0, tr_w = 0;
    for (int i = 0; i < 8; ++i) tr_h += tci::get_elem(ctx, herm, {i, i}).real(), tr_w += tci::get_elem(ctx, ew, {i});
    report("eigh", std::abs(tr_h - tr_w) + std::abs(tci::get_elem(ctx, ew2, {7}) - tci::get_elem(ctx, ew, {7})));
    auto lc = tci::linear_combine(ctx, list_of(tci::copy(ctx, a), tci::copy(ctx, a)), tci::List<Z>{Z(2), Z(-1)});
    report("linear_combine", maxdiff(host(ctx, lc), host(ctx, a)));

    // miscellaneous
    report("close", tci::close(ctx, a, l, 1e-15) ? 0.0 : 1.0);
    tci::Tensor<std::complex<float>> af;
    tci::convert(ctx, a, ctx, af);
    const Z x111 = tci::get_elem(ctx, a, {1, 1, 1});
    report("convert", std::abs(Z(tci::get_elem(ctx, af, {1, 1, 1})) - x111) <= 1e-6 * std::abs(x111) ? 0.0 : 1.0);
    auto small = tci::eye<DTen>(ctx, 2);
    tci::show(ctx, small);
    std::printf("DONE\n");
  } catch (const tci::error& ex) {
    std::printf("FAIL %s\n", ex.what());
    return 1;
  }
  return 0;
}
