"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point include/tci_c.h declares, and host-only calls behave."""
import ctypes
import os
import re

import pytest

from paper_2512_23917_amd import tci

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tci_c.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:tci_status|const char\*|void)\s+(tci_[a-z0-9_]+)\(", text, re.M)))


def test_header_declares_the_hot_path():
    names = declared_functions()
    for must in ["tci_contract", "tci_trunc_svd", "tci_qr", "tci_transpose", "tci_reshape", "tci_norm",
                 "tci_two_site_update_batched", "tci_heff_matvec", "tci_lanczos_ground", "tci_create_context"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(tci.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_the_header():
    L = tci.lib()
    for n in declared_functions():
        assert getattr(L, n).argtypes is not None or n in ("tci_version", "tci_last_error"), n


def test_version_and_error_string_without_gpu():
    assert tci.version() == "1.0"
    assert isinstance(tci.lib().tci_last_error(), bytes)


def test_update_params_defaults():
    p = tci.update_params()
    assert p.chi_min == 1 and p.chi_max == 2 ** 63 - 1 and p.direction == tci.DIR_RIGHT
    assert p.precision == tci.PREC_FP64 and p.svd_mode == tci.SVD_PLAIN and p.cert_tol == 1e-7


def test_null_arguments_are_rejected_on_the_host():
    L = tci.lib()
    assert L.tci_create_context(None, 0, None) == 1      # out NULL -> invalid argument
    assert L.tci_order(None, None, None) == 1
    assert b"null" in L.tci_last_error()


CPP_TYPES_AND_TEMPLATES = r'''
#include <tci/tci.h>
#include <complex>
using Z = tci::Tensor<std::complex<double>>;
static_assert(std::is_same<tci::real_ten_t<Z>, tci::Tensor<double>>::value, "real_ten_t");
static_assert(std::is_same<tci::cplx_ten_t<tci::Tensor<float>>, tci::Tensor<std::complex<float>>>::value, "cplx");
static_assert(std::is_same<tci::shape_t<Z>, tci::List<std::int64_t>>::value, "shape_t");
static_assert(std::is_same<tci::context_handle_t<Z>, tci::Context>::value, "context_handle_t");
void instantiate(tci::Context& ctx, Z& a, tci::Tensor<double>& s) {
  Z u, v, o;
  double err = 0;
  tci::svd(ctx, a, 2, u, s, v);
  tci::trunc_svd(ctx, a, 2, u, s, v, err, 1, 8, 1e-8, 0.0);
  tci::qr(ctx, a, 1, u, v);
  tci::lq(ctx, a, 1, u, v);
  tci::contract(ctx, a, {0, 1, 2}, a, {0, 1, 3}, o, {2, 3});
  tci::contract(ctx, a, "ijk", a, "ijl", o, "kl");
  tci::expand(ctx, a, {{0, 1}});
  tci::shrink(ctx, a, {{0, {0, 1}}});
  tci::extract_sub(ctx, a, {{0, 1}, {0, 1}, {0, 1}}, o);
  tci::trace(ctx, a, {{0, 1}}, o);
  tci::exp(ctx, a, 1);
  tci::inverse(ctx, a, 1, o);
  tci::diag(ctx, a, o);
  (void)tci::norm(ctx, a);
  (void)tci::normalize(ctx, a);
  (void)tci::to_cplx(ctx, s);
  (void)tci::real(ctx, a);
  (void)tci::concatenate(ctx, tci::List<Z>{}, 0);
  (void)tci::close(ctx, a, a, 1e-12);
}
'''


def test_cpp_header_compiles_on_the_host(tmp_path):
    """tci/tci.h builds with a plain host compiler (g++, C++17): the type
    system and the function templates instantiate without HIP."""
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    src = tmp_path / "hdr.cpp"
    src.write_text(CPP_TYPES_AND_TEMPLATES)
    r = subprocess.run([gxx, "-std=c++17", "-fsyntax-only", "-Wall", "-I", os.path.join(ROOT, "include"), str(src)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
