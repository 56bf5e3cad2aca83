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
                 "tci_two_site_update_batched", "tci_heff_matvec", "tci_lanczos_ground", "tci_create_context",
                 "tci_two_site_update", "tci_eigh", "tci_eigvalsh", "tci_context_opts_default"]:
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
    assert L.tci_create_context(None, 0, None, None) == 1      # out NULL -> invalid argument
    assert L.tci_order(None, None, None) == 1
    assert b"null" in L.tci_last_error()


def test_context_options_are_checked_on_the_host():
    """tci_context_opts: defaults, and invalid combinations rejected before
    any device is touched (so this runs without a GPU)."""
    L = tci.lib()
    o = tci.ContextOpts()
    L.tci_context_opts_default(ctypes.byref(o))
    assert o.precision == -1 and o.svd_mode == tci.SVD_PLAIN and o.verbosity == -1 and not o.autotune_cache
    h = ctypes.c_void_p()
    half = tci.ContextOpts()
    L.tci_context_opts_default(ctypes.byref(half))
    keep = tci.ALLOC_FN(lambda n, s, u: None)
    half.allocator.alloc = keep                    # alloc without free
    assert L.tci_create_context(ctypes.byref(h), 0, None, ctypes.byref(half)) == 1
    assert b"allocator" in L.tci_last_error()
    for field, bad in (("precision", 7), ("svd_mode", tci.SVD_LEARNED), ("verbosity", 3)):
        o2 = tci.ContextOpts()
        L.tci_context_opts_default(ctypes.byref(o2))
        setattr(o2, field, bad)
        assert L.tci_create_context(ctypes.byref(h), 0, None, ctypes.byref(o2)) == 1, field


def test_update_params_vidal_fields():
    p = tci.update_params(direction=tci.DIR_VIDAL)
    assert p.direction == 2 and not p.lambda_left and not p.lambda_right


def test_binding_structs_match_the_c_layout(tmp_path):
    """The ctypes structures of the binding have the sizes and field offsets
    a C compiler gives the header's structs."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no host C compiler")
    structs = {"tci_update_params": tci.UpdateParams, "tci_update_info": tci.UpdateInfo,
               "tci_context_opts": tci.ContextOpts, "tci_allocator": tci.Allocator}
    lines = ["#include <stdio.h>", "#include <stddef.h>", "#include <tci_c.h>", "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    r = subprocess.run([gcc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    for ln in filter(None, out):
        cname, what, val = ln.split()
        py = structs[cname]
        got = ctypes.sizeof(py) if what == "size" else getattr(py, what).offset
        assert got == int(val), (cname, what, got, val)


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
  tci::Tensor<double> w;
  tci::eigh(ctx, a, 1, w, u);
  tci::eigvalsh(ctx, a, 1, w);
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
