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
