"""CPU FP64 oracle for the two-site MPS update (arXiv:2512.23917).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The GPU library never imports,
links or executes anything from this package, and this package never imports
the GPU library.

The compiled part (``tci_oracle.c``) holds the brute-force primitives: label
contraction, transpose, one-sided Jacobi SVD, Householder QR, Jacobi eigh, the
truncation rule and the Philox generator.  This module marshals numpy arrays
into it and exposes the tensor-level operations of the paper's API
("Spec" = the appendix that specifies TCI):

    permute / transpose   Sec. II.B transpose equation; Spec, manipulation
    contract              Sec. II.B contraction equations; Spec, contract
    svd / trunc_svd       Sec. II.B decomposition; Spec, svd and trunc_svd
    qr                    Spec, qr
    eigh                  Spec, eigh
    norm / normalize      Spec, norm (Frobenius-norm equation) and normalize

Algorithm-level oracles live in the sibling modules: ``mps`` (two-site
update, open-chain sweep), ``dmrg`` (effective Hamiltonian, Lanczos),
``rsvd`` (randomized truncated SVD), ``mlp`` (sketch-rank network), ``bf16``
(split-BF16x3 emulation), ``u1`` (U(1) block-sparse update), ``itebd``,
``subtensor``, ``eig`` (general eigendecomposition) and ``bp``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tci_oracle.c")
_LIB = os.path.join(_HERE, "_tci_oracle.so")

OK, INVALID, SHAPE, LABEL, NOT_CONVERGED = 0, 1, 2, 3, 7


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"oracle {what} failed with status {status}")
        self.status = status


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain -O2, IEEE semantics, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        lib = ctypes.CDLL(build())
        p = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        lib.orc_permute.argtypes = [p, ctypes.c_int, p, p, p]
        lib.orc_contract_check.argtypes = [ctypes.c_int, p, p, ctypes.c_int, p, p, ctypes.c_int, p, p]
        lib.orc_contract.argtypes = [p, ctypes.c_int, p, p, p, ctypes.c_int, p, p, p, ctypes.c_int, p]
        lib.orc_svd.argtypes = [p, i64, i64, p, p, p, p]
        lib.orc_trunc_rule.argtypes = [p, i64, i64, i64, f64, f64, p, p]
        lib.orc_qr.argtypes = [p, i64, i64, p, p]
        lib.orc_eigh.argtypes = [p, i64, p, p, p]
        lib.orc_philox4x32_10_raw.argtypes = [p, p, p]
        lib.orc_philox4x32_10_raw.restype = None
        lib.orc_philox4x32_10.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, i64, p]
        lib.orc_philox4x32_10.restype = None
        for f in (lib.orc_permute, lib.orc_contract_check, lib.orc_contract, lib.orc_svd,
                  lib.orc_trunc_rule, lib.orc_qr, lib.orc_eigh):
            f.restype = i32
        _lib_handle = lib
    return _lib_handle


def _c128(x) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.complex128)


def _ptr(x: np.ndarray):
    return x.ctypes.data_as(ctypes.c_void_p)


def _labels(lab) -> np.ndarray:
    if isinstance(lab, str):
        return np.array([ord(ch) for ch in lab], dtype=np.int32)
    return np.array(list(lab), dtype=np.int32).reshape(-1)


# --------------------------------------------------------------------------
# manipulation
# --------------------------------------------------------------------------
def permute(a, perm) -> np.ndarray:
    """Spec, manipulation, transpose: out.shape[b] = a.shape[perm[b]]."""
    a = _c128(a)
    perm = np.array(perm, dtype=np.int32)
    shape = np.array(a.shape, dtype=np.int64)
    if len(perm) != a.ndim:
        raise OracleError(INVALID, "permute")
    out = np.empty(tuple(a.shape[p] for p in perm) if a.ndim else (), dtype=np.complex128)
    st = _lib().orc_permute(_ptr(a), a.ndim, _ptr(shape), _ptr(perm), _ptr(out))
    if st:
        raise OracleError(st, "permute")
    return out


transpose = permute


def contract(a, la, b, lb, lc) -> np.ndarray:
    """Spec, linear algebra, contract: sum over labels shared by a and b and
    absent from c; c's labels give its bonds in order.  Brute-force loops."""
    a, b = _c128(a), _c128(b)
    la, lb, lc = _labels(la), _labels(lb), _labels(lc)
    if len(la) != a.ndim or len(lb) != b.ndim:
        raise OracleError(INVALID, "contract")
    sa = np.array(a.shape, dtype=np.int64)
    sb = np.array(b.shape, dtype=np.int64)
    sc = np.zeros(max(len(lc), 1), dtype=np.int64)
    lib = _lib()
    st = lib.orc_contract_check(a.ndim, _ptr(sa), _ptr(la), b.ndim, _ptr(sb), _ptr(lb),
                                len(lc), _ptr(lc), _ptr(sc))
    if st:
        raise OracleError(st, "contract")
    out = np.empty(tuple(int(x) for x in sc[: len(lc)]), dtype=np.complex128)
    st = lib.orc_contract(_ptr(a), a.ndim, _ptr(sa), _ptr(la), _ptr(b), b.ndim, _ptr(sb),
                          _ptr(lb), _ptr(out), len(lc), _ptr(lc))
    if st:
        raise OracleError(st, "contract")
    return out


def norm(a) -> float:
    """Spec, linear algebra, norm: Frobenius-norm equation (modulus squared)."""
    a = _c128(a).reshape(-1)
    return float(np.sqrt(np.sum(a.real * a.real + a.imag * a.imag)))


def normalize(a):
    """Spec, linear algebra, normalize: returns (a / ||a||_F, ||a||_F)."""
    n = norm(a)
    return _c128(a) / n, n


# --------------------------------------------------------------------------
# decompositions
# --------------------------------------------------------------------------
def _matricize(a, k_rows: int):
    a = _c128(a)
    if not (1 <= k_rows < a.ndim):
        raise OracleError(INVALID, "matricize (need 1 <= k < order)")
    rows = int(np.prod(a.shape[:k_rows]))
    cols = int(np.prod(a.shape[k_rows:]))
    return a.reshape(rows, cols), a.shape[:k_rows], a.shape[k_rows:]


def svd_matrix(m):
    """Thin SVD of a matrix by one-sided Jacobi; s non-increasing; fixed gauge."""
    m = _c128(m)
    rows, cols = m.shape
    k = min(rows, cols)
    u = np.empty((rows, k), dtype=np.complex128)
    s = np.empty(k, dtype=np.float64)
    vh = np.empty((k, cols), dtype=np.complex128)
    sweeps = ctypes.c_int(0)
    st = _lib().orc_svd(_ptr(m), rows, cols, _ptr(u), _ptr(s), _ptr(vh), ctypes.byref(sweeps))
    if st:
        raise OracleError(st, "svd")
    return u, s, vh


def svd(a, k_rows: int):
    """Spec, linear algebra, svd: u {d_0..d_{k-1}, kappa}, s {kappa}, vh {kappa, d_k..}."""
    m, rshape, cshape = _matricize(a, k_rows)
    u, s, vh = svd_matrix(m)
    k = len(s)
    return u.reshape(tuple(rshape) + (k,)), s, vh.reshape((k,) + tuple(cshape))


def trunc_rule(s, chi_min: int, chi_max: int, target: float, s_min: float):
    """Spec, linear algebra, trunc_svd, rules a-c; returns (chi, relative error)."""
    s = np.ascontiguousarray(s, dtype=np.float64)
    chi = ctypes.c_int64(0)
    err = ctypes.c_double(0.0)
    st = _lib().orc_trunc_rule(_ptr(s), len(s), int(chi_min), int(chi_max), float(target),
                               float(s_min), ctypes.byref(chi), ctypes.byref(err))
    if st:
        raise OracleError(st, "trunc_rule")
    return int(chi.value), float(err.value)


def trunc_svd(a, k_rows: int, chi_min: int, chi_max: int, target: float = 0.0,
              s_min: float = 0.0):
    """Spec, linear algebra, trunc_svd form (2); form (1) is chi_min=1, target=0.

    Returns u, s, vh cut to chi and the relative truncation error."""
    u, s, vh = svd(a, k_rows)
    chi, err = trunc_rule(s, chi_min, chi_max, target, s_min)
    return u[..., :chi], s[:chi].copy(), vh[:chi], err


def qr_matrix(m):
    m = _c128(m)
    rows, cols = m.shape
    rho = min(rows, cols)
    q = np.empty((rows, rho), dtype=np.complex128)
    r = np.empty((rho, cols), dtype=np.complex128)
    st = _lib().orc_qr(_ptr(m), rows, cols, _ptr(q), _ptr(r))
    if st:
        raise OracleError(st, "qr")
    return q, r


def qr(a, k_rows: int):
    """Spec, linear algebra, qr: q {d_0..d_{k-1}, rho}, r {rho, d_k..}; diag(r) >= 0."""
    m, rshape, cshape = _matricize(a, k_rows)
    q, r = qr_matrix(m)
    rho = q.shape[1]
    return q.reshape(tuple(rshape) + (rho,)), r.reshape((rho,) + tuple(cshape))


def eigh(h):
    """Spec, linear algebra, eigh of a Hermitian matrix: ascending w, columns of v."""
    h = _c128(h)
    n = h.shape[0]
    if h.shape != (n, n):
        raise OracleError(SHAPE, "eigh")
    w = np.empty(n, dtype=np.float64)
    v = np.empty((n, n), dtype=np.complex128)
    sweeps = ctypes.c_int(0)
    st = _lib().orc_eigh(_ptr(h), n, _ptr(w), _ptr(v), ctypes.byref(sweeps))
    if st:
        raise OracleError(st, "eigh")
    return w, v


# --------------------------------------------------------------------------
# counter-based generator (Philox4x32-10, Salmon et al. SC'11)
# --------------------------------------------------------------------------
def philox_raw(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, dtype=np.uint32)
    _lib().orc_philox4x32_10_raw(_ptr(c), _ptr(k), _ptr(out))
    return out


def philox_blocks(seed: int, stream: int, first_block: int, n_blocks: int) -> np.ndarray:
    out = np.empty(4 * n_blocks, dtype=np.uint32)
    _lib().orc_philox4x32_10(int(seed) & (2 ** 64 - 1), int(stream) & 0xFFFFFFFF,
                             int(first_block), int(n_blocks), _ptr(out))
    return out


def philox_normal(seed: int, stream: int, n: int) -> np.ndarray:
    """n standard normals: block b gives (x0, x1, x2, x3); each pair (x0, x1) and
    (x2, x3) becomes two normals by Box-Muller with u = (x + 0.5) * 2^-32."""
    n_blocks = (n + 3) // 4
    x = philox_blocks(seed, stream, 0, n_blocks).astype(np.float64).reshape(-1, 2)
    u1 = (x[:, 0] + 0.5) * 2.0 ** -32
    u2 = (x[:, 1] + 0.5) * 2.0 ** -32
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.empty((x.shape[0], 2))
    z[:, 0] = r * np.cos(2.0 * np.pi * u2)
    z[:, 1] = r * np.sin(2.0 * np.pi * u2)
    return z.reshape(-1)[:n]
