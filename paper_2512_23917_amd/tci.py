"""Thin Python binding of libtci_mi355x.so (the C ABI in include/tci_c.h).

Only argument marshalling lives here: every numeric step runs in the HIP
library.  PyTorch provides device memory and the stream: tensors are wrapped
(borrowed) views of contiguous torch tensors, outputs are allocated as torch
tensors of sufficient capacity and reshaped to the size the library reports.
The library must be built (``python -m paper_2512_23917_amd.build``); there is
no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtci_mi355x.so")

F32, F64, C64, C128 = 0, 1, 2, 3
PREC_FP64, PREC_FP32, PREC_BF16X3 = 0, 1, 2
SVD_PLAIN, SVD_RANDOMIZED, SVD_LEARNED = 0, 1, 2
DIR_LEFT, DIR_RIGHT, DIR_VIDAL = 0, 1, 2

STATUS = {0: "OK", 1: "INVALID_ARGUMENT", 2: "SHAPE", 3: "LABEL", 4: "DTYPE", 5: "OUT_OF_MEMORY",
          6: "DEVICE", 7: "NOT_CONVERGED", 8: "NUMERIC", 9: "UNSUPPORTED", 10: "INTERNAL"}

TORCH_OF = {F32: torch.float32, F64: torch.float64, C64: torch.complex64, C128: torch.complex128}
DTYPE_OF = {v: k for k, v in TORCH_OF.items()}
NUMPY_OF = {F32: np.float32, F64: np.float64, C64: np.complex64, C128: np.complex128}
ELEM_BYTES = {F32: 4, F64: 8, C64: 8, C128: 16}


class TciError(RuntimeError):
    def __init__(self, status: int, func: str, msg: str):
        super().__init__(f"{func}: {STATUS.get(status, status)}: {msg}")
        self.status = status


class UpdateParams(ctypes.Structure):
    _fields_ = [("chi_min", ctypes.c_int64), ("chi_max", ctypes.c_int64),
                ("target_trunc_err", ctypes.c_double), ("s_min", ctypes.c_double),
                ("direction", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("svd_mode", ctypes.c_int32), ("sketch_rank", ctypes.c_int32),
                ("power_iters", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("cert_tol", ctypes.c_double),
                ("sketch_model", ctypes.c_void_p), ("prev_spectra", ctypes.POINTER(ctypes.c_void_p)),
                ("lambda_left", ctypes.POINTER(ctypes.c_void_p)),
                ("lambda_right", ctypes.POINTER(ctypes.c_void_p))]


class UpdateInfo(ctypes.Structure):
    _fields_ = [("chi", ctypes.c_int64), ("trunc_err", ctypes.c_double),
                ("discarded_abs", ctypes.c_double), ("norm2", ctypes.c_double),
                ("used_fallback", ctypes.c_int32), ("sketch_rank", ctypes.c_int32),
                ("max_residual", ctypes.c_double)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]


class ContextOpts(ctypes.Structure):
    _fields_ = [("allocator", Allocator), ("precision", ctypes.c_int32), ("svd_mode", ctypes.c_int32),
                ("autotune_cache", ctypes.c_char_p), ("verbosity", ctypes.c_int32)]


_lib = None


def lib():
    """Load the HIP library; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2512_23917_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    p, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "tci_version": (ctypes.c_char_p, []),
        "tci_last_error": (ctypes.c_char_p, []),
        "tci_context_opts_default": (None, [P(ContextOpts)]),
        "tci_create_context": (i32, [P(p), ctypes.c_int, p, P(ContextOpts)]),
        "tci_destroy_context": (i32, [p]),
        "tci_set_stream": (i32, [p, p]),
        "tci_set_precision": (i32, [p, ctypes.c_int]),
        "tci_allocate": (i32, [p, ctypes.c_int, ctypes.c_int, P(i64), P(p)]),
        "tci_zeros": (i32, [p, ctypes.c_int, ctypes.c_int, P(i64), P(p)]),
        "tci_wrap": (i32, [p, ctypes.c_int, ctypes.c_int, P(i64), p, P(p)]),
        "tci_copy": (i32, [p, p, P(p)]),
        "tci_move": (i32, [p, P(p), P(p)]),
        "tci_destroy": (i32, [p, p]),
        "tci_order": (i32, [p, p, P(ctypes.c_int)]),
        "tci_shape": (i32, [p, p, P(i64), ctypes.c_int]),
        "tci_size": (i32, [p, p, P(i64)]),
        "tci_size_bytes": (i32, [p, p, P(i64)]),
        "tci_dtype_of": (i32, [p, p, P(ctypes.c_int)]),
        "tci_data_ptr": (i32, [p, p, P(p)]),
        "tci_get_elem": (i32, [p, p, P(i64), p]),
        "tci_set_elem": (i32, [p, p, P(i64), p]),
        "tci_set_labels": (i32, [p, p, P(i32), ctypes.c_int]),
        "tci_get_labels": (i32, [p, p, P(i32), ctypes.c_int]),
        "tci_from_host": (i32, [p, p, p, ctypes.c_size_t]),
        "tci_to_host": (i32, [p, p, p, ctypes.c_size_t]),
        "tci_convert": (i32, [p, p, ctypes.c_int, P(p)]),
        "tci_reshape": (i32, [p, p, ctypes.c_int, P(i64), p]),
        "tci_transpose": (i32, [p, p, P(i32), p]),
        "tci_cplx_conj": (i32, [p, p, p]),
        "tci_scale": (i32, [p, p, p]),
        "tci_linear_combine": (i32, [p, ctypes.c_int, P(p), p, p]),
        "tci_norm": (i32, [p, p, P(f64)]),
        "tci_normalize": (i32, [p, p, P(f64)]),
        "tci_contract": (i32, [p, p, P(i32), ctypes.c_int, p, P(i32), ctypes.c_int, p, P(i32), ctypes.c_int]),
        "tci_contract_str": (i32, [p, p, ctypes.c_char_p, p, ctypes.c_char_p, p, ctypes.c_char_p]),
        "tci_svd": (i32, [p, p, ctypes.c_int, p, p, p]),
        "tci_trunc_svd": (i32, [p, p, ctypes.c_int, p, p, p, P(f64), i64, i64, f64, f64]),
        "tci_qr": (i32, [p, p, ctypes.c_int, p, p]),
        "tci_eigh": (i32, [p, p, ctypes.c_int, p, p]),
        "tci_eigvalsh": (i32, [p, p, ctypes.c_int, p]),
        "tci_eig": (i32, [p, p, ctypes.c_int, p, p]),
        "tci_eigvals": (i32, [p, p, ctypes.c_int, p]),
        "tci_close": (i32, [p, p, p, f64, P(ctypes.c_int)]),
        "tci_fill": (i32, [p, ctypes.c_int, ctypes.c_int, P(i64), p, P(p)]),
        "tci_eye": (i32, [p, ctypes.c_int, i64, P(p)]),
        "tci_extract_sub": (i32, [p, p, P(i64), P(i64), p]),
        "tci_shrink": (i32, [p, p, ctypes.c_int, P(i32), P(i64), P(i64), p]),
        "tci_expand": (i32, [p, p, ctypes.c_int, P(i32), P(i64), p]),
        "tci_replace_sub": (i32, [p, p, p, P(i64), p]),
        "tci_concatenate": (i32, [p, ctypes.c_int, P(p), ctypes.c_int, p]),
        "tci_stack": (i32, [p, ctypes.c_int, P(p), ctypes.c_int, p]),
        "tci_trace": (i32, [p, p, ctypes.c_int, P(i32), p]),
        "tci_exp": (i32, [p, p, ctypes.c_int, p]),
        "tci_lq": (i32, [p, p, ctypes.c_int, p, p]),
        "tci_inverse": (i32, [p, p, ctypes.c_int, p]),
        "tci_to_cplx": (i32, [p, p, p]),
        "tci_diag": (i32, [p, p, p]),
        "tci_real": (i32, [p, p, p]),
        "tci_imag": (i32, [p, p, p]),
        "tci_save": (i32, [p, p, ctypes.c_char_p]),
        "tci_load": (i32, [p, ctypes.c_char_p, P(p)]),
        "tci_show": (i32, [p, p]),
        "tci_update_params_default": (None, [P(UpdateParams)]),
        "tci_two_site_update_batched": (i32, [p, ctypes.c_int, P(p), P(p), P(p), P(UpdateParams),
                                              P(p), P(p), P(p), P(UpdateInfo)]),
        "tci_two_site_update": (i32, [p, p, p, p, P(UpdateParams), p, p, p, P(UpdateInfo)]),
        "tci_split_batched": (i32, [p, ctypes.c_int, P(p), P(UpdateParams), P(p), P(p), P(p), P(UpdateInfo)]),
        "tci_heff_matvec": (i32, [p, p, p, p, p, p, p]),
        "tci_heff_matvec_noalloc": (i32, [p, p, p, p, p, p, p]),
        "tci_lanczos_ground": (i32, [p, p, p, p, p, p, ctypes.c_int, P(f64)]),
        "tci_sketch_model_create": (i32, [p, ctypes.c_uint64, P(p)]),
        "tci_sketch_model_destroy": (i32, [p, p]),
        "tci_sketch_model_nparams": (i64, []),
        "tci_sketch_model_get_params": (i32, [p, p, p, i64]),
        "tci_sketch_model_set_params": (i32, [p, p, p, i64]),
        "tci_sketch_model_save": (i32, [p, p, ctypes.c_char_p]),
        "tci_sketch_model_load": (i32, [p, ctypes.c_char_p, P(p)]),
        "tci_sketch_predict": (i32, [p, p, p, ctypes.c_int, p]),
        "tci_sketch_grads": (i32, [p, p, p, p, ctypes.c_int, p, P(ctypes.c_float)]),
        "tci_sketch_train_step": (i32, [p, p, p, p, ctypes.c_int, ctypes.c_float, P(ctypes.c_float)]),
        "tci_sketch_features": (i32, [p, p, i64, p, ctypes.c_int, ctypes.c_int, ctypes.c_int, f64, p]),
        "tci_philox_blocks": (i32, [p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, i64, p]),
        "tci_profile_enable": (i32, [p, ctypes.c_int]),
        "tci_profile_query": (i32, [p, ctypes.c_char_p, P(i64), P(f64), P(f64)]),
        "tci_profile_tags": (i32, [p, ctypes.c_char_p, ctypes.c_int]),
        "tci_bs_create": (i32, [p, ctypes.c_int, ctypes.c_int, P(i32), P(i64), ctypes.c_int, P(i32), P(i64), P(p)]),
        "tci_bs_destroy": (i32, [p, p]),
        "tci_bs_dims": (i32, [p, p, P(ctypes.c_int), P(ctypes.c_int), P(ctypes.c_int), P(i64)]),
        "tci_bs_bonds": (i32, [p, p, P(i32), P(i64), P(i32), P(i64)]),
        "tci_bs_block_info": (i32, [p, p, ctypes.c_int, P(ctypes.c_int), P(ctypes.c_int), P(ctypes.c_int), P(i64)]),
        "tci_bs_from_host": (i32, [p, p, p, ctypes.c_size_t]),
        "tci_bs_to_host": (i32, [p, p, p, ctypes.c_size_t]),
        "tci_bs_two_site_update_batched": (i32, [p, ctypes.c_int, P(p), P(p), P(p), P(UpdateParams), P(i64),
                                                 P(p), P(p), P(p), P(UpdateInfo)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(st: int, func: str):
    if st != 0:
        raise TciError(st, func, lib().tci_last_error().decode())


def _i64(seq):
    seq = [int(x) for x in seq]
    return (ctypes.c_int64 * max(1, len(seq)))(*seq)


def _i32(seq):
    seq = [int(x) for x in seq]
    return (ctypes.c_int32 * max(1, len(seq)))(*seq)


class Context:
    """tci_create_context on a torch device, ordered on its current stream.

    torch_allocator: the library's device memory (workspace chunks and any
    storage it allocates) comes from torch's caching allocator through the
    tci_allocator callbacks, so it shows up in torch's memory statistics and
    is shared with torch's pool.  precision / svd_mode / autotune_cache /
    verbosity are the other tci_context_opts fields (None: library default).
    """

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None, torch_allocator: bool = True,
                 precision: int | None = None, svd_mode: int | None = None, autotune_cache: str | None = None,
                 verbosity: int | None = None, allocator: tuple | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the HIP library needs an MI355X")
        self.device = device
        self.torch_device = torch.device("cuda", device)
        st = stream if stream is not None else torch.cuda.current_stream(self.torch_device)
        self.stream = st
        opts = ContextOpts()
        lib().tci_context_opts_default(ctypes.byref(opts))
        self._callbacks = None
        if allocator is not None:                 # (alloc(bytes, stream) -> int, free(ptr, bytes, stream))
            fa, ff = allocator
            self._callbacks = (ALLOC_FN(lambda n, s, u: fa(n, s) or None),
                               FREE_FN(lambda ptr, n, s, u: ff(ptr, n, s)))
        elif torch_allocator:
            dev = device

            def _alloc(n, s, u):
                try:
                    return torch.cuda.caching_allocator_alloc(int(n), dev, torch.cuda.ExternalStream(s, device=dev)
                                                              if s else torch.cuda.default_stream(dev))
                except Exception:          # out of memory: the library reports TCI_ERR_OUT_OF_MEMORY
                    return None

            def _free(ptr, n, s, u):
                torch.cuda.caching_allocator_delete(ptr)

            self._callbacks = (ALLOC_FN(_alloc), FREE_FN(_free))
        if self._callbacks is not None:
            opts.allocator.alloc, opts.allocator.free = self._callbacks
        if precision is not None:
            opts.precision = precision
        if svd_mode is not None:
            opts.svd_mode = svd_mode
        if autotune_cache is not None:
            opts.autotune_cache = autotune_cache.encode()
        if verbosity is not None:
            opts.verbosity = verbosity
        h = ctypes.c_void_p()
        _check(lib().tci_create_context(ctypes.byref(h), device, ctypes.c_void_p(st.cuda_stream),
                                        ctypes.byref(opts)), "tci_create_context")
        self.h = h

    def set_precision(self, prec: int):
        _check(lib().tci_set_precision(self.h, prec), "tci_set_precision")

    def close(self):
        if self.h:
            _check(lib().tci_destroy_context(self.h), "tci_destroy_context")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tensor:
    """A tci_tensor borrowing the memory of a contiguous torch tensor."""

    def __init__(self, ctx: Context, buf: torch.Tensor, shape=None):
        if not buf.is_contiguous():
            buf = buf.contiguous()
        self.ctx = ctx
        self.buf = buf
        self.dtype = DTYPE_OF[buf.dtype]
        shape = list(buf.shape) if shape is None else list(shape)
        h = ctypes.c_void_p()
        _check(lib().tci_wrap(ctx.h, self.dtype, len(shape), _i64(shape), ctypes.c_void_p(buf.data_ptr()),
                              ctypes.byref(h)), "tci_wrap")
        self.h = h

    @classmethod
    def from_torch(cls, ctx, t: torch.Tensor):
        return cls(ctx, t.to(ctx.torch_device).contiguous())

    @classmethod
    def from_numpy(cls, ctx, a: np.ndarray, dtype: int | None = None):
        t = torch.from_numpy(np.ascontiguousarray(a))
        if dtype is not None:
            t = t.to(TORCH_OF[dtype])
        return cls(ctx, t.to(ctx.torch_device))

    @classmethod
    def empty(cls, ctx, dtype: int, capacity: int):
        """Output handle with room for `capacity` elements (shape set by the library)."""
        buf = torch.empty(max(1, int(capacity)), dtype=TORCH_OF[dtype], device=ctx.torch_device)
        return cls(ctx, buf, shape=[buf.numel()])

    def shape(self):
        n = ctypes.c_int()
        _check(lib().tci_order(self.ctx.h, self.h, ctypes.byref(n)), "tci_order")
        out = (ctypes.c_int64 * max(1, n.value))()
        _check(lib().tci_shape(self.ctx.h, self.h, out, n.value), "tci_shape")
        return tuple(out[i] for i in range(n.value))

    def current_dtype(self):
        d = ctypes.c_int()
        _check(lib().tci_dtype_of(self.ctx.h, self.h, ctypes.byref(d)), "tci_dtype_of")
        return d.value

    def torch(self) -> torch.Tensor:
        """View of the data with the current shape (shares memory)."""
        shp = self.shape()
        n = int(np.prod(shp)) if shp else 1
        dt = TORCH_OF[self.current_dtype()]
        ptr = ctypes.c_void_p()
        _check(lib().tci_data_ptr(self.ctx.h, self.h, ctypes.byref(ptr)), "tci_data_ptr")
        if ptr.value == self.buf.data_ptr() and dt == self.buf.dtype and n <= self.buf.numel():
            return self.buf.view(-1)[:n].view(shp)
        raise RuntimeError("tensor storage is not the wrapped torch buffer")

    def numpy(self) -> np.ndarray:
        torch.cuda.synchronize(self.ctx.torch_device)
        return self.torch().cpu().numpy()

    def __del__(self):
        try:
            if self.h:
                lib().tci_destroy(self.ctx.h, self.h)
                self.h = None
        except Exception:
            pass


# ---------------------------------------------------------------- operations
def version() -> str:
    return lib().tci_version().decode()


def norm(ctx: Context, t: Tensor) -> float:
    out = ctypes.c_double()
    _check(lib().tci_norm(ctx.h, t.h, ctypes.byref(out)), "tci_norm")
    return out.value


def normalize(ctx: Context, t: Tensor) -> float:
    out = ctypes.c_double()
    _check(lib().tci_normalize(ctx.h, t.h, ctypes.byref(out)), "tci_normalize")
    return out.value


def transpose(ctx: Context, t: Tensor, perm, out: Tensor | None = None) -> Tensor:
    if out is None:
        out = Tensor.empty(ctx, t.dtype, int(np.prod(t.shape())))
    _check(lib().tci_transpose(ctx.h, t.h, _i32(perm), out.h), "tci_transpose")
    return out


def reshape(ctx: Context, t: Tensor, shape, out: Tensor | None = None) -> Tensor:
    out = t if out is None else out
    _check(lib().tci_reshape(ctx.h, t.h, len(shape), _i64(shape), out.h), "tci_reshape")
    return out


def _labels(lab):
    if isinstance(lab, str):
        return [ord(c) for c in lab]
    return [int(x) for x in lab]


def contract(ctx: Context, a: Tensor, la, b: Tensor, lb, lc, out: Tensor | None = None) -> Tensor:
    la, lb, lc = _labels(la), _labels(lb), _labels(lc)
    if out is None:
        dims = dict(zip(la, a.shape()))
        dims.update(zip(lb, b.shape()))
        cap = int(np.prod([dims.get(x, 1) for x in lc])) if lc else 1
        out = Tensor.empty(ctx, a.dtype, cap)
    _check(lib().tci_contract(ctx.h, a.h, _i32(la), len(la), b.h, _i32(lb), len(lb), out.h, _i32(lc), len(lc)),
           "tci_contract")
    return out


def trunc_svd(ctx: Context, a: Tensor, k_rows: int, chi_min: int, chi_max: int, target: float = 0.0,
              s_min: float = 0.0):
    shp = a.shape()
    rows = int(np.prod(shp[:k_rows]))
    cols = int(np.prod(shp[k_rows:]))
    kap = min(rows, cols, chi_max)
    u = Tensor.empty(ctx, a.dtype, rows * kap)
    vh = Tensor.empty(ctx, a.dtype, kap * cols)
    s = Tensor.empty(ctx, F64 if a.dtype in (F64, C128) else F32, kap)
    err = ctypes.c_double()
    _check(lib().tci_trunc_svd(ctx.h, a.h, k_rows, u.h, s.h, vh.h, ctypes.byref(err), chi_min, chi_max, target,
                               s_min), "tci_trunc_svd")
    return u, s, vh, err.value


def svd(ctx: Context, a: Tensor, k_rows: int):
    shp = a.shape()
    rows = int(np.prod(shp[:k_rows]))
    cols = int(np.prod(shp[k_rows:]))
    kap = min(rows, cols)
    u = Tensor.empty(ctx, a.dtype, rows * kap)
    vh = Tensor.empty(ctx, a.dtype, kap * cols)
    s = Tensor.empty(ctx, F64 if a.dtype in (F64, C128) else F32, kap)
    _check(lib().tci_svd(ctx.h, a.h, k_rows, u.h, s.h, vh.h), "tci_svd")
    return u, s, vh


def qr(ctx: Context, a: Tensor, k_rows: int):
    shp = a.shape()
    rows = int(np.prod(shp[:k_rows]))
    cols = int(np.prod(shp[k_rows:]))
    rho = min(rows, cols)
    q = Tensor.empty(ctx, a.dtype, rows * rho)
    r = Tensor.empty(ctx, a.dtype, rho * cols)
    _check(lib().tci_qr(ctx.h, a.h, k_rows, q.h, r.h), "tci_qr")
    return q, r


def _real_of(dt: int) -> int:
    return F64 if dt in (F64, C128) else F32


def eigh(ctx: Context, a: Tensor, k_rows: int = 1):
    shp = a.shape()
    n = int(np.prod(shp[:k_rows]))
    w = Tensor.empty(ctx, _real_of(a.dtype), n)
    v = Tensor.empty(ctx, a.dtype, n * n)
    _check(lib().tci_eigh(ctx.h, a.h, k_rows, w.h, v.h), "tci_eigh")
    return w, v


def eigvalsh(ctx: Context, a: Tensor, k_rows: int = 1):
    n = int(np.prod(a.shape()[:k_rows]))
    w = Tensor.empty(ctx, _real_of(a.dtype), n)
    _check(lib().tci_eigvalsh(ctx.h, a.h, k_rows, w.h), "tci_eigvalsh")
    return w


def _cplx_of(dt: int) -> int:
    return C128 if dt in (F64, C128) else C64


def eig(ctx: Context, a: Tensor, k_rows: int = 1):
    """tci_eig: (w, v), eigenvalues ascending by (real, imaginary) part."""
    n = int(np.prod(a.shape()[:k_rows]))
    w = Tensor.empty(ctx, _cplx_of(a.dtype), n)
    v = Tensor.empty(ctx, _cplx_of(a.dtype), n * n)
    _check(lib().tci_eig(ctx.h, a.h, k_rows, w.h, v.h), "tci_eig")
    return w, v


def eigvals(ctx: Context, a: Tensor, k_rows: int = 1):
    n = int(np.prod(a.shape()[:k_rows]))
    w = Tensor.empty(ctx, _cplx_of(a.dtype), n)
    _check(lib().tci_eigvals(ctx.h, a.h, k_rows, w.h), "tci_eigvals")
    return w


def close(ctx: Context, a: Tensor, b: Tensor, eps: float) -> bool:
    r = ctypes.c_int()
    _check(lib().tci_close(ctx.h, a.h, b.h, eps, ctypes.byref(r)), "tci_close")
    return bool(r.value)


def lq(ctx: Context, a: Tensor, k_rows: int):
    shp = a.shape()
    rows = int(np.prod(shp[:k_rows]))
    cols = int(np.prod(shp[k_rows:]))
    rho = min(rows, cols)
    l = Tensor.empty(ctx, a.dtype, rows * rho)
    q = Tensor.empty(ctx, a.dtype, rho * cols)
    _check(lib().tci_lq(ctx.h, a.h, k_rows, l.h, q.h), "tci_lq")
    return l, q


def exp(ctx: Context, a: Tensor, k_rows: int, out: Tensor | None = None) -> Tensor:
    if out is None:
        out = Tensor.empty(ctx, a.dtype, int(np.prod(a.shape())))
    _check(lib().tci_exp(ctx.h, a.h, k_rows, out.h), "tci_exp")
    return out


def _scalar_bytes(dtype: int, value) -> ctypes.Array:
    v = np.array([value], dtype=NUMPY_OF[dtype])
    return (ctypes.c_char * v.nbytes).from_buffer_copy(v.tobytes())


def _adopt(ctx: Context, h: ctypes.c_void_p, dtype: int, shape) -> Tensor:
    """Copy an owning library tensor into a torch-backed Tensor and free it."""
    n = max(1, int(np.prod(shape)))
    out = Tensor(ctx, torch.empty(n, dtype=TORCH_OF[dtype], device=ctx.torch_device), shape=[n])
    try:
        _check(lib().tci_reshape(ctx.h, h, len(shape), _i64(shape), out.h), "tci_reshape")
    finally:
        lib().tci_destroy(ctx.h, h)
    return out


def fill(ctx: Context, dtype: int, shape, value) -> Tensor:
    h = ctypes.c_void_p()
    _check(lib().tci_fill(ctx.h, dtype, len(shape), _i64(shape), _scalar_bytes(dtype, value), ctypes.byref(h)),
           "tci_fill")
    return _adopt(ctx, h, dtype, list(shape))


def eye(ctx: Context, dtype: int, n: int) -> Tensor:
    h = ctypes.c_void_p()
    _check(lib().tci_eye(ctx.h, dtype, n, ctypes.byref(h)), "tci_eye")
    return _adopt(ctx, h, dtype, [n, n])


def extract_sub(ctx: Context, a: Tensor, ranges, out: Tensor | None = None) -> Tensor:
    first = [int(f) for f, _ in ranges]
    last = [int(l) for _, l in ranges]
    if out is None:
        out = Tensor.empty(ctx, a.dtype, int(np.prod([max(0, l - f) for f, l in zip(first, last)])))
    _check(lib().tci_extract_sub(ctx.h, a.h, _i64(first), _i64(last), out.h), "tci_extract_sub")
    return out


def shrink(ctx: Context, a: Tensor, ranges: dict, out: Tensor | None = None) -> Tensor:
    bonds = list(ranges)
    if out is None:
        shp = list(a.shape())
        for b, (f, l) in ranges.items():
            if 0 <= b < len(shp):   # bad bonds are reported by the library
                shp[b] = max(0, l - f)
        out = Tensor.empty(ctx, a.dtype, int(np.prod(shp)))
    _check(lib().tci_shrink(ctx.h, a.h, len(bonds), _i32(bonds), _i64([ranges[b][0] for b in bonds]),
                            _i64([ranges[b][1] for b in bonds]), out.h), "tci_shrink")
    return out


def expand(ctx: Context, a: Tensor, increments: dict, out: Tensor | None = None) -> Tensor:
    bonds = list(increments)
    if out is None:
        shp = list(a.shape())
        for b, inc in increments.items():
            if 0 <= b < len(shp):   # bad bonds are reported by the library
                shp[b] += max(0, inc)
        out = Tensor.empty(ctx, a.dtype, int(np.prod(shp)))
    _check(lib().tci_expand(ctx.h, a.h, len(bonds), _i32(bonds), _i64([increments[b] for b in bonds]), out.h),
           "tci_expand")
    return out


def replace_sub(ctx: Context, a: Tensor, sub: Tensor, begin, out: Tensor | None = None) -> Tensor:
    if out is None:
        out = Tensor.empty(ctx, a.dtype, int(np.prod(a.shape())))
    _check(lib().tci_replace_sub(ctx.h, a.h, sub.h, _i64(begin), out.h), "tci_replace_sub")
    return out


def _handles(ins):
    return (ctypes.c_void_p * len(ins))(*[t.h.value for t in ins])


def concatenate(ctx: Context, ins: list, bond: int, out: Tensor | None = None) -> Tensor:
    if out is None:
        out = Tensor.empty(ctx, ins[0].dtype, sum(int(np.prod(t.shape())) for t in ins))
    _check(lib().tci_concatenate(ctx.h, len(ins), _handles(ins), bond, out.h), "tci_concatenate")
    return out


def stack(ctx: Context, ins: list, bond: int, out: Tensor | None = None) -> Tensor:
    if out is None:
        out = Tensor.empty(ctx, ins[0].dtype, sum(int(np.prod(t.shape())) for t in ins))
    _check(lib().tci_stack(ctx.h, len(ins), _handles(ins), bond, out.h), "tci_stack")
    return out


def trace(ctx: Context, a: Tensor, pairs, out: Tensor | None = None) -> Tensor:
    flat = [int(x) for p in pairs for x in p]
    if out is None:
        shp = a.shape()
        used = set(flat)
        out = Tensor.empty(ctx, a.dtype, int(np.prod([d for b, d in enumerate(shp) if b not in used])))
    _check(lib().tci_trace(ctx.h, a.h, len(pairs), _i32(flat), out.h), "tci_trace")
    return out


def _attach_prev(params: UpdateParams, prev):
    if prev is None:
        return None
    arr = (ctypes.c_void_p * len(prev))(*[x.h.value for x in prev])
    params.prev_spectra = ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
    return arr


def _attach_lambdas(params: UpdateParams, lam_left, lam_right):
    """Vidal weights (lists of F64 Tensors); the returned arrays must stay alive."""
    if lam_left is None and lam_right is None:
        return None
    al = (ctypes.c_void_p * len(lam_left))(*[x.h.value for x in lam_left])
    ar = (ctypes.c_void_p * len(lam_right))(*[x.h.value for x in lam_right])
    params.lambda_left = ctypes.cast(al, ctypes.POINTER(ctypes.c_void_p))
    params.lambda_right = ctypes.cast(ar, ctypes.POINTER(ctypes.c_void_p))
    return al, ar


def _detach(params: UpdateParams, keep_prev, keep_lam):
    """Clear pointers that _attach_prev / _attach_lambdas set (their arrays die with the call)."""
    if keep_prev is not None:
        params.prev_spectra = None
    if keep_lam is not None:
        params.lambda_left = None
        params.lambda_right = None


def update_params(**kw) -> UpdateParams:
    p = UpdateParams()
    lib().tci_update_params_default(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def two_site_update_batched(ctx: Context, A: list, B: list, gates: list | None, params: UpdateParams,
                            prev_spectra: list | None = None, lambda_left: list | None = None,
                            lambda_right: list | None = None):
    """Returns (A_out, s_out, B_out, infos) lists; outputs are library-sized views.
    prev_spectra (learned sketch): per update the bond's spectrum before the update.
    lambda_left / lambda_right (DIR_VIDAL): per update the outer bond weights."""
    n = len(A)
    keep = _attach_prev(params, prev_spectra)
    keep_l = _attach_lambdas(params, lambda_left, lambda_right)
    P = ctypes.c_void_p * n
    chil, d, chim = A[0].shape()
    chir = B[0].shape()[2]
    kap = min(chil * d, d * chir, params.chi_max)
    dt = A[0].dtype
    A_out = [Tensor.empty(ctx, dt, chil * d * kap) for _ in range(n)]
    B_out = [Tensor.empty(ctx, dt, kap * d * chir) for _ in range(n)]
    s_out = [Tensor.empty(ctx, F64, kap) for _ in range(n)]
    infos = (UpdateInfo * n)()
    g = P(*[x.h.value if x is not None else None for x in gates]) if gates is not None else None
    try:
        _check(lib().tci_two_site_update_batched(ctx.h, n, P(*[x.h.value for x in A]), P(*[x.h.value for x in B]),
                                                 g, ctypes.byref(params), P(*[x.h.value for x in A_out]),
                                                 P(*[x.h.value for x in s_out]), P(*[x.h.value for x in B_out]),
                                                 infos), "tci_two_site_update_batched")
    finally:
        _detach(params, keep, keep_l)
    return A_out, s_out, B_out, list(infos)


def two_site_update(ctx: Context, A: Tensor, B: Tensor, gate: Tensor | None, params: UpdateParams | None = None):
    """tci_two_site_update: one update; returns (A_out, s_out, B_out, info)."""
    chil, d, _ = A.shape()
    chir = B.shape()[2]
    kap = min(chil * d, d * chir, params.chi_max if params is not None else chil * d)
    dt = A.dtype
    A_out = Tensor.empty(ctx, dt, chil * d * kap)
    B_out = Tensor.empty(ctx, dt, kap * d * chir)
    s_out = Tensor.empty(ctx, F64, kap)
    info = UpdateInfo()
    _check(lib().tci_two_site_update(ctx.h, A.h, B.h, gate.h if gate is not None else None,
                                     ctypes.byref(params) if params is not None else None, A_out.h, s_out.h,
                                     B_out.h, ctypes.byref(info)), "tci_two_site_update")
    return A_out, s_out, B_out, info


def split_batched(ctx: Context, thetas: list, params: UpdateParams, prev_spectra: list | None = None,
                  lambda_left: list | None = None, lambda_right: list | None = None):
    """trunc_svd + renormalisation + write-back of given (chi_l, d, d, chi_r) tensors."""
    n = len(thetas)
    keep = _attach_prev(params, prev_spectra)
    keep_l = _attach_lambdas(params, lambda_left, lambda_right)
    P = ctypes.c_void_p * n
    chil, d, _, chir = thetas[0].shape()
    kap = min(chil * d, d * chir, params.chi_max)
    dt = thetas[0].dtype
    A_out = [Tensor.empty(ctx, dt, chil * d * kap) for _ in range(n)]
    B_out = [Tensor.empty(ctx, dt, kap * d * chir) for _ in range(n)]
    s_out = [Tensor.empty(ctx, F64, kap) for _ in range(n)]
    infos = (UpdateInfo * n)()
    try:
        _check(lib().tci_split_batched(ctx.h, n, P(*[x.h.value for x in thetas]), ctypes.byref(params),
                                       P(*[x.h.value for x in A_out]), P(*[x.h.value for x in s_out]),
                                       P(*[x.h.value for x in B_out]), infos), "tci_split_batched")
    finally:
        _detach(params, keep, keep_l)
    return A_out, s_out, B_out, list(infos)


def heff_matvec(ctx: Context, L: Tensor, W1: Tensor, W2: Tensor, R: Tensor, x: Tensor,
                y: Tensor | None = None) -> Tensor:
    if y is None:
        y = Tensor.empty(ctx, x.dtype, int(np.prod(x.shape())))
    _check(lib().tci_heff_matvec(ctx.h, L.h, W1.h, W2.h, R.h, x.h, y.h), "tci_heff_matvec")
    return y


def heff_matvec_noalloc(ctx: Context, L: Tensor, W1: Tensor, W2: Tensor, R: Tensor, x: Tensor, y: Tensor) -> Tensor:
    """tci_heff_matvec_noalloc: y must already hold x's number of elements."""
    _check(lib().tci_heff_matvec_noalloc(ctx.h, L.h, W1.h, W2.h, R.h, x.h, y.h), "tci_heff_matvec_noalloc")
    return y


def lanczos_ground(ctx: Context, L: Tensor, W1: Tensor, W2: Tensor, R: Tensor, theta: Tensor,
                   n_matvec: int = 20) -> float:
    e = ctypes.c_double()
    _check(lib().tci_lanczos_ground(ctx.h, L.h, W1.h, W2.h, R.h, theta.h, n_matvec, ctypes.byref(e)),
           "tci_lanczos_ground")
    return e.value


def profile_enable(ctx: Context, on: bool = True):
    _check(lib().tci_profile_enable(ctx.h, 1 if on else 0), "tci_profile_enable")


def profile_tags(ctx: Context) -> list:
    buf = ctypes.create_string_buffer(8192)
    _check(lib().tci_profile_tags(ctx.h, buf, 8192), "tci_profile_tags")
    return [x for x in buf.value.decode().split("\n") if x]


def profile_query(ctx: Context, tag: str):
    """(launch count, total ms, total algorithmic work) for one tag."""
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    w = ctypes.c_double()
    _check(lib().tci_profile_query(ctx.h, tag.encode(), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(w)),
           "tci_profile_query")
    return n.value, ms.value, w.value


# ---------------------------------------------------------------- sketch-rank model
class SketchModel:
    """tci_sketch_model: the learned predictor of log2 chi* (FP32, on the GPU)."""

    def __init__(self, ctx: Context, seed: int = 0, path: str | None = None):
        self.ctx = ctx
        h = ctypes.c_void_p()
        if path is None:
            _check(lib().tci_sketch_model_create(ctx.h, seed, ctypes.byref(h)), "tci_sketch_model_create")
        else:
            _check(lib().tci_sketch_model_load(ctx.h, path.encode(), ctypes.byref(h)), "tci_sketch_model_load")
        self.h = h

    @staticmethod
    def nparams() -> int:
        return int(lib().tci_sketch_model_nparams())

    def params(self) -> np.ndarray:
        out = np.empty(self.nparams(), dtype=np.float32)
        _check(lib().tci_sketch_model_get_params(self.ctx.h, self.h, out.ctypes.data_as(ctypes.c_void_p), out.size),
               "tci_sketch_model_get_params")
        return out

    def set_params(self, p: np.ndarray):
        p = np.ascontiguousarray(p, dtype=np.float32)
        _check(lib().tci_sketch_model_set_params(self.ctx.h, self.h, p.ctypes.data_as(ctypes.c_void_p), p.size),
               "tci_sketch_model_set_params")

    def save(self, path: str):
        _check(lib().tci_sketch_model_save(self.ctx.h, self.h, path.encode()), "tci_sketch_model_save")

    def predict(self, X: torch.Tensor) -> torch.Tensor:
        X = X.to(self.ctx.torch_device, torch.float32).contiguous()
        y = torch.empty(X.shape[0], dtype=torch.float32, device=self.ctx.torch_device)
        _check(lib().tci_sketch_predict(self.ctx.h, self.h, ctypes.c_void_p(X.data_ptr()), X.shape[0],
                                        ctypes.c_void_p(y.data_ptr())), "tci_sketch_predict")
        torch.cuda.synchronize(self.ctx.torch_device)
        return y

    def grads(self, X: torch.Tensor, T: torch.Tensor):
        X = X.to(self.ctx.torch_device, torch.float32).contiguous()
        T = T.to(self.ctx.torch_device, torch.float32).contiguous()
        g = torch.empty(self.nparams(), dtype=torch.float32, device=self.ctx.torch_device)
        loss = ctypes.c_float()
        _check(lib().tci_sketch_grads(self.ctx.h, self.h, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(T.data_ptr()),
                                      X.shape[0], ctypes.c_void_p(g.data_ptr()), ctypes.byref(loss)), "tci_sketch_grads")
        return loss.value, g

    def train_step(self, X: torch.Tensor, T: torch.Tensor, lr: float = 1e-3) -> float:
        loss = ctypes.c_float()
        _check(lib().tci_sketch_train_step(self.ctx.h, self.h, ctypes.c_void_p(X.data_ptr()),
                                           ctypes.c_void_p(T.data_ptr()), X.shape[0], lr, ctypes.byref(loss)),
               "tci_sketch_train_step")
        return loss.value

    def close(self):
        if self.h:
            lib().tci_sketch_model_destroy(self.ctx.h, self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sketch_features(ctx: Context, spectra: list, chi_max: int, d: int, eps: float) -> torch.Tensor:
    """Feature rows (n x 35, FP32, device) of a list of descending spectra (numpy)."""
    n = len(spectra)
    L = max(1, max(len(s) for s in spectra))
    S = np.zeros((n, L))
    for i, s in enumerate(spectra):
        S[i, :len(s)] = s
    Sd = torch.from_numpy(S).to(ctx.torch_device)
    ln = torch.tensor([len(s) for s in spectra], dtype=torch.int32, device=ctx.torch_device)
    X = torch.empty((n, 35), dtype=torch.float32, device=ctx.torch_device)
    _check(lib().tci_sketch_features(ctx.h, ctypes.c_void_p(Sd.data_ptr()), L, ctypes.c_void_p(ln.data_ptr()), n,
                                     chi_max, d, eps, ctypes.c_void_p(X.data_ptr())), "tci_sketch_features")
    torch.cuda.synchronize(ctx.torch_device)
    return X


def philox_blocks(ctx: Context, seed: int, stream: int, first: int, n: int) -> np.ndarray:
    out = torch.empty(4 * n, dtype=torch.int32, device=ctx.torch_device)
    _check(lib().tci_philox_blocks(ctx.h, seed, stream, first, n, ctypes.c_void_p(out.data_ptr())), "tci_philox_blocks")
    torch.cuda.synchronize(ctx.torch_device)
    return out.cpu().numpy().view(np.uint32)


class BsTensor:
    """tci_bs_tensor: a U(1) block-sparse site tensor (F32).  Bonds are lists
    of (charge, dim); blocks are {(a, s, b): (D_l[a], D_r[b]) array}."""

    def __init__(self, ctx: Context, left=(), right=()):
        self.ctx = ctx
        h = ctypes.c_void_p()
        ql = (ctypes.c_int32 * max(1, len(left)))(*[q for q, _ in left])
        dl = (ctypes.c_int64 * max(1, len(left)))(*[d for _, d in left])
        qr = (ctypes.c_int32 * max(1, len(right)))(*[q for q, _ in right])
        dr = (ctypes.c_int64 * max(1, len(right)))(*[d for _, d in right])
        _check(lib().tci_bs_create(ctx.h, F32, len(left), ql, dl, len(right), qr, dr, ctypes.byref(h)),
               "tci_bs_create")
        self.h = h

    @classmethod
    def from_blocks(cls, ctx: Context, left, right, blocks: dict) -> "BsTensor":
        t = cls(ctx, left, right)
        buf = np.zeros(t.nelem(), dtype=np.float32)
        for (a, s, b), off in t.layout().items():
            blk = blocks.get((a, s, b))
            if blk is not None:
                buf[off:off + blk.size] = np.asarray(blk, dtype=np.float32).reshape(-1)
        _check(lib().tci_bs_from_host(ctx.h, t.h, buf.ctypes.data_as(ctypes.c_void_p), buf.nbytes),
               "tci_bs_from_host")
        return t

    def dims(self):
        nl, nr, nbk = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        ne = ctypes.c_int64()
        _check(lib().tci_bs_dims(self.ctx.h, self.h, ctypes.byref(nl), ctypes.byref(nr), ctypes.byref(nbk),
                                 ctypes.byref(ne)), "tci_bs_dims")
        return nl.value, nr.value, nbk.value, ne.value

    def nelem(self) -> int:
        return self.dims()[3]

    def bonds(self):
        nl, nr, _, _ = self.dims()
        ql, dl = (ctypes.c_int32 * max(1, nl))(), (ctypes.c_int64 * max(1, nl))()
        qr, dr = (ctypes.c_int32 * max(1, nr))(), (ctypes.c_int64 * max(1, nr))()
        _check(lib().tci_bs_bonds(self.ctx.h, self.h, ql, dl, qr, dr), "tci_bs_bonds")
        return [(ql[i], dl[i]) for i in range(nl)], [(qr[i], dr[i]) for i in range(nr)]

    def layout(self) -> dict:
        _, _, nbk, _ = self.dims()
        out = {}
        a, s, b = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        off = ctypes.c_int64()
        for i in range(nbk):
            _check(lib().tci_bs_block_info(self.ctx.h, self.h, i, ctypes.byref(a), ctypes.byref(s), ctypes.byref(b),
                                           ctypes.byref(off)), "tci_bs_block_info")
            out[(a.value, s.value, b.value)] = off.value
        return out

    def blocks(self) -> dict:
        left, right = self.bonds()
        buf = np.empty(self.nelem(), dtype=np.float32)
        if buf.size:
            _check(lib().tci_bs_to_host(self.ctx.h, self.h, buf.ctypes.data_as(ctypes.c_void_p), buf.nbytes),
                   "tci_bs_to_host")
        out = {}
        for (a, s, b), off in self.layout().items():
            r, c = left[a][1], right[b][1]
            out[(a, s, b)] = buf[off:off + r * c].reshape(r, c).copy()
        return out

    def close(self):
        if self.h:
            lib().tci_bs_destroy(self.ctx.h, self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bs_two_site_update_batched(ctx: Context, A: list, B: list, gates: list | None, params: UpdateParams,
                               chi_max_each: list | None = None):
    """Returns (A_out, s_out, B_out, infos); A_out / B_out are new BsTensor handles.
    chi_max_each: optional per-update caps (replacing params.chi_max)."""
    n = len(A)
    caps = (ctypes.c_int64 * n)(*chi_max_each) if chi_max_each is not None else None
    P = ctypes.c_void_p * n
    A_out = [BsTensor(ctx) for _ in range(n)]
    B_out = [BsTensor(ctx) for _ in range(n)]
    s_out = [Tensor.empty(ctx, F64, 2 * sum(d for _, d in A[i].bonds()[0]) + 1) for i in range(n)]
    infos = (UpdateInfo * n)()
    g = P(*[x.h.value if x is not None else None for x in gates]) if gates is not None else None
    _check(lib().tci_bs_two_site_update_batched(ctx.h, n, P(*[x.h.value for x in A]), P(*[x.h.value for x in B]), g,
                                                ctypes.byref(params), caps, P(*[x.h.value for x in A_out]),
                                                P(*[x.h.value for x in s_out]), P(*[x.h.value for x in B_out]),
                                                infos), "tci_bs_two_site_update_batched")
    return A_out, s_out, B_out, list(infos)


def inverse(ctx: Context, a: Tensor, k_rows: int, out: Tensor | None = None) -> Tensor:
    if out is None:
        out = Tensor.empty(ctx, a.dtype, int(np.prod(a.shape())))
    _check(lib().tci_inverse(ctx.h, a.h, k_rows, out.h), "tci_inverse")
    return out


COMPLEX_OF = {F32: C64, F64: C128, C64: C64, C128: C128}
REAL_OF = {F32: F32, F64: F64, C64: F32, C128: F64}


def to_cplx(ctx: Context, a: Tensor) -> Tensor:
    out = Tensor.empty(ctx, COMPLEX_OF[a.dtype], int(np.prod(a.shape())))
    _check(lib().tci_to_cplx(ctx.h, a.h, out.h), "tci_to_cplx")
    return out


def real(ctx: Context, a: Tensor) -> Tensor:
    out = Tensor.empty(ctx, REAL_OF[a.dtype], int(np.prod(a.shape())))
    _check(lib().tci_real(ctx.h, a.h, out.h), "tci_real")
    return out


def imag(ctx: Context, a: Tensor) -> Tensor:
    out = Tensor.empty(ctx, REAL_OF[a.dtype], int(np.prod(a.shape())))
    _check(lib().tci_imag(ctx.h, a.h, out.h), "tci_imag")
    return out


def save(ctx: Context, a: Tensor, path: str):
    _check(lib().tci_save(ctx.h, a.h, os.fsencode(path)), "tci_save")


def load(ctx: Context, path: str) -> Tensor:
    h = ctypes.c_void_p()
    _check(lib().tci_load(ctx.h, os.fsencode(path), ctypes.byref(h)), "tci_load")
    order = ctypes.c_int()
    dt = ctypes.c_int()
    _check(lib().tci_order(ctx.h, h, ctypes.byref(order)), "tci_order")
    shp = (ctypes.c_int64 * max(1, order.value))()
    _check(lib().tci_shape(ctx.h, h, shp, order.value), "tci_shape")
    _check(lib().tci_dtype_of(ctx.h, h, ctypes.byref(dt)), "tci_dtype_of")
    return _adopt(ctx, h, dt.value, [shp[i] for i in range(order.value)])


def show(ctx: Context, a: Tensor):
    _check(lib().tci_show(ctx.h, a.h), "tci_show")


def diag(ctx: Context, a: Tensor, out: Tensor | None = None) -> Tensor:
    if out is None:
        shp = a.shape()
        cap = shp[0] * shp[0] if len(shp) == 1 else (min(shp) if len(shp) == 2 else 1)
        out = Tensor.empty(ctx, a.dtype, cap)
    _check(lib().tci_diag(ctx.h, a.h, out.h), "tci_diag")
    return out


def cplx_conj(ctx: Context, a: Tensor, out: Tensor | None = None) -> Tensor:
    if out is None:
        out = Tensor.empty(ctx, a.dtype, int(np.prod(a.shape())))
    _check(lib().tci_cplx_conj(ctx.h, a.h, out.h), "tci_cplx_conj")
    return out


def scale(ctx: Context, a: Tensor, s) -> Tensor:
    """In place: a *= s (one scalar of a's dtype)."""
    _check(lib().tci_scale(ctx.h, a.h, _scalar_bytes(a.dtype, s)), "tci_scale")
    return a
