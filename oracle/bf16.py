"""Emulation of split-BF16x3 products: the expected-error reference of the
mixed-precision contractions.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The mixed-precision contractions store operands in FP32 and multiply them on
bf16 matrix cores.  Each FP32 value x is written as x ~ hi + lo with
    hi = RNE_bf16(x),  lo = RNE_bf16(x - hi)
(the difference x - hi is exact in FP32), and a product of two such values
keeps three of the four partial products:
    a b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi.
Here the partial products are formed exactly (a product of two 8-bit
significands fits a double) and every sum is an FP64 sum, so the only errors
left are the ones the split itself makes: the rounding of lo and the dropped
a_lo b_lo.  That is the error a kernel with exact accumulation would have;
the GPU's FP32 accumulation adds its own, much smaller, part on top.

RNE_bf16 follows the definition of rounding to the nearest value of the
bfloat16 format (8 significant bits, the exponent range of FP32, gradual
underflow with spacing 2^-133), ties to the value with an even last
significand bit; values whose rounding reaches 2^128 become infinite.
"""
from __future__ import annotations

import numpy as np

_MIN_EXP = -125        # frexp exponent of the smallest normal FP32 / bf16 value (2^-126 = 0.5 * 2^-125)
_SIG_BITS = 8          # significant bits of bfloat16 (1 implicit + 7 stored)


def round_bf16(x) -> np.ndarray:
    """Round FP32 values to the nearest bfloat16 value (ties to even).

    The spacing of bfloat16 values next to x is 2^(e - 8) for x = m 2^e with
    1/2 <= |m| < 1, and 2^-133 below the normal range; x / spacing is then
    rounded to the nearest integer, halves to even (numpy's rint).  Returns
    FP32 arrays holding the rounded values."""
    x = np.asarray(x, dtype=np.float32)
    xd = x.astype(np.float64)
    out = np.empty_like(xd)
    finite = np.isfinite(xd)
    _, e = np.frexp(np.where(finite, xd, 0.0))
    spacing = np.ldexp(1.0, np.maximum(e, _MIN_EXP) - _SIG_BITS)
    r = np.rint(np.where(finite, xd, 0.0) / spacing) * spacing
    out[finite] = r[finite]
    out[~finite] = xd[~finite]
    with np.errstate(over="ignore"):
        return out.astype(np.float32)      # 2^128 and beyond become +-inf


def split(x):
    """(hi, lo) of FP32 values: hi = RNE_bf16(x), lo = RNE_bf16(x - hi),
    the difference taken in FP32 (exact there)."""
    x = np.asarray(x, dtype=np.float32)
    hi = round_bf16(x)
    lo = round_bf16((x - hi).astype(np.float32))
    return hi, lo


def _real_x3(a, b) -> np.ndarray:
    """Real matrix product with three split partial products and FP64 sums."""
    ah, al = (p.astype(np.float64) for p in split(a))
    bh, bl = (p.astype(np.float64) for p in split(b))
    return ah @ bh + ah @ bl + al @ bh


def gemm_x3(a, b) -> np.ndarray:
    """C = A B with split-BF16x3 partial products and FP64 sums.

    A, B are rounded to FP32 (complex: complex64) first, the storage of the
    mixed paths.  Complex operands use the four real products
        Re C = Re A Re B - Im A Im B,   Im C = Re A Im B + Im A Re B,
    each one with three split partial products.  Returns float64 or
    complex128."""
    a = np.asarray(a)
    b = np.asarray(b)
    if np.iscomplexobj(a) or np.iscomplexobj(b):
        a = a.astype(np.complex64)
        b = b.astype(np.complex64)
        ar, ai = a.real.copy(), a.imag.copy()
        br, bi = b.real.copy(), b.imag.copy()
        re = _real_x3(ar, br) - _real_x3(ai, bi)
        im = _real_x3(ar, bi) + _real_x3(ai, br)
        return re + 1j * im
    return _real_x3(a.astype(np.float32), b.astype(np.float32))


def to_storage(x) -> np.ndarray:
    """Round to the mixed paths' storage type (FP32 / complex64), returned in
    FP64 / complex128."""
    x = np.asarray(x)
    if np.iscomplexobj(x):
        return x.astype(np.complex64).astype(np.complex128)
    return x.astype(np.float32).astype(np.float64)


def heff_x3_rows(left, w1, w2, right, x, rows):
    """Rows `rows` (values of the left index a) of the effective-Hamiltonian
    matvec y[a,s1,s2,b] = sum L[a,w,a'] W1[w,w',s1,s1'] W2[w',w'',s2,s2']
    R[b,w'',b'] x[a',s1',s2',b'] as the mixed path orders it:
        X1[(a,w),(s1',s2',b')] = L[(a,w),a'] x[a',(s1',s2',b')]        split-BF16x3
        X2[(a,s1,s2),(w'',b')] = sum W1 W2 X1 over w, w', s1', s2'     FP64, stored FP32
        y[(a,s1,s2),b]         = X2[(a,s1,s2),(w'',b')] R[b,(w'',b')]   split-BF16x3
    Operands are taken in their FP32 storage; X1 and X2 are rounded to it
    between the steps.  Returns y[rows] (complex128)."""
    left = to_storage(left)
    right = to_storage(right)
    x = to_storage(x)
    chi_l, wd, _ = left.shape
    d = w1.shape[2]
    chi_r = right.shape[0]
    rows = np.asarray(rows)
    lsub = left[rows].reshape(len(rows) * wd, chi_l)
    x1 = to_storage(gemm_x3(lsub, x.reshape(chi_l, d * d * chi_r)))
    x1 = x1.reshape(len(rows), wd, d, d, chi_r)
    w1 = np.asarray(w1, dtype=np.complex128)
    w2 = np.asarray(w2, dtype=np.complex128)
    # X2[a, s1, s2, w'', b'] = sum_{w, w', s1', s2'} W1[w,w',s1,s1'] W2[w',w'',s2,s2'] X1[a,w,s1',s2',b']
    x2 = np.zeros((len(rows), d, d, wd, chi_r), dtype=np.complex128)
    for w in range(wd):
        for wp in range(wd):
            for wpp in range(wd):
                for s1 in range(d):
                    for s1p in range(d):
                        for s2 in range(d):
                            for s2p in range(d):
                                c = w1[w, wp, s1, s1p] * w2[wp, wpp, s2, s2p]
                                if c != 0:
                                    x2[:, s1, s2, wpp, :] += c * x1[:, w, s1p, s2p, :]
    x2 = to_storage(x2).reshape(len(rows) * d * d, wd * chi_r)
    rmat = right.reshape(chi_r, wd * chi_r)
    y = gemm_x3(x2, rmat.T)
    return y.reshape(len(rows), d, d, chi_r)
