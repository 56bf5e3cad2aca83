"""CPU FP64 oracle for the sub-tensor, construction and matrix-function
operations of the TCI API (arXiv:2512.23917, the appendix that specifies TCI,
"Spec" below).

TEST INFRASTRUCTURE ONLY: the test-suite is the only caller; the GPU library
never imports this module and this module never imports the GPU library.

Every function writes out the definition the Spec entry gives, on numpy
arrays, in the bond order of the input (row-major, bond 0 slowest):

    fill, eye                 Spec, construction: fill, eye
    expand, shrink            Spec, manipulation: expand, shrink
    extract_sub, replace_sub  Spec, manipulation: extract_sub, replace_sub
    concatenate, stack        Spec, manipulation: concatenate, stack
    trace                     Spec, linear algebra: trace (partial trace)
    expm                      Spec, linear algebra: exp (matricised exponential)
    inverse                   Spec, linear algebra: inverse (matricised)
    lq                        Spec, linear algebra: lq
    to_cplx, real, imag       Spec, manipulation: to_cplx, real, imag
"""
from __future__ import annotations

import itertools

import numpy as np

from . import qr_matrix


def fill(shape, value, dtype=np.complex128) -> np.ndarray:
    """Spec, fill: every element equals the value."""
    out = np.empty(tuple(int(d) for d in shape), dtype=dtype)
    out[...] = value
    return out


def eye(n: int, dtype=np.complex128) -> np.ndarray:
    """Spec, eye: ones on the main diagonal of an n x n tensor, zeros elsewhere."""
    out = np.zeros((n, n), dtype=dtype)
    for i in range(n):
        out[i, i] = 1
    return out


def expand(a, increments: dict) -> np.ndarray:
    """Spec, expand: bond b grows by increments[b]; elements inside the old
    bounds are kept, every element with a coordinate in an appended range is
    zero."""
    a = np.asarray(a)
    shape = list(a.shape)
    for b, inc in increments.items():
        if inc < 0:
            raise ValueError("negative increment")
        shape[b] += int(inc)
    out = np.zeros(shape, dtype=a.dtype)
    out[tuple(slice(0, d) for d in a.shape)] = a
    return out


def extract_sub(a, ranges) -> np.ndarray:
    """Spec, extract_sub: per-bond half-open ranges [first, last), given for
    every bond in bond order."""
    a = np.asarray(a)
    if len(ranges) != a.ndim:
        raise ValueError("one range per bond")
    for (f, l), d in zip(ranges, a.shape):
        if not (0 <= f <= l <= d):
            raise ValueError("range outside the bond")
    return a[tuple(slice(int(f), int(l)) for f, l in ranges)].copy()


def shrink(a, ranges: dict) -> np.ndarray:
    """Spec, shrink: the listed bonds are cut to [first, last); the others keep
    their full range."""
    a = np.asarray(a)
    full = [(0, d) for d in a.shape]
    for b, (f, l) in ranges.items():
        full[b] = (f, l)
    return extract_sub(a, full)


def replace_sub(a, sub, begin) -> np.ndarray:
    """Spec, replace_sub: the origin of sub lands at the coordinate begin."""
    out = np.array(a, copy=True)
    sub = np.asarray(sub)
    if sub.ndim != out.ndim:
        raise ValueError("order differs")
    for b0, ds, d in zip(begin, sub.shape, out.shape):
        if b0 < 0 or b0 + ds > d:
            raise ValueError("sub does not fit")
    out[tuple(slice(int(b0), int(b0) + ds) for b0, ds in zip(begin, sub.shape))] = sub
    return out


def concatenate(ins, bond: int) -> np.ndarray:
    """Spec, concatenate: the inputs follow one another along `bond`; all other
    dimensions must agree."""
    ins = [np.asarray(x) for x in ins]
    ref = ins[0].shape
    for x in ins:
        if x.ndim != len(ref) or any(x.shape[b] != ref[b] for b in range(len(ref)) if b != bond):
            raise ValueError("inputs differ off the concatenated bond")
    shape = list(ref)
    shape[bond] = sum(x.shape[bond] for x in ins)
    out = np.zeros(shape, dtype=ins[0].dtype)
    off = 0
    for x in ins:
        idx = [slice(None)] * len(shape)
        idx[bond] = slice(off, off + x.shape[bond])
        out[tuple(idx)] = x
        off += x.shape[bond]
    return out


def stack(ins, bond: int) -> np.ndarray:
    """Spec, stack: a new bond of dimension len(ins) inserted at position
    `bond`; out[..., k, ...] = ins[k]."""
    ins = [np.asarray(x) for x in ins]
    ref = ins[0].shape
    for x in ins:
        if x.shape != ref:
            raise ValueError("inputs differ in shape")
    shape = list(ref)
    shape.insert(bond, len(ins))
    out = np.zeros(shape, dtype=ins[0].dtype)
    for k, x in enumerate(ins):
        idx = [slice(None)] * len(shape)
        idx[bond] = k
        out[tuple(idx)] = x
    return out


def trace(a, pairs) -> np.ndarray:
    """Spec, trace: sum over equal coordinates of each bond pair; the
    remaining bonds keep their order (a scalar when every bond is paired)."""
    a = np.asarray(a)
    used = set()
    for x, y in pairs:
        if x == y or x in used or y in used or a.shape[x] != a.shape[y]:
            raise ValueError("bad bond pair")
        used.update((x, y))
    keep = [b for b in range(a.ndim) if b not in used]
    out = np.zeros([a.shape[b] for b in keep], dtype=a.dtype)
    for t in itertools.product(*[range(a.shape[x]) for x, _ in pairs]):
        idx = [slice(None)] * a.ndim
        for (x, y), v in zip(pairs, t):
            idx[x] = v
            idx[y] = v
        out = out + a[tuple(idx)]
    return out


def expm_matrix(m) -> np.ndarray:
    """exp(M) = (exp(M / 2^s))^(2^s), the inner exponential summed as the
    power series sum_k X^k / k! until a term no longer changes the sum
    (X = M / 2^s with ||X||_F <= 1)."""
    m = np.asarray(m, dtype=np.complex128)
    n = m.shape[0]
    nrm = np.linalg.norm(m)
    s = 0
    while nrm / 2.0 ** s > 1.0:
        s += 1
    x = m / 2.0 ** s
    total = np.eye(n, dtype=np.complex128)
    term = np.eye(n, dtype=np.complex128)
    for k in range(1, 200):
        term = term @ x / k
        total = total + term
        if np.linalg.norm(term) <= 1e-18 * np.linalg.norm(total):
            break
    for _ in range(s):
        total = total @ total
    return total


def expm(a, k_rows: int) -> np.ndarray:
    """Spec, exp: matricise (first k_rows bonds as rows), exponentiate, fold
    back to the input shape; rows and columns must have equal size."""
    a = np.asarray(a)
    rows = int(np.prod(a.shape[:k_rows]))
    cols = int(np.prod(a.shape[k_rows:]))
    if rows != cols:
        raise ValueError("exp needs a square matricisation")
    return expm_matrix(a.reshape(rows, cols)).reshape(a.shape)


def lq_matrix(m):
    """A = L Q from the QR of A^H: A^H = Q' R' gives L = R'^H, Q = Q'^H
    (L lower triangular with a real non-negative diagonal, Q orthonormal rows)."""
    m = np.asarray(m, dtype=np.complex128)
    q1, r1 = qr_matrix(m.conj().T)
    return r1.conj().T, q1.conj().T


def lq(a, k_rows: int):
    """Spec, lq: l {d_0..d_{k-1}, rho}, q {rho, d_k..}, rho = min(I, J)."""
    a = np.asarray(a)
    rshape, cshape = a.shape[:k_rows], a.shape[k_rows:]
    rows, cols = int(np.prod(rshape)), int(np.prod(cshape))
    l, q = lq_matrix(a.reshape(rows, cols))
    rho = l.shape[1]
    return l.reshape(tuple(rshape) + (rho,)), q.reshape((rho,) + tuple(cshape))


def inverse(a, k_rows: int) -> np.ndarray:
    """Spec, inverse: matricise (first k_rows bonds as rows), take the X with
    A X = I (LAPACK's solve as the step), fold back to the input shape."""
    a = np.asarray(a)
    rows = int(np.prod(a.shape[:k_rows]))
    cols = int(np.prod(a.shape[k_rows:]))
    if rows != cols:
        raise ValueError("inverse needs a square matricisation")
    m = a.reshape(rows, cols).astype(np.complex128)
    return np.linalg.solve(m, np.eye(rows, dtype=np.complex128)).reshape(a.shape)


def to_cplx(a) -> np.ndarray:
    """Spec, to_cplx: real elements embedded with zero imaginary part."""
    a = np.asarray(a)
    out = np.zeros(a.shape, dtype=np.complex64 if a.dtype in (np.float32, np.complex64) else np.complex128)
    out.real = a.real
    if np.iscomplexobj(a):
        out.imag = a.imag
    return out


def real(a) -> np.ndarray:
    """Spec, real: elementwise real part (a copy for real input)."""
    a = np.asarray(a)
    return a.real.copy()


def imag(a) -> np.ndarray:
    """Spec, imag: elementwise imaginary part (zeros for real input)."""
    a = np.asarray(a)
    return a.imag.copy() if np.iscomplexobj(a) else np.zeros_like(a)


def diag(a) -> np.ndarray:
    """Spec, diag: a vector becomes the diagonal matrix; a matrix gives its
    main diagonal of length min(d0, d1)."""
    a = np.asarray(a)
    if a.ndim == 1:
        out = np.zeros((a.shape[0], a.shape[0]), dtype=a.dtype)
        for i in range(a.shape[0]):
            out[i, i] = a[i]
        return out
    if a.ndim == 2:
        return np.array([a[i, i] for i in range(min(a.shape))], dtype=a.dtype)
    raise ValueError("diag needs a first- or second-order tensor")
