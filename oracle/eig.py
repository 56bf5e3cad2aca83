"""CPU FP64 oracle for the general (non-Hermitian) eigendecomposition of the
TCI API (arXiv:2512.23917, the appendix that specifies TCI, "Spec" below:
eigvals and eig).

TEST INFRASTRUCTURE ONLY: the test-suite is the only caller; the GPU library
never imports this module and this module never imports the GPU library.

Spec, eig: the tensor is matricised with the first k bonds as rows (the
matrix must be square); the right eigendecomposition A'V = V Lambda gives the
eigenvalues w (a complex first-order tensor) and the eigenvectors, folded
back so that the last bond indexes them.  Spec, eigvals returns w alone.

The textbook route, in complex128 throughout:
  1. Householder reduction to upper Hessenberg form, A = Q H Q^H;
  2. single-shift QR iteration with Wilkinson shifts and deflation of
     negligible subdiagonal entries (|h_{i+1,i}| <= u (|h_ii| + |h_{i+1,i+1}|)),
     accumulating the rotations: H = Z T Z^H with T upper triangular (the
     complex Schur form);
  3. eigenvectors of T by back substitution, x_k = 1 and
     (T_{0:k,0:k} - t_kk I) x_{0:k} = -T_{0:k,k}, with a denominator that
     would vanish replaced by u ||T||_F (a repeated eigenvalue);
  4. V = Q Z X, each column scaled to unit 2-norm.
The paper fixes neither the order of the eigenvalues nor the scaling of the
eigenvectors.  Reading taken here (and by the library): eigenvalues sorted by
ascending real part, then ascending imaginary part; eigenvectors of unit
2-norm whose largest-modulus entry (the first one on exact ties) is real and
positive.
"""
from __future__ import annotations

import numpy as np

U = 2.0 ** -53


def hessenberg(m):
    """Householder reduction: returns (H, Q) with m = Q H Q^H, H upper
    Hessenberg, Q unitary."""
    h = np.array(m, dtype=np.complex128)
    n = h.shape[0]
    q = np.eye(n, dtype=np.complex128)
    for j in range(n - 2):
        x = h[j + 1:, j].copy()
        alpha = np.linalg.norm(x)
        if alpha == 0.0:
            continue
        phase = x[0] / abs(x[0]) if x[0] != 0 else 1.0
        v = x.copy()
        v[0] += phase * alpha                 # v = x + e^{i arg x0} ||x|| e_1
        v /= np.linalg.norm(v)
        # H <- P H P with P = I - 2 v v^H acting on rows / columns j+1..n-1
        h[j + 1:, :] -= 2.0 * np.outer(v, v.conj() @ h[j + 1:, :])
        h[:, j + 1:] -= 2.0 * np.outer(h[:, j + 1:] @ v, v.conj())
        q[:, j + 1:] -= 2.0 * np.outer(q[:, j + 1:] @ v, v.conj())
        h[j + 2:, j] = 0.0
    return h, q


def _givens(a, b):
    """c (real), s with [[c, s], [-conj(s), c]] [a; b] = [r; 0]."""
    if b == 0:
        return 1.0, 0.0
    if a == 0:
        return 0.0, np.conj(b) / abs(b)
    na = abs(a)
    r = np.hypot(na, abs(b))
    c = na / r
    s = (a / na) * np.conj(b) / r
    return c, s


def schur(h, z, max_sweeps_per_eig: int = 60):
    """Complex Schur form of an upper Hessenberg h by single-shift QR with
    Wilkinson shifts; z accumulates the transformations (z <- z G).  Returns
    (T, Z) with Z T Z^H = z_in h z_in^H."""
    t = np.array(h, dtype=np.complex128)
    z = np.array(z, dtype=np.complex128)
    n = t.shape[0]
    hi = n - 1
    sweeps = 0
    while hi > 0:
        # deflate: find the active block [lo, hi]
        lo = hi
        while lo > 0:
            if abs(t[lo, lo - 1]) <= U * (abs(t[lo - 1, lo - 1]) + abs(t[lo, lo])):
                t[lo, lo - 1] = 0.0
                break
            lo -= 1
        if lo == hi:
            hi -= 1
            sweeps = 0
            continue
        sweeps += 1
        if sweeps > max_sweeps_per_eig:
            raise RuntimeError("QR iteration did not converge")
        # Wilkinson shift: eigenvalue of the trailing 2 x 2 block nearer t[hi, hi]
        a, b = t[hi - 1, hi - 1], t[hi - 1, hi]
        c, d = t[hi, hi - 1], t[hi, hi]
        tr, det = a + d, a * d - b * c
        disc = np.sqrt(tr * tr / 4 - det)
        l1, l2 = tr / 2 + disc, tr / 2 - disc
        mu = l1 if abs(l1 - d) < abs(l2 - d) else l2
        if sweeps % 11 == 10:                 # exceptional shift against cycling
            mu = d + abs(t[hi, hi - 1])
        # one implicit QR step on the active block: H - mu I = QR, H <- RQ + mu I
        x, y = t[lo, lo] - mu, t[lo + 1, lo]
        for k in range(lo, hi):
            cs, sn = _givens(x, y)
            g = np.array([[cs, sn], [-np.conj(sn), cs]], dtype=np.complex128)
            c0 = max(lo, k - 1)
            t[k:k + 2, c0:] = g @ t[k:k + 2, c0:]
            r1 = min(hi, k + 2)
            t[:r1 + 1, k:k + 2] = t[:r1 + 1, k:k + 2] @ g.conj().T
            z[:, k:k + 2] = z[:, k:k + 2] @ g.conj().T
            if k + 1 < hi:
                x, y = t[k + 1, k], t[k + 2, k]
    # exact zeros below the diagonal
    return np.triu(t), z


def triangular_eigvecs(t):
    """Columns x_k with T x_k = t_kk x_k, x_k[k] = 1, zero below k."""
    n = t.shape[0]
    x = np.zeros((n, n), dtype=np.complex128)
    small = U * max(np.linalg.norm(t), np.finfo(float).tiny)
    for k in range(n):
        lam = t[k, k]
        x[k, k] = 1.0
        for i in range(k - 1, -1, -1):
            acc = -t[i, k] - t[i, i + 1:k] @ x[i + 1:k, k]
            den = t[i, i] - lam
            if abs(den) < small:
                den = small
            x[i, k] = acc / den
    return x


def _order(w):
    return sorted(range(len(w)), key=lambda i: (w[i].real, w[i].imag))


def _gauge(v):
    out = v.copy()
    for k in range(v.shape[1]):
        col = out[:, k] / np.linalg.norm(out[:, k])
        j = int(np.argmax(np.abs(col)))
        out[:, k] = col * (abs(col[j]) / col[j])
    return out


def eig_matrix(m):
    """(w, V) of a square matrix: A V = V diag(w), ordered and scaled as the
    module docstring states."""
    a = np.asarray(m, dtype=np.complex128)
    n = a.shape[0]
    if a.shape != (n, n):
        raise ValueError("eig needs a square matricisation")
    if n == 0:
        return np.zeros(0, dtype=np.complex128), np.zeros((0, 0), dtype=np.complex128)
    h, q = hessenberg(a)
    t, z = schur(h, q)
    x = triangular_eigvecs(t)
    v = z @ x
    w = np.diag(t).copy()
    idx = _order(w)
    return w[idx], _gauge(v[:, idx])


def eigvals(a, k_rows: int):
    """Spec, eigvals: eigenvalues of the matricised tensor (first k bonds as rows)."""
    a = np.asarray(a)
    rows = int(np.prod(a.shape[:k_rows]))
    w, _ = eig_matrix(a.reshape(rows, -1))
    return w


def eig(a, k_rows: int):
    """Spec, eig: (w, v) with v of shape (d_0, ..., d_{k-1}, I)."""
    a = np.asarray(a)
    rows = int(np.prod(a.shape[:k_rows]))
    w, v = eig_matrix(a.reshape(rows, -1))
    return w, v.reshape(tuple(a.shape[:k_rows]) + (rows,))
