"""Oracle for the randomized truncated SVD with a plain-SVD fallback.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Randomized range finder with power iterations (Halko, Martinsson, Tropp,
SIAM Rev. 53, 2011, Alg. 4.4) and Cholesky-QR2 orthonormalisation (Fukaya et
al., ScalA 2014), cut by the truncation rule of the paper's trunc_svd
(Spec, linear algebra, trunc_svd) with the relative error measured against the
exact total weight ||theta||_F^2.

    Y = theta Omega                         (Omega n x k Gaussian, Philox)
    repeat q times:  Y <- theta (theta^dagger orth(Y))
    Q = CholQR2(Y);  B = Q^dagger theta
    B B^dagger = W Lambda W^dagger, sigma = sqrt(Lambda) descending
    U = Q W;  V^dagger = Sigma^-1 W^dagger B
    chi, eps from the rule with total = ||theta||_F^2
    residuals r_i = || theta v_i - sigma_i u_i ||_2 for the kept i
    accept iff eps <= target and max r_i <= cert * sigma_1, else plain SVD.
"""
from __future__ import annotations

import numpy as np

from . import eigh, philox_normal, svd_matrix, trunc_rule


def gaussian_sketch(n: int, k: int, seed: int, complex_: bool, stream: int = 0) -> np.ndarray:
    """Omega[i, j]: real case z[i*k+j]; complex case (z[2t] + i z[2t+1]) / sqrt 2
    with t = i*k + j, z the Philox normal stream `stream` under key `seed`."""
    if complex_:
        z = philox_normal(seed, stream, 2 * n * k).reshape(n * k, 2)
        return ((z[:, 0] + 1j * z[:, 1]) / np.sqrt(2.0)).reshape(n, k)
    return philox_normal(seed, stream, n * k).reshape(n, k).astype(np.complex128)


def cholesky_drop(g, tau=1e-12):
    """Upper-triangular R with R^dagger R = G restricted to the columns kept.

    Column j is dropped when its pivot (the squared distance of y_j from the
    span of the kept earlier columns) is <= tau * G[j, j] or not positive:
    y_j is then numerically inside that span.  Dropped rows of R stay zero."""
    k = g.shape[0]
    r = np.zeros_like(g)
    keep = np.zeros(k, dtype=bool)
    for j in range(k):
        p = g[j, j].real - np.sum(np.abs(r[:j, j]) ** 2)
        if not (p > tau * g[j, j].real and p > 0.0):
            continue
        keep[j] = True
        r[j, j] = np.sqrt(p)
        if j + 1 < k:
            r[j, j + 1:] = (g[j, j + 1:] - r[:j, j].conj() @ r[:j, j + 1:]) / r[j, j]
    return r, keep


def chol_qr(y, tau=1e-12):
    """One Cholesky-QR pass with column dropping: G = Y^dagger Y = R^dagger R,
    Q = Y R^-1 by forward substitution over the columns; dropped columns of Q
    are zero."""
    g = y.conj().T @ y
    r, keep = cholesky_drop(g, tau)
    q = np.zeros_like(y)
    for j in range(y.shape[1]):
        if keep[j]:
            q[:, j] = (y[:, j] - q[:, :j] @ r[:j, j]) / r[j, j]
    return q


def chol_qr2(y):
    """Cholesky-QR2 (Fukaya et al. 2014): a second pass repairs the loss of
    orthogonality of the first."""
    return chol_qr(chol_qr(y))


def rule_with_total(sig, total, chi_min, chi_max, target, s_min):
    """The trunc_svd rule with eps(chi) = (total - sum_{i<chi} sig_i^2) / total."""
    k = len(sig)
    n_a = 0
    while n_a < k and sig[n_a] >= s_min:
        n_a += 1
    kept = np.concatenate([[0.0], np.cumsum(sig ** 2)])

    def eps(c):
        return max(total - kept[c], 0.0) / total if total > 0 else 0.0

    if n_a <= chi_min:
        chi = n_a
    else:
        chi = chi_min
        lim = min(chi_max, n_a)
        while chi < lim and eps(chi) > target:
            chi += 1
    chi = max(chi, 1)
    return chi, eps(chi)


def randomized_tsvd(theta, k, q=2, seed=0, chi_min=1, chi_max=None, target=0.0,
                    s_min=0.0, cert=1e-7, stream=0, complex_=None):
    """Returns dict(u, s, vh, chi, err, accepted, residual, sig_all)."""
    theta = np.asarray(theta, dtype=np.complex128)
    m, n = theta.shape
    if chi_max is None:
        chi_max = min(m, n)
    if complex_ is None:
        complex_ = bool(np.any(theta.imag != 0))
    omega = gaussian_sketch(n, k, seed, complex_, stream)
    y = theta @ omega
    for _ in range(q):
        z = theta.conj().T @ chol_qr2(y)
        y = theta @ chol_qr2(z)
    qm = chol_qr2(y)
    b = qm.conj().T @ theta
    lam, w = eigh(b @ b.conj().T)
    order = np.arange(len(lam))[::-1]
    lam, w = lam[order], w[:, order]
    sig = np.sqrt(np.maximum(lam, 0.0))
    u = qm @ w
    total = float(np.sum(np.abs(theta) ** 2))
    chi, err = rule_with_total(sig, total, chi_min, chi_max, target, s_min)
    s = sig[:chi]
    vh = (w[:, :chi].conj().T @ b) / s[:, None]
    resid = np.linalg.norm(theta @ vh.conj().T - u[:, :chi] * s[None, :], axis=0)
    accepted = bool(err <= target and np.max(resid) <= cert * sig[0])
    return dict(u=u[:, :chi], s=s, vh=vh, chi=chi, err=err, accepted=accepted,
                residual=resid, sig_all=sig)


def tsvd_with_fallback(theta, k, q=2, seed=0, chi_min=1, chi_max=None, target=0.0,
                       s_min=0.0, cert=1e-7, stream=0, complex_=None):
    """Randomized first; the plain truncated SVD when it is not accepted."""
    r = randomized_tsvd(theta, k, q, seed, chi_min, chi_max, target, s_min, cert, stream, complex_)
    if r["accepted"]:
        r["fallback"] = False
        return r
    u, s, vh = svd_matrix(theta)
    m, n = theta.shape
    chi, err = trunc_rule(s, chi_min, chi_max if chi_max else min(m, n), target, s_min)
    return dict(u=u[:, :chi], s=s[:chi], vh=vh[:chi], chi=chi, err=err, accepted=False,
                fallback=True, residual=None, sig_all=s)
