"""Oracle for the effective-Hamiltonian matvec and the Lanczos ground-state step.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper names DMRG among the algorithms its interface serves (Sec. I) but
prints no DMRG code; the two-site DMRG update used here is the textbook one
written in the paper's contraction primitive:

    y[a,s1,s2,b] = sum L[a,w,a'] W[w,w',s1,s1'] W[w',w'',s2,s2'] R[b,w'',b']
                       theta[a',s1',s2',b']

evaluated as four label contractions (Spec, contract), followed by a Lanczos
iteration with full re-orthogonalisation.
"""
from __future__ import annotations

import numpy as np

from . import contract, eigh, norm


def heff_apply(left, w1, w2, right, theta):
    """H_eff theta by four pairwise label contractions (brute-force loops)."""
    x1 = contract(left, "awp", theta, "pstq", "awstq")          # sum a'
    x2 = contract(x1, "awstq", w1, "wvus", "avutq")            # sum w, s1'
    x3 = contract(x2, "avutq", w2, "vxet", "auxeq")            # sum w', s2'
    return contract(x3, "auxeq", right, "bxq", "aueb")         # sum w'', b'


def heff_dense(left, w1, w2, right):
    """The dense matrix of H_eff (tiny chi only), by the definition's loops."""
    chi_l, chi_r = left.shape[0], right.shape[0]
    d = w1.shape[2]
    dim = chi_l * d * d * chi_r
    h = np.zeros((dim, dim), dtype=np.complex128)
    for a in range(chi_l):
        for s1 in range(d):
            for s2 in range(d):
                for b in range(chi_r):
                    row = ((a * d + s1) * d + s2) * chi_r + b
                    for ap in range(chi_l):
                        for t1 in range(d):
                            for t2 in range(d):
                                for bp in range(chi_r):
                                    col = ((ap * d + t1) * d + t2) * chi_r + bp
                                    acc = 0.0
                                    for w in range(left.shape[1]):
                                        for wp in range(w1.shape[1]):
                                            for wpp in range(w2.shape[1]):
                                                acc += (left[a, w, ap] * w1[w, wp, s1, t1]
                                                        * w2[wp, wpp, s2, t2]
                                                        * right[b, wpp, bp])
                                    h[row, col] = acc
    return h


def _vdot(x, y):
    return complex(np.sum(np.conj(x) * y))


def lanczos_ground(matvec, theta, n_matvec=20, breakdown=1e-13):
    """Lowest Ritz pair of H after at most n_matvec matvecs, started at theta.

    v_0 = theta / ||theta||; for j = 0, 1, ...: w = H v_j, alpha_j = Re<v_j, w>,
    w -= alpha_j v_j + beta_{j-1} v_{j-1}, then two passes of classical
    Gram-Schmidt against v_0..v_j, beta_j = ||w||; stop on
    beta_j <= breakdown * max|T| or after n_matvec matvecs, else
    v_{j+1} = w / beta_j.  T = tridiag(alpha, beta) -> lowest (lambda, y);
    psi = sum y_i v_i normalised, phase fixed so <theta, psi> is real > 0.
    Returns (energy, psi, alphas, betas)."""
    v0, _ = theta / norm(theta), None
    basis = [v0]
    alphas, betas = [], []
    tmax = 0.0
    for j in range(n_matvec):
        w = matvec(basis[j])
        alpha = _vdot(basis[j], w).real
        alphas.append(alpha)
        w = w - alpha * basis[j]
        if j > 0:
            w = w - betas[j - 1] * basis[j - 1]
        for _ in range(2):
            coefs = [_vdot(v, w) for v in basis]
            for c, v in zip(coefs, basis):
                w = w - c * v
        beta = norm(w)
        tmax = max(tmax, abs(alpha), abs(beta))
        if j == n_matvec - 1:
            break
        if beta <= breakdown * tmax:
            break
        betas.append(beta)
        basis.append(w / beta)
    m = len(alphas)
    t = np.diag(np.array(alphas, dtype=np.complex128))
    for i in range(m - 1):
        t[i, i + 1] = t[i + 1, i] = betas[i]
    evals, evecs = eigh(t)
    y = evecs[:, 0]
    psi = np.zeros_like(v0)
    for i in range(m):
        psi = psi + y[i] * basis[i]
    psi = psi / norm(psi)
    ov = _vdot(theta, psi)
    if abs(ov) > 0:
        psi = psi * (np.conj(ov) / abs(ov))
    return float(evals[0]), psi, np.array(alphas), np.array(betas[: m - 1])


def heisenberg_chain_dense(n_sites: int) -> np.ndarray:
    """Dense Hamiltonian of the open spin-1/2 Heisenberg chain,
    H = sum_i S_i . S_{i+1} (J = 1), basis index 0 = up, site 0 the most
    significant factor of the Kronecker products."""
    sp = np.array([[0.0, 1.0], [0.0, 0.0]])
    sm = sp.T
    sz = np.diag([0.5, -0.5])
    dim = 2 ** n_sites
    h = np.zeros((dim, dim))
    for i in range(n_sites - 1):
        left = np.eye(2 ** i)
        right = np.eye(2 ** (n_sites - i - 2))
        bond = 0.5 * (np.kron(sp, sm) + np.kron(sm, sp)) + np.kron(sz, sz)
        h += np.kron(np.kron(left, bond), right)
    return h


def heisenberg_ground_energy(n_sites: int) -> float:
    """Exact ground-state energy of the open chain by dense diagonalisation."""
    return float(np.linalg.eigvalsh(heisenberg_chain_dense(n_sites))[0])
