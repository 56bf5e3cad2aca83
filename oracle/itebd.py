"""Oracle for the infinite-TEBD application (the paper's App. A, Vidal form).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The same steps as App. A with the oracle's contraction and truncated SVD
(one-sided Jacobi), FP64: theta = diag(l_o) G_X diag(l_i) G_Y diag(l_o),
theta' = U theta, trunc_svd with 2 row bonds, l_i = s / ||s||,
G_X = diag(1/l_o) U_, G_Y = V^dag diag(1/l_o), for the bonds (A, B) then
(B, A).  Energy per site: the mean over the two bonds of <theta|h|theta> /
<theta|theta>.  The physics pin is the exact ground-state energy per site of
the transverse-field Ising chain, e0(g) = -(1/pi) int_0^pi sqrt(1 + g^2 +
2 g cos k) dk (e0(1) = -4/pi).
"""
from __future__ import annotations

import numpy as np

from . import contract, trunc_svd


def e0_exact(g: float) -> float:
    from scipy.integrate import quad
    val, _ = quad(lambda k: np.sqrt(1.0 + g * g + 2.0 * g * np.cos(k)), 0.0, np.pi, epsabs=1e-13, epsrel=1e-13,
                  limit=200)
    return -val / np.pi


def run(g: float, chi: int, schedule, J: float = 1.0, s_min: float = 1e-13):
    X = np.array([[0.0, 1.0], [1.0, 0.0]])
    Z = np.diag([1.0, -1.0])
    I = np.eye(2)
    h = -J * np.kron(Z, Z) - 0.5 * g * (np.kron(X, I) + np.kron(I, X))
    up = np.zeros((1, 2, 1))
    up[0, 0, 0] = 1.0
    G = [up.copy(), up.copy()]
    lam = [np.ones(1), np.ones(1)]

    def theta(x):
        y = 1 - x
        t = contract(np.diag(lam[y]), "ax", G[x], "xsm", "asm")
        t = contract(t, "asm", np.diag(lam[x]), "mn", "asn")
        t = contract(t, "asn", G[y], "ntx", "astx")
        return contract(t, "astx", np.diag(lam[y]), "xb", "astb")

    for dt, n in schedule:
        w, v = np.linalg.eigh(h)
        u4 = ((v * np.exp(-dt * w)) @ v.T).reshape(2, 2, 2, 2)
        for _ in range(n):
            for x in (0, 1):
                y = 1 - x
                th = contract(theta(x), "astb", u4, "uvst", "auvb")
                u, s, vh, _ = trunc_svd(th, 2, 1, chi, 0.0, s_min)
                lam[x] = s / np.linalg.norm(s)
                G[x] = contract(np.diag(1.0 / lam[y]), "ax", u, "xsk", "ask").real
                G[y] = contract(vh, "ktx", np.diag(1.0 / lam[y]), "xb", "ktb").real
    es = []
    h4 = h.reshape(2, 2, 2, 2)
    for x in (0, 1):
        th = theta(x)
        hth = contract(th, "astb", h4, "uvst", "auvb")
        es.append(np.vdot(th, hth).real / np.vdot(th, th).real)
    return float(np.mean(es))
