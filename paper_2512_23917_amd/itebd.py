"""Infinite TEBD for the transverse-field Ising chain on the library (the
application of the paper's App. A, in the Vidal form with inverse singular
values).

Model (Sec. IV, eq. (1)): H = -J sum_i Z_i Z_{i+1} - g sum_i X_i, split into
bond terms h = -J Z Z - (g/2)(X I + I X).  The imaginary-time gate
U = exp(-dt h) is symmetric, so contracting either of its index pairs gives
the same update; the library applies rows = outgoing pair.

Two-site unit cell (Gamma_A, lambda_A, Gamma_B, lambda_B); lambda_A sits on
the A-B bond, lambda_B on the B-A bond.  One step updates the bond (X, Y)
with inner weights l_i and outer weights l_o:

    theta = diag(l_o) Gamma_X diag(l_i) Gamma_Y diag(l_o)      (chi, 2, 2, chi)
    theta' = U theta;   U_, s, V^dag = trunc_svd(theta', 2 row bonds)
    l_i <- s / ||s||;   Gamma_X <- diag(1/l_o) U_;   Gamma_Y <- V^dag diag(1/l_o)

first for (A, B), then for (B, A).  Every contraction, the gate and the
truncated SVD run in the library (FP64); the weights are moved to the host
only to build the diagonal factors.  The energy per site is the mean over
the two bonds of <theta|h|theta> / <theta|theta>.
"""
from __future__ import annotations

import numpy as np

from . import tci

PAULI_X = np.array([[0.0, 1.0], [1.0, 0.0]])
PAULI_Z = np.array([[1.0, 0.0], [0.0, -1.0]])


def bond_hamiltonian(g: float, J: float = 1.0) -> np.ndarray:
    """4 x 4 bond term, rows and columns ordered (s1 s2)."""
    eye = np.eye(2)
    return -J * np.kron(PAULI_Z, PAULI_Z) - 0.5 * g * (np.kron(PAULI_X, eye) + np.kron(eye, PAULI_X))


def imaginary_time_gate(h: np.ndarray, dt: float) -> np.ndarray:
    """exp(-dt h) of the real symmetric 4 x 4 bond term."""
    w, v = np.linalg.eigh(h)
    return (v * np.exp(-dt * w)) @ v.T


class ITEBD:
    def __init__(self, ctx: tci.Context, chi: int, g: float, J: float = 1.0, s_min: float = 1e-13):
        self.ctx, self.chi, self.g, self.J, self.s_min = ctx, chi, g, J, s_min
        up = np.zeros((1, 2, 1))
        up[0, 0, 0] = 1.0
        self.G = [self._t(up), self._t(up)]
        self.lam = [np.ones(1), np.ones(1)]
        self.h4 = self._t(bond_hamiltonian(g, J).reshape(2, 2, 2, 2))

    def _t(self, a: np.ndarray) -> tci.Tensor:
        return tci.Tensor.from_numpy(self.ctx, np.ascontiguousarray(a, dtype=np.float64), tci.F64)

    def _theta(self, X: int) -> tci.Tensor:
        Y = 1 - X
        c = self.ctx
        do, di = self._t(np.diag(self.lam[Y])), self._t(np.diag(self.lam[X]))
        t = tci.contract(c, do, "ax", self.G[X], "xsm", "asm")
        t = tci.contract(c, t, "asm", di, "mn", "asn")
        t = tci.contract(c, t, "asn", self.G[Y], "ntx", "astx")
        return tci.contract(c, t, "astx", do, "xb", "astb")

    def step(self, gate4: tci.Tensor):
        c = self.ctx
        for X in (0, 1):
            Y = 1 - X
            th = tci.contract(c, self._theta(X), "astb", gate4, "uvst", "auvb")
            u, s, vh, _ = tci.trunc_svd(c, th, 2, 1, self.chi, 0.0, self.s_min)
            sv = s.numpy().astype(np.float64)
            self.lam[X] = sv / np.linalg.norm(sv)
            dinv = self._t(np.diag(1.0 / self.lam[Y]))
            self.G[X] = tci.contract(c, dinv, "ax", u, "xsk", "ask")
            self.G[Y] = tci.contract(c, vh, "ktx", dinv, "xb", "ktb")

    def energy(self) -> float:
        c = self.ctx
        es = []
        for X in (0, 1):
            th = self._theta(X)
            hth = tci.contract(c, th, "astb", self.h4, "uvst", "auvb")
            num = tci.contract(c, th, "astb", hth, "astb", "").numpy().reshape(-1)[0]
            den = tci.contract(c, th, "astb", th, "astb", "").numpy().reshape(-1)[0]
            es.append(num / den)
        return float(np.mean(es))

    def run(self, schedule) -> float:
        """schedule: [(dt, steps), ...]; returns the energy per site."""
        h = bond_hamiltonian(self.g, self.J)
        for dt, n in schedule:
            gate4 = self._t(imaginary_time_gate(h, dt).reshape(2, 2, 2, 2))
            for _ in range(n):
                self.step(gate4)
        return self.energy()
