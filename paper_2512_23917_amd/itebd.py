"""Infinite TEBD for the transverse-field Ising chain on the library (the
application of the paper's App. A, in the Vidal form).

Model (Sec. IV, eq. (1)): H = -J sum_i Z_i Z_{i+1} - g sum_i X_i, split into
bond terms h = -J Z Z - (g/2)(X I + I X).  The imaginary-time gate
U = exp(-dt h) is symmetric, so contracting either of its index pairs gives
the same update; the library applies rows = outgoing pair.

State: a two-site unit cell (Gamma_A, lambda_A, Gamma_B, lambda_B), where
lambda_A sits on the A-B bond and lambda_B on the B-A bond.  Updating the
bond (X, Y) with inner weights l_i and outer weights l_o is one two-site
update of the pair

    A' = diag(l_o) Gamma_X diag(l_i),   B' = Gamma_Y diag(l_o)

(so that theta = A' B' carries every weight of the bond's environment): the
composite forms theta, applies the gate, truncates, renormalises the kept
values into the new l_i and writes the Vidal factors
Gamma_X = diag(1/l_o) U and Gamma_Y = V^dag diag(1/l_o) on the device.  The
weights never leave the device; the bond (A, B) is updated first, then
(B, A).  The energy per site is the mean over the two bonds of
<theta|h|theta> / <theta|theta>.
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
        self.lam = [self._t(np.ones(1)), self._t(np.ones(1))]
        self.h4 = self._t(bond_hamiltonian(g, J).reshape(2, 2, 2, 2))
        self.params = tci.update_params(chi_min=1, chi_max=chi, target_trunc_err=0.0, s_min=s_min,
                                        direction=tci.DIR_VIDAL, precision=tci.PREC_FP64)

    def _t(self, a: np.ndarray) -> tci.Tensor:
        return tci.Tensor.from_numpy(self.ctx, np.ascontiguousarray(a, dtype=np.float64), tci.F64)

    def _pair(self, X: int):
        """The bond's site tensors with the environment weights absorbed."""
        Y = 1 - X
        c = self.ctx
        lo, li = tci.diag(c, self.lam[Y]), tci.diag(c, self.lam[X])
        a = tci.contract(c, lo, "ax", self.G[X], "xsm", "asm")
        a = tci.contract(c, a, "asm", li, "mn", "asn")
        b = tci.contract(c, self.G[Y], "ntx", lo, "xb", "ntb")
        return a, b

    def step(self, gate4: tci.Tensor):
        for X in (0, 1):
            Y = 1 - X
            a, b = self._pair(X)
            lam_o = self.lam[Y]
            A_out, s_out, B_out, _ = tci.two_site_update_batched(self.ctx, [a], [b], [gate4], self.params,
                                                                 lambda_left=[lam_o], lambda_right=[lam_o])
            self.G[X], self.lam[X], self.G[Y] = A_out[0], s_out[0], B_out[0]

    def energy(self) -> float:
        c = self.ctx
        es = []
        for X in (0, 1):
            a, b = self._pair(X)
            th = tci.contract(c, a, "asm", b, "mtb", "astb")
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
