"""Finite two-site DMRG sweeps on the library: the effective-Hamiltonian
Lanczos step, the truncated split and the environment updates of an open
spin-1/2 Heisenberg chain (the DMRG form of the two-site update, Sec. II.B
contraction and decomposition equations).

Conventions (as in tci_heff_matvec): the MPO W[w, w', s_out, s_in] is the
bond-dimension-5 Heisenberg operator; a left environment L[a, w, a'] has the
bra index a and the ket index a', likewise R[b, w, b'].  The open ends are
the one-dimensional environments that select channel 4 on the left and
channel 0 on the right.

    L_{i+1}[b, w', b'] = sum conj(A_i[a, s, b]) L_i[a, w, a'] W[w, w', s, s'] A_i[a', s', b']
    R_i[a, w, a']      = sum conj(B_i[a, s, b]) W[w, w'', s, s'] R_{i+1}[b, w'', b'] B_i[a', s', b']

A sweep visits the bonds left to right (the split keeps U as the new
left-isometric site and diag(s) V^dagger as the centre) and then right to
left (U diag(s) as the centre, V^dagger right-isometric).  Every contraction,
Lanczos solve and split runs in the library; the initial state is
right-canonicalised on the host (input preparation).
"""
from __future__ import annotations

import numpy as np

from . import synth, tci


def conj(ctx: tci.Context, t: tci.Tensor) -> tci.Tensor:
    out = tci.Tensor.empty(ctx, t.dtype, int(np.prod(t.shape())))
    tci._check(tci.lib().tci_cplx_conj(ctx.h, t.h, out.h), "tci_cplx_conj")
    return out


def right_canonical(mps):
    """Right-canonical copy of an open MPS (host QR, last site to second)."""
    out = [np.array(a, dtype=np.complex128) for a in mps]
    for i in range(len(out) - 1, 0, -1):
        chil, d, chir = out[i].shape
        q, r = np.linalg.qr(out[i].reshape(chil, d * chir).T)
        k = q.shape[1]
        out[i] = q.T.reshape(k, d, chir)
        out[i - 1] = np.einsum("asm,km->ask", out[i - 1], r)
    out[0] = out[0] / np.linalg.norm(out[0])
    return out


class DMRG:
    def __init__(self, ctx: tci.Context, n_sites: int, chi: int, seed: int = 0, dtype: int = tci.C128,
                 n_matvec: int = 20, eps: float = 1e-12):
        self.ctx, self.n, self.chi, self.n_matvec, self.eps = ctx, n_sites, chi, n_matvec, eps
        self.dt = dtype
        np_dt = np.complex128 if dtype == tci.C128 else np.complex64
        mps = right_canonical(synth.random_open_mps(synth.rng(6, seed), n_sites, 2, chi))
        self.M = [tci.Tensor.from_numpy(ctx, a.astype(np_dt), dtype) for a in mps]
        self.W = tci.Tensor.from_numpy(ctx, synth.heisenberg_mpo().astype(np_dt), dtype)
        left, right = synth.trivial_environments()
        self.L = [None] * (n_sites + 1)
        self.R = [None] * (n_sites + 1)
        self.L[0] = tci.Tensor.from_numpy(ctx, left.astype(np_dt), dtype)
        self.R[n_sites] = tci.Tensor.from_numpy(ctx, right.astype(np_dt), dtype)
        for i in range(n_sites - 1, 1, -1):
            self.R[i] = self._right_env(self.R[i + 1], self.M[i])
        self.energy = None

    def _left_env(self, L, A):
        c = self.ctx
        t = tci.contract(c, L, "awx", A, "xtb", "awtb")
        t = tci.contract(c, t, "awtb", self.W, "wvst", "avsb")
        return tci.contract(c, conj(c, A), "asc", t, "avsb", "cvb")

    def _right_env(self, R, B):
        c = self.ctx
        t = tci.contract(c, B, "atx", R, "bvx", "atbv")
        t = tci.contract(c, t, "atbv", self.W, "wvst", "asbw")
        return tci.contract(c, conj(c, B), "csb", t, "asbw", "cwa")

    def _update(self, i: int, direction: int):
        c = self.ctx
        th = tci.contract(c, self.M[i], "asm", self.M[i + 1], "mtb", "astb")
        self.energy = tci.lanczos_ground(c, self.L[i], self.W, self.W, self.R[i + 2], th, self.n_matvec)
        p = tci.update_params(chi_min=1, chi_max=self.chi, target_trunc_err=self.eps, direction=direction,
                              precision=tci.PREC_FP64 if self.dt == tci.C128 else tci.PREC_BF16X3)
        Ao, so, Bo, _ = tci.split_batched(c, [th], p)
        self.M[i], self.M[i + 1] = Ao[0], Bo[0]

    def sweep(self) -> float:
        for i in range(self.n - 1):
            self._update(i, tci.DIR_LEFT)
            if i < self.n - 2:
                self.L[i + 1] = self._left_env(self.L[i], self.M[i])
        for i in range(self.n - 2, -1, -1):
            self._update(i, tci.DIR_RIGHT)
            if i > 0:
                self.R[i + 1] = self._right_env(self.R[i + 2], self.M[i + 1])
        return self.energy
