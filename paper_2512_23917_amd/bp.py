"""Belief-propagation update of a tensor-network state on a graph, on the
library (the TNO-TNS scheme of the paper's App. B: gate layers attached as
tensor-network operators, BP messages converged on the norm network, then
square-root messages and an SVD of their product to regauge and truncate
every updated bond).

Conventions:
  * sites 0..n-1, undirected edges (i, j), i < j; the bonds of a site are
    ordered by the neighbour's index; V_i has indices [s, b_1, ..., b_deg];
  * M_{i->j}[a, a'] is the environment of bond (i, j) from i's side (a ket,
    a' bra), Hermitian, unit trace; one BP sweep recomputes every M_{i->j}
    from V_i, conj(V_i) and the messages M_{k->i}, k != j, of the previous
    sweep;
  * edge (i, j) is regauged with X = M_{i->j}^{1/2}, Y = M_{j->i}^{1/2}:
    R = X^T Y = U S V^H, and the bond matrices X^{-T} U S^{1/2} (on V_i) and
    Y^{-T} conj(V) S^{1/2} (on V_j), kept to the chi largest singular
    values; inverse square roots drop eigenvalues below 1e-10 of the
    largest (their relative error from FP64 rounding would exceed ~5e-6),
    and singular values below sv_cut (default 1e-6) of the largest are not
    bond directions (FP64 rounding of R, amplified up to 1e10 by the two
    inverse square roots, reaches that level); the SVD of R runs on the
    library's one-sided Jacobi path, which resolves its small values;
  * a gate G[s_i, s_j, s_i', s_j'] is split by an SVD of its
    (s_i s_i') x (s_j s_j') matrix into O_i U S^{1/2} and O_j (S^{1/2} V^H)^T,
    whose shared index becomes the faster half of the bond (i, j).

Every contraction, eigendecomposition, SVD, trace, transpose, scaling and
sub-tensor extraction runs in the library (complex128, FP64 matrix cores);
the host only reads the small spectra of the messages and of R to build the
diagonal factors and the cut (as in the App. A driver) and keeps the graph.
"""
from __future__ import annotations

import numpy as np

from . import tci

INV_SQRT_CUT = 1e-10   # message eigenvalues kept by the inverse square root (relative)
SV_CUT = 1e-6          # default floor of the singular values of R kept as bond directions (relative)
S_LABEL, KET, BRA, NEW, GATE = 1, 100, 200, 300, 400


def neighbours(n, edges):
    nb = [[] for _ in range(n)]
    for i, j in edges:
        nb[i].append(j)
        nb[j].append(i)
    return [sorted(x) for x in nb]


class BPState:
    def __init__(self, ctx: tci.Context, n: int, edges, tensors):
        self.ctx, self.n = ctx, n
        self.edges = [tuple(sorted(e)) for e in edges]
        self.nb = neighbours(n, self.edges)
        self.V = [tci.Tensor.from_numpy(ctx, np.ascontiguousarray(v, dtype=np.complex128), tci.C128)
                  for v in tensors]
        self.M = {}

    # ------------------------------------------------------------ helpers
    def _t(self, a) -> tci.Tensor:
        return tci.Tensor.from_numpy(self.ctx, np.ascontiguousarray(a, dtype=np.complex128), tci.C128)

    def _labels(self, i):
        return [S_LABEL] + [KET + p for p in range(len(self.nb[i]))]

    def host_tensors(self):
        return [v.numpy().copy() for v in self.V]

    # ------------------------------------------------------------ BP
    def init_messages(self):
        self.M = {}
        for i in range(self.n):
            for pos, j in enumerate(self.nb[i]):
                d = self.V[i].shape()[1 + pos]
                self.M[(i, j)] = self._t(np.eye(d) / d)

    def message(self, i, j, M):
        c = self.ctx
        lab = self._labels(i)
        a = self.V[i]
        for pos, k in enumerate(self.nb[i]):
            if k == j:
                continue
            out = [BRA + pos if x == KET + pos else x for x in lab]
            a = tci.contract(c, a, lab, M[(k, i)], [KET + pos, BRA + pos], out)
            lab = out
        pj = self.nb[i].index(j)
        bra = [S_LABEL] + [BRA + p for p in range(len(self.nb[i]))]
        m = tci.contract(c, a, lab, tci.cplx_conj(c, self.V[i]), bra, [KET + pj, BRA + pj])
        tr = tci.trace(c, m, [(0, 1)]).numpy().reshape(-1)[0]
        return tci.scale(c, m, 1.0 / tr)

    def sweep(self):
        self.M = {(i, j): self.message(i, j, self.M) for (i, j) in self.M}

    def run_bp(self, iters: int):
        self.init_messages()
        for _ in range(iters):
            self.sweep()

    def bp_norm(self) -> complex:
        c = self.ctx
        z = 1.0 + 0.0j
        for i in range(self.n):
            lab = self._labels(i)
            a = self.V[i]
            for pos, k in enumerate(self.nb[i]):
                out = [BRA + pos if x == KET + pos else x for x in lab]
                a = tci.contract(c, a, lab, self.M[(k, i)], [KET + pos, BRA + pos], out)
                lab = out
            bra = [S_LABEL] + [BRA + p for p in range(len(self.nb[i]))]
            z *= tci.contract(c, a, lab, tci.cplx_conj(c, self.V[i]), bra, []).numpy().reshape(-1)[0]
        for i, j in self.edges:
            z /= tci.contract(c, self.M[(i, j)], "ab", self.M[(j, i)], "ab", "").numpy().reshape(-1)[0]
        return z

    # ------------------------------------------------------------ regauge + truncation
    def _sqrt_and_inv(self, m):
        c = self.ctx
        w, u = tci.eigh(c, m)
        w = np.clip(w.numpy(), 0.0, None)
        keep = w > INV_SQRT_CUT * w.max()
        uc = tci.cplx_conj(c, u)
        ds = self._t(np.diag(np.sqrt(w)))
        di = self._t(np.diag(np.where(keep, 1.0 / np.sqrt(np.where(keep, w, 1.0)), 0.0)))
        x = tci.contract(c, tci.contract(c, u, "ac", ds, "cd", "ad"), "ad", uc, "bd", "ab")
        xi = tci.contract(c, tci.contract(c, u, "ac", di, "cd", "ad"), "ad", uc, "bd", "ab")
        return x, xi

    def _on_bond(self, i, pos, mat):
        lab = self._labels(i)
        out = [NEW if x == KET + pos else x for x in lab]
        return tci.contract(self.ctx, self.V[i], lab, mat, [KET + pos, NEW], out)

    def truncate_edge(self, i, j, chi: int, sv_cut: float = SV_CUT) -> np.ndarray:
        c = self.ctx
        X, Xi = self._sqrt_and_inv(self.M[(i, j)])
        Y, Yi = self._sqrt_and_inv(self.M[(j, i)])
        R = tci.contract(c, X, "ab", Y, "ac", "bc")
        u, s, vh = tci.svd(c, R, 1)
        sv = s.numpy().copy()
        k = max(1, min(chi, int(np.sum(sv > sv_cut * sv[0])) if sv[0] > 0 else 1))
        d = sv.shape[0]
        u = tci.extract_sub(c, u, [(0, d), (0, k)])
        vh = tci.extract_sub(c, vh, [(0, k), (0, d)])
        rs = self._t(np.diag(np.sqrt(sv[:k])))
        ai = tci.contract(c, tci.contract(c, Xi, "ba", u, "bk", "ak"), "ak", rs, "kl", "al")
        aj = tci.contract(c, tci.contract(c, Yi, "ba", vh, "kb", "ak"), "ak", rs, "kl", "al")
        vi = self._on_bond(i, self.nb[i].index(j), ai)
        vj = self._on_bond(j, self.nb[j].index(i), aj)
        self.V[i], self.V[j] = vi, vj
        return sv[:k]

    # ------------------------------------------------------------ gates
    def split_gate(self, gate):
        c = self.ctx
        g = self._t(np.asarray(gate).reshape(2, 2, 2, 2))
        m = tci.transpose(c, g, [0, 2, 1, 3])                 # [s_i, s_i', s_j, s_j']
        u, s, vh = tci.svd(c, m, 2)
        sv = s.numpy().copy()
        r = int(np.sum(sv > 1e-14 * sv[0]))
        u = tci.extract_sub(c, u, [(0, 2), (0, 2), (0, r)])
        vh = tci.extract_sub(c, vh, [(0, r), (0, 2), (0, 2)])
        rs = self._t(np.diag(np.sqrt(sv[:r])))
        oi = tci.contract(c, u, "abk", rs, "kl", "abl")
        oj = tci.contract(c, vh, "kab", rs, "kl", "abl")
        return oi, oj

    def apply_gate(self, i, j, gate):
        c = self.ctx
        oi, oj = self.split_gate(gate)
        for site, other, o in ((i, j, oi), (j, i, oj)):
            lab = self._labels(site)
            pos = self.nb[site].index(other)
            vin = [200 + 99] + lab[1:]                       # the old physical index
            out = [S_LABEL] + lab[1:2 + pos] + [GATE] + lab[2 + pos:]
            w = tci.contract(c, o, [S_LABEL, 299, GATE], self.V[site], vin, out)
            shp = list(w.shape())
            shp[1 + pos] = shp[1 + pos] * shp[2 + pos]
            del shp[2 + pos]
            self.V[site] = tci.reshape(c, w, shp)

    def apply_layer(self, gates: dict, chi: int, bp_iters: int, sv_cut: float = SV_CUT) -> dict:
        """Attach the gates ({(i, j): 4x4 matrix}), run bp_iters BP sweeps
        from identity messages, truncate every gated bond to chi; returns the
        kept singular values per bond."""
        for (i, j), g in gates.items():
            self.apply_gate(i, j, g)
        self.run_bp(bp_iters)
        return {e: self.truncate_edge(e[0], e[1], chi, sv_cut) for e in gates}
