"""Oracle for the U(1) block-sparse two-site update.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The conserved quantity is the total 2 S^z.  A bond is a list of sectors
(charge q, dimension D).  The physical index carries the charges +1 (index 0,
spin up) and -1 (index 1, spin down).  A site tensor M[(q_l, i), s, (q_r, j)]
is non-zero only in the blocks with q_r = q_l + s (charge flows from left to
right), stored as a dict {(a, s, b): D_l[a] x D_r[b] array} over sector
indices a, b.  This is the symmetric-tensor form that the paper names as the
natural extension of its dense interface (Sec. V, future work); the update
below is the block form of the dense two-site update.

    theta(a, s1, s2, b) = A[a, s1, m] B[m, s2, b]      (m the sector q_l + s1)
    theta'(a, s1', s2', b) = sum over s1 + s2 = s1' + s2' of
                             G[(s1' s2'), (s1 s2)] theta(a, s1, s2, b)
    sector Q of the new bond: rows (a, i, s1') with q_l[a] + s1' = Q in the
        order of the dense row index (a, i), columns (s2', b, j) with
        q_r[b] - s2' = Q in the order of the dense column index (s2', b, j)
    one SVD per sector; all singular values merged in descending order (ties:
        sector charge ascending, then in-sector index) and cut once by the
        truncation rule (Spec, trunc_svd) with the total weight
        W = sum of all squared singular values; s renormalised over the kept set.

The pin is the dense embedding (tests/test_oracle_u1.py): the same update of
the dense tensors gives the same multiset of singular values, the same chi
and truncation error, and the same truncated two-site tensor.
"""
from __future__ import annotations

import numpy as np

from . import svd_matrix, trunc_rule

SPIN_CHARGE = (1, -1)   # physical index 0 = up (+1), 1 = down (-1)


def offsets(bond):
    out, acc = [], 0
    for _, dim in bond:
        out.append(acc)
        acc += dim
    return out, acc


def allowed_blocks(bl, br):
    """(a, s, b) with q_r[b] = q_l[a] + charge(s)."""
    idx = {q: k for k, (q, _) in enumerate(br)}
    out = []
    for a, (ql, _) in enumerate(bl):
        for s, cs in enumerate(SPIN_CHARGE):
            b = idx.get(ql + cs)
            if b is not None:
                out.append((a, s, b))
    return out


def dense_site(blocks, bl, br):
    ol, nl = offsets(bl)
    orr, nr = offsets(br)
    m = np.zeros((nl, 2, nr), dtype=np.complex128)
    for (a, s, b), blk in blocks.items():
        m[ol[a]:ol[a] + bl[a][1], s, orr[b]:orr[b] + br[b][1]] = blk
    return m


def sector_layout(bl, br):
    """For every new-bond charge Q: row pieces [(a, s1')] and column pieces [(s2', b)]."""
    rows, cols = {}, {}
    for a, (ql, _) in enumerate(bl):
        for s1, c1 in enumerate(SPIN_CHARGE):
            rows.setdefault(ql + c1, []).append((a, s1))
    for s2, c2 in enumerate(SPIN_CHARGE):
        for b, (qr, _) in enumerate(br):
            cols.setdefault(qr - c2, []).append((s2, b))
    qs = sorted(set(rows) & set(cols))
    return [(q, rows[q], cols[q]) for q in qs]


def theta_blocks(A, B, bl, bm, br):
    """theta[(a, s1, s2, b)] = A[a, s1, m] B[m, s2, b], one plain product per block."""
    im = {q: k for k, (q, _) in enumerate(bm)}
    ib = {q: k for k, (q, _) in enumerate(br)}
    out = {}
    for (a, s1, m), ablk in A.items():
        assert bm[m][0] == bl[a][0] + SPIN_CHARGE[s1]
        for s2, c2 in enumerate(SPIN_CHARGE):
            b = ib.get(bm[m][0] + c2)
            if b is None or (m, s2, b) not in B:
                continue
            assert im[bm[m][0]] == m
            key = (a, s1, s2, b)
            prod = np.asarray(ablk, dtype=np.complex128) @ np.asarray(B[(m, s2, b)], dtype=np.complex128)
            out[key] = out.get(key, 0) + prod
    return out


def gate_blocks(theta, gate):
    """theta'(a, u, v, b) = sum_{s, t} G[(u v), (s t)] theta(a, s, t, b) (charge-conserving G)."""
    g = np.asarray(gate, dtype=np.complex128).reshape(2, 2, 2, 2)
    out = {}
    for (a, s, t, b), blk in theta.items():
        for u in range(2):
            for v in range(2):
                c = g[u, v, s, t]
                if c == 0:
                    continue
                assert SPIN_CHARGE[u] + SPIN_CHARGE[v] == SPIN_CHARGE[s] + SPIN_CHARGE[t]
                key = (a, u, v, b)
                out[key] = out.get(key, 0) + c * blk
    return out


def sector_matrix(thp, bl, br, rows, cols):
    """Dense matrix of one sector from its (a, s1') row pieces and (s2', b) column pieces."""
    nr = sum(bl[a][1] for a, _ in rows)
    nc = sum(br[b][1] for _, b in cols)
    m = np.zeros((nr, nc), dtype=np.complex128)
    r0 = 0
    for a, s1 in rows:
        c0 = 0
        for s2, b in cols:
            blk = thp.get((a, s1, s2, b))
            if blk is not None:
                m[r0:r0 + bl[a][1], c0:c0 + br[b][1]] = blk
            c0 += br[b][1]
        r0 += bl[a][1]
    return m


def block_update(A, B, bl, bm, br, gate=None, chi_min=1, chi_max=None, target=0.0, s_min=0.0):
    """Returns dict: sectors [(Q, rows, cols, u_kept, s_kept, vh_kept)], s (all kept,
    merged order, renormalised), chi, trunc_err, total, discarded_abs."""
    th = theta_blocks(A, B, bl, bm, br)
    if gate is not None:
        th = gate_blocks(th, gate)
    layout = sector_layout(bl, br)
    svals = []   # (sigma, Q, j)
    facts = {}
    total = 0.0
    for q, rows, cols in layout:
        m = sector_matrix(th, bl, br, rows, cols)
        if m.size == 0:
            continue
        total += float(np.sum(np.abs(m) ** 2))
        u, s, vh = svd_matrix(m)
        facts[q] = (rows, cols, u, s, vh)
        svals += [(float(s[j]), q, j) for j in range(len(s))]
    svals.sort(key=lambda e: (-e[0], e[1], e[2]))
    merged = np.array([e[0] for e in svals])
    if chi_max is None:
        chi_max = len(merged)
    chi, err = trunc_rule(merged, chi_min, chi_max, target, s_min)
    kept = {}
    for _, q, j in svals[:chi]:
        kept[q] = kept.get(q, 0) + 1
    nrm = float(np.sqrt(np.sum(merged[:chi] ** 2)))
    sectors = []
    for q in sorted(kept):
        rows, cols, u, s, vh = facts[q]
        k = kept[q]
        sectors.append((q, rows, cols, u[:, :k], s[:k] / nrm if nrm > 0 else s[:k], vh[:k, :]))
    return dict(sectors=sectors, s=merged[:chi] / nrm if nrm > 0 else merged[:chi], chi=chi, trunc_err=err,
                total=total, discarded_abs=err * total)


def truncated_theta_dense(res, bl, br):
    """Dense (sum D_l, 2, 2, sum D_r) tensor U s V^dagger of the kept sectors (renormalised s)."""
    ol, nl = offsets(bl)
    orr, nr = offsets(br)
    out = np.zeros((nl, 2, 2, nr), dtype=np.complex128)
    for q, rows, cols, u, s, vh in res["sectors"]:
        m = (u * s[None, :]) @ vh
        r0 = 0
        for a, s1 in rows:
            c0 = 0
            for s2, b in cols:
                out[ol[a]:ol[a] + bl[a][1], s1, s2, orr[b]:orr[b] + br[b][1]] = \
                    m[r0:r0 + bl[a][1], c0:c0 + br[b][1]]
                c0 += br[b][1]
            r0 += bl[a][1]
    return out
