"""CPU FP64 oracle for the belief-propagation (BP) update of a tensor-network
state on a graph: App. B (the TNO-TNS update with BP regauging and
message-SVD truncation).

TEST INFRASTRUCTURE ONLY: the test-suite is the only caller; the GPU library
never imports this module and this module never imports the GPU library.

Conventions (shared by the GPU driver only through this description):
  * graph: sites 0..n-1, undirected edges (i, j) with i < j; the bonds of a
    site are ordered by the index of the neighbour;
  * site tensor V_i has indices [s, b_1, ..., b_deg] (s physical, dim 2),
    complex128;
  * message M_{i->j}[a, a'] is the environment of bond (i, j) seen from i's
    side: a is the ket index, a' the bra index; Hermitian and positive
    semi-definite, normalised to unit trace;
  * BP update (App. B, fixed-point relation of the messages): M_{i->j} is
    the contraction of V_i, conj(V_i) and the messages M_{k->i} of every
    other neighbour k of i, with the physical index traced; one sweep
    updates every directed edge from the messages of the previous sweep
    (parallel schedule);
  * regauge and truncation of edge (i, j) (App. B, square-root messages and
    the SVD of the message tensors): X = M_{i->j}^{1/2}, Y = M_{j->i}^{1/2}
    (Hermitian square roots from the eigendecomposition), R = X^T Y =
    U S V^H, keep the chi largest s, then on the shared bond
        V_i <- V_i . X^{-T} U_chi S_chi^{1/2},
        V_j <- V_j . Y^{-T} conj(V_chi) S_chi^{1/2},
    so that (X^{-T} U S^{1/2})(Y^{-T} conj(V) S^{1/2})^T = X^{-T} R Y^{-1} = I
    when nothing is cut.  Two thresholds follow from the FP64 arithmetic
    of these steps (the paper fixes neither):
      - the messages come out of sums of products, so their entries carry
        relative rounding of about 10 u (u = 2^-53) and, by Weyl's bound,
        their eigenvalues an absolute error delta ~ 10 u w_max; the inverse
        square root turns it into a relative error delta / (2 w), so only
        the eigen-directions with w > INV_SQRT_CUT * w_max = 1e-10 w_max
        are inverted, where that error stays below about 5e-6;
      - R = X^T Y carries an absolute rounding of about u ||X|| ||Y||,
        and the regauged bond X^{-T} R Y^{-1} multiplies it by
        ||X^{-1}|| ||Y^{-1}||, up to INV_SQRT_CUT^-1 = 1e10 relative to the
        largest scale: rounding can reach 1e10 u ~ 1e-6 of s_0 there.  A
        singular value of R below SV_CUT * s_0 = 1e-6 s_0 is therefore not a
        bond direction that FP64 resolves after the regauging, and is cut
        (the relative form of trunc_svd's rule (a), s_i < s_min, with
        s_min = SV_CUT * s_0).  sv_cut is an argument, so a caller can ask
        for a smaller floor;
  * a two-site gate G[s_i, s_j, s_i', s_j'] on edge (i, j) enters as a
    tensor-network operator: G reshaped (s_i s_i') x (s_j s_j') is split by
    an SVD into O_i[s_i, s_i', k] (U sqrt(S)) and O_j[s_j, s_j', k]
    (sqrt(S) V^H), and O_i, O_j are contracted into V_i, V_j with the gate
    bond k merged into the bond (i, j) as its faster index.
"""
from __future__ import annotations

import numpy as np

INV_SQRT_CUT = 1e-10   # message eigenvalues kept by the inverse square root (relative)
SV_CUT = 1e-6          # default floor of the singular values of R kept as bond directions (relative)


# ------------------------------------------------------------------ graphs
def heavy_hex_patch():
    """One heavy hexagon (6 corner sites, 6 edge-midpoint sites on a 12-site
    ring) with a pendant site on three alternate corners: 15 sites, 15
    edges, one loop; degrees 1, 2 and 3 as on a heavy-hex device."""
    ring = list(range(12))                       # even: corners, odd: midpoints
    edges = [(ring[k], ring[(k + 1) % 12]) for k in range(12)]
    pend = {0: 12, 4: 13, 8: 14}
    edges += [(c, p) for c, p in pend.items()]
    return 15, sorted(tuple(sorted(e)) for e in edges)


def neighbours(n, edges):
    nb = [[] for _ in range(n)]
    for i, j in edges:
        nb[i].append(j)
        nb[j].append(i)
    return [sorted(x) for x in nb]


def product_state(n, edges, seed=0):
    """Random product state with bond dimension 1 on every edge."""
    g = np.random.default_rng(seed)
    nb = neighbours(n, edges)
    out = []
    for i in range(n):
        v = g.standard_normal(2) + 1j * g.standard_normal(2)
        out.append((v / np.linalg.norm(v)).reshape((2,) + (1,) * len(nb[i])))
    return out


# ------------------------------------------------------------------ exact contraction
def state_vector(n, edges, V):
    """Contract the whole network into the 2^n amplitudes (site 0 slowest)."""
    nb = neighbours(n, edges)
    letters = iter("ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz")
    phys = [next(letters) for _ in range(n)]
    bond = {e: next(letters) for e in edges}
    subs = [phys[i] + "".join(bond[tuple(sorted((i, k)))] for k in nb[i]) for i in range(n)]
    expr = ",".join(subs) + "->" + "".join(phys)
    return np.einsum(expr, *V, optimize="greedy").reshape(-1)


# ------------------------------------------------------------------ BP messages
def init_messages(n, edges, V):
    nb = neighbours(n, edges)
    M = {}
    for i in range(n):
        for pos, j in enumerate(nb[i]):
            d = V[i].shape[1 + pos]
            M[(i, j)] = np.eye(d, dtype=np.complex128) / d
    return M


def message(i, j, V, M, nb):
    """App. B fixed-point relation: M_{i->j} from V_i, conj(V_i) and the
    messages into i from its other neighbours, normalised to unit trace."""
    v = V[i]
    deg = len(nb[i])
    letters = "abcdefgh"
    primes = "ABCDEFGH"
    ket = "s" + letters[:deg]
    bra = "s" + primes[:deg]
    subs, ops = [ket, bra], [v, np.conj(v)]
    out = ""
    for pos, k in enumerate(nb[i]):
        if k == j:
            out = letters[pos] + primes[pos]
            continue
        subs.append(letters[pos] + primes[pos])
        ops.append(M[(k, i)])
    m = np.einsum(",".join(subs) + "->" + out, *ops)
    return m / np.trace(m)


def bp_sweep(n, edges, V, M):
    nb = neighbours(n, edges)
    return {(i, j): message(i, j, V, M, nb) for (i, j) in M}


def bp_run(n, edges, V, iters=None, tol=1e-12, max_iters=200):
    """Parallel BP sweeps from identity messages: a fixed number of sweeps,
    or until the largest change of a message is below tol."""
    M = init_messages(n, edges, V)
    done = 0
    while True:
        if iters is not None and done >= iters:
            return M, done
        Mn = bp_sweep(n, edges, V, M)
        delta = max(np.abs(Mn[k] - M[k]).max() for k in M)
        M = Mn
        done += 1
        if iters is None and (delta < tol or done >= max_iters):
            return M, done


def bp_norm(n, edges, V, M):
    """BP estimate of <psi|psi>: product of the site contractions with all
    incoming messages over the product of the edge overlaps
    Tr(M_{i->j} M_{j->i}^T); exact on trees."""
    nb = neighbours(n, edges)
    z = 1.0 + 0.0j
    letters, primes = "abcdefgh", "ABCDEFGH"
    for i in range(n):
        deg = len(nb[i])
        subs = ["s" + letters[:deg], "s" + primes[:deg]] + [letters[p] + primes[p] for p in range(deg)]
        ops = [V[i], np.conj(V[i])] + [M[(k, i)] for k in nb[i]]
        z *= np.einsum(",".join(subs) + "->", *ops)
    for i, j in edges:
        z /= np.sum(M[(i, j)] * M[(j, i)])
    return z


# ------------------------------------------------------------------ regauge + truncation
def _sqrt_and_inv(m):
    m = 0.5 * (m + m.conj().T)
    w, u = np.linalg.eigh(m)
    w = np.clip(w, 0.0, None)
    keep = w > INV_SQRT_CUT * w.max()
    sq = (u * np.sqrt(w)) @ u.conj().T
    inv = (u[:, keep] / np.sqrt(w[keep])) @ u[:, keep].conj().T
    return sq, inv


def _apply_on_bond(v, pos, mat):
    """v[..., a (bond pos), ...] -> sum_a v[..., a, ...] mat[a, c]."""
    axis = 1 + pos
    out = np.tensordot(v, mat, axes=([axis], [0]))
    return np.moveaxis(out, -1, axis)


def truncate_edge(i, j, V, M, nb, chi, sv_cut=SV_CUT):
    """App. B message-SVD truncation of bond (i, j): at most chi values,
    none below sv_cut * s_0; returns the kept singular values (descending)
    and updates V_i, V_j in place."""
    X, Xi = _sqrt_and_inv(M[(i, j)])
    Y, Yi = _sqrt_and_inv(M[(j, i)])
    R = X.T @ Y
    u, s, vh = np.linalg.svd(R)
    k = min(chi, int(np.sum(s > sv_cut * s[0])) if s[0] > 0 else 1)
    k = max(k, 1)
    u, s, vh = u[:, :k], s[:k], vh[:k]
    rs = np.sqrt(s)
    V[i] = _apply_on_bond(V[i], nb[i].index(j), Xi.T @ u * rs)
    V[j] = _apply_on_bond(V[j], nb[j].index(i), Yi.T @ vh.T * rs)
    return s


# ------------------------------------------------------------------ gates as operators
def split_gate(gate):
    """G[s_i, s_j, s_i', s_j'] -> O_i[s_i, s_i', k], O_j[s_j, s_j', k]."""
    g = np.asarray(gate, dtype=np.complex128).reshape(2, 2, 2, 2)
    m = g.transpose(0, 2, 1, 3).reshape(4, 4)          # (s_i s_i') x (s_j s_j')
    u, s, vh = np.linalg.svd(m)
    r = int(np.sum(s > 1e-14 * s[0]))
    rs = np.sqrt(s[:r])
    oi = (u[:, :r] * rs).reshape(2, 2, r)
    oj = (vh[:r].T * rs).reshape(2, 2, r)
    return oi, oj


def apply_gate_operator(i, j, gate, V, nb):
    """Contract the split gate into V_i and V_j; the gate bond becomes the
    faster half of the merged bond (i, j)."""
    oi, oj = split_gate(gate)
    for site, other, o in ((i, j, oi), (j, i, oj)):
        v = V[site]
        pos = nb[site].index(other)
        w = np.tensordot(o, v, axes=([1], [0]))          # [s, k, s', ...] -> [s, k, b...]
        w = np.moveaxis(w, 1, 1 + 1 + pos)               # k right after bond pos
        shp = list(w.shape)
        shp[1 + pos] = shp[1 + pos] * shp[2 + pos]
        del shp[2 + pos]
        V[site] = w.reshape(shp)


def apply_layer(n, edges, V, gates, chi, bp_iters, sv_cut=SV_CUT):
    """One TNO layer (App. B): attach the gates of `gates` ({edge: 4x4x...}),
    converge BP with a fixed number of sweeps, then truncate every gated
    bond to chi.  Returns the BP messages used and the kept spectra."""
    nb = neighbours(n, edges)
    for (i, j), g in gates.items():
        apply_gate_operator(i, j, g, V, nb)
    M, _ = bp_run(n, edges, V, iters=bp_iters)
    spectra = {}
    for (i, j) in gates:
        spectra[(i, j)] = truncate_edge(i, j, V, M, nb, chi, sv_cut)
    return M, spectra


def apply_gate_statevector(psi, n, i, j, gate):
    """Exact two-site gate on the 2^n amplitudes (site 0 slowest)."""
    g = np.asarray(gate, dtype=np.complex128).reshape(2, 2, 2, 2)
    t = psi.reshape((2,) * n)
    t = np.tensordot(g, t, axes=([2, 3], [i, j]))
    t = np.moveaxis(t, [0, 1], [i, j])
    return t.reshape(-1)
