"""Seeded synthetic inputs for the two-site MPS update.

This module only *draws* inputs; it holds none of the update's arithmetic, so
both the GPU path and the CPU oracle can consume exactly the same arrays.
Everything is produced on the host in float64 / complex128 from
``numpy.random.Generator(PCG64(seed))`` and the caller rounds to the working
precision it needs.

Seeds: ``seed(config, update) = 251223917 + 1000 * config + update``.

Distributions
    complex Gaussian  (N(0,1) + i N(0,1)) / sqrt(2)
    real Gaussian     N(0,1)
    Haar unitary      QR of a Gaussian matrix with the phases of diag(R)
                      moved into Q (Mezzadri, Notices AMS 54, 2007); the real
                      orthogonal case uses the signs of diag(R).

Workloads (shapes follow the spin-1/2 chains the paper's applications use,
Sec. IV "Two representative TN applications"):
    * open MPS of N sites, d = 2, bond dims min(2^i, 2^(N-i), chi_cap);
    * dense two-site blocks A, B of shape (chi, 2, chi);
    * Heisenberg MPO of bond dimension 5 and Hermitian environments L, R of
      shape (chi, 5, chi) for the effective-Hamiltonian matvec;
    * matrices with prescribed singular values U diag(s) V^dagger (exponential
      or power-law spectra) so the exact truncation error is known.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 251223917


def seed(config: int, update: int = 0) -> int:
    return SEED_BASE + 1000 * int(config) + int(update)


def rng(config: int, update: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed(config, update)))


def complex_gaussian(g: np.random.Generator, shape) -> np.ndarray:
    re = g.standard_normal(shape)
    im = g.standard_normal(shape)
    return (re + 1j * im) / math.sqrt(2.0)


def real_gaussian(g: np.random.Generator, shape) -> np.ndarray:
    return g.standard_normal(shape)


def haar(g: np.random.Generator, rows: int, cols: int | None = None,
         complex_: bool = True) -> np.ndarray:
    """rows x cols matrix with Haar-distributed orthonormal columns (rows >= cols)."""
    cols = rows if cols is None else cols
    if complex_:
        z = complex_gaussian(g, (rows, cols))
    else:
        z = real_gaussian(g, (rows, cols))
    q, r = np.linalg.qr(z)
    d = np.diagonal(r).copy()
    ph = d / np.where(np.abs(d) > 0, np.abs(d), 1.0)
    ph = np.where(np.abs(d) > 0, ph, 1.0)
    return q * ph[None, :]


def haar_gate(g: np.random.Generator, d: int = 2, complex_: bool = True) -> np.ndarray:
    """Two-site gate as a (d*d, d*d) matrix, rows = outgoing (s1', s2')."""
    return haar(g, d * d, d * d, complex_)


# --------------------------------------------------------------------------
# Open MPS for the small sweep (N sites, d = 2, capped bond dimension)
# --------------------------------------------------------------------------
def open_mps_bond_dims(n_sites: int, d: int, chi_cap: int) -> list[int]:
    return [min(d ** i, d ** (n_sites - i), chi_cap) for i in range(n_sites + 1)]


def random_open_mps(g: np.random.Generator, n_sites: int = 16, d: int = 2,
                    chi_cap: int = 32) -> list[np.ndarray]:
    dims = open_mps_bond_dims(n_sites, d, chi_cap)
    return [complex_gaussian(g, (dims[i], d, dims[i + 1])) for i in range(n_sites)]


# --------------------------------------------------------------------------
# Matrices with a prescribed spectrum
# --------------------------------------------------------------------------
def exp_spectrum(n: int, scale: float = 200.0) -> np.ndarray:
    s = np.exp(-np.arange(n, dtype=np.float64) / scale)
    return s / np.linalg.norm(s)


def power_spectrum(n: int, alpha: float) -> np.ndarray:
    s = np.arange(1, n + 1, dtype=np.float64) ** (-float(alpha))
    return s / np.linalg.norm(s)


def two_site_blocks_from_spectrum(g: np.random.Generator, chi: int, d: int,
                                  s: np.ndarray, complex_: bool = True):
    """A (chi, d, k) = U diag(s) and B (k, d, chi) = V^dagger with k = len(s).

    U is (chi*d) x k and V is (d*chi) x k, both Haar; then the matricised
    product A.B = U diag(s) V^dagger has exactly the singular values s.
    """
    k = len(s)
    u = haar(g, chi * d, k, complex_)
    v = haar(g, d * chi, k, complex_)
    a = (u * s[None, :]).reshape(chi, d, k)
    b = v.conj().T.reshape(k, d, chi)
    return a, b


def isometry_pool(config: int, n_pool: int, rows: int, cols: int, complex_: bool = True) -> list:
    """n_pool Haar isometries rows x cols from the generator of (config, 0)."""
    g = rng(config, 0)
    return [haar(g, rows, cols, complex_) for _ in range(n_pool)]


def power_law_update(g: np.random.Generator, us: list, vs: list, chi: int, d: int = 2,
                     alpha_range=(1.0, 3.0)):
    """Inputs of one two-site update with a power-law bond: alpha ~ U[alpha_range],
    s_k ~ k^-alpha (k = 1..chi, unit 2-norm), A = U diag(s) as (chi, d, chi) and
    B = V^dagger as (chi, d, chi) with U, V drawn from the pools (Haar
    (chi d) x chi isometries), and a Haar two-site gate.
    Returns (alpha, s, A, B, gate)."""
    alpha = float(g.uniform(*alpha_range))
    s = power_spectrum(chi, alpha)
    i, j = (int(x) for x in g.integers(len(us), size=2))
    a = (us[i] * s[None, :]).reshape(chi, d, chi)
    b = vs[j].conj().T.reshape(chi, d, chi)
    return alpha, s, a, b, haar_gate(g, d)


def gaussian_two_site_blocks(g: np.random.Generator, chi: int, d: int = 2,
                             complex_: bool = True):
    if complex_:
        return complex_gaussian(g, (chi, d, chi)), complex_gaussian(g, (chi, d, chi))
    return real_gaussian(g, (chi, d, chi)), real_gaussian(g, (chi, d, chi))


# --------------------------------------------------------------------------
# Heisenberg chain: MPO (bond dimension 5) and Hermitian environments
# --------------------------------------------------------------------------
def heisenberg_mpo() -> np.ndarray:
    """W[w_l, w_r, s_out, s_in] of H = sum_i S_i . S_{i+1} (J = 1, spin 1/2).

    Channels (identity, S+, S-, Sz, H).  Lower-triangular convention:
    W[0,0]=I, W[1,0]=S+, W[2,0]=S-, W[3,0]=Sz,
    W[4,1]=S-/2, W[4,2]=S+/2, W[4,3]=Sz, W[4,4]=I.
    Physical basis index 0 = up, 1 = down.
    """
    eye = np.eye(2)
    sp = np.array([[0.0, 1.0], [0.0, 0.0]])
    sm = sp.T.copy()
    sz = np.diag([0.5, -0.5])
    w = np.zeros((5, 5, 2, 2), dtype=np.complex128)
    w[0, 0] = eye
    w[1, 0] = sp
    w[2, 0] = sm
    w[3, 0] = sz
    w[4, 1] = 0.5 * sm
    w[4, 2] = 0.5 * sp
    w[4, 3] = sz
    w[4, 4] = eye
    return w


def hermitian_environment(g: np.random.Generator, chi: int, complex_: bool = True,
                          left: bool = True) -> np.ndarray:
    """Environment E[a, w, a'] of shape (chi, 5, chi) that makes H_eff Hermitian.

    Channels pair up with the MPO: the slices for the self-adjoint channels
    (identity, Sz, H) are Hermitian matrices, and the S+ / S- channels carry
    mutually adjoint slices.  For the left environment W's S+ in row 1 meets
    L channel 1, so L_2 = L_1^dagger; the right environment mirrors it.
    """
    x = complex_gaussian(g, (5, chi, chi)) if complex_ else real_gaussian(g, (5, chi, chi))
    e = np.empty_like(x)
    for w in (0, 3, 4):
        e[w] = 0.5 * (x[w] + x[w].conj().T)
    e[1] = x[1]
    e[2] = x[1].conj().T
    return np.ascontiguousarray(e.transpose(1, 0, 2))


def trivial_environments():
    """chi = 1 environments that reduce H_eff to the two-site Heisenberg bond."""
    left = np.zeros((1, 5, 1), dtype=np.complex128)
    right = np.zeros((1, 5, 1), dtype=np.complex128)
    left[0, 4, 0] = 1.0
    right[0, 0, 0] = 1.0
    return left, right


# --------------------------------------------------------------------------
# U(1) block-sparse sector profiles
# --------------------------------------------------------------------------
def binomial_sector_sizes(total: int, n_sectors: int) -> list[int]:
    """Split `total` over `n_sectors` sectors following binomial(n_sectors-1, 1/2)
    weights: quotas w_k * total, floored and raised to at least 1, then the
    difference to `total` is given to (or, if negative, taken from sectors
    above 1 with) the largest (smallest) fractional parts, ties to the
    lower index."""
    n = n_sectors - 1
    w = np.array([math.comb(n, k) for k in range(n_sectors)], dtype=np.float64)
    w /= w.sum()
    if total < n_sectors:
        raise ValueError("total smaller than the number of sectors")
    quota = w * total
    fl = np.maximum(np.floor(quota).astype(np.int64), 1)
    frac = quota - np.floor(quota)
    rem = total - int(fl.sum())
    if rem > 0:
        order = np.argsort(-frac, kind="stable")
        fl[order[:rem]] += 1
    while rem < 0:
        cand = [k for k in np.argsort(frac, kind="stable") if fl[k] > 1]
        fl[cand[0]] -= 1
        rem += 1
    return [int(x) for x in fl]


def u1_bond(chi: int, n_sectors: int) -> list[tuple[int, int]]:
    """Bond of U(1) sectors: charges 2Sz = -(n_sectors-1), ..., n_sectors-1 in
    steps of 2 (even charges for an odd count, odd for an even count), sizes
    from binomial_sector_sizes."""
    dims = binomial_sector_sizes(chi, n_sectors)
    return [(2 * k - (n_sectors - 1), dims[k]) for k in range(n_sectors)]


U1_SPIN_CHARGE = (1, -1)   # physical index 0 = up, 1 = down


def u1_site_blocks(g: np.random.Generator, bl, br, complex_: bool = False) -> dict:
    """Gaussian blocks {(a, s, b): D_l[a] x D_r[b]} of a site tensor whose
    non-zero blocks satisfy q_r[b] = q_l[a] + charge(s)."""
    idx = {q: k for k, (q, _) in enumerate(br)}
    out = {}
    for a, (ql, dl) in enumerate(bl):
        for s, cs in enumerate(U1_SPIN_CHARGE):
            b = idx.get(ql + cs)
            if b is None:
                continue
            dr = br[b][1]
            out[(a, s, b)] = complex_gaussian(g, (dl, dr)) if complex_ else real_gaussian(g, (dl, dr))
    return out


def u1_gate(g: np.random.Generator) -> np.ndarray:
    """Charge-conserving two-site gate (4 x 4, rows = outgoing pair, real
    orthogonal): +-1 on up-up and down-down, a Haar 2 x 2 rotation on the
    (up-down, down-up) pair."""
    gm = np.zeros((4, 4))
    gm[0, 0] = 1.0 if g.standard_normal() >= 0 else -1.0
    gm[1:3, 1:3] = haar(g, 2, 2, complex_=False)
    gm[3, 3] = 1.0 if g.standard_normal() >= 0 else -1.0
    return gm
