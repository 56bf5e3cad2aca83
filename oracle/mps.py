"""Oracle for the two-site MPS update and the small open-chain sweep.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The update follows the paper's Application A listing (appendix
"Implementation of Application A using TCI") in TCI operations:
    theta = contract(A, B)                                   (site tensors)
    theta' = contract(theta, gate)                           (two-site gate)
    u, s, vh, err = trunc_svd(theta', 2, chi_min, chi_max, target, s_min)
    s <- s / ||s||_2                                         (normalize)
and then writes the factors back as new site tensors.  The gate convention
is rows = outgoing indices: theta'(a,s1',s2',b) = sum G[(s1' s2'),(s1 s2)]
theta(a,s1,s2,b).  (The paper's listing contracts the incoming legs with the
gate's row indices, which is the same thing for its symmetric gate; random
gates need the convention fixed.)
"""
from __future__ import annotations

import numpy as np

from . import contract, norm, qr, trunc_svd

LEFT, RIGHT, VIDAL = 0, 1, 2   # write-back direction


def theta_of(a, b):
    """theta(a, s1, s2, b) = sum_m A(a, s1, m) B(m, s2, b) (contraction eq.)."""
    return contract(a, "asm", b, "mtb", "astb")


def apply_gate(theta, gate):
    """theta'(a,u,v,b) = sum_{s,t} G[(u v),(s t)] theta(a,s,t,b)."""
    d = theta.shape[1]
    g4 = np.asarray(gate, dtype=np.complex128).reshape(d, d, d, d)
    return contract(theta, "astb", g4, "uvst", "auvb")


def two_site_update(a, b, gate=None, chi_min=1, chi_max=None, target=0.0, s_min=0.0,
                    direction=RIGHT, lam_left=None, lam_right=None):
    """One two-site update.  Returns dict with a_out, s, b_out, trunc_err, chi,
    theta (after the gate), discarded_abs.

    direction LEFT:  a_out = U,          b_out = diag(s) V^dagger
    direction RIGHT: a_out = U diag(s),  b_out = V^dagger
    direction VIDAL: a_out = diag(1/lam_left) U, b_out = V^dagger diag(1/lam_right)
    (the Gamma tensors of the Vidal form, as in the Application A listing).
    """
    theta = theta_of(a, b)
    if gate is not None:
        theta = apply_gate(theta, gate)
    chi_l, d1, d2, chi_r = theta.shape
    if chi_max is None:
        chi_max = min(chi_l * d1, d2 * chi_r)
    u, s, vh, err = trunc_svd(theta, 2, chi_min, chi_max, target, s_min)
    total = float(np.sum(np.abs(theta) ** 2))
    s_kept_norm = float(np.sqrt(np.sum(s * s)))
    s_n = s / s_kept_norm if s_kept_norm > 0 else s
    if direction == LEFT:
        a_out = u
        b_out = s_n[:, None, None] * vh
    elif direction == RIGHT:
        a_out = u * s_n[None, None, :]
        b_out = vh
    elif direction == VIDAL:
        a_out = u / np.asarray(lam_left)[:, None, None]
        b_out = vh / np.asarray(lam_right)[None, None, :]
    else:
        raise ValueError("direction")
    return dict(a_out=a_out, s=s_n, s_raw=s, b_out=b_out, trunc_err=err, chi=len(s),
                theta=theta, discarded_abs=err * total)


# --------------------------------------------------------------------------
# open chain: canonical form, sweep, exact state vector
# --------------------------------------------------------------------------
def left_canonicalize(mps):
    """QR left to right, R absorbed into the next site; last site normalised."""
    out = [np.asarray(t, dtype=np.complex128) for t in mps]
    for i in range(len(out) - 1):
        q, r = qr(out[i], 2)
        out[i] = q
        out[i + 1] = contract(r, "km", out[i + 1], "msb", "ksb")
    out[-1] = out[-1] / norm(out[-1])
    return out


def sweep_right_to_left(mps, gates, chi_max=32, target=1e-10, s_min=0.0):
    """Apply gates[i] on bonds (i, i+1) for i = n-2 ... 0 (centre moves left).

    Each step: theta, gate, trunc_svd(chi_min 1, chi_max, target, s_min),
    renormalise s, write back A = U diag(s), B = V^dagger.  Returns the new
    MPS and the list of truncation errors."""
    out = list(mps)
    errs = []
    for i in range(len(out) - 2, -1, -1):
        r = two_site_update(out[i], out[i + 1], gates[i], 1, chi_max, target, s_min, RIGHT)
        out[i], out[i + 1] = r["a_out"], r["b_out"]
        errs.append(r["trunc_err"])
    return out, errs


def state_vector(mps):
    """Contract an open MPS (boundary dims 1) into the full 2^N amplitude vector."""
    psi = np.asarray(mps[0], dtype=np.complex128)[0]          # (d, D1)
    for t in mps[1:]:
        t = np.asarray(t, dtype=np.complex128)
        psi = np.tensordot(psi, t, axes=([psi.ndim - 1], [0]))
    return psi.reshape(-1)


def exact_gate_evolution(psi, n_sites, gates, d=2):
    """Apply gates[i] on sites (i, i+1) for i = n-2 ... 0 to a state vector."""
    psi = psi.reshape((d,) * n_sites)
    for i in range(n_sites - 2, -1, -1):
        g4 = np.asarray(gates[i]).reshape(d, d, d, d)
        psi = np.tensordot(g4, psi, axes=([2, 3], [i, i + 1]))
        psi = np.moveaxis(psi, [0, 1], [i, i + 1])
    return psi.reshape(-1)
