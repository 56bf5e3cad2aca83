"""Shared helpers for the GPU parity tests (comparison metrics only)."""
import numpy as np


def rel_fro(x, ref):
    x = np.asarray(x)
    ref = np.asarray(ref)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / (den if den > 0 else 1.0))


def gauge_ok_columns(s, tol=1e-6):
    """Indices i whose singular value is separated from its neighbours by a
    relative gap >= tol (so u_i and v_i are unique up to the fixed phase)."""
    s = np.asarray(s)
    if len(s) == 0:
        return []
    s1 = s[0] if s[0] > 0 else 1.0
    ok = []
    for i in range(len(s)):
        lo = s[i - 1] - s[i] if i > 0 else np.inf
        hi = s[i] - s[i + 1] if i + 1 < len(s) else np.inf
        if min(lo, hi) / s1 >= tol:
            ok.append(i)
    return ok


def isometry_err(u, axis_cols=True):
    u = np.asarray(u)
    m = u.reshape(-1, u.shape[-1]) if axis_cols else u.reshape(u.shape[0], -1)
    g = m.conj().T @ m if axis_cols else m @ m.conj().T
    return float(np.abs(g - np.eye(g.shape[0])).max())


def chi_allowed(chi, chi_ref, s_kept_raw, total, err_ref, target, chi_max, rel=1e-3):
    """Kept bond dimensions a mixed-precision path may return next to the
    oracle's chi_ref: chi_ref itself; chi_ref - 1 only when the oracle's
    eps(chi_ref - 1) lies within a factor 1 + rel of the target (the last
    kept value sits on the threshold); chi_ref + 1 only when eps(chi_ref)
    lies within 1 - rel of it and the cap allows it.  s_kept_raw: the oracle's
    kept values before renormalisation, total: ||theta||_F^2, err_ref: the
    oracle's relative truncation error eps(chi_ref)."""
    ok = {chi_ref}
    if chi_ref >= 2 and target > 0:
        e_prev = err_ref + float(s_kept_raw[chi_ref - 1]) ** 2 / total
        if e_prev <= target * (1 + rel):
            ok.add(chi_ref - 1)
    if chi_ref < chi_max and target > 0 and err_ref >= target * (1 - rel):
        ok.add(chi_ref + 1)
    return chi in ok
