"""Pins of the general eigendecomposition oracle (Spec, eig / eigvals):
LAPACK's eigenvalues (the oracle runs its own Hessenberg + shifted QR), the
eigen-equation residual, closed forms (triangular, rotation, companion
matrix of known roots, similarity transforms of a known spectrum), Hermitian
input against LAPACK's Hermitian solver, and the Spec example's shapes."""
import numpy as np
import pytest

from oracle import eig as oe


def match(w, ref):
    """Max distance after pairing each reference eigenvalue with the nearest
    unused computed one (conjugate pairs of real matrices may come in either order)."""
    w = list(np.asarray(w))
    worst = 0.0
    for r in np.asarray(ref):
        j = int(np.argmin([abs(x - r) for x in w]))
        worst = max(worst, abs(w[j] - r))
        w.pop(j)
    return worst


@pytest.mark.parametrize("n", [1, 2, 3, 7, 24])
@pytest.mark.parametrize("cplx", [True, False])
def test_eigenvalues_match_lapack_and_residual(n, cplx):
    g = np.random.default_rng(100 + n)
    a = g.standard_normal((n, n)) + (1j * g.standard_normal((n, n)) if cplx else 0)
    w, v = oe.eig_matrix(a)
    scale = np.linalg.norm(a)
    assert match(w, np.linalg.eigvals(a)) <= 1e-12 * scale
    assert np.linalg.norm(a @ v - v * w[None, :]) <= 1e-13 * scale * n
    assert np.abs(np.linalg.norm(v, axis=0) - 1).max() <= 1e-14
    for k in range(n):
        j = int(np.argmax(np.abs(v[:, k])))
        assert abs(v[j, k].imag) <= 1e-15 and v[j, k].real > 0


def test_order_ascending_real_then_imaginary():
    g = np.random.default_rng(5)
    w, _ = oe.eig_matrix(g.standard_normal((12, 12)) + 1j * g.standard_normal((12, 12)))
    keys = [(x.real, x.imag) for x in w]
    assert keys == sorted(keys)


def test_triangular_gives_its_diagonal():
    g = np.random.default_rng(6)
    t = np.triu(g.standard_normal((9, 9)) + 1j * g.standard_normal((9, 9)))
    w, v = oe.eig_matrix(t)
    assert match(w, np.diag(t)) <= 1e-14
    assert np.linalg.norm(t @ v - v * w[None, :]) <= 1e-13 * np.linalg.norm(t)


def test_rotation_closed_form():
    th = 0.7
    r = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    w, v = oe.eig_matrix(r)
    assert abs(w[0] - np.exp(-1j * th)) <= 1e-15 and abs(w[1] - np.exp(1j * th)) <= 1e-15
    # eigenvectors (1, +-i)/sqrt(2) up to the fixed phase
    assert abs(abs(v[0, 0]) - 2 ** -0.5) <= 1e-15 and abs(abs(v[1, 0]) - 2 ** -0.5) <= 1e-15


def test_companion_matrix_of_known_roots():
    roots = np.array([1.0, 2.0, 3.0, -4.0, 1 + 1j, 1 - 1j, 0.5j])
    c = np.poly(roots)                      # monic coefficients, highest first
    n = len(roots)
    comp = np.zeros((n, n), dtype=np.complex128)
    comp[0, :] = -c[1:]
    comp[1:, :-1] = np.eye(n - 1)
    w, v = oe.eig_matrix(comp)
    assert match(w, roots) <= 1e-9
    assert np.linalg.norm(comp @ v - v * w[None, :]) <= 1e-12 * np.linalg.norm(comp)


def test_similarity_of_a_known_spectrum():
    g = np.random.default_rng(7)
    lam = np.array([3.0, -1.0 + 2j, 0.25, 5j, -2.5, 1.5 - 0.5j])
    q, _ = np.linalg.qr(g.standard_normal((6, 6)) + 1j * g.standard_normal((6, 6)))
    s = q @ np.diag([1.0, 2.0, 0.5, 1.5, 1.0, 3.0]) @ q.conj().T     # well-conditioned, not unitary
    a = s @ np.diag(lam) @ np.linalg.inv(s)
    w, v = oe.eig_matrix(a)
    assert match(w, lam) <= 1e-13 * np.linalg.norm(a)
    # A = V diag(w) V^-1
    assert np.linalg.norm(v @ np.diag(w) @ np.linalg.inv(v) - a) <= 1e-12 * np.linalg.norm(a)


def test_hermitian_input_gives_lapack_hermitian_spectrum():
    g = np.random.default_rng(8)
    h = g.standard_normal((10, 10)) + 1j * g.standard_normal((10, 10))
    h = h + h.conj().T
    w, v = oe.eig_matrix(h)
    assert np.abs(w.imag).max() <= 1e-13 * np.linalg.norm(h)
    assert np.abs(w.real - np.linalg.eigvalsh(h)).max() <= 1e-13 * np.linalg.norm(h)
    assert np.abs(v.conj().T @ v - np.eye(10)).max() <= 1e-13


def test_repeated_eigenvalue_identity():
    w, v = oe.eig_matrix(np.eye(4))
    assert np.all(w == 1.0)
    assert np.abs(v - np.eye(4)).max() <= 1e-15


def test_spec_example_shapes():
    g = np.random.default_rng(9)
    a = g.standard_normal((3, 4, 12))
    w = oe.eigvals(a, 2)
    assert w.shape == (12,) and w.dtype == np.complex128
    w2, v = oe.eig(a, 2)
    assert v.shape == (3, 4, 12)
    m = a.reshape(12, 12)
    vm = v.reshape(12, 12)
    assert np.linalg.norm(m @ vm - vm * w2[None, :]) <= 1e-13 * np.linalg.norm(m) * 12
    assert np.array_equal(w, w2)
