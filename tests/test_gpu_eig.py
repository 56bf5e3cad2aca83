"""GPU parity of the general eigendecomposition (Spec, eig / eigvals) against
the CPU oracle: eigenvalues matched pairwise, eigenvectors of separated
eigenvalues compared under the fixed scaling, the eigen-equation residual,
all four dtypes, the Spec example's shapes and the error paths."""
import numpy as np
import pytest

from oracle import eig as oe

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    from paper_2512_23917_amd import tci
    return tci


@pytest.fixture(scope="module")
def ctx(T):
    c = T.Context(0)
    yield c
    c.close()


NP = {0: np.float32, 1: np.float64, 2: np.complex64, 3: np.complex128}


def matrix(n, dt, seed):
    g = np.random.default_rng(4000 + 7 * n + dt)
    a = g.standard_normal((n, n))
    if dt in (2, 3):
        a = a + 1j * g.standard_normal((n, n))
    return a.astype(NP[dt])


def pairing(w, ref):
    """For each reference eigenvalue the index of the nearest unused computed one."""
    free = list(range(len(w)))
    out = []
    for r in ref:
        j = min(free, key=lambda i: abs(w[i] - r))
        out.append(j)
        free.remove(j)
    return out


@pytest.mark.parametrize("n", [1, 2, 5, 64, 130])
@pytest.mark.parametrize("dt", [3, 1, 2, 0])
def test_eig_matches_oracle(T, ctx, n, dt):
    a = matrix(n, dt, 0)
    print(f"eig n={n} dtype={dt}", flush=True)
    wg, vg = T.eig(ctx, T.Tensor.from_numpy(ctx, a, dt), 1)
    w, v = wg.numpy(), vg.numpy().reshape(n, n)
    assert v.shape == (n, n) and w.shape == (n,)
    assert w.dtype == (np.complex128 if dt in (1, 3) else np.complex64)
    ref_w, ref_v = oe.eig_matrix(a.astype(np.complex128))       # the oracle on the rounded input
    scale = max(np.abs(ref_w).max(), 1e-300)
    tol = 1e-10 if dt in (1, 3) else 1e-6                       # single-precision outputs are rounded
    idx = pairing(w.astype(np.complex128), ref_w)
    assert max(abs(w[j] - r) for j, r in zip(idx, ref_w)) <= tol * scale
    keys = [(x.real, x.imag) for x in w]
    assert keys == sorted(keys)
    a64 = a.astype(np.complex128)
    v64 = v.astype(np.complex128)
    assert np.linalg.norm(a64 @ v64 - v64 * w.astype(np.complex128)[None, :]) <= tol * np.linalg.norm(a64) * max(n, 1)
    assert np.abs(np.linalg.norm(v64, axis=0) - 1).max() <= tol
    # eigenvectors of eigenvalues separated from all others by >= 1e-3 of the scale
    for i, j in enumerate(idx):
        gap = min([abs(ref_w[i] - ref_w[q]) for q in range(n) if q != i], default=np.inf)
        col = np.abs(ref_v[:, i])
        top2 = np.sort(col)[-2:] if n > 1 else col
        if gap < 1e-3 * scale or (n > 1 and top2[1] - top2[0] < 1e-6):
            continue
        assert np.abs(v64[:, j] - ref_v[:, i]).max() <= 1e3 * tol, (n, dt, i)


def test_eigvals_matches_eig_and_spec_example(T, ctx):
    g = np.random.default_rng(11)
    a = g.standard_normal((3, 4, 12))
    t = T.Tensor.from_numpy(ctx, a, T.F64)
    w = T.eigvals(ctx, t, 2).numpy()
    w2, v = T.eig(ctx, t, 2)
    assert w.shape == (12,) and tuple(v.shape()) == (3, 4, 12)
    assert np.array_equal(w, w2.numpy())
    ref = oe.eigvals(a, 2)
    idx = pairing(w, ref)
    assert max(abs(w[j] - r) for j, r in zip(idx, ref)) <= 1e-10 * np.abs(ref).max()


def test_eig_closed_forms(T, ctx):
    th = 0.7
    r = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    w = T.eigvals(ctx, T.Tensor.from_numpy(ctx, r, T.F64), 1).numpy()
    assert abs(w[0] - np.exp(-1j * th)) <= 1e-14 and abs(w[1] - np.exp(1j * th)) <= 1e-14
    tri = np.triu(np.random.default_rng(3).standard_normal((40, 40)))
    w = T.eigvals(ctx, T.Tensor.from_numpy(ctx, tri, T.F64), 1).numpy()
    assert np.abs(np.sort(w.real) - np.sort(np.diag(tri))).max() <= 1e-13 and np.abs(w.imag).max() == 0
    w, v = T.eig(ctx, T.Tensor.from_numpy(ctx, np.eye(6), T.C128), 1)
    assert np.all(w.numpy() == 1.0) and np.abs(v.numpy() - np.eye(6)).max() <= 1e-15


def test_eig_errors(T, ctx):
    with pytest.raises(T.TciError) as e:
        T.eig(ctx, T.Tensor.from_numpy(ctx, np.zeros((3, 4)), T.F64), 1)
    assert e.value.status == 2
    with pytest.raises(T.TciError) as e:
        T.eigvals(ctx, T.Tensor.from_numpy(ctx, np.zeros((4, 4)), T.F64), 2)
    assert e.value.status == 1
    with pytest.raises(T.TciError) as e:
        T.eigvals(ctx, T.Tensor.from_numpy(ctx, np.zeros((1025, 1025), dtype=np.float32), T.F32), 1)
    assert e.value.status == 9
