"""Pins for the sub-tensor, construction and matrix-function oracle: the
paper's printed examples, brute-force loops over coordinates, closed forms of
the exponential, and LAPACK (through numpy and scipy) special cases."""
import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import subtensor as st
from paper_2512_23917_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


EX = _gold("paper_examples.json")


def cg(seed, shape):
    return synth.complex_gaussian(np.random.default_rng(seed), shape)


# ---------------------------------------------------------------- construction
def test_eye_and_fill_paper_examples():
    ex = EX["eye"]
    e = st.eye(ex["n"])
    for coord, v in ex["checks"]:
        assert e[tuple(coord)] == v
    assert np.array_equal(e, np.eye(ex["n"]))
    ex = EX["fill"]
    f = st.fill(ex["shape"], ex["value"])
    assert list(f.shape) == ex["shape"] and f[tuple(ex["coord"])] == ex["expected"]
    assert np.all(f == ex["value"])


# ---------------------------------------------------------------- expand / shrink
def test_expand_paper_example_and_zero_padding():
    ex = EX["expand"]
    a = cg(1, ex["shape"])
    out = st.expand(a, {b: inc for b, inc in ex["increments"]})
    assert list(out.shape) == ex["expected_shape"]
    assert out[tuple(ex["zero_coord"])] == 0
    # brute force: an element is kept iff every coordinate is inside the old bounds
    for c in itertools.product(*[range(d) for d in out.shape]):
        inside = all(ci < di for ci, di in zip(c, a.shape))
        assert out[c] == (a[c] if inside else 0)


def test_shrink_paper_example_and_coordinates():
    ex = EX["shrink"]
    a = cg(2, ex["shape"])
    ranges = {b: tuple(r) for b, r in ex["ranges"]}
    out = st.shrink(a, ranges)
    assert list(out.shape) == ex["expected_shape"]
    assert out[tuple(ex["coord_after"])] == a[tuple(ex["coord_before"])]
    first = [ranges.get(b, (0, d))[0] for b, d in enumerate(a.shape)]
    for c in itertools.product(*[range(d) for d in out.shape]):
        assert out[c] == a[tuple(ci + fi for ci, fi in zip(c, first))]


def test_expand_then_shrink_is_identity():
    a = cg(3, (3, 5, 2))
    big = st.expand(a, {0: 2, 2: 3})
    assert np.array_equal(st.shrink(big, {0: (0, 3), 2: (0, 2)}), a)


# ---------------------------------------------------------------- extract / replace
def test_extract_sub_paper_example():
    ex = EX["extract_sub"]
    a = cg(4, ex["shape"])
    sub = st.extract_sub(a, ex["ranges"])
    assert sub.shape == tuple(l - f for f, l in ex["ranges"])
    assert sub[tuple(ex["coord_after"])] == a[tuple(ex["coord_before"])]


def test_replace_sub_paper_example_and_untouched_rest():
    ex = EX["replace_sub"]
    a = np.zeros(ex["shape"], dtype=np.complex128)
    sub = cg(5, ex["sub_shape"])
    out = st.replace_sub(a, sub, ex["begin"])
    assert out[tuple(ex["coord_in"])] == sub[tuple(ex["coord_sub"])]
    for c in itertools.product(*[range(d) for d in out.shape]):
        rel = [ci - bi for ci, bi in zip(c, ex["begin"])]
        inside = all(0 <= r < d for r, d in zip(rel, sub.shape))
        assert out[c] == (sub[tuple(rel)] if inside else 0)


def test_replace_then_extract_round_trip():
    a = cg(6, (4, 6, 3))
    sub = cg(7, (2, 3, 3))
    out = st.replace_sub(a, sub, (1, 2, 0))
    assert np.array_equal(st.extract_sub(out, [(1, 3), (2, 5), (0, 3)]), sub)


@pytest.mark.parametrize("bad", [[(0, 4), (0, 4), (0, 2)], [(2, 1), (0, 4), (0, 2)], [(0, 3), (0, 4)]])
def test_extract_sub_rejects_bad_ranges(bad):
    with pytest.raises(ValueError):
        st.extract_sub(np.zeros((3, 4, 2)), bad)


# ---------------------------------------------------------------- concatenate / stack
def test_concatenate_paper_example_and_numpy():
    ex = EX["concatenate"]
    ins = [cg(10 + k, ex["shape"]) for k in range(ex["n"])]
    out = st.concatenate(ins, ex["bond"])
    assert list(out.shape) == ex["expected_shape"]
    assert out[tuple(ex["coord_out"])] == ins[ex["input"]][tuple(ex["coord_in"])]
    assert np.array_equal(out, np.concatenate(ins, axis=ex["bond"]))
    three = [cg(10 + k, ex["shape"]) for k in range(ex["n_printed"])]
    assert list(st.concatenate(three, ex["bond"]).shape) == ex["expected_shape_printed_inputs"]


def test_concatenate_uneven_dimensions():
    ins = [cg(20, (2, 1, 3)), cg(21, (2, 4, 3)), cg(22, (2, 2, 3))]
    out = st.concatenate(ins, 1)
    assert out.shape == (2, 7, 3)
    assert np.array_equal(out[:, 1:5], ins[1])
    with pytest.raises(ValueError):
        st.concatenate([np.zeros((2, 3)), np.zeros((3, 3))], 1)


def test_stack_paper_example_and_numpy():
    ex = EX["stack"]
    ins = [cg(30 + k, ex["shape"]) for k in range(ex["n"])]
    out = st.stack(ins, ex["bond"])
    assert list(out.shape) == ex["expected_shape"]
    assert out[tuple(ex["coord_out"])] == ins[ex["input"]][tuple(ex["coord_in"])]
    for b in range(len(ex["shape"]) + 1):
        assert np.array_equal(st.stack(ins, b), np.stack(ins, axis=b))


# ---------------------------------------------------------------- trace
def test_trace_paper_example_against_loops():
    ex = EX["trace"]
    a = cg(40, ex["shape"])
    out = st.trace(a, [tuple(p) for p in ex["pairs"]])
    assert list(out.shape) == ex["expected_shape"]
    ref = np.zeros(3, dtype=np.complex128)
    for i in range(3):
        for j in range(4):
            for k in range(2):
                ref[i] += a[i, j, k, j, k]
    assert np.allclose(out, ref, rtol=0, atol=1e-14)


def test_trace_matrix_and_full_contraction():
    m = cg(41, (7, 7))
    assert np.isclose(st.trace(m, [(0, 1)]), np.trace(m), rtol=1e-15)
    a = cg(42, (3, 5, 5, 3))
    assert np.isclose(st.trace(a, [(0, 3), (1, 2)]), np.einsum("ijji->", a), rtol=1e-14)
    # keep the order of the untraced bonds
    b = cg(43, (2, 4, 3, 4, 5))
    assert np.allclose(st.trace(b, [(3, 1)]), np.einsum("ajbjc->abc", b), atol=1e-14)
    with pytest.raises(ValueError):
        st.trace(b, [(0, 1)])


# ---------------------------------------------------------------- exp
def test_exp_paper_example_eye3():
    ex = EX["exp_eye3"]
    out = st.expm(np.eye(ex["n"]), ex["k_rows"])
    assert abs(out[tuple(ex["coord"])] - ex["expected"]) < 1e-14
    assert np.abs(out - math.e * np.eye(3)).max() < 1e-14


def test_exp_closed_forms():
    # nilpotent: exp([[0, t], [0, 0]]) = [[1, t], [0, 1]]
    t = 2.5
    assert np.abs(st.expm_matrix([[0, t], [0, 0]]) - [[1, t], [0, 1]]).max() < 1e-14
    # rotation generator
    th = 1.3
    r = st.expm_matrix([[0, -th], [th, 0]])
    assert np.abs(r - [[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]]).max() < 1e-14
    # Hermitian: exp(H) = V diag(exp(w)) V^H, with the spectrum from LAPACK
    a = cg(50, (12, 12))
    h = (a + a.conj().T) / 4
    w, v = np.linalg.eigh(h)
    ref = (v * np.exp(w)) @ v.conj().T
    assert np.linalg.norm(st.expm_matrix(h) - ref) / np.linalg.norm(ref) < 1e-13
    # exp(A) exp(-A) = I
    g = cg(51, (9, 9))
    assert np.abs(st.expm_matrix(g) @ st.expm_matrix(-g) - np.eye(9)).max() < 1e-11


def test_exp_matches_scipy_and_tensor_fold():
    a = cg(52, (2, 3, 6)) * 0.7
    out = st.expm(a, 2)
    ref = scipy.linalg.expm(a.reshape(6, 6)).reshape(2, 3, 6)
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref) < 1e-13
    with pytest.raises(ValueError):
        st.expm(np.zeros((2, 3)), 1)


# ---------------------------------------------------------------- lq
@pytest.mark.parametrize("m,n", [(5, 12), (8, 8), (1, 6)])
def test_lq_properties_and_lapack(m, n):
    a = cg(60 + m, (m, n))
    l, q = st.lq_matrix(a)
    assert l.shape == (m, m) and q.shape == (m, n)
    assert np.abs(l @ q - a).max() < 1e-13
    assert np.abs(q @ q.conj().T - np.eye(m)).max() < 1e-13
    assert np.abs(np.triu(l, 1)).max() == 0
    d = np.diagonal(l)
    assert np.all(np.abs(d.imag) < 1e-15) and np.all(d.real >= 0)
    # unique for full rank: |diag(L)| equals |diag(R)| of LAPACK's QR of A^H
    _, rn = np.linalg.qr(a.conj().T)
    assert np.allclose(np.abs(np.diagonal(rn)), d.real, atol=1e-12)


def test_lq_paper_shapes():
    ex = EX["lq_shapes"]
    l, q = st.lq(cg(70, ex["shape"]), ex["k_rows"])
    assert list(l.shape) == ex["l"] and list(q.shape) == ex["q"]


# ---------------------------------------------------------------- inverse
def test_inverse_paper_example_and_special_cases():
    ex = EX["inverse_eye3"]
    out = st.inverse(np.eye(ex["n"]), ex["k_rows"])
    assert out[tuple(ex["coord"])] == ex["expected"] and np.array_equal(out, np.eye(3))
    # 2 x 2 closed form
    a, b, c, d = 2.0, -1.5, 0.5, 3.0
    det = a * d - b * c
    assert np.abs(st.inverse(np.array([[a, b], [c, d]]), 1) - np.array([[d, -b], [-c, a]]) / det).max() < 1e-15
    # unitary: the inverse is the conjugate transpose
    q, _ = np.linalg.qr(cg(80, (9, 9)))
    assert np.abs(st.inverse(q, 1) - q.conj().T).max() < 1e-13


def test_inverse_hilbert_integer_closed_form():
    n = 6
    h = np.array([[1.0 / (i + j + 1) for j in range(n)] for i in range(n)])
    exact = np.zeros((n, n))
    for i in range(1, n + 1):
        for j in range(1, n + 1):
            exact[i - 1, j - 1] = ((-1) ** (i + j) * (i + j - 1) * math.comb(n + i - 1, n - j)
                                   * math.comb(n + j - 1, n - i) * math.comb(i + j - 2, i - 1) ** 2)
    out = st.inverse(h, 1)
    assert np.abs(out - exact).max() / np.abs(exact).max() < 1e-8   # cond(H_6) ~ 1.5e7


def test_inverse_tensor_fold_and_errors():
    a = cg(81, (2, 3, 6)) + 4 * np.eye(6).reshape(2, 3, 6)
    out = st.inverse(a, 2)
    assert out.shape == a.shape
    assert np.abs(a.reshape(6, 6) @ out.reshape(6, 6) - np.eye(6)).max() < 1e-13
    with pytest.raises(ValueError):
        st.inverse(np.zeros((2, 3)), 1)


# ---------------------------------------------------------------- to_cplx / real / imag
def test_to_cplx_real_imag_paper_examples():
    ex = EX["to_cplx_eye3"]
    c = st.to_cplx(np.eye(ex["n"]))
    assert c.dtype == np.complex128 and c[tuple(ex["coord"])] == complex(*ex["expected"])
    ex = EX["real_imag"]
    a = cg(90, ex["shape"])
    el = a[tuple(ex["coord"])]
    assert st.real(a)[tuple(ex["coord"])] == el.real and st.imag(a)[tuple(ex["coord"])] == el.imag
    assert np.array_equal(st.real(a) + 1j * st.imag(a), a)
    r = np.arange(6, dtype=np.float32).reshape(2, 3)
    assert np.array_equal(st.real(r), r) and np.array_equal(st.imag(r), np.zeros((2, 3), np.float32))
    assert st.to_cplx(r).dtype == np.complex64 and np.array_equal(st.to_cplx(r).real, r)
    assert np.array_equal(st.to_cplx(a), a)


def test_diag_paper_example_and_numpy():
    e = np.eye(3)
    d = st.diag(e)
    assert d.ndim == 1 and np.array_equal(st.diag(d), e)
    v = cg(91, (5,))
    assert np.array_equal(st.diag(v), np.diag(v))
    m = cg(92, (4, 7))
    assert np.array_equal(st.diag(m), np.diagonal(m))
    with pytest.raises(ValueError):
        st.diag(np.zeros((2, 2, 2)))
