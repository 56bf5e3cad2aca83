"""GPU parity of the sub-tensor, construction, trace, exp and LQ entry points
against the CPU oracle, through the C ABI.

Data movement (fill, eye, extract_sub, shrink, expand, replace_sub,
concatenate, stack) is bit-exact.  The partial trace accumulates in FP64
(<= 1e-13 relative per element for double types, 1e-6 for single).  exp and
lq (both computed in FP64 for every dtype): <= 1e-10 relative Frobenius for
F64/C128, <= 1e-6 (exp) and 1e-5 (lq) for F32/C64."""
import numpy as np
import pytest

from oracle import subtensor as ost
from paper_2512_23917_amd import synth

from gpu_util import isometry_err, rel_fro

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DTYPES = ["F32", "F64", "C64", "C128"]
NP = {"F32": np.float32, "F64": np.float64, "C64": np.complex64, "C128": np.complex128}


@pytest.fixture(scope="module")
def T():
    from paper_2512_23917_amd import tci
    return tci


@pytest.fixture(scope="module")
def ctx(T):
    c = T.Context(0)
    yield c
    c.close()


def rand(seed, shape, dtype):
    g = np.random.default_rng(seed)
    if dtype.startswith("C"):
        return synth.complex_gaussian(g, shape).astype(NP[dtype])
    return g.standard_normal(shape).astype(NP[dtype])


def up(T, ctx, a, dtype):
    return T.Tensor.from_numpy(ctx, np.ascontiguousarray(a), getattr(T, dtype))


# ------------------------------------------------------------------ construction
@pytest.mark.parametrize("dtype", DTYPES)
def test_fill_and_eye(T, ctx, dtype):
    v = (2.0 - 0.5j) if dtype.startswith("C") else 2.0
    f = T.fill(ctx, getattr(T, dtype), (3, 2, 4), v)
    assert f.shape() == (3, 2, 4)
    assert np.array_equal(f.numpy(), ost.fill((3, 2, 4), v, NP[dtype]))
    big = T.fill(ctx, getattr(T, dtype), (1000, 1001), v)   # several workgroups, ragged tail
    assert np.array_equal(big.numpy(), ost.fill((1000, 1001), v, NP[dtype]))
    for n in (0, 1, 3, 517):
        e = T.eye(ctx, getattr(T, dtype), n)
        assert e.shape() == (n, n)
        assert np.array_equal(e.numpy(), ost.eye(n, NP[dtype]))


# ------------------------------------------------------------------ box copies
@pytest.mark.parametrize("dtype", DTYPES)
def test_extract_shrink_expand(T, ctx, dtype):
    a = rand(1, (37, 65, 3, 5), dtype)
    ta = up(T, ctx, a, dtype)
    ranges = [(4, 30), (0, 65), (1, 3), (2, 5)]
    assert np.array_equal(T.extract_sub(ctx, ta, ranges).numpy(), ost.extract_sub(a, ranges))
    empty = T.extract_sub(ctx, ta, [(3, 3), (0, 65), (0, 3), (0, 5)])
    assert empty.shape() == (0, 65, 3, 5)
    sh = {1: (7, 64), 3: (0, 1)}
    assert np.array_equal(T.shrink(ctx, ta, sh).numpy(), ost.shrink(a, sh))
    inc = {0: 5, 2: 2}
    assert np.array_equal(T.expand(ctx, ta, inc).numpy(), ost.expand(a, inc))
    assert np.array_equal(T.expand(ctx, ta, {}).numpy(), a)


@pytest.mark.parametrize("dtype", ["F32", "C128"])
def test_extract_in_place_and_errors(T, ctx, dtype):
    a = rand(2, (9, 10, 11), dtype)
    ta = up(T, ctx, a, dtype)
    ranges = [(1, 8), (2, 10), (0, 5)]
    T.extract_sub(ctx, ta, ranges, out=ta)
    assert ta.shape() == (7, 8, 5)
    assert np.array_equal(ta.numpy(), ost.extract_sub(a, ranges))
    with pytest.raises(T.TciError):
        T.extract_sub(ctx, up(T, ctx, a, dtype), [(0, 10), (0, 10), (0, 11)])
    with pytest.raises(T.TciError):
        T.shrink(ctx, up(T, ctx, a, dtype), {3: (0, 1)})


@pytest.mark.parametrize("dtype", DTYPES)
def test_replace_sub(T, ctx, dtype):
    a = rand(3, (40, 70, 3), dtype)
    sub = rand(4, (13, 66, 2), dtype)
    ta, ts = up(T, ctx, a, dtype), up(T, ctx, sub, dtype)
    ref = ost.replace_sub(a, sub, (20, 4, 1))
    assert np.array_equal(T.replace_sub(ctx, ta, ts, (20, 4, 1)).numpy(), ref)
    assert np.array_equal(ta.numpy(), a)            # out-of-place leaves the input
    T.replace_sub(ctx, ta, ts, (20, 4, 1), out=ta)  # in place
    assert np.array_equal(ta.numpy(), ref)
    with pytest.raises(T.TciError):
        T.replace_sub(ctx, ta, ts, (28, 4, 1))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("bond", [0, 1, 2])
def test_concatenate_and_stack(T, ctx, dtype, bond):
    shapes = [[6, 7, 9], [6, 7, 9], [6, 7, 9]]
    shapes[1][bond] = 13
    shapes[2][bond] = 1
    ins = [rand(10 + k, s, dtype) for k, s in enumerate(shapes)]
    out = T.concatenate(ctx, [up(T, ctx, x, dtype) for x in ins], bond)
    assert np.array_equal(out.numpy(), ost.concatenate(ins, bond))
    same = [rand(20 + k, (6, 7, 9), dtype) for k in range(4)]
    for b in range(4):
        st = T.stack(ctx, [up(T, ctx, x, dtype) for x in same], b)
        assert np.array_equal(st.numpy(), ost.stack(same, b))


def test_concatenate_and_stack_errors(T, ctx):
    a = up(T, ctx, rand(30, (2, 3), "F64"), "F64")
    b = up(T, ctx, rand(31, (3, 3), "F64"), "F64")
    with pytest.raises(T.TciError):
        T.concatenate(ctx, [a, b], 1)
    with pytest.raises(T.TciError):
        T.stack(ctx, [a, b], 0)


# ------------------------------------------------------------------ trace
@pytest.mark.parametrize("dtype", DTYPES)
def test_trace(T, ctx, dtype):
    tol = 1e-13 if dtype in ("F64", "C128") else 1e-5
    a = rand(40, (3, 4, 2, 4, 2), dtype)
    out = T.trace(ctx, up(T, ctx, a, dtype), [(1, 3), (2, 4)])
    assert out.shape() == (3,)
    ref = ost.trace(a.astype(np.complex128), [(1, 3), (2, 4)])
    assert rel_fro(out.numpy(), ref) < tol
    b = rand(41, (70, 5, 3, 70, 5), dtype)
    out = T.trace(ctx, up(T, ctx, b, dtype), [(3, 0)])
    assert out.shape() == (5, 3, 5)
    assert rel_fro(out.numpy(), ost.trace(b.astype(np.complex128), [(3, 0)])) < tol
    c = rand(42, (33, 33), dtype)
    full = T.trace(ctx, up(T, ctx, c, dtype), [(0, 1)])
    assert full.shape() == ()
    assert abs(full.numpy() - np.trace(c.astype(np.complex128))) <= tol * np.linalg.norm(c)


def test_trace_in_place_and_errors(T, ctx):
    a = rand(43, (4, 6, 4), "C128")
    ta = up(T, ctx, a, "C128")
    T.trace(ctx, ta, [(0, 2)], out=ta)
    assert ta.shape() == (6,)
    assert rel_fro(ta.numpy(), ost.trace(a, [(0, 2)])) < 1e-13
    with pytest.raises(T.TciError):
        T.trace(ctx, up(T, ctx, a, "C128"), [(0, 1)])


# ------------------------------------------------------------------ exp
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,scale", [(3, 0.0), (50, 0.3), (200, 0.08), (129, 1.5)])
def test_exp(T, ctx, dtype, n, scale):
    # computed in FP64 for every dtype: single types only see the final rounding
    tol = 1e-10 if dtype in ("F64", "C128") else 1e-6
    a = np.eye(n) if scale == 0.0 else rand(50 + n, (n, n), dtype) * scale
    a = a.astype(NP[dtype])
    out = T.exp(ctx, up(T, ctx, a, dtype), 1)
    ref = ost.expm_matrix(a.astype(np.complex128))
    assert rel_fro(out.numpy(), ref) < tol


def test_exp_paper_example_and_tensor_fold(T, ctx):
    e = T.exp(ctx, T.eye(ctx, T.F64, 3), 1).numpy()
    assert abs(e[1, 1] - np.e) < 1e-14 and abs(e[1, 2]) == 0
    a = rand(60, (2, 3, 6), "C128") * 0.5
    ta = up(T, ctx, a, "C128")
    T.exp(ctx, ta, 2, out=ta)
    assert ta.shape() == (2, 3, 6)
    assert rel_fro(ta.numpy(), ost.expm(a, 2)) < 1e-10
    with pytest.raises(T.TciError):
        T.exp(ctx, up(T, ctx, rand(61, (2, 3), "F64"), "F64"), 1)


# ------------------------------------------------------------------ lq
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("shape,k", [((3, 4, 12), 2), ((30, 2, 70), 1), ((40, 2, 65, 2), 2)])
def test_lq(T, ctx, dtype, shape, k):
    tol = 1e-10 if dtype in ("F64", "C128") else 1e-5
    a = rand(70, shape, dtype)
    l, q = T.lq(ctx, up(T, ctx, a, dtype), k)
    lo, qo = ost.lq(a.astype(np.complex128), k)
    assert l.shape() == lo.shape and q.shape() == qo.shape
    assert rel_fro(l.numpy(), lo) < tol
    assert rel_fro(q.numpy(), qo) < tol
    assert isometry_err(q.numpy(), axis_cols=False) < (1e-12 if tol == 1e-10 else 1e-5)


def test_lq_rejects_tall(T, ctx):
    with pytest.raises(T.TciError):
        T.lq(ctx, up(T, ctx, rand(71, (12, 5), "F64"), "F64"), 1)


# ------------------------------------------------------------------ TCI_VERBOSE
@pytest.mark.parametrize("level", ["0", "1", "2"])
def test_verbose_levels(T, level, capfd, monkeypatch):
    """Spec, environment variables: 0 silent, 1 one line per call with the
    function name and input shape, 2 the same line with the call's time."""
    monkeypatch.setenv("TCI_VERBOSE", level)
    c = T.Context(0)
    try:
        capfd.readouterr()
        a = up(T, c, rand(80, (4, 6, 4), "C128"), "C128")
        T.trace(c, a, [(0, 2)])
        T.expand(c, a, {1: 2})
        torch.cuda.synchronize()
        err = capfd.readouterr().err
    finally:
        c.close()
    lines = [ln for ln in err.splitlines() if ln.startswith("TCI_VERBOSE:")]
    if level == "0":
        assert lines == []
        return
    assert any("trace {4,6,4}" in ln for ln in lines) and any("expand {4,6,4}" in ln for ln in lines)
    timed = [ln for ln in lines if ln.rstrip().endswith(" us")]
    assert (len(timed) == len(lines)) if level == "2" else not timed


# ------------------------------------------------------------------ inverse
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [1, 3, 70, 300])
def test_inverse(T, ctx, dtype, n):
    tol = 1e-10 if dtype in ("F64", "C128") else 1e-5
    a = rand(90 + n, (n, n), dtype) + (2.0 * np.sqrt(n) * np.eye(n)).astype(NP[dtype])
    out = T.inverse(ctx, up(T, ctx, a, dtype), 1).numpy()
    ref = ost.inverse(a.astype(np.complex128), 1)
    assert rel_fro(out, ref) < tol
    if tol == 1e-10:
        assert np.abs(a.astype(np.complex128) @ out - np.eye(n)).max() < 1e-11


def test_inverse_paper_example_pivoting_fold_and_errors(T, ctx):
    e = T.inverse(ctx, T.eye(ctx, T.F64, 3), 1).numpy()
    assert e[1, 1] == 1.0 and np.array_equal(e, np.eye(3))
    # a zero leading entry needs a row swap
    p = np.array([[0.0, 2.0, 1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 3.0]])
    assert rel_fro(T.inverse(ctx, up(T, ctx, p, "F64"), 1).numpy(), np.linalg.inv(p)) < 1e-14
    a = rand(95, (2, 3, 6), "C128") + 4 * np.eye(6).reshape(2, 3, 6)
    ta = up(T, ctx, a, "C128")
    T.inverse(ctx, ta, 2, out=ta)
    assert ta.shape() == (2, 3, 6) and rel_fro(ta.numpy(), ost.inverse(a, 2)) < 1e-12
    with pytest.raises(T.TciError):   # exactly singular: second pivot 4 - 2 * 2 = 0
        T.inverse(ctx, up(T, ctx, np.array([[1.0, 2.0], [2.0, 4.0]]), "F64"), 1)
    with pytest.raises(T.TciError):
        T.inverse(ctx, up(T, ctx, rand(96, (2, 3), "F64"), "F64"), 1)


# ------------------------------------------------------------------ to_cplx / real / imag
@pytest.mark.parametrize("dtype", DTYPES)
def test_to_cplx_real_imag(T, ctx, dtype):
    a = rand(100, (33, 65, 3), dtype)
    ta = up(T, ctx, a, dtype)
    assert np.array_equal(T.to_cplx(ctx, ta).numpy(), ost.to_cplx(a))
    assert np.array_equal(T.real(ctx, ta).numpy(), ost.real(a))
    assert np.array_equal(T.imag(ctx, ta).numpy(), ost.imag(a))
    c = T.to_cplx(ctx, T.eye(ctx, getattr(T, dtype), 3)).numpy()
    assert c[1, 1] == 1.0 + 0.0j


# ------------------------------------------------------------------ save / load / show
@pytest.mark.parametrize("dtype", DTYPES)
def test_save_load_round_trip_and_format(T, ctx, dtype, tmp_path):
    a = rand(110, (5, 1, 7, 3), dtype)
    path = str(tmp_path / f"a_{dtype}.ten")
    T.save(ctx, up(T, ctx, a, dtype), path)
    raw = open(path, "rb").read()
    assert raw[:8] == b"TCIMI355"
    ver, dt, order, _ = np.frombuffer(raw[8:24], dtype="<i4")
    assert (ver, dt, order) == (1, getattr(T, dtype), 4)
    assert list(np.frombuffer(raw[24:56], dtype="<i8")) == [5, 1, 7, 3]
    assert raw[56:] == np.ascontiguousarray(a).tobytes()
    b = T.load(ctx, path)
    assert b.shape() == (5, 1, 7, 3) and b.current_dtype() == getattr(T, dtype)
    assert np.array_equal(b.numpy(), a)
    bad = tmp_path / "bad.ten"
    bad.write_bytes(raw[:60])
    with pytest.raises(T.TciError):
        T.load(ctx, str(bad))


def test_show_prints_every_element(T, ctx, capfd):
    a = np.array([[1.5, -2.0], [0.25, 3.0]])
    capfd.readouterr()
    T.show(ctx, up(T, ctx, a, "F64"))
    lines = capfd.readouterr().out.strip().splitlines()
    assert lines[0] == "tensor F64 shape {2,2}"
    vals = {tuple(int(x) for x in ln.split(")")[0].strip(" (").split(",")): float(ln.split(")")[1]) for ln in lines[1:]}
    assert vals == {(0, 0): 1.5, (0, 1): -2.0, (1, 0): 0.25, (1, 1): 3.0}


@pytest.mark.parametrize("dtype", DTYPES)
def test_diag(T, ctx, dtype):
    v = rand(120, (300,), dtype)
    m = T.diag(ctx, up(T, ctx, v, dtype))
    assert m.shape() == (300, 300) and np.array_equal(m.numpy(), ost.diag(v))
    for shp in [(70, 45), (45, 70), (33, 33)]:
        a = rand(121, shp, dtype)
        d = T.diag(ctx, up(T, ctx, a, dtype))
        assert np.array_equal(d.numpy(), ost.diag(a))
    e = T.eye(ctx, getattr(T, dtype), 3)   # the paper's example: twice in place is the identity
    T.diag(ctx, e, out=e)
    assert e.shape() == (3,)
    T.diag(ctx, e, out=e)
    assert np.array_equal(e.numpy(), np.eye(3))


# ------------------------------------------------------------------ C++17 header
def test_cpp_header_program(tmp_path):
    """tests/cpp/tci_header_check.cpp calls every function of tci/tci.h on
    the GPU (built by the build step); each check prints its residual."""
    import os
    import subprocess
    exe = os.path.join(os.path.dirname(__file__), "cpp", "tci_header_check")
    if not os.path.exists(exe):
        pytest.fail(f"{exe} is missing: run the build step first")
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, timeout=100)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = r.stdout.splitlines()
    assert lines[0] == "version 1.0" and "DONE" in lines
    checks = {ln.split()[1]: float(ln.split()[2]) for ln in lines if ln.startswith("CHECK ")}
    assert len(checks) >= 38, sorted(checks)
    bad = {k: v for k, v in checks.items() if not v <= 1e-10}
    assert not bad, bad
    assert "tensor F64 shape {2,2}" in lines
