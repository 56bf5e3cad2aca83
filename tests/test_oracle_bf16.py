"""Pins of the split-BF16x3 emulation (the expected-error reference of the
mixed-precision contractions) against the bfloat16 format's definition,
hand-worked splits, exact cases and the error bound of the split."""
import numpy as np
import pytest

from oracle import bf16
from oracle import dmrg as odmrg


def _all_bf16_values():
    """Every finite bfloat16 value, from its 65536 bit patterns (the upper
    16 bits of an FP32 word), with the pattern's last significand bit."""
    pat = np.arange(1 << 16, dtype=np.uint32)
    vals = (pat << 16).view(np.float32)
    fin = np.isfinite(vals)
    vals, pat = vals[fin].astype(np.float64), pat[fin]
    order = np.argsort(vals, kind="stable")
    vals, pat = vals[order], pat[order]
    # +0 and -0 compare equal; keep one
    keep = np.concatenate([[True], np.diff(vals) > 0])
    return vals[keep], (pat[keep] & 1).astype(bool)


def _rne_by_search(x):
    """Nearest bfloat16 value by search over the sorted finite values; ties to
    the value whose last significand bit is 0."""
    vals, odd = _all_bf16_values()
    xd = np.asarray(x, dtype=np.float32).astype(np.float64)
    hi_i = np.clip(np.searchsorted(vals, xd, side="left"), 1, len(vals) - 1)
    lo_i = hi_i - 1
    dlo = xd - vals[lo_i]
    dhi = vals[hi_i] - xd
    pick_hi = (dhi < dlo) | ((dhi == dlo) & odd[lo_i])
    out = np.where(pick_hi, vals[hi_i], vals[lo_i])
    exact = vals[np.clip(np.searchsorted(vals, xd), 0, len(vals) - 1)] == xd
    return np.where(exact, xd, out)


def test_rne_matches_nearest_value_search():
    g = np.random.default_rng(1)
    x = np.concatenate([
        g.standard_normal(20000),
        g.standard_normal(2000) * 1e-38,            # FP32 subnormal range
        g.standard_normal(2000) * 1e30,
        np.ldexp(1.0 + np.arange(1, 256) / 256.0, 0),  # 1 + k 2^-8: every tie and non-tie
        -np.ldexp(1.0 + np.arange(1, 256) / 256.0, 3),
    ]).astype(np.float32)
    got = bf16.round_bf16(x).astype(np.float64)
    want = _rne_by_search(x)
    assert np.array_equal(got, want)


def test_hand_worked_splits():
    # 1 + 2^-8 + 2^-10: above the half-way point -> hi = 1 + 2^-7, lo = -3 2^-10
    x = np.float32(1.0 + 2.0 ** -8 + 2.0 ** -10)
    hi, lo = bf16.split(np.array([x]))
    assert hi[0] == np.float32(1.0 + 2.0 ** -7)
    assert lo[0] == np.float32(-3.0 * 2.0 ** -10)
    # ties go to the even significand
    assert bf16.round_bf16(np.float32(1.0 + 2.0 ** -8)) == np.float32(1.0)
    assert bf16.round_bf16(np.float32(1.0 + 2.0 ** -7 + 2.0 ** -8)) == np.float32(1.0 + 2.0 ** -6)
    assert bf16.round_bf16(np.float32(-(1.0 + 2.0 ** -7 + 2.0 ** -8))) == np.float32(-(1.0 + 2.0 ** -6))
    # gradual underflow: spacing 2^-133 below 2^-126
    assert bf16.round_bf16(np.float32(2.0 ** -140)) == 0.0
    assert bf16.round_bf16(np.float32(1.5 * 2.0 ** -133)) == np.float32(2.0 ** -132)
    # overflow of the rounding
    assert np.isinf(bf16.round_bf16(np.float32(3.4028235e38)))
    # 1/3: hi = 0.333984375 (0x3EAB), lo = RNE(1/3 - hi)
    third = np.float32(1.0) / np.float32(3.0)
    hi, lo = bf16.split(np.array([third]))
    assert hi[0] == np.float32(0.333984375)
    assert lo[0] == bf16.round_bf16(np.float32(third - np.float32(0.333984375)))
    assert abs(float(third) - float(hi[0]) - float(lo[0])) <= 2.0 ** -16 * float(third)


def test_split_error_bound():
    g = np.random.default_rng(2)
    x = (g.standard_normal(100000) * np.exp(g.uniform(-20, 20, 100000))).astype(np.float32)
    hi, lo = bf16.split(x)
    xd = x.astype(np.float64)
    r = np.abs(xd - hi.astype(np.float64) - lo.astype(np.float64))
    assert np.all(r <= 2.0 ** -16 * np.abs(xd))
    assert np.all(np.abs(lo.astype(np.float64)) <= 2.0 ** -8 * np.abs(xd))
    assert r.max() > 0        # the split is not exact in general


def test_product_exact_on_bf16_values():
    g = np.random.default_rng(3)
    a = g.integers(-255, 256, size=(17, 40)).astype(np.float64)
    b = g.integers(-255, 256, size=(40, 9)).astype(np.float64)
    assert np.array_equal(bf16.gemm_x3(a, b), a @ b)
    ac = a + 1j * g.integers(-255, 256, size=a.shape)
    bc = b + 1j * g.integers(-255, 256, size=b.shape)
    assert np.array_equal(bf16.gemm_x3(ac, bc), ac @ bc)


@pytest.mark.parametrize("cplx", [False, True])
def test_product_error_bound_and_size(cplx):
    """|C_x3 - C| <= 3.001 * 2^-16 * (|A| |B|) elementwise, from
    a b - (a_hi b_hi + a_hi b_lo + a_lo b_hi) = a r_b + r_a b - r_a r_b + a_lo b_lo
    with |r| <= 2^-16 |x|, |x_lo| <= 2^-8 |x|; and on Gaussian data at K = 1024
    the relative Frobenius error lies between 1e-6 and 1e-5."""
    g = np.random.default_rng(4)
    shp_a, shp_b = (64, 1024), (1024, 48)
    if cplx:
        a = (g.standard_normal(shp_a) + 1j * g.standard_normal(shp_a)).astype(np.complex64)
        b = (g.standard_normal(shp_b) + 1j * g.standard_normal(shp_b)).astype(np.complex64)
        ar, ai, br, bi = (np.abs(z).astype(np.float64) for z in (a.real, a.imag, b.real, b.imag))
        bound_re = ar @ br + ai @ bi
        bound_im = ar @ bi + ai @ br
    else:
        a = g.standard_normal(shp_a).astype(np.float32)
        b = g.standard_normal(shp_b).astype(np.float32)
        bound_re = np.abs(a).astype(np.float64) @ np.abs(b).astype(np.float64)
        bound_im = None
    exact = a.astype(np.complex128 if cplx else np.float64) @ b.astype(np.complex128 if cplx else np.float64)
    c = bf16.gemm_x3(a, b)
    d = c - exact
    tol = 3.001 * 2.0 ** -16
    assert np.all(np.abs(d.real) <= tol * bound_re)
    if cplx:
        assert np.all(np.abs(d.imag) <= tol * bound_im)
    rel = np.linalg.norm(d) / np.linalg.norm(exact)
    assert 1e-6 < rel < 1e-5, rel


def test_heff_x3_rows_exact_on_representable_data():
    """With entries in {-1, 0, 1} at chi = 3 every intermediate (X1 <= 3 in
    modulus, X2 a multiple of 1/4 below 16) is a bf16 value, so the emulated
    chain equals the exact matvec of the brute-force oracle."""
    g = np.random.default_rng(5)
    chi = 3
    from paper_2512_23917_amd import synth
    w = synth.heisenberg_mpo()
    left = (g.integers(-1, 2, (chi, 5, chi)) + 1j * g.integers(-1, 2, (chi, 5, chi))).astype(np.complex128)
    right = (g.integers(-1, 2, (chi, 5, chi)) + 1j * g.integers(-1, 2, (chi, 5, chi))).astype(np.complex128)
    x = (g.integers(-1, 2, (chi, 2, 2, chi)) + 1j * g.integers(-1, 2, (chi, 2, 2, chi))).astype(np.complex128)
    ref = odmrg.heff_apply(left, w, w, right, x)
    rows = [0, 2]
    got = bf16.heff_x3_rows(left, w, w, right, x, rows)
    assert np.array_equal(got, ref[rows])


def test_heff_x3_rows_error_size():
    """On Gaussian data the emulated chain differs from the exact matvec by
    the split's error (relative Frobenius between 1e-6 and 1e-5)."""
    from paper_2512_23917_amd import synth
    g = synth.rng(2, 901)
    chi = 24
    w = synth.heisenberg_mpo()
    left = synth.hermitian_environment(g, chi)
    right = synth.hermitian_environment(g, chi)
    x = synth.complex_gaussian(g, (chi, 2, 2, chi))
    ls, rs, xs = (bf16.to_storage(z) for z in (left, right, x))
    ref = odmrg.heff_apply(ls, w, w, rs, xs)
    rows = np.arange(chi)
    got = bf16.heff_x3_rows(left, w, w, right, x, rows)
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert 1e-7 < rel < 1e-5, rel
