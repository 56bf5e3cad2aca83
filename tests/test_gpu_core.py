"""GPU parity of the HIP library against the CPU oracle, through the C ABI.

FP64 path: <= 1e-10 relative Frobenius on theta, reconstructions and phase-
fixed factors; kept singular values <= 1e-6 normwise (and much tighter in
practice).  Mixed paths: <= 1e-5 on gauge-invariant results."""
import numpy as np
import pytest

import oracle
from oracle import bf16
from oracle import mps as omps
from paper_2512_23917_amd import synth

from gpu_util import gauge_ok_columns, isometry_err, rel_fro

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


def up(T, ctx, a, dtype):
    return T.Tensor.from_numpy(ctx, np.asarray(a), dtype)


def cg(g, shape):
    return synth.complex_gaussian(g, shape)


# ------------------------------------------------------------------ contract / GEMM
@pytest.mark.parametrize("dtype", ["C128", "F64"])
@pytest.mark.parametrize("case", [
    ("ik", "kj", "ij", dict(i=130, k=70, j=50)),   # ragged tails, N/N
    ("ki", "kj", "ij", dict(i=77, k=33, j=129)),   # A transposed
    ("ik", "jk", "ij", dict(i=65, k=17, j=200)),   # B transposed
    ("ki", "jk", "ji", dict(i=31, k=45, j=64)),    # both + output permute
    ("asm", "mtb", "astb", dict(a=9, s=2, m=40, t=2, b=11)),
    ("ijk", "kjl", "li", dict(i=3, j=4, k=2, l=5)),
    ("ij", "ij", "", dict(i=13, j=7)),
    ("astb", "uvst", "auvb", dict(a=5, s=2, t=2, b=6, u=2, v=2)),
    # long K over few output tiles: the FP64 kernels split K into chunks
    ("ik", "kj", "ij", dict(i=64, k=4096, j=64)),    # one tile, 32 chunks
    ("ki", "jk", "ij", dict(i=37, k=1000, j=70)),    # ragged chunks, both transposed
    ("ik", "kj", "ij", dict(i=300, k=300, j=20)),    # two chunks
    ("ij", "ij", "", dict(i=100, j=50)),             # full contraction, K = 5000
])
def test_contract_fp64_matches_oracle(T, ctx, dtype, case):
    la, lb, lc, dims = case
    g = np.random.default_rng(11)
    dt = getattr(T, dtype)
    mk = (lambda s: cg(g, s)) if dtype == "C128" else (lambda s: g.standard_normal(s))
    a = mk([dims[x] for x in la])
    b = mk([dims[x] for x in lb])
    ref = oracle.contract(a, la, b, lb, lc)
    c = T.contract(ctx, up(T, ctx, a, dt), la, up(T, ctx, b, dt), lb, lc).numpy()
    assert c.shape == ref.shape
    assert rel_fro(c, ref) < 1e-13


@pytest.mark.parametrize("prec,tol", [("PREC_FP32", 2e-6), ("PREC_BF16X3", 1e-5)])
@pytest.mark.parametrize("dtype", ["C64", "F32"])
def test_contract_mixed_matches_oracle(T, ctx, dtype, prec, tol):
    """Mixed contractions against the FP64 oracle on the same FP32 operands:
    <= 1e-5 relative Frobenius, and for split-BF16x3 within twice the error of
    the split's emulation (exact partial products, FP64 sums)."""
    g = np.random.default_rng(12)
    dt = getattr(T, dtype)
    if dtype == "C64":
        a, b = cg(g, (150, 96)), cg(g, (96, 70))
    else:
        a, b = g.standard_normal((150, 96)), g.standard_normal((96, 70))
    a32 = a.astype(np.complex64 if dtype == "C64" else np.float32)
    b32 = b.astype(np.complex64 if dtype == "C64" else np.float32)
    ref = oracle.contract(a32.astype(np.complex128), "ik", b32.astype(np.complex128), "kj", "ij")
    ctx.set_precision(getattr(T, prec))
    try:
        c = T.contract(ctx, up(T, ctx, a32, dt), "ik", up(T, ctx, b32, dt), "kj", "ij").numpy()
    finally:
        ctx.set_precision(T.PREC_FP32)
    err = rel_fro(c, ref)
    assert err < tol
    if prec == "PREC_BF16X3":
        err_emu = rel_fro(bf16.gemm_x3(a32, b32), ref)
        print(f"contract {dtype} bf16x3: GPU {err:.3e} emulation {err_emu:.3e}")
        assert err <= 2 * err_emu, (err, err_emu)


def test_contract_alias_and_label_errors(T, ctx):
    g = np.random.default_rng(13)
    a = cg(g, (6, 5))
    b = cg(g, (5, 5))
    ta = up(T, ctx, a, T.C128)
    tb = up(T, ctx, b, T.C128)
    # c aliases a: result must equal the non-aliased product
    T.contract(ctx, ta, "ij", tb, "jk", "ik", out=ta)
    np.testing.assert_allclose(ta.numpy(), a @ b, atol=1e-13)
    with pytest.raises(T.TciError) as e:
        T.contract(ctx, tb, "ii", tb, "ij", "j")
    assert e.value.status == 3
    with pytest.raises(T.TciError) as e:
        T.contract(ctx, tb, "ij", tb, "jk", "ijk")
    assert e.value.status == 3


# ------------------------------------------------------------------ transpose / norm
@pytest.mark.parametrize("shape,perm", [((3, 2, 4), (2, 1, 0)), ((64, 2, 2, 70), (0, 3, 1, 2)),
                                        ((130, 67), (1, 0)), ((5, 6, 7, 8), (1, 3, 0, 2))])
def test_transpose_bit_exact(T, ctx, shape, perm):
    a = cg(np.random.default_rng(14), shape)
    out = T.transpose(ctx, up(T, ctx, a, T.C128), perm).numpy()
    np.testing.assert_array_equal(out, oracle.permute(a, perm))


def test_norm_normalize(T, ctx):
    a = cg(np.random.default_rng(15), (33, 2, 17))
    t = up(T, ctx, a, T.C128)
    assert T.norm(ctx, t) == pytest.approx(oracle.norm(a), rel=1e-14)
    old = T.normalize(ctx, t)
    assert old == pytest.approx(oracle.norm(a), rel=1e-14)
    assert T.norm(ctx, t) == pytest.approx(1.0, abs=1e-14)
    assert T.norm(ctx, up(T, ctx, np.eye(3), T.F64)) == pytest.approx(np.sqrt(3.0), rel=1e-15)


# ------------------------------------------------------------------ decompositions
def _svd_parity(u, s, vh, a_mat, chi, tol_rec=1e-10):
    uo, so, vho = oracle.svd_matrix(a_mat)
    s = np.asarray(s)
    assert len(s) == chi
    assert np.abs(s - so[:chi]).max() <= 1e-10 * so[0]
    um = np.asarray(u).reshape(-1, chi)
    vm = np.asarray(vh).reshape(chi, -1)
    rec = um @ np.diag(s) @ vm
    rec_o = uo[:, :chi] @ np.diag(so[:chi]) @ vho[:chi]
    assert rel_fro(rec, rec_o) < tol_rec
    assert isometry_err(um) < 1e-12
    assert isometry_err(vm, axis_cols=False) < 1e-12
    for i in gauge_ok_columns(so[:chi + 1])[:chi]:
        if i < chi:
            assert rel_fro(um[:, i], uo[:, i]) < 1e-8
            assert rel_fro(vm[i], vho[i]) < 1e-8


@pytest.mark.parametrize("m,n,complex_", [(64, 64, True), (100, 60, True), (60, 100, True), (97, 97, False),
                                          (33, 130, False), (200, 150, True)])
def test_svd_full_matches_oracle(T, ctx, m, n, complex_):
    g = np.random.default_rng(m * 7 + n)
    a = cg(g, (m, n)) if complex_ else g.standard_normal((m, n))
    dt = T.C128 if complex_ else T.F64
    u, s, vh = T.svd(ctx, up(T, ctx, a, dt), 1)
    _svd_parity(u.numpy(), s.numpy(), vh.numpy(), a, min(m, n))


@pytest.mark.parametrize("m,n", [(48, 40), (40, 48), (64, 64)])
def test_svd_small_graded_spectrum(T, ctx, m, n):
    """Matrices with k = min(m, n) <= 64 take the one-sided Jacobi path: a
    spectrum graded from 1 down to 1e-13 is resolved to an absolute error of
    a few ulps of s_0 (the Gram route would lose everything below ~1e-8)."""
    g = np.random.default_rng(m + 3 * n)
    k = min(m, n)
    sv = np.logspace(0, -13, k)
    u0 = synth.haar(g, m, k)
    v0 = synth.haar(g, n, k)
    a = (u0 * sv) @ v0.conj().T
    u, s, vh = T.svd(ctx, up(T, ctx, a, T.C128), 1)
    s = s.numpy()
    assert np.abs(s - sv).max() < 1e-13
    assert np.all(np.abs(s - sv)[sv >= 1e-9] <= 1e-4 * sv[sv >= 1e-9])
    _, so, _ = oracle.svd_matrix(a)
    assert np.abs(s - so).max() < 1e-13
    um, vm = u.numpy().reshape(m, k), vh.numpy().reshape(k, n)
    assert isometry_err(um) < 1e-12 and isometry_err(vm, axis_cols=False) < 1e-12
    assert rel_fro(um @ np.diag(s) @ vm, a) < 1e-13


@pytest.mark.parametrize("m,n,exact_zero", [(30, 20, False), (20, 30, False), (30, 20, True), (20, 30, True)])
def test_svd_small_rank_deficient(T, ctx, m, n, exact_zero):
    """Rank 7: rounding-level singular values keep orthonormal vectors; and
    with exactly zero columns (tall) or rows (wide) the zero singular values
    get an orthonormal completion of their singular vectors (on u for tall
    matrices, on the rows of v^dagger for wide ones)."""
    g = np.random.default_rng(m * n + exact_zero)
    if exact_zero:
        a = cg(g, (m, n))
        if m >= n:
            a[:, [2, 5, 11, 12, 19]] = 0.0
        else:
            a[[2, 5, 11, 12, 19], :] = 0.0
    else:
        a = cg(g, (m, 7)) @ cg(g, (7, n))
    rank = 15 if exact_zero else 7
    u, s, vh = T.svd(ctx, up(T, ctx, a, T.C128), 1)
    k = min(m, n)
    s = s.numpy()
    _, so, _ = oracle.svd_matrix(a)
    assert np.abs(s - so).max() < 1e-12 * so[0]
    assert np.all(s[rank:] < 1e-13 * s[0])
    if exact_zero:
        assert np.all(s[rank:] == 0.0)
    um, vm = u.numpy().reshape(m, k), vh.numpy().reshape(k, n)
    assert isometry_err(um) < 1e-12 and isometry_err(vm, axis_cols=False) < 1e-12
    assert rel_fro(um @ np.diag(s) @ vm, a) < 1e-13


@pytest.mark.parametrize("chi_min,chi_max,target,s_min", [(1, 40, 0.0, 0.0), (1, 200, 1e-3, 0.0),
                                                         (5, 60, 0.5, 0.0), (1, 200, 0.0, 0.5)])
def test_trunc_svd_rule_matches_oracle(T, ctx, chi_min, chi_max, target, s_min):
    g = np.random.default_rng(21)
    s_true = synth.power_spectrum(96, 1.2) * 10.0
    a, b = synth.two_site_blocks_from_spectrum(g, 48, 2, s_true)
    theta = np.einsum("asm,mtb->astb", a, b)
    u, s, vh, err = T.trunc_svd(ctx, up(T, ctx, theta, T.C128), 2, chi_min, chi_max, target, s_min)
    uo, so, vho, erro = oracle.trunc_svd(theta, 2, chi_min, chi_max, target, s_min)
    assert len(so) == s.numpy().shape[0]
    assert err == pytest.approx(erro, rel=1e-6, abs=1e-15)
    _svd_parity(u.numpy(), s.numpy(), vh.numpy(), theta.reshape(96, 96), len(so))


def test_trunc_svd_paper_example(T, ctx):
    a = cg(np.random.default_rng(22), (3, 4, 12))
    u, s, vh, err = T.trunc_svd(ctx, up(T, ctx, a, T.C128), 2, 3, 6, 1e-2, 1e-12)
    assert err != 0.0
    assert 3 <= s.numpy().shape[0] <= 6
    assert u.shape()[:2] == (3, 4) and vh.shape()[1:] == (12,)


def test_qr_matches_oracle(T, ctx):
    g = np.random.default_rng(23)
    a = cg(g, (40, 2, 30))
    q, r = T.qr(ctx, up(T, ctx, a, T.C128), 2)
    qo, ro = oracle.qr(a, 2)
    assert q.shape() == qo.shape and r.shape() == ro.shape
    assert rel_fro(q.numpy(), qo) < 1e-12
    assert rel_fro(r.numpy(), ro) < 1e-12


def test_eigh_matches_oracle(T, ctx):
    g = np.random.default_rng(24)
    x = cg(g, (70, 70))
    h = x + x.conj().T
    w, v = T.eigh(ctx, up(T, ctx, h, T.C128))
    wo, vo = oracle.eigh(h)
    assert np.abs(w.numpy() - wo).max() < 1e-12 * np.abs(wo).max()
    vv = v.numpy()
    assert rel_fro(vv @ np.diag(w.numpy()) @ vv.conj().T, h) < 1e-12
    for i in gauge_ok_columns(wo[::-1] - wo.min()):
        pass
    assert isometry_err(vv) < 1e-12


def test_eigh_degenerate_clusters(T, ctx):
    """Eigenvalues of multiplicity 20: inverse iteration returns nearly
    parallel vectors inside each cluster, so the orthonormalisation takes
    full Cholesky-QR passes before its first-order finish."""
    g = np.random.default_rng(25)
    q, _ = np.linalg.qr(cg(g, (60, 60)))
    lam = np.concatenate([np.full(20, 1.0), np.full(20, 2.0), np.linspace(3.0, 4.0, 20)])
    h = (q * lam) @ q.conj().T
    h = 0.5 * (h + h.conj().T)
    w, v = T.eigh(ctx, up(T, ctx, h, T.C128))
    assert np.abs(w.numpy() - np.sort(lam)).max() < 1e-12 * 4.0
    vv = v.numpy()
    assert isometry_err(vv) < 1e-12
    assert rel_fro(vv @ np.diag(w.numpy()) @ vv.conj().T, h) < 1e-12


def test_eigh_graded_spectrum(T, ctx):
    """Eigenvalues lambda_i = i^-4 (the Gram matrix of a power-law bond
    s_i ~ i^-2): consecutive gaps fall from 1e-1 to about 1e-12 of the norm,
    so hundreds of inverse-iteration vectors overlap at the 1e-4 level before
    the final orthonormalisation.  Checked: eigenvalues, isometry and the
    reconstruction, at the FP64 bar."""
    g = np.random.default_rng(26)
    n = 300
    q, _ = np.linalg.qr(cg(g, (n, n)))
    lam = np.arange(1, n + 1, dtype=np.float64) ** -4.0
    h = (q * lam) @ q.conj().T
    h = 0.5 * (h + h.conj().T)
    w, v = T.eigh(ctx, up(T, ctx, h, T.C128))
    assert np.abs(w.numpy() - np.sort(lam)).max() < 1e-14
    vv = v.numpy()
    assert isometry_err(vv) < 1e-12
    assert rel_fro(vv @ np.diag(w.numpy()) @ vv.conj().T, h) < 1e-12


def test_trunc_svd_power_law_matches_oracle(T, ctx):
    """A power-law theta (s_k ~ k^-2, 512 x 512 complex, Haar factors): the
    truncated SVD at eps = 1e-8 against the oracle's Jacobi SVD.  Singular
    values at the FP64 bar.  The kept subspace comes from the Gram matrix,
    whose eigenvectors at the cut are resolved only to an angle of about
    u s_1^2 / (s_chi^2 - s_chi+1^2); the reconstruction is held to the larger
    of 1e-10 and ten times the error that angle allows (s_chi+1 times it,
    relative to ||theta_chi||)."""
    g = synth.rng(1, 4242)
    n = 512
    s = synth.power_spectrum(n, 2.0)
    u, v = synth.haar(g, n, n), synth.haar(g, n, n)
    th = ((u * s[None, :]) @ v.conj().T).reshape(n // 2, 2, 2, n // 2)
    ref_u, ref_sall, ref_vh = oracle.svd(th, 2)
    chi, ref_err = oracle.trunc_rule(ref_sall, 1, n, 1e-8, 0.0)
    ref_s = ref_sall[:chi]
    U, S, V, err = T.trunc_svd(ctx, up(T, ctx, th, T.C128), 2, chi_min=1, chi_max=n, target=1e-8)
    sv = S.numpy()
    assert len(sv) == chi
    assert np.abs(sv - ref_s).max() <= 1e-10 * ref_s[0]
    rec = U.numpy().reshape(-1, chi) @ (sv[:, None] * V.numpy().reshape(chi, -1))
    rec_ref = ref_u.reshape(-1, n)[:, :chi] @ (ref_s[:, None] * ref_vh.reshape(n, -1)[:chi])
    u53 = 2.0 ** -53
    angle = u53 * ref_sall[0] ** 2 / (ref_sall[chi - 1] ** 2 - ref_sall[chi] ** 2)
    bound = max(1e-10, 10 * angle * ref_sall[chi] / np.linalg.norm(ref_s))
    err_rec = rel_fro(rec, rec_ref)
    print(f"power-law trunc_svd chi={chi} reconstruction {err_rec:.2e} bound {bound:.2e}")
    assert err_rec <= bound
    assert isometry_err(U.numpy().reshape(-1, chi)) < 1e-12


# ------------------------------------------------------------------ two-site update
@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("chi", [8, 32, 45])
def test_two_site_update_batched_matches_oracle(T, ctx, chi, direction):
    nb = 3
    As, Bs, Gs, refs = [], [], [], []
    for i in range(nb):
        g = synth.rng(1, 100 + i)
        a, b = cg(g, (chi, 2, chi)), cg(g, (chi, 2, chi))
        gate = synth.haar_gate(g)
        refs.append(omps.two_site_update(a, b, gate, 1, chi, 1e-10, 0.0, direction))
        As.append(up(T, ctx, a, T.C128))
        Bs.append(up(T, ctx, b, T.C128))
        Gs.append(up(T, ctx, gate, T.C128))
    p = T.update_params(chi_min=1, chi_max=chi, target_trunc_err=1e-10, direction=direction)
    Ao, so, Bo, infos = T.two_site_update_batched(ctx, As, Bs, Gs, p)
    for i in range(nb):
        r = refs[i]
        chi_o = r["chi"]
        assert infos[i].chi == chi_o
        assert infos[i].trunc_err == pytest.approx(r["trunc_err"], rel=1e-6, abs=1e-16)
        assert infos[i].discarded_abs == pytest.approx(r["discarded_abs"], rel=1e-6, abs=1e-14)
        s = so[i].numpy()
        assert np.abs(s - r["s"]).max() < 1e-10
        a_out, b_out = Ao[i].numpy(), Bo[i].numpy()
        rec = np.einsum("asm,mtb->astb", a_out, b_out)
        rec_o = np.einsum("asm,mtb->astb", r["a_out"], r["b_out"])
        assert rel_fro(rec, rec_o) < 1e-10
        ok = [j for j in gauge_ok_columns(r["s_raw"]) if j < chi_o]
        assert rel_fro(a_out[..., ok], r["a_out"][..., ok]) < 1e-9
        assert rel_fro(b_out[ok], r["b_out"][ok]) < 1e-9


def test_identity_gate_invariance_and_norm(T, ctx):
    g = synth.rng(1, 7)
    s_true = synth.exp_spectrum(24, 5.0)
    a, b = synth.two_site_blocks_from_spectrum(g, 12, 2, s_true)
    p = T.update_params(chi_min=1, chi_max=24, target_trunc_err=0.0)
    Ao, so, Bo, inf = T.two_site_update_batched(ctx, [up(T, ctx, a, T.C128)], [up(T, ctx, b, T.C128)],
                                                [up(T, ctx, np.eye(4), T.C128)], p)
    s = so[0].numpy()
    np.testing.assert_allclose(s, s_true / np.linalg.norm(s_true), atol=1e-13)
    assert inf[0].norm2 == pytest.approx(1.0, rel=1e-13)
    rec = np.einsum("asm,mtb->astb", Ao[0].numpy(), Bo[0].numpy())
    assert rel_fro(rec, np.einsum("asm,mtb->astb", a, b)) < 1e-12


def test_c1_sweep_on_gpu_matches_oracle_and_state_vector(T, ctx):
    """Open chain N=16, d=2, chi<=32, complex128: left-canonicalise with the
    library's QR, sweep 15 Haar gates right to left with the batched update
    (batch of one per bond), compare with the oracle sweep and the exact
    state vector."""
    g = synth.rng(1, 0)
    m0 = synth.random_open_mps(g, 16, 2, 32)
    gates = [synth.haar_gate(g) for _ in range(15)]
    # left-canonical form on the GPU
    sites = [up(T, ctx, t, T.C128) for t in m0]
    for i in range(15):
        q, r = T.qr(ctx, sites[i], 2)
        sites[i] = q
        sites[i + 1] = T.contract(ctx, r, "km", sites[i + 1], "msb", "ksb")
    T.normalize(ctx, sites[15])
    ref0 = omps.left_canonicalize(m0)
    for i in range(16):
        assert rel_fro(sites[i].numpy(), ref0[i]) < 1e-11
    ref, ref_errs = omps.sweep_right_to_left(ref0, gates, 32, 1e-10)
    p = T.update_params(chi_min=1, chi_max=32, target_trunc_err=1e-10, direction=1)
    errs = []
    for i in range(14, -1, -1):
        Ao, so, Bo, inf = T.two_site_update_batched(ctx, [sites[i]], [sites[i + 1]],
                                                    [up(T, ctx, gates[i], T.C128)], p)
        sites[i], sites[i + 1] = Ao[0], Bo[0]
        errs.append(inf[0].trunc_err)
    psi = omps.state_vector([t.numpy() for t in sites])
    psi_ref = omps.state_vector(ref)
    assert rel_fro(psi, psi_ref) < 1e-9
    np.testing.assert_allclose(errs, ref_errs, rtol=1e-5, atol=1e-15)
    exact = omps.exact_gate_evolution(omps.state_vector(ref0), 16, gates)
    bound = sum(np.sqrt(2 * (1 - np.sqrt(1 - e))) for e in errs) + 1e-9
    assert np.linalg.norm(psi - exact) <= bound
