"""Full-size parity on the GPU (chi = 1024 and 2048): sampled outputs that the
oracle computes one by one, closed-form spectra, and properties that hold at
any size (isometries, discarded weight = sum of the cut squares)."""
import math

import numpy as np
import pytest

import oracle
from oracle import bf16
from oracle import dmrg as odmrg
from paper_2512_23917_amd import synth

from gpu_util import chi_allowed, rel_fro

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


def up(T, ctx, a, dt):
    return T.Tensor.from_numpy(ctx, np.asarray(a), dt)


@pytest.fixture(scope="module")
def c3_inputs():
    """chi = 2048, real: theta = U diag(s) V^T with Haar U, V (4096 x 2048) and
    s_k = exp(-k/200) normalised, so the exact truncation is known:
    chi*(1e-8) = 1831 with eps(1831) = 9.895e-9 and eps(1830) = 1.001e-8."""
    g = synth.rng(3, 0)
    s = synth.exp_spectrum(2048, 200.0)
    a, b = synth.two_site_blocks_from_spectrum(g, 2048, 2, s, complex_=False)
    return a.real.copy(), b.real.copy(), s


@pytest.mark.parametrize("mode", ["fp64", "fp32", "bf16x3"])
def test_c3_precision_variant_exact_spectrum(T, ctx, c3_inputs, mode):
    a, b, s = c3_inputs
    chi_ref, err_ref = oracle.trunc_rule(s, 1, 2048, 1e-8, 0.0)
    assert chi_ref == 1831
    if mode == "fp64":
        dt, prec, ta, tb = T.F64, T.PREC_FP64, a, b
    else:
        dt = T.F32
        prec = T.PREC_FP32 if mode == "fp32" else T.PREC_BF16X3
        ta, tb = a.astype(np.float32), b.astype(np.float32)
    p = T.update_params(chi_min=1, chi_max=2048, target_trunc_err=1e-8, direction=1, precision=prec)
    Ao, so, Bo, inf = T.two_site_update_batched(ctx, [up(T, ctx, ta, dt)], [up(T, ctx, tb, dt)], None, p)
    chi = inf[0].chi
    sn = so[0].numpy()
    s_ref = s[:chi] / np.linalg.norm(s[:chi])
    if mode == "fp64":
        assert chi == chi_ref
        assert inf[0].trunc_err == pytest.approx(err_ref, rel=1e-6)
        assert np.abs(sn - s_ref).max() < 1e-10
    else:
        # the cut may move by one value only where eps(chi_ref - 1) is within 1e-3 of the target
        _, e_prev = oracle.trunc_rule(s, chi_ref - 1, chi_ref - 1, 0.0, 0.0)
        allowed = {chi_ref} | ({chi_ref - 1} if abs(e_prev / 1e-8 - 1) < 1e-3 else set())
        assert chi in allowed
        c = min(chi, chi_ref)
        assert np.abs(sn[:c] - s_ref[:c]).max() <= 1e-6 * s_ref[0]
        assert abs(inf[0].trunc_err - err_ref) < 2e-10
    # reconstruction against the exact truncated product
    u = a.reshape(4096, 2048)[:, :chi] / s[None, :chi]          # U columns
    vt = b.reshape(2048, 4096)[:chi]
    exact = (u * s_ref[None, :]) @ vt
    rec = Ao[0].numpy().reshape(4096, chi).astype(np.float64) @ Bo[0].numpy().reshape(chi, 4096).astype(np.float64)
    assert rel_fro(rec, exact) < (1e-10 if mode == "fp64" else 1e-5)


@pytest.fixture(scope="module")
def c2_update():
    g = synth.rng(2, 0)
    chi = 1024
    a = synth.complex_gaussian(g, (chi, 2, chi))
    b = synth.complex_gaussian(g, (chi, 2, chi))
    left = synth.hermitian_environment(g, chi)
    right = synth.hermitian_environment(g, chi)
    return a, b, left, right


def test_c2_theta_and_heff_sampled(T, ctx, c2_update):
    """theta = A.B and H_eff theta at chi = 1024: sampled rows recomputed by the oracle."""
    a, b, left, right = c2_update
    w = synth.heisenberg_mpo()
    th = T.contract(ctx, up(T, ctx, a, T.C128), "asm", up(T, ctx, b, T.C128), "mtb", "astb")
    thn = th.numpy()
    rows = [0, 517, 1023]
    for r in rows:
        ref = oracle.contract(a[r:r + 1], "asm", b, "mtb", "astb")
        assert rel_fro(thn[r:r + 1], ref) < 1e-13
    y = T.heff_matvec(ctx, up(T, ctx, left, T.C128), up(T, ctx, w, T.C128), up(T, ctx, w, T.C128),
                      up(T, ctx, right, T.C128), th).numpy()
    for r in [3, 700]:
        ref = odmrg.heff_apply(np.ascontiguousarray(left[r:r + 1]), w, w, right, thn)
        assert rel_fro(y[r:r + 1], ref) < 1e-12


def test_c2_heff_mixed_sampled_rows(T, ctx, c2_update):
    """The benchmark's mixed matvec at chi = 1024 (complex64 storage,
    split-BF16x3 L- and R-steps, FP32 middle step): sampled rows of H_eff x
    against the FP64 oracle on the same complex64-rounded operands, <= 1e-5
    relative, and within twice the error of the split's emulation."""
    a, b, left, right = c2_update
    w = synth.heisenberg_mpo()
    x = synth.complex_gaussian(synth.rng(2, 1), (1024, 2, 2, 1024))
    c64 = lambda z: np.asarray(z).astype(np.complex64)
    ctx.set_precision(T.PREC_BF16X3)
    try:
        y = T.heff_matvec(ctx, up(T, ctx, c64(left), T.C64), up(T, ctx, c64(w), T.C64), up(T, ctx, c64(w), T.C64),
                          up(T, ctx, c64(right), T.C64), up(T, ctx, c64(x), T.C64)).numpy()
    finally:
        ctx.set_precision(T.PREC_FP32)
    st = bf16.to_storage
    for rows in ([5], [400, 1022]):
        ref = odmrg.heff_apply(np.ascontiguousarray(st(left)[rows]), st(w), st(w), st(right), st(x))
        emu = bf16.heff_x3_rows(left, w, w, right, x, rows)
        err, err_emu = rel_fro(y[rows], ref), rel_fro(emu, ref)
        print(f"heff chi=1024 rows {rows} bf16x3: GPU {err:.3e} emulation {err_emu:.3e}")
        assert err <= 1e-5 and err <= 2 * err_emu, (rows, err, err_emu)


def test_c2_mixed_update_power_law_exact_spectrum(T, ctx):
    """The benchmark's mixed update at chi = 1024 (complex64 A, B; split-
    BF16x3 theta = A.B; FP64 Gram, eigensolve and orthogonalisation) on
    theta = U diag(s) V^H with Haar U, V (2048 x 1024) and s_k ~ k^-2, whose
    truncation is known in closed form: kept values within 1e-6 normwise of
    s / ||s_kept||, chi by the rule (shifted only at the threshold),
    isometric U and a truncated product within 1e-5 of the exact one."""
    g = synth.rng(2, 4000)
    s = synth.power_spectrum(1024, 2.0)
    a, b = synth.two_site_blocks_from_spectrum(g, 1024, 2, s)
    chi_ref, err_ref = oracle.trunc_rule(s, 1, 1024, 1e-8, 0.0)
    p = T.update_params(chi_min=1, chi_max=1024, target_trunc_err=1e-8, direction=1, precision=T.PREC_BF16X3)
    Ao, so, Bo, inf = T.two_site_update_batched(ctx, [up(T, ctx, a.astype(np.complex64), T.C64)],
                                                [up(T, ctx, b.astype(np.complex64), T.C64)], None, p)
    chi = inf[0].chi
    assert chi_allowed(chi, chi_ref, s, float(np.sum(s ** 2)), err_ref, 1e-8, 1024), (chi, chi_ref)
    c = min(chi, chi_ref)
    sn = so[0].numpy()
    s_ref = s[:chi_ref] / np.linalg.norm(s[:chi_ref])
    assert np.abs(sn[:c] - s_ref[:c]).max() <= 1e-6 * s_ref[0]
    eps_exact = float(np.sum(s[chi:] ** 2) / np.sum(s ** 2))        # the rule's error at the GPU's chi
    assert inf[0].trunc_err <= 1e-8 and abs(inf[0].trunc_err - eps_exact) <= 1e-3 * 1e-8
    vh = Bo[0].numpy().reshape(chi, 2048).astype(np.complex128)
    assert np.abs(vh @ vh.conj().T - np.eye(chi)).max() < 1e-5
    u = a.reshape(2048, 1024)[:, :chi] / s[None, :chi]
    exact = (u * (s[:chi] / np.linalg.norm(s[:chi]))[None, :]) @ b.reshape(1024, 2048)[:chi]
    rec = Ao[0].numpy().reshape(2048, chi).astype(np.complex128) @ vh
    assert rel_fro(rec, exact) < 1e-5


def test_c2_split_properties_full_size(T, ctx, c2_update):
    """trunc_svd of a 2048 x 2048 theta (eps 1e-8, cap 1024): isometric factors,
    discarded weight equals ||theta - U S V^H||^2, and the Lanczos Ritz value
    agrees with the Rayleigh quotient of the returned vector."""
    a, b, left, right = c2_update
    w = synth.heisenberg_mpo()
    th = T.contract(ctx, up(T, ctx, a, T.C128), "asm", up(T, ctx, b, T.C128), "mtb", "astb")
    e = T.lanczos_ground(ctx, up(T, ctx, left, T.C128), up(T, ctx, w, T.C128), up(T, ctx, w, T.C128),
                         up(T, ctx, right, T.C128), th, 20)
    psi = th.numpy()
    assert np.linalg.norm(psi) == pytest.approx(1.0, abs=1e-12)
    hpsi = T.heff_matvec(ctx, up(T, ctx, left, T.C128), up(T, ctx, w, T.C128), up(T, ctx, w, T.C128),
                         up(T, ctx, right, T.C128), th).numpy()
    rq = np.vdot(psi.reshape(-1), hpsi.reshape(-1))
    assert abs(rq.imag) < 1e-9 * abs(rq.real)
    assert rq.real == pytest.approx(e, rel=1e-10)
    p = T.update_params(chi_min=1, chi_max=1024, target_trunc_err=1e-8, direction=0)
    Ao, so, Bo, inf = T.split_batched(ctx, [th], p)
    chi = inf[0].chi
    assert chi == 1024 and inf[0].trunc_err > 1e-8          # the cap binds for this spectrum
    U = Ao[0].numpy().reshape(2048, chi)
    Vh = Bo[0].numpy().reshape(chi, 2048)
    sn = so[0].numpy()
    assert np.abs(U.conj().T @ U - np.eye(chi)).max() < 1e-11
    Vr = Vh / sn[:, None]                                    # direction LEFT: B' = diag(s) V^H
    assert np.abs(Vr @ Vr.conj().T - np.eye(chi)).max() < 1e-10
    W = inf[0].norm2
    kept = W - inf[0].discarded_abs
    rec = (U * (sn * math.sqrt(kept))[None, :]) @ Vr
    resid2 = np.linalg.norm(psi.reshape(2048, 2048) - rec) ** 2
    assert resid2 == pytest.approx(inf[0].discarded_abs, rel=1e-6)


def test_c5_randomized_power_law_full_size(T, ctx):
    """2048 x 2048 float32 theta = U diag(s) V^T with s_k ~ k^-alpha: the
    randomized path with a sketch covering chi* accepts and reproduces the
    known singular values; alpha = 1.2 exceeds the cap and falls back."""
    for alpha, expect_fallback in [(2.5, False), (1.2, True)]:
        g = synth.rng(5, int(alpha * 100))
        s = synth.power_spectrum(2048, alpha)
        a, b = synth.two_site_blocks_from_spectrum(g, 1024, 2, s, complex_=False)
        theta = np.einsum("asm,mtb->astb", a, b).astype(np.float32)
        chi_ref, _ = oracle.trunc_rule(s, 1, 1024, 1e-8, 0.0)
        p = T.update_params(chi_min=1, chi_max=1024, target_trunc_err=1e-8, direction=1,
                            svd_mode=T.SVD_RANDOMIZED, sketch_rank=min(2048, chi_ref + 64), power_iters=2, seed=9,
                            precision=T.PREC_BF16X3)
        Ao, so, Bo, inf = T.split_batched(ctx, [up(T, ctx, theta, T.F32)], p)
        assert bool(inf[0].used_fallback) == expect_fallback
        c = min(inf[0].chi, chi_ref)
        _, err_ref = oracle.trunc_rule(s, 1, 1024, 1e-8, 0.0)
        assert chi_allowed(inf[0].chi, chi_ref, s, float(np.sum(s ** 2)), err_ref, 1e-8, 1024)
        sn = so[0].numpy()
        s_ref = s[:chi_ref] / np.linalg.norm(s[:chi_ref])
        assert np.abs(sn[:c] - s_ref[:c]).max() <= 1e-6 * s_ref[0]


@pytest.mark.slow
@pytest.mark.parametrize("dt", ["C128", "C64"])
def test_split_batch_of_64_matches_single_problems(T, ctx, dt):
    """The benchmark's launch configuration: one split of 64 full-size
    (1024, 2, 2, 1024) two-site tensors.  Sampled problems of the batch must
    equal the same problem split alone (the batch shares launches, not
    arithmetic), and every problem's factors are isometric with
    discarded weight = ||theta - U S V^H||^2."""
    g = torch.Generator(device="cuda")
    g.manual_seed(251223917 + 2000)
    tdt = torch.complex128 if dt == "C128" else torch.complex64
    thetas_t = [torch.randn((1024, 2, 2, 1024), dtype=tdt, device="cuda", generator=g) for _ in range(64)]
    thetas = [T.Tensor.from_torch(ctx, x) for x in thetas_t]
    p = T.update_params(chi_min=1, chi_max=1024, target_trunc_err=1e-8, direction=0,
                        precision=T.PREC_FP64 if dt == "C128" else T.PREC_BF16X3)
    Ao, so, Bo, inf = T.split_batched(ctx, thetas, p)
    assert all(i.chi == 1024 for i in inf)
    for k in (0, 29, 63):
        A1, s1, B1, i1 = T.split_batched(ctx, [thetas[k]], p)
        assert i1[0].chi == inf[k].chi
        assert i1[0].trunc_err == pytest.approx(inf[k].trunc_err, rel=1e-12)
        np.testing.assert_allclose(s1[0].numpy(), so[k].numpy(), rtol=0, atol=1e-13)
        ra = Ao[k].numpy().reshape(2048, -1) @ Bo[k].numpy().reshape(-1, 2048)
        rb = A1[0].numpy().reshape(2048, -1) @ B1[0].numpy().reshape(-1, 2048)
        assert rel_fro(ra, rb) < (1e-12 if dt == "C128" else 1e-6)
        U = Ao[k].numpy().reshape(2048, -1).astype(np.complex128)
        tol = 1e-11 if dt == "C128" else 1e-5
        assert np.abs(U.conj().T @ U - np.eye(U.shape[1])).max() < tol
        th = thetas_t[k].cpu().numpy().reshape(2048, 2048).astype(np.complex128)
        Vh = Bo[k].numpy().reshape(-1, 2048).astype(np.complex128)
        sn = so[k].numpy()
        kept = inf[k].norm2 - inf[k].discarded_abs
        rec = U @ (Vh * math.sqrt(kept))
        resid2 = np.linalg.norm(th - rec) ** 2
        assert resid2 == pytest.approx(inf[k].discarded_abs, rel=1e-6 if dt == "C128" else 1e-4)
        assert np.sum(sn ** 2) == pytest.approx(1.0, rel=1e-12)


def test_headline_batch_learned_matches_plain_fp64(T, ctx):
    """The headline batch (64 TEBD updates at chi = 1024, power-law bonds, Haar
    gates) through the learned + mixed path, which reduces the problems the
    network sends to the plain SVD on the second stream and sketches the
    rest, against the plain FP64 path on the same inputs: kept singular
    values at 1e-6 of s_1, chi under the threshold rule, and the truncated
    reconstruction A'.B' at the mixed bar (1e-5)."""
    import bench
    from paper_2512_23917_amd import sketch_train
    host = bench.headline_inputs(64, 1024)
    ins_m = bench.upload_headline(T, ctx, host, T.C64)
    ins_p = bench.upload_headline(T, ctx, host, T.C128)
    model = T.SketchModel(ctx, path=sketch_train.DEFAULT_WEIGHTS)
    pm = T.update_params(chi_min=1, chi_max=1024, target_trunc_err=1e-8, direction=T.DIR_RIGHT,
                         precision=T.PREC_BF16X3, svd_mode=T.SVD_LEARNED, power_iters=2, seed=1)
    pm.sketch_model = model.h.value
    Am, sm, Bm, im = T.two_site_update_batched(ctx, *ins_m[:3], pm, prev_spectra=ins_m[3])
    pp = T.update_params(chi_min=1, chi_max=1024, target_trunc_err=1e-8, direction=T.DIR_RIGHT,
                         precision=T.PREC_FP64)
    Ap, sp, Bp, ip = T.two_site_update_batched(ctx, *ins_p[:3], pp)
    plain = sum(1 for i in im if i.sketch_rank == 0 or i.used_fallback)
    print(f"learned batch: {plain} plain, {64 - plain} sketched", flush=True)
    assert plain >= 12 and plain < 64          # the second-stream batch and the sketches both ran
    for u in range(64):
        i_m, i_p = im[u], ip[u]
        s_p = sp[u].numpy()
        kept_p = i_p.norm2 - i_p.discarded_abs
        s_raw = s_p * math.sqrt(kept_p)
        assert chi_allowed(i_m.chi, i_p.chi, s_raw, i_p.norm2, i_p.trunc_err, 1e-8, 1024), (u, i_m.chi, i_p.chi)
        c = min(i_m.chi, i_p.chi)
        s_m = sm[u].numpy()
        assert np.abs(s_m[:c] - s_p[:c]).max() <= 1e-6 * s_p[0], u
        am = Am[u].numpy().reshape(-1, i_m.chi)[:, :c].astype(np.complex128)
        bm = Bm[u].numpy().reshape(i_m.chi, -1)[:c].astype(np.complex128)
        ap = Ap[u].numpy().reshape(-1, i_p.chi)[:, :c]
        bp = Bp[u].numpy().reshape(i_p.chi, -1)[:c]
        assert rel_fro(am @ bm, ap @ bp) <= 1e-5, u
    model.close()
