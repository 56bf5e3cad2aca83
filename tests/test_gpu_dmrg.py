"""GPU parity of the DMRG pieces (effective-Hamiltonian matvec, Lanczos,
split of a given two-site tensor) against the CPU oracle."""
import numpy as np
import pytest

import oracle
from oracle import bf16
from oracle import dmrg as odmrg
from oracle import mps as omps
from paper_2512_23917_amd import synth

from gpu_util import rel_fro

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


def env(chi, seed, complex_=True):
    g = synth.rng(2, seed)
    left = synth.hermitian_environment(g, chi, complex_)
    right = synth.hermitian_environment(g, chi, complex_)
    w = synth.heisenberg_mpo()
    x = synth.complex_gaussian(g, (chi, 2, 2, chi)) if complex_ else synth.real_gaussian(g, (chi, 2, 2, chi))
    if not complex_:
        w = w.real
    return left, w, right, x


@pytest.mark.parametrize("chi", [1, 3, 16, 40])
def test_heff_matvec_fp64(T, ctx, chi):
    left, w, right, x = env(chi, chi)
    ref = odmrg.heff_apply(left, w, w, right, x)
    y = T.heff_matvec(ctx, up(T, ctx, left, T.C128), up(T, ctx, w, T.C128), up(T, ctx, w, T.C128),
                      up(T, ctx, right, T.C128), up(T, ctx, x, T.C128)).numpy()
    assert rel_fro(y, ref) < 1e-13


def test_heff_matvec_real(T, ctx):
    left, w, right, x = env(12, 5, complex_=False)
    ref = odmrg.heff_apply(left, w, w, right, x)
    y = T.heff_matvec(ctx, up(T, ctx, left, T.F64), up(T, ctx, w, T.F64), up(T, ctx, w, T.F64),
                      up(T, ctx, right, T.F64), up(T, ctx, x, T.F64)).numpy()
    assert rel_fro(y, ref) < 1e-13


@pytest.mark.parametrize("prec,tol,chi,complex_", [("PREC_FP32", 3e-6, 24, True), ("PREC_BF16X3", 1e-5, 24, True),
                                                   ("PREC_BF16X3", 1e-5, 200, True),
                                                   ("PREC_BF16X3", 1e-5, 72, False),
                                                   ("PREC_FP32", 3e-6, 72, False)])
def test_heff_matvec_mixed(T, ctx, prec, tol, chi, complex_):
    """Mixed H_eff matvec against the FP64 oracle on the same FP32 operands:
    <= 1e-5 relative Frobenius; split-BF16x3 also within twice the error of
    its emulation (the same three steps with exact partial products and FP64
    sums, FP32 storage between the steps).  chi = 200: the environment planes
    are 1000 x 200 and the vector planes 800 x 200, i.e. ragged in every
    padded dimension of the plane GEMM."""
    left, w, right, x = env(chi, 9, complex_)
    lo = np.complex64 if complex_ else np.float32
    dt = T.C64 if complex_ else T.F32
    c64 = lambda a: np.asarray(a).astype(lo)
    ref = odmrg.heff_apply(c64(left).astype(np.complex128), c64(w).astype(np.complex128),
                           c64(w).astype(np.complex128), c64(right).astype(np.complex128),
                           c64(x).astype(np.complex128))
    ctx.set_precision(getattr(T, prec))
    try:
        y = T.heff_matvec(ctx, up(T, ctx, c64(left), dt), up(T, ctx, c64(w), dt), up(T, ctx, c64(w), dt),
                          up(T, ctx, c64(right), dt), up(T, ctx, c64(x), dt)).numpy()
    finally:
        ctx.set_precision(T.PREC_FP32)
    err = rel_fro(y, ref)
    assert err < tol
    if prec == "PREC_BF16X3":
        emu = bf16.heff_x3_rows(left, w, w, right, x, np.arange(chi))
        err_emu = rel_fro(emu, ref)
        print(f"heff chi={chi} complex={complex_} bf16x3: GPU {err:.3e} emulation {err_emu:.3e}")
        assert err <= 2 * err_emu, (err, err_emu)


def test_heff_trivial_environment_spectrum(T, ctx):
    left, right = synth.trivial_environments()
    w = synth.heisenberg_mpo()
    cols = []
    for k in range(4):
        e = np.zeros(4, dtype=np.complex128)
        e[k] = 1.0
        y = T.heff_matvec(ctx, up(T, ctx, left, T.C128), up(T, ctx, w, T.C128), up(T, ctx, w, T.C128),
                          up(T, ctx, right, T.C128), up(T, ctx, e.reshape(1, 2, 2, 1), T.C128)).numpy()
        cols.append(y.reshape(-1))
    h = np.stack(cols, axis=1)
    np.testing.assert_allclose(np.linalg.eigvalsh(h), [-0.75, 0.25, 0.25, 0.25], atol=1e-15)


@pytest.mark.parametrize("chi,nmv", [(2, 16), (6, 20), (16, 20)])
def test_lanczos_matches_oracle(T, ctx, chi, nmv):
    left, w, right, x = env(chi, 100 + chi)
    mv = lambda v: odmrg.heff_apply(left, w, w, right, v)
    e_ref, psi_ref, _, _ = odmrg.lanczos_ground(mv, x, n_matvec=nmv)
    th = up(T, ctx, x, T.C128)
    e = T.lanczos_ground(ctx, up(T, ctx, left, T.C128), up(T, ctx, w, T.C128), up(T, ctx, w, T.C128),
                         up(T, ctx, right, T.C128), th, nmv)
    assert e == pytest.approx(e_ref, rel=1e-10)
    assert rel_fro(th.numpy(), psi_ref) < 1e-8
    if chi == 2:
        h = odmrg.heff_dense(left, w, w, right)
        assert e == pytest.approx(np.linalg.eigvalsh(h)[0], rel=1e-11)


@pytest.mark.parametrize("prec,chi", [("PREC_FP32", 16), ("PREC_BF16X3", 16), ("PREC_BF16X3", 128)])
def test_lanczos_mixed_energy(T, ctx, prec, chi):
    """The mixed path's Ritz value (complex64 storage of the operands and of
    the Krylov basis, FP64 recurrence) against the oracle's FP64 Lanczos on
    the same complex64-rounded operands: relative 1e-5."""
    left, w, right, x = env(chi, 77)
    s = bf16.to_storage
    mv = lambda v: odmrg.heff_apply(s(left), s(w), s(w), s(right), v)
    e_ref, psi_ref, _, _ = odmrg.lanczos_ground(mv, s(x), n_matvec=20)
    c64 = lambda a: np.asarray(a).astype(np.complex64)
    th = up(T, ctx, c64(x), T.C64)
    ctx.set_precision(getattr(T, prec))
    try:
        e = T.lanczos_ground(ctx, up(T, ctx, c64(left), T.C64), up(T, ctx, c64(w), T.C64),
                             up(T, ctx, c64(w), T.C64), up(T, ctx, c64(right), T.C64), th, 20)
    finally:
        ctx.set_precision(T.PREC_FP32)
    assert e == pytest.approx(e_ref, rel=1e-5)


def test_split_batched_matches_oracle(T, ctx):
    g = synth.rng(2, 5)
    thetas = [synth.complex_gaussian(g, (20, 2, 2, 24)) for _ in range(3)]
    p = T.update_params(chi_min=1, chi_max=30, target_trunc_err=1e-4, direction=1)
    Ao, so, Bo, infos = T.split_batched(ctx, [up(T, ctx, t, T.C128) for t in thetas], p)
    for i, th in enumerate(thetas):
        u, s, vh, err = oracle.trunc_svd(th, 2, 1, 30, 1e-4, 0.0)
        assert infos[i].chi == len(s)
        assert infos[i].trunc_err == pytest.approx(err, rel=1e-8)
        sn = s / np.linalg.norm(s)
        np.testing.assert_allclose(so[i].numpy(), sn, atol=1e-12)
        rec = np.einsum("asm,mtb->astb", Ao[i].numpy(), Bo[i].numpy())
        rec_o = np.einsum("asm,mtb->astb", u * sn[None, None, :], vh)
        assert rel_fro(rec, rec_o) < 1e-10


def test_dmrg_update_pipeline_matches_oracle(T, ctx):
    """theta0 = A.B, 20 Lanczos matvecs, trunc_svd (eps 1e-8, chi <= 24), renormalise."""
    chi = 12
    g = synth.rng(2, 9)
    a, b = synth.complex_gaussian(g, (chi, 2, chi)), synth.complex_gaussian(g, (chi, 2, chi))
    left = synth.hermitian_environment(g, chi)
    right = synth.hermitian_environment(g, chi)
    w = synth.heisenberg_mpo()
    theta0 = omps.theta_of(a, b)
    mv = lambda v: odmrg.heff_apply(left, w, w, right, v)
    e_ref, psi, _, _ = odmrg.lanczos_ground(mv, theta0, 20)
    u, s, vh, err = oracle.trunc_svd(psi, 2, 1, 24, 1e-8, 0.0)
    th = T.contract(ctx, up(T, ctx, a, T.C128), "asm", up(T, ctx, b, T.C128), "mtb", "astb")
    e = T.lanczos_ground(ctx, up(T, ctx, left, T.C128), up(T, ctx, w, T.C128), up(T, ctx, w, T.C128),
                         up(T, ctx, right, T.C128), th, 20)
    assert e == pytest.approx(e_ref, rel=1e-10)
    p = T.update_params(chi_min=1, chi_max=24, target_trunc_err=1e-8, direction=1)
    Ao, so, Bo, infos = T.split_batched(ctx, [th], p)
    assert infos[0].chi == len(s)
    rec = np.einsum("asm,mtb->astb", Ao[0].numpy(), Bo[0].numpy())
    sn = s / np.linalg.norm(s)
    assert rel_fro(rec, np.einsum("asm,mtb->astb", u * sn[None, None, :], vh)) < 1e-8


def test_lanczos_second_gram_schmidt_pass(T, capfd):
    """Non-Hermitian environments on a 16-dimensional space: the residual of
    the three-term recurrence keeps large components along the older Krylov
    vectors, so the first Gram-Schmidt pass removes most of its norm and the
    conditional second pass runs (the device takes that decision; the call
    reports how often at verbosity 1).  The result must still equal the
    oracle's, which always takes two passes (the same quantities in exact
    arithmetic)."""
    g = synth.rng(2, 4242)
    chi = 2
    left = synth.complex_gaussian(g, (chi, 5, chi))
    right = synth.complex_gaussian(g, (chi, 5, chi))
    w = synth.heisenberg_mpo()
    x = synth.complex_gaussian(g, (chi, 2, 2, chi))
    mv = lambda v: odmrg.heff_apply(left, w, w, right, v)
    e_ref, psi_ref, _, _ = odmrg.lanczos_ground(mv, x, n_matvec=15)
    e, psi, fields = lanczos_logged(T, capfd, left, w, right, x, 15)
    assert 1 <= fields["krylov"] <= 15
    assert fields["reorth"] >= 1
    assert fields["host_syncs"] == 1
    assert e == pytest.approx(e_ref, rel=1e-9)
    assert rel_fro(psi, psi_ref) < 1e-7


def lanczos_logged(T, capfd, left, w, right, x, nmv):
    """Runs the solve on a verbosity-1 context; returns (energy, psi, fields
    of the call's log line)."""
    c = T.Context(0, verbosity=1)
    try:
        th = up(T, c, x, T.C128)
        capfd.readouterr()
        e = T.lanczos_ground(c, up(T, c, left, T.C128), up(T, c, w, T.C128), up(T, c, w, T.C128),
                             up(T, c, right, T.C128), th, nmv)
        psi = th.numpy()
        del th
    finally:
        c.close()
    err = capfd.readouterr().err
    line = [l for l in err.splitlines() if l.startswith("TCI_VERBOSE: lanczos_ground")]
    assert len(line) == 1, err
    fields = dict(f.split("=") for f in line[0].split() if f.count("=") == 1 and not f.startswith("m="))
    return e, psi, {k: int(v) for k, v in fields.items()}


def test_lanczos_breakdown_matches_oracle(T, capfd):
    """Trivial environments reduce H_eff to the two-site Heisenberg bond, whose
    two distinct eigenvalues (-3/4 and 1/4) make the Krylov space of any start
    vector at most two-dimensional: beta_1 vanishes and the recurrence stops
    after the second matvec although ten were allowed.  The device decides the
    breakdown on its own; T has the oracle's order, the energy is -3/4 and the
    Ritz vector the oracle's.  One host synchronisation per solve."""
    left, right = synth.trivial_environments()
    w = synth.heisenberg_mpo()
    x = synth.complex_gaussian(synth.rng(2, 31), (1, 2, 2, 1))
    mv = lambda v: odmrg.heff_apply(left, w, w, right, v)
    e_ref, psi_ref, alphas, _ = odmrg.lanczos_ground(mv, x, n_matvec=10)
    e, psi, f = lanczos_logged(T, capfd, left, w, right, x, 10)
    assert f["krylov"] == len(alphas) == 2
    assert f["host_syncs"] == 1
    assert e == pytest.approx(-0.75, abs=1e-13)
    assert e == pytest.approx(e_ref, abs=1e-13)
    assert rel_fro(psi, psi_ref) < 1e-12


def test_lanczos_eigenvector_start(T, capfd):
    """Started at the singlet (an eigenvector), the first residual is zero:
    T is the single entry -3/4 and theta comes back as the singlet."""
    left, right = synth.trivial_environments()
    w = synth.heisenberg_mpo()
    x = np.zeros((1, 2, 2, 1), dtype=np.complex128)
    x[0, 0, 1, 0], x[0, 1, 0, 0] = 1 / np.sqrt(2), -1 / np.sqrt(2)
    e, psi, f = lanczos_logged(T, capfd, left, w, right, x, 20)
    assert f["krylov"] == 1
    assert e == pytest.approx(-0.75, abs=1e-15)
    np.testing.assert_allclose(psi, x, atol=1e-15)


@pytest.mark.parametrize("bad", ["zero", "nan"])
def test_lanczos_bad_start_vector(T, ctx, bad):
    """A start vector with zero or non-finite norm is reported as
    TCI_ERR_NUMERIC after the queued solve, and theta is left as it was."""
    left, w, right, x = env(3, 55)
    x = np.zeros_like(x) if bad == "zero" else x.copy()
    if bad == "nan":
        x[1, 0, 1, 2] = np.nan
    th = up(T, ctx, x, T.C128)
    with pytest.raises(T.TciError) as ei:
        T.lanczos_ground(ctx, up(T, ctx, left, T.C128), up(T, ctx, w, T.C128), up(T, ctx, w, T.C128),
                         up(T, ctx, right, T.C128), th, 12)
    assert T.STATUS[ei.value.status] == "NUMERIC"
    np.testing.assert_array_equal(th.numpy(), x)
    # the context is usable afterwards
    e = T.lanczos_ground(ctx, up(T, ctx, left, T.C128), up(T, ctx, w, T.C128), up(T, ctx, w, T.C128),
                         up(T, ctx, right, T.C128), up(T, ctx, env(3, 55)[3], T.C128), 12)
    assert np.isfinite(e)
