"""GPU checks of the C-ABI boundary: context options (allocator callbacks,
svd mode, autotune cache, verbosity), the Vidal write-back of the update
composite, the single-update entry point, and eigh / eigvalsh on matricised
tensors -- each against the CPU oracle or the definition it follows."""
import ctypes
import os

import numpy as np
import pytest

import oracle
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


def up(T, ctx, a, dtype):
    return T.Tensor.from_numpy(ctx, np.asarray(a), dtype)


def _vidal_rebuild(a_out, s, b_out, lam_l, lam_r):
    """theta_trunc = diag(l_l) Gamma_A diag(s) Gamma_B diag(l_r) (App. A)."""
    return np.einsum("a,asm,m,mtb,b->astb", lam_l, a_out, s, b_out, lam_r)


@pytest.mark.parametrize("dtype,chi_l,chi_m,chi_r,chi_max,tol", [
    ("C128", 12, 20, 9, 14, 1e-10),       # Jacobi route (min(m, n) <= 64)
    ("C128", 48, 80, 40, 60, 1e-10),      # Gram route
    ("F64", 33, 40, 35, 50, 1e-10),
    ("C64", 40, 64, 36, 50, 1e-5),        # mixed: gauge-invariant rebuild only
])
def test_vidal_write_back_matches_oracle(T, ctx, dtype, chi_l, chi_m, chi_r, chi_max, tol):
    """Gamma_A = diag(1/l_l) U, Gamma_B = V^dag diag(1/l_r), Lambda = s/||s||
    (App. A); the oracle's VIDAL branch on the same inputs."""
    g = np.random.default_rng(77)
    cplx = dtype in ("C128", "C64")
    mk = (lambda s: synth.complex_gaussian(g, s)) if cplx else (lambda s: g.standard_normal(s))
    a, b = mk((chi_l, 2, chi_m)), mk((chi_m, 2, chi_r))
    gate = synth.haar_gate(g) if cplx else np.linalg.qr(g.standard_normal((4, 4)))[0]
    lam_l = np.sort(g.uniform(0.05, 1.0, chi_l))[::-1].copy()
    lam_r = np.sort(g.uniform(0.05, 1.0, chi_r))[::-1].copy()
    ref = omps.two_site_update(a, b, gate, 1, chi_max, 1e-10, 0.0, omps.VIDAL, lam_l, lam_r)
    dt = getattr(T, dtype)
    prec = {"C128": T.PREC_FP64, "F64": T.PREC_FP64, "C64": T.PREC_BF16X3}[dtype]
    p = T.update_params(chi_min=1, chi_max=chi_max, target_trunc_err=1e-10, direction=T.DIR_VIDAL, precision=prec)
    Ao, so, Bo, inf = T.two_site_update_batched(ctx, [up(T, ctx, a, dt)], [up(T, ctx, b, dt)], [up(T, ctx, gate, dt)],
                                                p, lambda_left=[up(T, ctx, lam_l, T.F64)],
                                                lambda_right=[up(T, ctx, lam_r, T.F64)])
    assert inf[0].chi == ref["chi"]
    s = so[0].numpy()
    assert np.abs(s - ref["s"]).max() <= (1e-12 if tol < 1e-6 else 1e-6)
    rec = _vidal_rebuild(Ao[0].numpy().astype(np.complex128), s, Bo[0].numpy().astype(np.complex128), lam_l, lam_r)
    rec_ref = _vidal_rebuild(ref["a_out"], ref["s"], ref["b_out"], lam_l, lam_r)
    assert rel_fro(rec, rec_ref) <= tol
    # pointers set for the call are cleared afterwards
    assert not p.lambda_left and not p.lambda_right


def test_vidal_needs_positive_weights(T, ctx):
    g = np.random.default_rng(3)
    a, b = synth.complex_gaussian(g, (4, 2, 5)), synth.complex_gaussian(g, (5, 2, 6))
    p = T.update_params(chi_min=1, chi_max=8, direction=T.DIR_VIDAL)
    bad = np.ones(4)
    bad[2] = 0.0
    with pytest.raises(T.TciError) as e:
        T.two_site_update_batched(ctx, [up(T, ctx, a, T.C128)], [up(T, ctx, b, T.C128)], None, p,
                                  lambda_left=[up(T, ctx, bad, T.F64)], lambda_right=[up(T, ctx, np.ones(6), T.F64)])
    assert e.value.status == 8
    with pytest.raises(T.TciError) as e:       # wrong length
        T.two_site_update_batched(ctx, [up(T, ctx, a, T.C128)], [up(T, ctx, b, T.C128)], None, p,
                                  lambda_left=[up(T, ctx, np.ones(5), T.F64)], lambda_right=[up(T, ctx, np.ones(6), T.F64)])
    assert e.value.status == 2
    with pytest.raises(T.TciError) as e:       # no weights
        T.two_site_update_batched(ctx, [up(T, ctx, a, T.C128)], [up(T, ctx, b, T.C128)], None, p)
    assert e.value.status == 1


@pytest.mark.parametrize("direction", [0, 1])
def test_single_update_equals_oracle(T, ctx, direction):
    g = np.random.default_rng(5)
    a, b = synth.complex_gaussian(g, (70, 2, 90)), synth.complex_gaussian(g, (90, 2, 66))
    gate = synth.haar_gate(g)
    ref = omps.two_site_update(a, b, gate, 1, 100, 1e-9, 0.0, direction)
    p = T.update_params(chi_min=1, chi_max=100, target_trunc_err=1e-9, direction=direction)
    Ao, so, Bo, inf = T.two_site_update(ctx, up(T, ctx, a, T.C128), up(T, ctx, b, T.C128), up(T, ctx, gate, T.C128), p)
    assert inf.chi == ref["chi"]
    assert np.abs(so.numpy() - ref["s"]).max() < 1e-12
    rec = np.einsum("asm,mtb->astb", Ao.numpy(), Bo.numpy())
    rec_ref = np.einsum("asm,mtb->astb", ref["a_out"], ref["b_out"])
    assert rel_fro(rec, rec_ref) < 1e-10


@pytest.mark.parametrize("dtype", ["C128", "F64", "C64", "F32"])
def test_eigh_and_eigvalsh_on_matricised_tensors(T, ctx, dtype):
    """tci_eigh / tci_eigvalsh with k_rows = 2 on an order-3 tensor
    {3, 4, 12}: eigenvalues ascending (oracle Jacobi eigensolver), vectors
    {3, 4, 12} with A V = V diag(w)."""
    g = np.random.default_rng(19)
    cplx = dtype in ("C128", "C64")
    m = synth.complex_gaussian(g, (12, 12)) if cplx else g.standard_normal((12, 12))
    h = m + m.conj().T
    w_ref, _ = oracle.eigh(h)
    dt = getattr(T, dtype)
    a = up(T, ctx, h.reshape(3, 4, 12), dt)
    w, v = T.eigh(ctx, a, 2)
    assert tuple(v.shape()) == (3, 4, 12) and tuple(w.shape()) == (12,)
    single = dtype in ("C64", "F32")
    tol = 1e-5 if single else 1e-12
    hq = h.astype(np.complex64 if cplx else np.float32).astype(np.complex128) if single else h
    wn = w.numpy().astype(np.float64)
    assert np.abs(wn - w_ref).max() <= tol * np.abs(w_ref).max()
    vm = v.numpy().reshape(12, 12).astype(np.complex128)
    assert np.abs(hq @ vm - vm * wn[None, :]).max() <= 10 * tol * np.abs(w_ref).max()
    w2 = T.eigvalsh(ctx, a, 2).numpy()
    assert np.abs(w2.astype(np.float64) - wn).max() <= tol * np.abs(w_ref).max()
    with pytest.raises(T.TciError) as e:
        T.eigvalsh(ctx, up(T, ctx, h.reshape(3, 4, 12), dt), 1)    # 3 x 48: not square
    assert e.value.status == 2


def test_eigh_large_matches_oracle(T, ctx):
    """A 300 x 300 Hermitian matrix (several reduction panels) through
    eigvalsh: ascending values against the oracle to 1e-12 relative."""
    g = np.random.default_rng(23)
    m = synth.complex_gaussian(g, (300, 300))
    h = m + m.conj().T
    w_ref, _ = oracle.eigh(h)
    w = T.eigvalsh(ctx, up(T, ctx, h, T.C128), 1).numpy()
    assert np.abs(w - w_ref).max() <= 1e-12 * np.abs(w_ref).max()


def test_context_allocator_callbacks(T):
    """Every device buffer of the context comes from the callbacks and goes
    back through them; an allocator that fails yields TCI_ERR_OUT_OF_MEMORY
    (and no C++ exception crosses the ABI)."""
    live = {}
    log = {"alloc": 0, "free": 0}

    def alloc(n, s):
        ptr = torch.cuda.caching_allocator_alloc(int(n), 0)
        live[ptr] = n
        log["alloc"] += 1
        return ptr

    def free(ptr, n, s):
        assert live.pop(ptr) == n
        torch.cuda.caching_allocator_delete(ptr)
        log["free"] += 1

    c = T.Context(0, allocator=(alloc, free))
    g = np.random.default_rng(1)
    a = synth.complex_gaussian(g, (100, 2, 100))
    ta = up(T, c, a, T.C128)
    u, s, vh, _ = T.trunc_svd(c, ta, 2, 1, 50)
    ref = oracle.trunc_svd(a, 2, 1, 50)
    assert np.abs(s.numpy() - ref[1]).max() < 1e-12
    assert log["alloc"] >= 1
    c.close()
    assert not live and log["free"] == log["alloc"]

    def failing(n, s):
        return None

    c2 = T.Context(0, allocator=(failing, lambda p, n, s: None))
    with pytest.raises(T.TciError) as e:
        T.trunc_svd(c2, up(T, c2, a, T.C128), 2, 1, 50)
    assert e.value.status == 5
    c2.close()


def test_torch_allocator_is_the_default(T):
    """The binding hands torch's caching allocator to the library: the
    workspace of an SVD is counted in torch's allocated bytes."""
    c = T.Context(0)
    g = np.random.default_rng(2)
    a = up(T, c, synth.complex_gaussian(g, (200, 2, 200)), T.C128)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated(0)
    T.trunc_svd(c, a, 2, 1, 100)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated(0) - before >= 256 << 20      # one arena chunk
    c.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated(0) - before < 256 << 20


def test_context_svd_mode_randomized_trunc_svd(T, capfd):
    """opts.svd_mode = RANDOMIZED: tci_trunc_svd with a cap and a positive
    target sketches (rank chi_max + 64) and keeps the result when the
    discarded weight and the residual certificate pass; the values equal the
    oracle's exact truncated SVD."""
    c = T.Context(0, svd_mode=T.SVD_RANDOMIZED, verbosity=1)
    a, b, s_true = _low_rank_pair(np.random.default_rng(8), 150, 6)
    theta = np.einsum("asm,mtb->astb", a, b)
    u, s, vh, err = T.trunc_svd(c, up(T, c, theta, T.C128), 2, 1, 40, 1e-10)
    ref = oracle.trunc_svd(theta, 2, 1, 40, 1e-10)
    assert len(s.numpy()) == len(ref[1]) == 6
    np.testing.assert_allclose(s.numpy(), ref[1], rtol=0, atol=1e-12)
    rec = np.einsum("ask,k,ktb->astb", u.numpy(), s.numpy(), vh.numpy())
    assert rel_fro(rec, theta) < 1e-10
    # a full-rank matrix misses the target at the cap: the plain SVD decides
    g = np.random.default_rng(9)
    full = synth.complex_gaussian(g, (150, 2, 2, 150))
    u2, s2, vh2, err2 = T.trunc_svd(c, up(T, c, full, T.C128), 2, 1, 40, 1e-10)
    ref2 = oracle.trunc_svd(full, 2, 1, 40, 1e-10)
    np.testing.assert_allclose(s2.numpy(), ref2[1], rtol=0, atol=1e-10 * ref2[1][0])
    c.close()
    err_text = capfd.readouterr().err
    assert "randomized k=128\n" in err_text and "randomized k=128 fallback\n" in err_text


def _low_rank_pair(g, chi, r):
    """A (chi, 2, chi), B (chi, 2, chi) whose theta has rank r with known s."""
    s = np.linspace(1.0, 0.3, r)
    u = np.linalg.qr(synth.complex_gaussian(g, (2 * chi, r)))[0]
    v = np.linalg.qr(synth.complex_gaussian(g, (2 * chi, r)))[0]
    a = np.zeros((2 * chi, chi), dtype=np.complex128)
    a[:, :r] = u * s
    b = np.zeros((chi, 2 * chi), dtype=np.complex128)
    b[:r] = v.conj().T
    return a.reshape(chi, 2, chi), b.reshape(chi, 2, chi), s


def test_autotune_cache_round_trip(T, tmp_path):
    """The grouped-GEMM tile choices of a block-sparse update are written to
    the cache file when the context is destroyed and read by the next one."""
    path = str(tmp_path / "tiles.txt")
    c = T.Context(0, autotune_cache=path)
    g = synth.rng(4, 1)
    bl, bm, br = synth.u1_bond(64, 21), synth.u1_bond(64, 22), synth.u1_bond(64, 21)
    A = T.BsTensor.from_blocks(c, bl, bm, {k: v.astype(np.float32) for k, v in synth.u1_site_blocks(g, bl, bm).items()})
    B = T.BsTensor.from_blocks(c, bm, br, {k: v.astype(np.float32) for k, v in synth.u1_site_blocks(g, bm, br).items()})
    p = T.update_params(chi_min=1, chi_max=64, target_trunc_err=1e-8, direction=T.DIR_LEFT, precision=T.PREC_FP32)
    T.bs_two_site_update_batched(c, [A], [B], [None], p)
    del A, B
    c.close()
    lines = open(path).read().split("\n")
    rows = [ln.split() for ln in lines if ln.strip()]
    assert rows and all(len(r) == 39 for r in rows)
    c2 = T.Context(0, autotune_cache=path)
    c2.close()
    assert os.path.getsize(path) > 0


def test_verbosity_option_logs_calls(T, capfd):
    c = T.Context(0, verbosity=1)
    g = np.random.default_rng(4)
    T.norm(c, up(T, c, g.standard_normal((5, 5)), T.F64))
    c.close()
    assert "TCI_VERBOSE: norm" in capfd.readouterr().err
