"""Pins for the U(1) block-sparse oracle: the dense embedding of the same
update (Jacobi SVD of the dense two-site matrix) fixes the singular values,
chi, the truncation error and the truncated tensor; charge conservation and
per-sector isometry are checked directly."""
import numpy as np
import pytest

from oracle import mps as omps
from oracle import u1
from paper_2512_23917_amd import synth


def _case(chi_l, chi_m, chi_r, seed, outer=21, middle=22):
    g = synth.rng(4, seed)
    bl, bm, br = synth.u1_bond(chi_l, outer), synth.u1_bond(chi_m, middle), synth.u1_bond(chi_r, outer)
    A = synth.u1_site_blocks(g, bl, bm)
    B = synth.u1_site_blocks(g, bm, br)
    return bl, bm, br, A, B, synth.u1_gate(g)


def test_sector_profile_recipe():
    assert synth.binomial_sector_sizes(1024, 21) == [1, 1, 1, 1, 4, 15, 37, 75, 123, 164, 180, 164, 123, 75, 37,
                                                     15, 4, 1, 1, 1, 1]
    assert synth.binomial_sector_sizes(2048, 21) == [1, 1, 1, 2, 9, 30, 75, 151, 246, 328, 360, 328, 246, 151, 75,
                                                     30, 9, 2, 1, 1, 1]
    assert [q for q, _ in synth.u1_bond(64, 22)] == list(range(-21, 22, 2))


def test_gate_conserves_charge_and_is_orthogonal():
    gm = synth.u1_gate(synth.rng(4, 1))
    np.testing.assert_allclose(gm @ gm.T, np.eye(4), atol=1e-15)
    q = np.array([2, 0, 0, -2])
    assert np.all(gm[q[:, None] != q[None, :]] == 0)


@pytest.mark.parametrize("target,chi_max", [(1e-3, None), (0.0, 40), (1e-2, 25)])
def test_block_update_equals_dense_embedding(target, chi_max):
    bl, bm, br, A, B, gm = _case(32, 32, 32, 3)
    res = u1.block_update(A, B, bl, bm, br, gm, 1, chi_max, target, 0.0)
    ad, bd = u1.dense_site(A, bl, bm), u1.dense_site(B, bm, br)
    dense = omps.two_site_update(ad, bd, gm, 1, chi_max, target, 0.0, direction=omps.LEFT)
    assert res["chi"] == dense["chi"]
    assert res["trunc_err"] == pytest.approx(dense["trunc_err"], rel=1e-10, abs=1e-15)
    np.testing.assert_allclose(np.sort(res["s"])[::-1], dense["s"], atol=1e-12)
    # truncated two-site tensor (gauge free) against the dense U s V^dagger
    th = u1.truncated_theta_dense(res, bl, br)
    s = dense["s"]
    ref = np.einsum("asm,m,mtb->astb", dense["a_out"], np.ones_like(s), dense["b_out"])
    np.testing.assert_allclose(th, ref, atol=1e-11)


def test_theta_respects_charge_and_sectors_are_isometric():
    bl, bm, br, A, B, gm = _case(40, 48, 36, 5)
    th = u1.gate_blocks(u1.theta_blocks(A, B, bl, bm, br), gm)
    for (a, s1, s2, b) in th:
        assert bl[a][0] + u1.SPIN_CHARGE[s1] + u1.SPIN_CHARGE[s2] == br[b][0]
    res = u1.block_update(A, B, bl, bm, br, gm, 1, None, 1e-4, 0.0)
    for q, rows, cols, u, s, vh in res["sectors"]:
        np.testing.assert_allclose(u.conj().T @ u, np.eye(u.shape[1]), atol=1e-12)
        np.testing.assert_allclose(vh @ vh.conj().T, np.eye(vh.shape[0]), atol=1e-12)
    assert np.sum(res["s"] ** 2) == pytest.approx(1.0, rel=1e-14)
    # dense theta' from the embedding has no weight outside the allowed blocks
    ad, bd = u1.dense_site(A, bl, bm), u1.dense_site(B, bm, br)
    thd = omps.apply_gate(omps.theta_of(ad, bd), gm)
    ql = np.repeat([q for q, _ in bl], [d for _, d in bl])
    qr = np.repeat([q for q, _ in br], [d for _, d in br])
    c = np.array(u1.SPIN_CHARGE)
    bad = (ql[:, None, None, None] + c[None, :, None, None] + c[None, None, :, None]) != qr[None, None, None, :]
    assert np.abs(thd[bad]).max() == 0.0
