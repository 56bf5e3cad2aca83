"""Pins for the CPU oracle: every check compares it with something other than
itself -- the paper's printed examples, brute-force loops, LAPACK through
numpy, closed forms, invariants and special cases with known answers."""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import dmrg, mps, rsvd
from paper_2512_23917_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def cg(g, shape):
    return synth.complex_gaussian(g, shape)


# ---------------------------------------------------------------- permute
def test_transpose_paper_example():
    ex = _gold("paper_examples.json")["transpose"]
    g = np.random.default_rng(1)
    a = cg(g, ex["shape"])
    b = oracle.permute(a, ex["perm1"])
    assert a[tuple(ex["coord_before"])] == b[tuple(ex["coord_after"])]
    c = oracle.permute(b, ex["perm2"])
    assert list(c.shape) == ex["shape_after_perm2"]


@pytest.mark.parametrize("shape", [(2, 3, 4), (5, 1, 3, 2), (7,), (2, 2, 2, 2, 2)])
def test_permute_matches_numpy_transpose(shape):
    g = np.random.default_rng(2)
    a = cg(g, shape)
    for perm in itertools.permutations(range(len(shape))):
        np.testing.assert_array_equal(oracle.permute(a, perm), np.transpose(a, perm))


def test_permute_rejects_bad_perm():
    with pytest.raises(oracle.OracleError):
        oracle.permute(np.zeros((2, 3)), [0, 0])


# ---------------------------------------------------------------- contract
def _contract_loops(a, la, b, lb, lc):
    """Independent brute force: enumerate every assignment of every label."""
    dims = {}
    for lab, d in list(zip(la, a.shape)) + list(zip(lb, b.shape)):
        dims[lab] = d
    summed = [x for x in dims if x not in lc]
    out = np.zeros([dims[x] for x in lc], dtype=np.complex128)
    for oc in itertools.product(*[range(dims[x]) for x in lc]):
        acc = 0j
        for sc in itertools.product(*[range(dims[x]) for x in summed]):
            val = dict(zip(lc, oc))
            val.update(zip(summed, sc))
            acc += a[tuple(val[x] for x in la)] * b[tuple(val[x] for x in lb)]
        out[oc] = acc
    return out


def test_contract_paper_example_list_and_string():
    ex = _gold("paper_examples.json")["contract"]
    g = np.random.default_rng(3)
    a, b = cg(g, ex["shape_a"]), cg(g, ex["shape_b"])
    c1 = oracle.contract(a, ex["labels_a"], b, ex["labels_b"], ex["labels_c"])
    c2 = oracle.contract(a, ex["str_a"], b, ex["str_b"], ex["str_c"])
    assert list(c1.shape) == ex["expected_shape"]
    np.testing.assert_array_equal(c1, c2)
    np.testing.assert_allclose(c1, _contract_loops(a, "ijk", b, "kjl", "li"), atol=1e-13)


@pytest.mark.parametrize("case", [
    ("ijk", "jkl", "il"), ("ijk", "jklm", "ilm"), ("ij", "jk", "ik"), ("ij", "ij", ""),
    ("i", "j", "ij"), ("abc", "cde", "ebda"), ("astb", "uvst", "auvb"), ("ab", "bc", "ca")])
def test_contract_matches_loops_and_einsum(case):
    la, lb, lc = case
    g = np.random.default_rng(4)
    dims = {ch: 2 + (ord(ch) % 3) for ch in set(la + lb)}
    a = cg(g, [dims[x] for x in la])
    b = cg(g, [dims[x] for x in lb])
    c = oracle.contract(a, la, b, lb, lc)
    np.testing.assert_allclose(c, _contract_loops(a, la, b, lb, lc), atol=1e-12)
    np.testing.assert_allclose(c, np.einsum(f"{la},{lb}->{lc}", a, b), atol=1e-12)


@pytest.mark.parametrize("bad", [
    ("iij", "jk", "ik"),      # repeated label inside an operand
    ("ij", "jk", "ikk"),      # repeated label in the result
    ("ij", "jk", "ijk"),      # a shared label kept in the result (batch)
    ("ij", "jk", "i"),        # label of b in neither the sum nor the result
    ("ij", "jk", "ikz"),      # result label found in neither operand
])
def test_contract_rejects_bad_labels(bad):
    la, lb, lc = bad
    a = np.ones([2] * len(la))
    b = np.ones([2] * len(lb))
    with pytest.raises(oracle.OracleError) as e:
        oracle.contract(a, la, b, lb, lc)
    assert e.value.status == oracle.LABEL


def test_contract_rejects_dim_mismatch():
    with pytest.raises(oracle.OracleError) as e:
        oracle.contract(np.ones((2, 3)), "ij", np.ones((4, 2)), "jk", "ik")
    assert e.value.status == oracle.SHAPE


# ---------------------------------------------------------------- norms
def test_norm_eye3_paper_example():
    ex = _gold("paper_examples.json")["norm_eye3"]
    assert oracle.norm(np.eye(3)) == pytest.approx(ex["expected"], rel=1e-15)


def test_norm_complex_modulus():
    a = np.array([3 + 4j, 0, 0])
    assert oracle.norm(a) == 5.0
    b, n = oracle.normalize(np.array([[3.0, 4.0]]))
    assert n == 5.0 and oracle.norm(b) == pytest.approx(1.0, abs=1e-15)


# ---------------------------------------------------------------- svd
@pytest.mark.parametrize("m,n", [(40, 30), (30, 40), (64, 64), (1, 5), (5, 1), (17, 3)])
def test_svd_reconstruction_isometry_lapack(m, n):
    g = np.random.default_rng(m * 100 + n)
    a = cg(g, (m, n))
    u, s, vh = oracle.svd_matrix(a)
    k = min(m, n)
    assert u.shape == (m, k) and s.shape == (k,) and vh.shape == (k, n)
    assert np.all(np.diff(s) <= 0) and np.all(s >= 0)
    assert np.linalg.norm(u @ np.diag(s) @ vh - a) / np.linalg.norm(a) < 1e-13
    assert np.abs(u.conj().T @ u - np.eye(k)).max() < 1e-13
    assert np.abs(vh @ vh.conj().T - np.eye(k)).max() < 1e-13
    ref = np.linalg.svd(a, compute_uv=False)
    assert np.abs(s - ref).max() <= 1e-13 * ref[0]
    # gauge: largest-modulus entry of every u column is real and positive
    idx = np.argmax(np.abs(u), axis=0)
    top = u[idx, np.arange(k)]
    assert np.all(np.abs(top.imag) < 1e-14) and np.all(top.real > 0)


def test_svd_closed_form_spectrum():
    g = np.random.default_rng(5)
    s_true = synth.exp_spectrum(48, 6.0)
    a, b = synth.two_site_blocks_from_spectrum(g, 24, 2, s_true)
    m = np.einsum("asm,mtb->astb", a, b).reshape(48, 48)
    _, s, _ = oracle.svd_matrix(m)
    assert np.abs(s - s_true).max() < 1e-14


def test_svd_rank_deficient_completion():
    g = np.random.default_rng(6)
    x = cg(g, (20, 4)) @ cg(g, (4, 12))            # rank 4
    x[:, 0] = 0.0
    u, s, vh = oracle.svd_matrix(x)
    assert np.abs(u.conj().T @ u - np.eye(12)).max() < 1e-12
    assert np.linalg.norm(u @ np.diag(s) @ vh - x) < 1e-12 * np.linalg.norm(x)
    assert np.all(s[4:] < 1e-12 * s[0])


def test_svd_tensor_fold_back_paper_shapes():
    ex = _gold("paper_examples.json")["svd_shapes"]
    a = cg(np.random.default_rng(7), ex["shape"])
    u, s, vh = oracle.svd(a, ex["k_rows"])
    assert list(u.shape) == ex["u"] and list(s.shape) == ex["s"] and list(vh.shape) == ex["vh"]
    with pytest.raises(oracle.OracleError):
        oracle.svd(a, 3)  # k must satisfy 1 <= k < order


def test_svd_real_input_stays_real():
    a = np.random.default_rng(8).standard_normal((9, 7))
    u, s, vh = oracle.svd_matrix(a)
    assert np.abs(u.imag).max() == 0 and np.abs(vh.imag).max() == 0


# ---------------------------------------------------------------- truncation
def test_trunc_rule_hand_worked():
    for c in _gold("trunc_rule_closed_forms.json")["hand_worked"]:
        chi, err = oracle.trunc_rule(c["s"], c["chi_min"], c["chi_max"], c["target"], c["s_min"])
        assert chi == c["chi"], c["why"]
        assert err == pytest.approx(c["err"], rel=1e-14, abs=0), c["why"]


def _brute_chistar(s, target):
    s2 = [x * x for x in s]
    total = math.fsum(s2)
    for c in range(1, len(s) + 1):
        if math.fsum(s2[c:]) / total <= target:
            return c
    return len(s)


def test_trunc_rule_closed_form_spectra():
    gold = _gold("trunc_rule_closed_forms.json")
    s = synth.exp_spectrum(2048, 200.0)
    chi, err = oracle.trunc_rule(s, 1, 2048, 1e-8, 0.0)
    assert chi == gold["exp_spectrum_2048_scale200"]["chi_at_1e-8"] == _brute_chistar(s, 1e-8)
    assert err == pytest.approx(gold["exp_spectrum_2048_scale200"]["err_at_1e-8"], rel=1e-9)
    chi, _ = oracle.trunc_rule(s, 1, 2048, 1e-10, 0.0)
    assert chi == gold["exp_spectrum_2048_scale200"]["chi_at_1e-10"]
    for alpha, want in gold["power_law_2048_chi_at_1e-8"].items():
        s = synth.power_spectrum(2048, float(alpha))
        chi, _ = oracle.trunc_rule(s, 1, 2048, 1e-8, 0.0)
        assert chi == want
        chi_cap, err_cap = oracle.trunc_rule(s, 1, 1024, 1e-8, 0.0)
        assert chi_cap == min(want, 1024)
        if want > 1024:
            assert err_cap > 1e-8


def test_trunc_rule_invalid_arguments():
    for args in [(0, 4), (3, 2), (1, 0)]:
        with pytest.raises(oracle.OracleError) as e:
            oracle.trunc_rule([3.0, 2.0], args[0], args[1], 0.0, 0.0)
        assert e.value.status == oracle.INVALID


def test_trunc_svd_paper_example_and_discarded_weight():
    ex = _gold("paper_examples.json")["trunc_svd"]
    a = cg(np.random.default_rng(9), ex["shape"])
    u, s, vh, err = oracle.trunc_svd(a, ex["k_rows"], ex["chi_min"], ex["chi_max"],
                                     ex["target"], ex["s_min"])
    assert err != 0.0
    assert ex["chi_min"] <= len(s) <= ex["chi_max"]
    _, s_all, _ = oracle.svd(a, ex["k_rows"])
    # discarded weight = sum of the squares of the cut values = eps * total
    total = np.sum(np.abs(a) ** 2)
    assert np.sum(s_all[len(s):] ** 2) == pytest.approx(err * total, rel=1e-12)


def test_minimal_example_overlap():
    """Sec. III: normalised 6-qubit state, trunc_svd keeping 2 values at 3|3.
    The overlap <psi|psi_trunc> equals 1 - trunc_err (the printed 'fide'
    squares it, which only matches for the overlap itself)."""
    g = np.random.default_rng(10)
    psi = g.uniform(-1, 1, (2,) * 6)
    psi, _ = oracle.normalize(psi)
    u, s, vh, err = oracle.trunc_svd(psi, 3, 1, 2, 0.0, 0.0)
    psi1 = oracle.contract(u * s[None, None, None, :], "ijkl", vh, "lmno", "ijkmno")
    ov = oracle.contract(psi, "ijklmn", psi1, "ijklmn", "")
    assert complex(ov).real == pytest.approx(1.0 - err, abs=1e-13)


# ---------------------------------------------------------------- qr / eigh
@pytest.mark.parametrize("m,n", [(12, 5), (5, 12), (8, 8)])
def test_qr_properties(m, n):
    a = cg(np.random.default_rng(11 + m), (m, n))
    q, r = oracle.qr_matrix(a)
    rho = min(m, n)
    assert np.abs(q @ r - a).max() < 1e-13
    assert np.abs(q.conj().T @ q - np.eye(rho)).max() < 1e-13
    assert np.abs(np.tril(r, -1)).max() == 0
    d = np.diagonal(r)
    assert np.all(np.abs(d.imag) < 1e-15) and np.all(d.real >= 0)
    qn, rn = np.linalg.qr(a)
    assert np.allclose(np.abs(np.diagonal(rn)), d.real, atol=1e-12)


def test_qr_paper_shapes():
    ex = _gold("paper_examples.json")["qr_shapes"]
    q, r = oracle.qr(cg(np.random.default_rng(12), ex["shape"]), ex["k_rows"])
    assert list(q.shape) == ex["q"] and list(r.shape) == ex["r"]


def test_eigh_vs_lapack_and_heisenberg_bond():
    a = cg(np.random.default_rng(13), (30, 30))
    h = a + a.conj().T
    w, v = oracle.eigh(h)
    assert np.abs(w - np.linalg.eigvalsh(h)).max() < 1e-13 * np.abs(w).max()
    assert np.abs(v @ np.diag(w) @ v.conj().T - h).max() < 1e-12 * np.abs(w).max()
    assert np.abs(v.conj().T @ v - np.eye(30)).max() < 1e-13
    # two-site Heisenberg bond S1.S2: singlet -3/4, triplet 1/4
    sx = np.array([[0, 0.5], [0.5, 0]])
    sy = np.array([[0, -0.5j], [0.5j, 0]])
    sz = np.diag([0.5, -0.5])
    hb = sum(np.kron(o, o) for o in (sx, sy, sz))
    w, _ = oracle.eigh(hb)
    np.testing.assert_allclose(w, [-0.75, 0.25, 0.25, 0.25], atol=1e-15)


# ---------------------------------------------------------------- gate / update
def test_gate_norm_identity_and_inverse():
    g = np.random.default_rng(14)
    a, b = cg(g, (6, 2, 5)), cg(g, (5, 2, 7))
    theta = mps.theta_of(a, b)
    np.testing.assert_allclose(theta, np.einsum("asm,mtb->astb", a, b), atol=1e-13)
    gate = synth.haar_gate(g)
    t2 = mps.apply_gate(theta, gate)
    assert oracle.norm(t2) == pytest.approx(oracle.norm(theta), rel=1e-14)
    np.testing.assert_allclose(mps.apply_gate(theta, np.eye(4)), theta, atol=1e-15)
    back = mps.apply_gate(t2, gate.conj().T)
    np.testing.assert_allclose(back, theta, atol=1e-13)
    # orientation: rows of the gate are the outgoing (s1', s2') indices
    perm = np.zeros((4, 4))
    perm[1, 2] = perm[2, 1] = perm[0, 0] = perm[3, 3] = 1.0   # SWAP
    np.testing.assert_allclose(mps.apply_gate(theta, perm), theta.transpose(0, 2, 1, 3), atol=0)


@pytest.mark.parametrize("direction", [mps.LEFT, mps.RIGHT])
def test_two_site_update_invariants(direction):
    g = np.random.default_rng(15)
    a, b = cg(g, (8, 2, 8)), cg(g, (8, 2, 8))
    gate = synth.haar_gate(g)
    r = mps.two_site_update(a, b, gate, 1, 6, 1e-12, 0.0, direction)
    s = r["s"]
    assert np.sum(s ** 2) == pytest.approx(1.0, abs=1e-14)
    theta = r["theta"].reshape(16, 16)
    _, s_all, _ = oracle.svd_matrix(theta)
    assert r["discarded_abs"] == pytest.approx(np.sum(s_all[6:] ** 2), rel=1e-12)
    u = r["a_out"] if direction == mps.LEFT else r["a_out"] / s[None, None, :]
    um = u.reshape(16, -1)
    assert np.abs(um.conj().T @ um - np.eye(um.shape[1])).max() < 1e-13
    vh = r["b_out"] if direction == mps.RIGHT else r["b_out"] / s[:, None, None]
    vm = vh.reshape(vh.shape[0], -1)
    assert np.abs(vm @ vm.conj().T - np.eye(vm.shape[0])).max() < 1e-13


def test_c1_sweep_against_state_vector():
    """Small open chain (N=16, d=2, chi 32): right-to-left gate sweep on the
    left-canonical MPS.  Uncapped (chi 64) the MPS equals the exact
    state-vector evolution; at chi 32 the deviation obeys the sum of the
    per-bond truncation bounds."""
    g = synth.rng(1, 0)
    m0 = synth.random_open_mps(g, 16, 2, 32)
    gates = [synth.haar_gate(g) for _ in range(15)]
    m0 = mps.left_canonicalize(m0)
    psi0 = mps.state_vector(m0)
    assert np.linalg.norm(psi0) == pytest.approx(1.0, abs=1e-12)
    exact = mps.exact_gate_evolution(psi0, 16, gates)
    m_full, errs_full = mps.sweep_right_to_left(m0, gates, chi_max=64, target=0.0)
    assert np.linalg.norm(mps.state_vector(m_full) - exact) < 1e-11
    m_cut, errs = mps.sweep_right_to_left(m0, gates, chi_max=32, target=1e-10)
    bound = sum(math.sqrt(2 * (1 - math.sqrt(1 - e))) for e in errs) + 1e-10
    assert np.linalg.norm(mps.state_vector(m_cut) - exact) <= bound


# ---------------------------------------------------------------- H_eff / Lanczos
def test_heff_matches_dense_definition_and_is_hermitian():
    g = np.random.default_rng(16)
    w = synth.heisenberg_mpo()
    left = synth.hermitian_environment(g, 2)
    right = synth.hermitian_environment(g, 2)
    h = dmrg.heff_dense(left, w, w, right)
    assert np.abs(h - h.conj().T).max() < 1e-14 * np.abs(h).max()
    x = cg(g, (2, 2, 2, 2))
    y = dmrg.heff_apply(left, w, w, right, x)
    np.testing.assert_allclose(y.reshape(-1), h @ x.reshape(-1), atol=1e-13)


def test_heff_trivial_environment_is_heisenberg_bond():
    left, right = synth.trivial_environments()
    w = synth.heisenberg_mpo()
    h = dmrg.heff_dense(left, w, w, right)
    np.testing.assert_allclose(np.linalg.eigvalsh(h), [-0.75, 0.25, 0.25, 0.25], atol=1e-15)


def test_lanczos_exact_in_small_space_and_monotone():
    g = np.random.default_rng(17)
    w = synth.heisenberg_mpo()
    left = synth.hermitian_environment(g, 2)
    right = synth.hermitian_environment(g, 2)
    h = dmrg.heff_dense(left, w, w, right)
    x0 = cg(g, (2, 2, 2, 2))
    mv = lambda v: dmrg.heff_apply(left, w, w, right, v)
    e, psi, al, be = dmrg.lanczos_ground(mv, x0, n_matvec=16)
    lam = np.linalg.eigvalsh(h)
    assert e == pytest.approx(lam[0], abs=1e-12 * np.abs(lam).max())
    r = h @ psi.reshape(-1) - e * psi.reshape(-1)
    assert np.linalg.norm(r) < 1e-10 * np.abs(lam).max()
    es = [dmrg.lanczos_ground(mv, x0, n_matvec=j)[0] for j in range(1, 9)]
    assert all(es[i + 1] <= es[i] + 1e-12 for i in range(len(es) - 1))
    assert all(x >= lam[0] - 1e-12 for x in es)
    ov = complex(np.vdot(x0.reshape(-1), psi.reshape(-1)))
    assert abs(ov.imag) < 1e-12 and ov.real > 0


# ---------------------------------------------------------------- randomized SVD
def test_randomized_exact_for_low_rank():
    g = np.random.default_rng(18)
    x = cg(g, (60, 7)) @ cg(g, (7, 50))
    r = rsvd.randomized_tsvd(x, k=12, q=1, seed=3, chi_max=20, target=1e-12)
    _, s_ref, _ = oracle.svd_matrix(x)
    assert r["accepted"] and r["chi"] == 7
    assert np.abs(r["s"] - s_ref[:7]).max() < 1e-12 * s_ref[0]
    rec = r["u"] @ np.diag(r["s"]) @ r["vh"]
    assert np.linalg.norm(rec - x) < 1e-12 * np.linalg.norm(x)


def test_randomized_falls_back_when_sketch_too_small():
    g = np.random.default_rng(19)
    s_true = synth.power_spectrum(64, 1.0)
    a, b = synth.two_site_blocks_from_spectrum(g, 32, 2, s_true)
    theta = np.einsum("asm,mtb->astb", a, b).reshape(64, 64)
    r = rsvd.tsvd_with_fallback(theta, k=8, q=1, seed=1, chi_max=64, target=1e-8)
    assert r["fallback"] and r["chi"] == _brute_chistar(s_true, 1e-8)
    assert np.abs(r["s"] - s_true[: r["chi"]]).max() < 1e-13


def test_randomized_matches_plain_on_decaying_spectrum():
    g = np.random.default_rng(20)
    s_true = synth.power_spectrum(128, 3.0)
    a, b = synth.two_site_blocks_from_spectrum(g, 64, 2, s_true)
    theta = np.einsum("asm,mtb->astb", a, b).reshape(128, 128)
    want = _brute_chistar(s_true, 1e-8)
    r = rsvd.tsvd_with_fallback(theta, k=want + 16, q=2, seed=5, chi_max=128, target=1e-8)
    assert not r["fallback"] and r["chi"] == want
    assert np.abs(r["s"] - s_true[:want]).max() < 1e-10


# ---------------------------------------------------------------- Philox
def test_philox_published_known_answers():
    """Known-answer vectors published with the Random123 library (Salmon et al.)."""
    kat = [([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
           ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
           ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
            [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1])]
    for ctr, key, want in kat:
        assert [int(x) for x in oracle.philox_raw(ctr, key)] == want


def test_philox_normal_moments():
    z = oracle.philox_normal(1234, 0, 200000)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1.0) < 0.01


def test_heisenberg_chain_exact_energy_and_mpo():
    """Dense open-chain Hamiltonian: E0(2) = -3/4 and E0(4) = -3/4 - sqrt(3)/2
    (closed forms); the bond-dimension-5 MPO with the one-dimensional end
    environments (channel 4 on the left, channel 0 on the right) contracts to
    the same dense operator."""
    import math
    from oracle import dmrg as od
    assert od.heisenberg_ground_energy(2) == pytest.approx(-0.75, abs=1e-14)
    assert od.heisenberg_ground_energy(4) == pytest.approx(-0.75 - math.sqrt(3) / 2, abs=1e-13)
    w = synth.heisenberg_mpo()
    n = 4
    vec = np.zeros(5)
    vec[4] = 1.0
    op = np.einsum("w,wvst->vst", vec, w)                   # (5, 2, 2) after site 0
    for _ in range(n - 1):
        op = np.einsum("vST,vust->uSsTt", op, w).reshape(5, op.shape[1] * 2, op.shape[2] * 2)
    dense = op[0]
    np.testing.assert_allclose(dense, od.heisenberg_chain_dense(n), atol=1e-14)


def test_philox_normal_box_muller_pairs_from_known_answer_block():
    """Key (0, 0), counter (0, 0, 0, 0) is the first published known-answer
    block (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8).  Each normal pair
    (z0, z1) of the block is a point in the plane with squared radius
    -2 ln u1 and angle 2 pi u2, where u = (x + 1/2) 2^-32 maps the words
    (x0, x1) and (x2, x3) into (0, 1)."""
    import math
    words = [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    z = oracle.philox_normal(0, 0, 4)
    for p in range(2):
        u1 = (words[2 * p] + 0.5) / 2.0 ** 32
        u2 = (words[2 * p + 1] + 0.5) / 2.0 ** 32
        z0, z1 = z[2 * p], z[2 * p + 1]
        assert z0 * z0 + z1 * z1 == pytest.approx(-2.0 * math.log(u1), rel=1e-14)
        ang = math.atan2(z1, z0) % (2.0 * math.pi)
        assert ang == pytest.approx(2.0 * math.pi * u2, rel=1e-13)


def test_philox_normal_distribution():
    """Kolmogorov-Smirnov tests: the normals against N(0, 1), the halved
    squared radii of the pairs against Exp(1), the pair angles against
    U(0, 2 pi)."""
    from scipy import stats
    z = oracle.philox_normal(251223917, 3, 200000)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    pairs = z.reshape(-1, 2)
    assert stats.kstest(0.5 * (pairs ** 2).sum(1), "expon").pvalue > 1e-3
    ang = np.arctan2(pairs[:, 1], pairs[:, 0]) % (2 * np.pi)
    assert stats.kstest(ang, "uniform", args=(0.0, 2 * np.pi)).pvalue > 1e-3


def test_vidal_write_back_reconstructs_theta():
    """Vidal form (App. A): with Gamma_A = Lambda_l^-1 U, Gamma_B = V^dagger
    Lambda_r^-1 and Lambda = s / ||s||, the chain Lambda_l Gamma_A Lambda
    Gamma_B Lambda_r reproduces theta' / ||theta'||_F when nothing is cut,
    and Lambda_l Gamma_A has orthonormal columns (Lambda_l^2-weighted
    left-canonical condition)."""
    g = np.random.default_rng(31)
    chi = 5
    a = synth.complex_gaussian(g, (chi, 2, chi))
    b = synth.complex_gaussian(g, (chi, 2, chi))
    gate = synth.haar_gate(g)
    lam_l = np.sort(g.uniform(0.1, 1.0, chi))[::-1]
    lam_r = np.sort(g.uniform(0.1, 1.0, chi))[::-1]
    r = mps.two_site_update(a, b, gate, 1, 2 * chi, 0.0, 0.0, mps.VIDAL, lam_left=lam_l, lam_right=lam_r)
    rec = np.einsum("a,asm,m,mtb,b->astb", lam_l, r["a_out"], r["s"], r["b_out"], lam_r)
    th = r["theta"]
    np.testing.assert_allclose(rec, th / np.linalg.norm(th), atol=1e-13)
    left = (lam_l[:, None, None] * r["a_out"]).reshape(2 * chi, -1)
    np.testing.assert_allclose(left.conj().T @ left, np.eye(left.shape[1]), atol=1e-13)
    right = (r["b_out"] * lam_r[None, None, :]).reshape(left.shape[1], -1)
    np.testing.assert_allclose(right @ right.conj().T, np.eye(left.shape[1]), atol=1e-13)
