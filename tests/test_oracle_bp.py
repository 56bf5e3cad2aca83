"""Pins for the BP oracle (App. B): exactness of BP on trees, exact
regauging when nothing is cut, gate layers against a state-vector
simulation, and the discarded weight of a single-bond cut on a tree."""
import numpy as np
import pytest

from oracle import bp
from paper_2512_23917_amd import synth


def random_tns(n, edges, dim, seed):
    g = np.random.default_rng(seed)
    nb = bp.neighbours(n, edges)
    return [synth.complex_gaussian(g, (2,) + (dim,) * len(nb[i])) for i in range(n)]


def tree_of(n, edges):
    return [e for e in edges if e != (0, 11)]


def test_heavy_hex_patch_shape():
    n, edges = bp.heavy_hex_patch()
    deg = [len(x) for x in bp.neighbours(n, edges)]
    assert n == 15 and len(edges) == 15
    assert sorted(deg).count(1) == 3 and sorted(deg).count(3) == 3 and sorted(deg).count(2) == 9
    tree = tree_of(n, edges)
    assert len(tree) == n - 1   # connected with n - 1 edges: a tree


def test_bp_exact_on_a_tree():
    n, edges = bp.heavy_hex_patch()
    tree = tree_of(n, edges)
    V = random_tns(n, tree, 2, 1)
    psi = bp.state_vector(n, tree, V)
    M, it = bp.bp_run(n, tree, V, tol=1e-14)
    assert it < 200
    z = bp.bp_norm(n, tree, V, M)
    ref = np.vdot(psi, psi).real
    assert abs(z.imag) < 1e-10 * ref and abs(z.real - ref) < 1e-10 * ref


def test_messages_hermitian_psd_unit_trace():
    n, edges = bp.heavy_hex_patch()
    V = random_tns(n, edges, 3, 2)
    M, _ = bp.bp_run(n, edges, V, iters=20)
    for m in M.values():
        assert abs(np.trace(m) - 1) < 1e-13
        assert np.abs(m - m.conj().T).max() < 1e-13
        assert np.linalg.eigvalsh(m).min() > -1e-13


def test_regauge_without_cut_keeps_the_state_on_a_loop():
    n, edges = bp.heavy_hex_patch()
    V = random_tns(n, edges, 2, 3)
    psi = bp.state_vector(n, edges, V)
    M, _ = bp.bp_run(n, edges, V, iters=30)
    nb = bp.neighbours(n, edges)
    for i, j in edges:
        s = bp.truncate_edge(i, j, V, M, nb, chi=64)
        assert len(s) == 2
    out = bp.state_vector(n, edges, V)
    assert np.linalg.norm(out - psi) / np.linalg.norm(psi) < 1e-10


def test_gate_layers_match_state_vector_when_nothing_is_cut():
    n, edges = bp.heavy_hex_patch()
    V = bp.product_state(n, edges, seed=4)
    psi = bp.state_vector(n, edges, V)
    g = synth.rng(4, 0)
    layers = [[(0, 1), (2, 3), (4, 5), (6, 7), (8, 14)], [(1, 2), (3, 4), (0, 12), (8, 9)]]
    for layer in layers:
        gates = {e: synth.haar_gate(g) for e in layer}
        for (i, j), gate in gates.items():
            psi = bp.apply_gate_statevector(psi, n, i, j, gate)
        bp.apply_layer(n, edges, V, gates, chi=16, bp_iters=10)
    out = bp.state_vector(n, edges, V)
    assert np.linalg.norm(out - psi) / np.linalg.norm(psi) < 1e-10


def test_single_bond_cut_on_a_tree_discards_the_cut_weight():
    """On a tree the converged messages are the exact environments, so the
    relative error of cutting one bond is the discarded weight of R."""
    n, edges = bp.heavy_hex_patch()
    tree = tree_of(n, edges)
    V = random_tns(n, tree, 3, 5)
    psi = bp.state_vector(n, tree, V)
    M, _ = bp.bp_run(n, tree, V, tol=1e-14)
    nb = bp.neighbours(n, tree)
    W = [v.copy() for v in V]
    s_all = bp.truncate_edge(2, 3, W, M, nb, chi=64)
    W = [v.copy() for v in V]
    s = bp.truncate_edge(2, 3, W, M, nb, chi=1)
    assert len(s_all) == 3 and len(s) == 1
    out = bp.state_vector(n, tree, W)
    # the kept part is the projection of psi: <psi|out> = <out|out>
    assert abs(np.vdot(psi, out) - np.vdot(out, out)) < 1e-10 * np.vdot(psi, psi).real
    err = np.linalg.norm(psi - out) ** 2 / np.linalg.norm(psi) ** 2
    disc = np.sum(s_all[1:] ** 2) / np.sum(s_all ** 2)
    assert abs(err - disc) < 1e-10


def test_gate_split_reproduces_the_gate():
    g = synth.haar_gate(synth.rng(6, 0)).reshape(2, 2, 2, 2)
    oi, oj = bp.split_gate(g)
    back = np.einsum("aik,bjk->abij", oi, oj)
    assert np.abs(back - g).max() < 1e-14
    assert oi.shape[2] <= 4


def _graded_tree(seed=4):
    """Tree patch whose bond (4, 5) has dimension 4 with weights
    (1, 1e-1, 1e-2, 1e-4) on both of its site tensors: the singular values of
    R on that bond reach ~1e-9 of the largest, the message eigenvalues stay
    above the inverse-square-root cut."""
    n, edges = bp.heavy_hex_patch()
    tree = tree_of(n, edges)
    nb = bp.neighbours(n, tree)
    g = np.random.default_rng(seed)
    dims = {e: 2 for e in tree}
    dims[(4, 5)] = 4
    V = [synth.complex_gaussian(g, (2,) + tuple(dims[tuple(sorted((i, k)))] for k in nb[i])) for i in range(n)]
    lam = np.array([1.0, 1e-1, 1e-2, 1e-4])
    for site, other in ((4, 5), (5, 4)):
        p = nb[site].index(other)
        V[site] = np.moveaxis(np.moveaxis(V[site], 1 + p, -1) * lam, -1, 1 + p)
    return n, tree, nb, V


def test_regauge_exact_with_graded_bond_when_nothing_is_cut():
    """With a singular-value floor below the bond's smallest value the
    regauging keeps the state exactly; the default floor cuts the ~1e-9
    direction and changes the state by about that much."""
    n, tree, nb, V = _graded_tree()
    psi = bp.state_vector(n, tree, V)
    M, _ = bp.bp_run(n, tree, V, tol=1e-15)
    Vk = [v.copy() for v in V]
    s = bp.truncate_edge(4, 5, Vk, M, nb, 16, sv_cut=1e-12)
    assert len(s) == 4 and 1e-10 < s[-1] / s[0] < 1e-8
    out = bp.state_vector(n, tree, Vk)
    assert np.linalg.norm(out - psi) / np.linalg.norm(psi) < 1e-12
    Vc = [v.copy() for v in V]
    s6 = bp.truncate_edge(4, 5, Vc, M, nb, 16)
    assert len(s6) == 3
    out6 = bp.state_vector(n, tree, Vc)
    assert 1e-10 < np.linalg.norm(out6 - psi) / np.linalg.norm(psi) < 1e-7
