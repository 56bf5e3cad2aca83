"""GPU parity of the BP update (App. B) against the CPU oracle, through the
library: messages, the BP norm, kept spectra and the state vector after
truncating gate layers on a 15-site heavy-hex patch (complex128, FP64;
<= 1e-10 relative on gauge-invariant results)."""
import time

import numpy as np
import pytest

from oracle import bp as obp
from paper_2512_23917_amd import synth

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


def random_tns(n, edges, seed, dims=(2, 3)):
    g = np.random.default_rng(seed)
    nb = obp.neighbours(n, edges)
    dim = {e: dims[k % len(dims)] for k, e in enumerate(edges)}
    return [synth.complex_gaussian(g, (2,) + tuple(dim[tuple(sorted((i, k)))] for k in nb[i])) for i in range(n)]


def test_messages_and_norm_match_oracle(ctx):
    from paper_2512_23917_amd import bp
    n, edges = obp.heavy_hex_patch()
    V = random_tns(n, edges, 1)
    st = bp.BPState(ctx, n, edges, V)
    st.run_bp(12)
    M, _ = obp.bp_run(n, edges, [v.copy() for v in V], iters=12)
    err = max(np.abs(st.M[k].numpy() - M[k]).max() for k in M)
    assert err < 1e-12, err
    z, zo = st.bp_norm(), obp.bp_norm(n, edges, V, M)
    assert abs(z - zo) < 1e-10 * abs(zo)


def test_bp_norm_exact_on_a_tree(ctx):
    from paper_2512_23917_amd import bp
    n, edges = obp.heavy_hex_patch()
    tree = [e for e in edges if e != (0, 11)]
    V = random_tns(n, tree, 2)
    st = bp.BPState(ctx, n, tree, V)
    st.run_bp(40)
    psi = obp.state_vector(n, tree, V)
    ref = np.vdot(psi, psi).real
    assert abs(st.bp_norm() - ref) < 1e-10 * ref


@pytest.mark.parametrize("chi", [16, 2])
def test_gate_layers_match_oracle(ctx, chi):
    from paper_2512_23917_amd import bp
    n, edges = obp.heavy_hex_patch()
    V0 = obp.product_state(n, edges, seed=3)
    st = bp.BPState(ctx, n, edges, V0)
    Vo = [v.copy() for v in V0]
    psi = obp.state_vector(n, edges, V0)
    g = synth.rng(7, 0)
    layers = [[(0, 1), (2, 3), (4, 5), (6, 7), (8, 14)], [(1, 2), (3, 4), (0, 12), (8, 9), (10, 11)],
              [(0, 1), (2, 3), (4, 13), (6, 7), (9, 10)]]
    t0 = time.perf_counter()
    for layer in layers:
        gates = {e: synth.haar_gate(g) for e in layer}
        for (i, j), gate in gates.items():
            psi = obp.apply_gate_statevector(psi, n, i, j, gate)
        spec = st.apply_layer(gates, chi, bp_iters=10)
        _, spec_o = obp.apply_layer(n, edges, Vo, gates, chi, bp_iters=10)
        for e in gates:
            assert spec[e].shape == spec_o[e].shape
            assert np.abs(spec[e] - spec_o[e]).max() < 1e-10 * spec_o[e][0]
    dt = (time.perf_counter() - t0) / len(layers)
    out = obp.state_vector(n, edges, st.host_tensors())
    ref = obp.state_vector(n, edges, Vo)
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref) < 1e-10
    if chi == 16:   # nothing is cut: the exact state
        assert np.linalg.norm(out - psi) / np.linalg.norm(psi) < 1e-10
    else:
        assert max(max(v.shape[1:]) for v in st.host_tensors()) <= chi
        fid = abs(np.vdot(psi, out)) / (np.linalg.norm(psi) * np.linalg.norm(out))
        assert 0.5 < fid < 1.0
    print(f"BP layer (5 gates, 10 sweeps, chi={chi}): {dt * 1e3:.1f} ms")


def test_graded_bond_resolved_by_the_library_svd(ctx):
    """A tree bond whose R has singular values down to ~1e-9 of the largest:
    the library's SVD of R (one-sided Jacobi) resolves them, so the kept
    spectrum matches the oracle to 1e-12 of s_0 and, with a floor below the
    smallest value, the regauged state is the exact one."""
    from paper_2512_23917_amd import bp
    n, edges = obp.heavy_hex_patch()
    tree = [e for e in edges if e != (0, 11)]
    nb = obp.neighbours(n, tree)
    g = np.random.default_rng(4)
    dims = {e: 2 for e in tree}
    dims[(4, 5)] = 4
    V = [synth.complex_gaussian(g, (2,) + tuple(dims[tuple(sorted((i, k)))] for k in nb[i])) for i in range(n)]
    lam = np.array([1.0, 1e-1, 1e-2, 1e-4])
    for site, other in ((4, 5), (5, 4)):
        p = nb[site].index(other)
        V[site] = np.moveaxis(np.moveaxis(V[site], 1 + p, -1) * lam, -1, 1 + p)
    psi = obp.state_vector(n, tree, V)
    for cut in (1e-12, 1e-6):
        st = bp.BPState(ctx, n, tree, V)
        st.run_bp(30)
        s = st.truncate_edge(4, 5, 16, sv_cut=cut)
        Vo = [v.copy() for v in V]
        M, _ = obp.bp_run(n, tree, Vo, iters=30)
        so = obp.truncate_edge(4, 5, Vo, M, nb, 16, cut)
        assert s.shape == so.shape
        assert np.abs(s - so).max() < 1e-12 * so[0], (cut, s, so)
        out = obp.state_vector(n, tree, st.host_tensors())
        ref = obp.state_vector(n, tree, Vo)
        assert np.linalg.norm(out - ref) / np.linalg.norm(ref) < 1e-9
        if cut == 1e-12:
            assert len(s) == 4
            assert np.linalg.norm(out - psi) / np.linalg.norm(psi) < 1e-9
