"""Host-side logic of the benchmark (no GPU): the headline input recipe, the
choice of the oracle's sample updates and the parity report, checked on a
small bond dimension with the oracle's own update standing in for the GPU's
outputs (where the errors must vanish) and with a planted error."""
import numpy as np

import bench
from paper_2512_23917_amd import synth


class _T:
    def __init__(self, a):
        self.a = a

    def numpy(self):
        return self.a


class _Info:
    def __init__(self, chi, err):
        self.chi, self.trunc_err, self.sketch_rank, self.used_fallback = chi, err, 0, 0


def test_headline_inputs_follow_the_recipe():
    host = bench.headline_inputs(5, 16)
    assert len(host) == 5
    for alpha, s, a, b, gate in host:
        assert 1.0 <= alpha <= 3.0
        np.testing.assert_allclose(s, synth.power_spectrum(16, alpha), rtol=0, atol=0)
        assert a.shape == (16, 2, 16) and b.shape == (16, 2, 16) and gate.shape == (4, 4)
        # theta = A.B has exactly the bond spectrum s (isometric U, V)
        th = np.einsum("asm,mtb->astb", a, b).reshape(32, 32)
        np.testing.assert_allclose(np.linalg.svd(th, compute_uv=False)[:16], s, atol=1e-13)
        np.testing.assert_allclose(gate.conj().T @ gate, np.eye(4), atol=1e-13)
    # seeded: the same batch twice
    again = bench.headline_inputs(5, 16)
    assert all(np.array_equal(x[2], y[2]) for x, y in zip(host, again))


def test_sample_updates_alternates_fast_and_slow_bonds():
    host = [(a, None, None, None, None) for a in (1.1, 2.5, 1.5, 2.9, 2.0, 2.3)]
    assert bench.sample_updates(host, 2) == [1, 0]
    assert bench.sample_updates(host, 4) == [1, 0, 3, 2]
    assert bench.sample_updates(host, 9) == [1, 0, 3, 2, 5]


def test_parity_report_zero_for_the_oracle_and_catches_a_planted_error():
    host = bench.headline_inputs(3, 24)
    ref, times = bench.oracle_updates(host, [0], 24, 1e-8)
    r = ref[0]
    out = bench.parity(r, _T(r["a_out"]), _T(r["s"]), _T(r["b_out"]), _Info(r["chi"], r["trunc_err"]), 24, 1e-8)
    assert out["chi_valid"] and out["sigma_normwise"] == 0.0 and out["recon_rel_fro"] == 0.0
    bad = r["b_out"].copy()
    bad[0] *= 1.0 + 1e-4
    out = bench.parity(r, _T(r["a_out"]), _T(r["s"]), _T(bad), _Info(r["chi"], r["trunc_err"]), 24, 1e-8)
    assert 1e-6 < out["recon_rel_fro"] < 1e-3
    s_bad = r["s"].copy()
    s_bad[-1] *= 1.5
    out = bench.parity(r, _T(r["a_out"]), _T(s_bad), _T(r["b_out"]), _Info(r["chi"], r["trunc_err"]), 24, 1e-8)
    assert out["sigma_normwise"] > 0.0
    # a chi one below the reference is valid only when the cut sits on the threshold
    c = r["chi"] - 1
    out = bench.parity(r, _T(r["a_out"][..., :c]), _T(r["s"][:c]), _T(r["b_out"][:c]), _Info(c, r["trunc_err"]), 24,
                       1e-8)
    e_prev = r["trunc_err"] + float(r["s_raw"][r["chi"] - 1]) ** 2 / float(np.sum(np.abs(r["theta"]) ** 2))
    assert out["chi_valid"] == (e_prev <= 1e-8 * (1 + 1e-3))
