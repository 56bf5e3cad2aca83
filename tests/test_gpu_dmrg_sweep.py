"""Finite two-site DMRG sweeps on the GPU library (Lanczos, split and
environment updates) for the open spin-1/2 Heisenberg chain, against the
exact ground-state energy from dense diagonalisation (N = 10, where
chi = 32 is exact)."""
import pytest

from oracle import dmrg as odmrg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2512_23917_amd import tci
    c = tci.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("dtype,tol", [("C128", 1e-9), ("C64", 2e-5)])
def test_dmrg_sweeps_reach_exact_energy(ctx, dtype, tol):
    from paper_2512_23917_amd import dmrg_sweep, tci
    e0 = odmrg.heisenberg_ground_energy(10)
    if dtype == "C64":
        ctx.set_precision(tci.PREC_BF16X3)
    try:
        run = dmrg_sweep.DMRG(ctx, 10, 32, seed=3, dtype=getattr(tci, dtype))
        energies = [run.sweep() for _ in range(4)]
    finally:
        ctx.set_precision(tci.PREC_FP32)
    print(dtype, energies, e0)
    assert energies[-1] >= e0 - tol
    assert abs(energies[-1] - e0) < tol * abs(e0)
    assert energies[-1] <= energies[0] + tol * abs(e0)   # sweeping does not raise the energy
