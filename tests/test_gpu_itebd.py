"""The infinite-TEBD application on the GPU library: the same trajectory as
the oracle (FP64 throughout) and the exact transverse-field Ising energy
within the Trotter and truncation bias."""
import pytest

from oracle import itebd as oitebd

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SCHEDULE = [(0.1, 60), (0.01, 200), (0.002, 300)]


@pytest.fixture(scope="module")
def ctx():
    from paper_2512_23917_amd import tci
    c = tci.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("g,tol", [(0.5, 1e-5), (1.0, 3e-4)])
def test_itebd_matches_oracle_and_exact_energy(ctx, g, tol):
    from paper_2512_23917_amd import itebd
    e_gpu = itebd.ITEBD(ctx, 16, g).run(SCHEDULE)
    e_orc = oitebd.run(g, 16, SCHEDULE)
    assert e_gpu == pytest.approx(e_orc, rel=1e-9)
    e0 = oitebd.e0_exact(g)
    assert e0 - 1e-9 <= e_gpu < e0 + tol
