"""Pins for the infinite-TEBD oracle (App. A): the exact ground-state energy
per site of the transverse-field Ising chain, and imaginary-time evolution
converging to it within the Trotter and truncation bias."""
import math

import pytest

from oracle import itebd

SCHEDULE = [(0.1, 60), (0.01, 200), (0.002, 300)]


def test_exact_energy_closed_forms():
    # Sec. IV: e0(1) = -4/pi at the critical point; e0(0.5) from the same integral
    assert itebd.e0_exact(1.0) == pytest.approx(-4.0 / math.pi, abs=1e-12)
    assert itebd.e0_exact(0.5) == pytest.approx(-1.063544409973, abs=1e-12)
    assert itebd.e0_exact(0.0) == pytest.approx(-1.0, abs=1e-12)       # classical Ising, g = 0


@pytest.mark.parametrize("g,tol", [(0.5, 1e-5), (1.0, 3e-4)])
def test_imaginary_time_evolution_reaches_ground_state(g, tol):
    e = itebd.run(g, 16, SCHEDULE)
    e0 = itebd.e0_exact(g)
    assert e >= e0 - 1e-9          # variational: a matrix-product state cannot go below e0
    assert e - e0 < tol
