"""Pins of the oracle's topological charge (Results, skyrmion phase diagram:
skyrmions classified by Q) and of the input generators' skyrmion seeds."""
import math

import numpy as np
import pytest

from oracle import Grid, Material
from oracle import integrators as it
from oracle import observables as ob
from workloads import neel_skyrmions, uniform


def test_uniform_state_has_zero_charge():
    grid = Grid((16, 12, 1), (2e-9, 2e-9, 1e-9), pbc=(1, 1, 0))
    assert ob.topological_charge(uniform(grid.n, (0.1, 0.2, 0.97)), grid) == pytest.approx(0.0, abs=1e-14)


@pytest.mark.parametrize("count", [1, 3])
def test_core_down_skyrmions_have_charge_minus_count(count):
    """A smooth core-down skyrmion on a +z background carries Q = -1; the
    central-difference sum converges to the integer as the texture is resolved."""
    n, cell = (128, 128, 1), (1e-9, 1e-9, 0.6e-9)
    grid = Grid(n, cell, pbc=(1, 1, 0))
    m, _, _ = neel_skyrmions(n, cell, count, 12e-9, 14e-9, seed=2, width=4e-9)
    Q = ob.topological_charge(m, grid)
    assert abs(Q + count) < 0.02 * count


def test_charge_converges_with_resolution():
    errs = []
    for h in (2e-9, 1e-9, 0.5e-9):
        N = int(round(96e-9 / h))
        grid = Grid((N, N, 1), (h, h, 0.6e-9), pbc=(1, 1, 0))
        m, _, _ = neel_skyrmions(grid.n, grid.cell, 1, 15e-9, 15e-9, seed=7, width=5e-9)
        errs.append(abs(ob.topological_charge(m, grid) + 1))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 2e-3


def test_relaxing_skyrmion_keeps_charge_near_minus_one():
    """Damped dynamics lower the energy; the metastable skyrmion (D < D_c)
    shrinks towards a few cells, so the discrete charge drifts from -1 by the
    discretisation error only."""
    n, cell = (48, 48, 1), (2e-9, 2e-9, 0.6e-9)
    grid = Grid(n, cell, pbc=(1, 1, 0), images=(1, 1, 0))
    mat = Material(Ms=5.8e5, A=1.5e-11, D=3e-3, Ku=0.8e6, alpha=0.5, B=(0, 0, 0.1))
    m0, _, _ = neel_skyrmions(n, cell, 1, 12e-9, 12e-9, seed=1, width=5.05e-9)
    res = it.rk45_run(m0, grid, mat, 0.0, 5e-11, tol=1e-5, dt0=1e-14, energy=True)
    assert abs(ob.topological_charge(res.m, grid) + 1) < 0.15
    assert res.energy[-1] < res.energy[0]


def test_neel_brown_sun_limits_and_half_crossing():
    """Switching law (Results, replica-batched STT switching sweep), pinned by
    what its definition fixes independently of its code: no barrier at and
    above J_c0 (P = 1 - exp(-t f0) for every j >= 1), the zero-current limit
    1 - exp(-t f0 e^-Delta), strict increase below J_c0, and the half-switching
    current solved by hand, j* = 1 - sqrt(ln(t f0 / ln 2) / Delta)."""
    from oracle.observables import switching_probability_neel_brown_sun as psw
    t, f0, delta = 2e-9, 4.9e10, 121.0
    assert np.allclose(psw([1.0, 1.2, 3.0], t, f0, delta), -np.expm1(-t * f0), rtol=0, atol=1e-15)
    assert abs(psw(0.0, t, f0, delta) - (-math.expm1(-t * f0 * math.exp(-delta)))) < 1e-60
    j = np.linspace(0.0, 1.0, 401)
    p = psw(j, t, f0, delta)
    assert np.all(np.diff(p) >= 0) and p[-1] > p[0]
    js = 1.0 - math.sqrt(math.log(t * f0 / math.log(2.0)) / delta)
    assert abs(psw(js, t, f0, delta) - 0.5) < 1e-12
    # a longer window or a faster attempt rate lowers the half-switching current
    assert psw(js, 2 * t, f0, delta) > 0.5 and psw(js, t, 2 * f0, delta) > 0.5
