"""Pins of the oracle's fixed-step RK4 and damping-only relaxer (Methods,
"Integrators": RK4 fixed step, damping-only relax): fourth order against the
damped-macrospin closed form, the damping-only macrospin closed form (no
precession), and relaxed states that are stationary points of the full LLG
equation with lower energy."""
import dataclasses
import math

import numpy as np

from oracle import GAMMA0, Grid, Material
from oracle import integrators as it
from oracle import observables
from workloads import random_unit


def _macrospin(alpha, B=0.2, precess=True):
    return Grid((1, 1, 1), (4e-9, 4e-9, 4e-9)), Material(Ms=8e5, alpha=alpha, B=(0.0, 0.0, B),
                                                          demag=False, precess=precess)


def _exact(theta0, phi0, alpha, B, t, precess=True):
    gp = GAMMA0 / (1 + alpha ** 2)
    th = 2 * np.arctan(np.tan(theta0 / 2) * np.exp(-gp * alpha * B * t))
    ph = phi0 + (gp * B * t if precess else 0.0)
    return np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])


def test_rk4_is_fourth_order():
    alpha, B = 0.1, 0.2
    grid, mat = _macrospin(alpha, B)
    m0 = _exact(1.0, 0.0, alpha, B, 0.0).reshape(3, 1, 1, 1)
    T = 2e-10
    errs = []
    for n in (25, 50, 100):
        m = it.rk4_run(m0, grid, mat, T / n, n)
        errs.append(np.abs(m[:, 0, 0, 0] - _exact(1.0, 0.0, alpha, B, T)).max())
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert 3.7 < min(slopes) and max(slopes) < 4.4
    assert errs[-1] < 1e-6


def test_damping_only_macrospin_closed_form():
    """Without precession the moment turns straight towards the field: the
    azimuth stays fixed and the polar angle follows the damped closed form."""
    alpha, B = 0.3, 0.2
    grid, mat = _macrospin(alpha, B, precess=False)
    th0, ph0 = 2.0, 0.7
    m0 = _exact(th0, ph0, alpha, B, 0.0).reshape(3, 1, 1, 1)
    t_end = 0.2e-9
    res = it.rk45_run(m0, grid, mat, 0.0, t_end, tol=1e-11, dt0=1e-13)
    ref = _exact(th0, ph0, alpha, B, t_end, precess=False)
    assert np.abs(res.m[:, 0, 0, 0] - ref).max() < 1e-7
    assert abs(math.atan2(res.m[1, 0, 0, 0], res.m[0, 0, 0, 0]) - ph0) < 1e-12


def test_relaxed_film_is_a_stationary_point_with_lower_energy():
    grid = Grid((16, 12, 1), (4e-9, 4e-9, 4e-9))
    mat = Material(Ms=8e5, A=1.3e-11, alpha=0.5, Ku=2e5, u=(0, 0, 1))
    m0 = random_unit(grid.n, seed=21, replicas=1)[0]
    m, t, acc, rej, tq = it.relax_run(m0, grid, mat, torque_tol=1e8, t_max=2e-9, tol=1e-6)
    assert tq <= 1e8 and t < 2e-9
    E0 = observables.energies(m0, grid, mat)["total"]
    E1 = observables.energies(m, grid, mat)["total"]
    assert E1 < E0
    # per cell |full LLG torque| = |damping-only torque| sqrt(1 + alpha^2) /
    # alpha (both are |m x H| times a constant): the full torque vanishes
    # with the relaxer's
    full = np.sqrt((it.rhs(m, grid, mat) ** 2).sum(axis=0))
    damp = np.sqrt((it.rhs(m, grid, dataclasses.replace(mat, precess=False)) ** 2).sum(axis=0))
    assert np.allclose(full, damp * math.sqrt(1 + mat.alpha ** 2) / mat.alpha, rtol=1e-10)
    assert abs(damp.max() - tq) <= 1e-12 * tq
    assert np.abs(np.linalg.norm(m, axis=0) - 1).max() < 1e-14
