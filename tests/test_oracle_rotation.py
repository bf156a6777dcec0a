"""Pins of the oracle's norm-exact rotation integrator and of the retire/refill
trials (Results, "A replica-batched engine"; Methods, "Integrators" and
"Replica batching"; Depondt & Mertens 2009): Rodrigues' formula against an
independent rotation routine, the rotation form of the LLG equation, exact
precession for any step at zero damping, second order against the damped
macrospin closed form, |m| = 1 without normalisation, energy decay, the
Langevin law, and the trial bookkeeping of retire/refill."""
import json
import math
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import GAMMA0, KB, MU0, Grid, Material
from oracle import integrators as it
from oracle import llg, observables, rotation
from workloads import random_unit, replica_seeds

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_rodrigues_matches_an_independent_rotation_routine():
    rng = np.random.default_rng(4)
    v = rng.standard_normal((3, 1, 1, 50))
    w = rng.standard_normal((3, 1, 1, 50)) * rng.uniform(0, 3, 50)
    got = rotation.rotate(v, w)[:, 0, 0, :].T
    ref = Rotation.from_rotvec(w[:, 0, 0, :].T).apply(v[:, 0, 0, :].T)
    assert np.abs(got - ref).max() < 1e-14
    # zero angle: identity; quarter turn about z maps x to y
    assert np.array_equal(rotation.rotate(v, np.zeros_like(v)), v)
    e = rotation.rotate(np.array([1.0, 0, 0]).reshape(3, 1, 1, 1),
                        np.array([0, 0, math.pi / 2]).reshape(3, 1, 1, 1))
    assert np.abs(e[:, 0, 0, 0] - [0, 1, 0]).max() < 1e-16


def test_rotation_form_is_the_llg_equation():
    """Omega x m equals the Landau-Lifshitz-Gilbert torque for any m, H."""
    rng = np.random.default_rng(5)
    m = random_unit((6, 5, 2), seed=3, replicas=1)[0]
    H = 1e5 * rng.standard_normal(m.shape)
    for alpha in (0.0, 0.02, 0.7):
        o = rotation.omega(m, H, alpha)
        assert np.allclose(np.cross(o, m, axis=0), llg.llg_rhs(m, H, alpha), rtol=1e-13,
                           atol=1e-13 * np.abs(llg.llg_rhs(m, H, alpha)).max())


def _macrospin(alpha, B=0.2, T=0.0):
    return Grid((1, 1, 1), (4e-9, 4e-9, 4e-9)), Material(Ms=8e5, alpha=alpha, B=(0.0, 0.0, B),
                                                          T=T, demag=False)


def _macrospin_exact(theta0, phi0, alpha, B, t):
    gp = GAMMA0 / (1 + alpha ** 2)
    th = 2 * np.arctan(np.tan(theta0 / 2) * np.exp(-gp * alpha * B * t))
    ph = phi0 + gp * B * t
    return np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])


def test_exact_precession_for_any_step_without_damping():
    """At alpha = 0 in a uniform field both evaluations give the same Omega and
    each step is the exact rotation: the closed form holds at a step of 0.05
    precession periods, where Heun is far off."""
    B = 0.2
    grid, mat = _macrospin(0.0, B)
    period = 2 * math.pi / (GAMMA0 * B)
    dt, n = 0.05 * period, 400
    m0 = _macrospin_exact(1.1, 0.4, 0.0, B, 0.0).reshape(3, 1, 1, 1)
    got = rotation.depondt_run(m0, grid, mat, dt, n)[:, 0, 0, 0]
    ref = _macrospin_exact(1.1, 0.4, 0.0, B, n * dt)
    assert np.abs(got - ref).max() < 1e-11
    heun = it.heun_run(m0, grid, mat, dt, n)[:, 0, 0, 0]
    assert np.abs(heun - ref).max() > 1e-3


def test_second_order_against_the_damped_macrospin():
    alpha, B = 0.1, 0.2
    grid, mat = _macrospin(alpha, B)
    m0 = _macrospin_exact(1.0, 0.0, alpha, B, 0.0).reshape(3, 1, 1, 1)
    T = 2e-10
    errs = []
    for n in (100, 200, 400):
        m = rotation.depondt_run(m0, grid, mat, T / n, n)
        errs.append(np.abs(m[:, 0, 0, 0] - _macrospin_exact(1.0, 0.0, alpha, B, T)).max())
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert 1.8 < min(slopes) and max(slopes) < 2.3
    assert errs[-1] < 5e-5


def test_unit_norm_without_normalisation_and_energy_decay():
    """A damped film with exchange, anisotropy and demag: |m| stays 1 to
    round-off over 300 steps without any normalisation, and the energy (no
    drive, T = 0) does not increase."""
    grid = Grid((16, 8, 1), (4e-9, 4e-9, 4e-9))
    mat = Material(Ms=8e5, A=1.3e-11, alpha=0.5, Ku=3e5, u=(0, 0, 1))
    m = random_unit(grid.n, seed=11, replicas=1)[0]
    E = [observables.energies(m, grid, mat)["total"]]
    for k in range(30):
        m = rotation.depondt_run(m, grid, mat, 1e-13, 10)
        E.append(observables.energies(m, grid, mat)["total"])
    assert np.abs(np.linalg.norm(m, axis=0) - 1).max() < 1e-13
    assert np.all(np.diff(E) <= 1e-12 * np.abs(E[:-1]))
    assert E[-1] < E[0]


@pytest.mark.slow
def test_langevin_law_with_the_rotation_scheme():
    with open(os.path.join(GOLDEN, "paper_values.json")) as fh:
        g = json.load(fh)["langevin"]
    xi = g["xi"]
    cell = (4e-9, 4e-9, 4e-9)
    Ms, T = 8e5, 300.0
    V = cell[0] * cell[1] * cell[2]
    B = xi * KB * T / (Ms * V)
    grid = Grid((1, 1, 1), cell)
    mat = Material(Ms=Ms, alpha=0.1, B=(0, 0, B), T=T, demag=False)
    R = 4096
    seeds = replica_seeds(19, R)
    m = np.zeros((R, 3, 1, 1, 1)); m[:, 2] = 1.0
    dt = 1e-13
    # the ensemble relaxes from m_z = 1 over a few 0.1 ns: average over
    # 0.6-1.2 ns, where the transient has died out
    m = rotation.depondt_run(m, grid, mat, dt, 6000, seed=seeds)
    acc, n = 0.0, 0
    for k in range(6000, 12000, 3):
        m = rotation.depondt_run(m, grid, mat, dt, 3, seed=seeds, step0=k)
        acc += m[:, 2].mean()
        n += 1
    L = 1.0 / math.tanh(xi) - 1.0 / xi
    assert abs(acc / n - L) < 0.005
    assert abs(np.linalg.norm(m, axis=1) - 1).max() < 1e-13


def _switch_case(T):
    grid = Grid((1, 1, 1), (4e-9, 4e-9, 4e-9))
    mat = Material(Ms=8e5, alpha=0.2, Ku=2e5, u=(0, 0, 1), B=(0, 0, -1.0), T=T, demag=False)
    th = 0.3
    m_init = np.array([math.sin(th), 0.0, math.cos(th)]).reshape(3, 1, 1, 1)
    return grid, mat, m_init


def test_refill_at_zero_temperature_repeats_the_plain_switching_time():
    """T = 0: every trial is the same trajectory, so each recorded time equals
    the plain run's switching time and the slot finishes nsteps // s* trials."""
    grid, mat, m_init = _switch_case(0.0)
    dt = 1e-13
    tsw = [-1.0]
    rotation.depondt_run(m_init[None], grid, mat, dt, 2000, seed=np.array([1], np.uint64),
                         t_switch=tsw)
    assert tsw[0] > 0
    s_star = round(tsw[0] / dt)
    nsteps = 3 * s_star + s_star // 2
    times, done, m, g, s, _ = rotation.refill_slot(m_init, grid, mat, dt, nsteps, 1, cap=8)
    assert done == 3 and g == 3 and s == nsteps - 3 * s_star
    assert times == [s_star * dt] * 3
    # the running trial is the plain run from the initial state
    assert np.array_equal(m, rotation.depondt_run(m_init, grid, mat, dt, s))
    times2, done2, *_ = rotation.refill_slot(m_init, grid, mat, dt, nsteps, 1, cap=2)
    assert times2 == times[:2] and done2 == 3


def test_refill_trials_use_fresh_noise_streams():
    """T > 0: trial g equals a standalone run with counter word 3 = g from the
    initial state; trial 0 is the plain run's noise."""
    grid, mat, m_init = _switch_case(300.0)
    dt, seed = 1e-13, 77
    times, done, *_ = rotation.refill_slot(m_init, grid, mat, dt, 5000, seed, cap=16)
    assert done >= 2
    for g in range(min(done, 3)):
        m, s = m_init.copy(), 0
        while True:
            m = rotation.depondt_step(m, grid, mat, dt, seed, s, g)
            s += 1
            if m[2].mean() < 0:
                break
        assert times[g] == s * dt
    assert len(set(times)) > 1
