"""Pins of the oracle's local field terms and torque (Methods, "Physics and
discretization"; LLG equation) against closed forms and invariants."""
import math

import numpy as np
import pytest

from oracle import GAMMA0, MU0, Grid, Material
from oracle import fields as fl
from oracle import llg, observables
from workloads import neel_skyrmions, random_unit, uniform


def test_uniform_state_has_no_exchange_field():
    for grid in (Grid((5, 4, 3), (2e-9, 3e-9, 1e-9)),
                 Grid((6, 4, 1), (2e-9, 2e-9, 1e-9), pbc=(1, 1, 0))):
        m = uniform(grid.n, (0.3, -0.4, 0.866))
        H = fl.exchange_field(m, grid, Material())
        assert np.abs(H).max() < 1e-6


def test_exchange_field_of_spin_wave_closed_form():
    """For m_i = (s cos(k x_i), s sin(k x_i), c) on a periodic chain,
    H_ex = -(2A/mu0 Ms)(4/dx^2) sin^2(k dx/2) (m - c z)."""
    N, dx = 40, 5e-9
    grid = Grid((N, 1, 1), (dx, 3e-9, 3e-9), pbc=(1, 0, 0))
    mat = Material(Ms=8e5, A=1.3e-11)
    th = 0.4
    for nk in (1, 3, 7, 20):
        k = 2 * math.pi * nk / (N * dx)
        x = np.arange(N) * dx
        m = np.zeros((3, 1, 1, N))
        m[0, 0, 0] = math.sin(th) * np.cos(k * x)
        m[1, 0, 0] = math.sin(th) * np.sin(k * x)
        m[2, 0, 0] = math.cos(th)
        C = 2 * mat.A / (MU0 * mat.Ms) * 4 / dx ** 2 * math.sin(k * dx / 2) ** 2
        ref = -C * m.copy()
        ref[2] += C * math.cos(th)
        H = fl.exchange_field(m, grid, mat)
        assert np.abs(H - ref).max() <= 1e-9 * C


def test_dmi_field_of_cycloid_closed_form():
    """m = (sin kx, 0, cos kx) on a periodic chain: central differences give
    H_dmi = -(2D/mu0 Ms)(sin(k dx)/dx) m, so the DMI energy per volume is
    D sin(k dx)/dx: negative for k < 0 when D > 0."""
    N, dx = 32, 2e-9
    grid = Grid((N, 1, 1), (dx, 2e-9, 1e-9), pbc=(1, 0, 0))
    mat = Material(Ms=5.8e5, A=1.5e-11, D=3e-3)
    for nk in (-5, -1, 1, 4):
        k = 2 * math.pi * nk / (N * dx)
        x = np.arange(N) * dx
        m = np.zeros((3, 1, 1, N))
        m[0, 0, 0] = np.sin(k * x)
        m[2, 0, 0] = np.cos(k * x)
        H = fl.dmi_field(m, grid, mat)
        pref = 2 * mat.D / (MU0 * mat.Ms) * math.sin(k * dx) / dx
        assert np.abs(H + pref * m).max() <= 1e-9 * abs(pref)
        e = observables.energies(m, grid, Material(Ms=mat.Ms, A=mat.A, D=mat.D, demag=False))["dmi"]
        assert e == pytest.approx(mat.D * math.sin(k * dx) / dx * N * grid.volume, rel=1e-12)


def test_dmi_energy_negative_for_outward_neel_skyrmion():
    n, cell = (64, 64, 1), (2e-9, 2e-9, 0.6e-9)
    m, _, _ = neel_skyrmions(n, cell, 1, 15e-9, 15e-9, seed=5, width=5e-9)
    grid = Grid(n, cell, pbc=(1, 1, 0))
    mat = Material(Ms=5.8e5, A=1.5e-11, D=3e-3, demag=False)
    assert observables.energies(m, grid, mat)["dmi"] < 0
    assert observables.energies(m, grid, Material(Ms=5.8e5, A=1.5e-11, D=-3e-3, demag=False))["dmi"] > 0


def test_dmi_edge_ghost_satisfies_boundary_condition():
    """At an open x edge the ghost makes the one-sided derivative equal
    (D/2A)(m_z, 0, -m_x), the free boundary condition of the paper."""
    grid = Grid((6, 5, 1), (2e-9, 2e-9, 1e-9))
    mat = Material(Ms=5.8e5, A=1.5e-11, D=3e-3)
    m = random_unit(grid.n, seed=3)
    mm, mp = fl.neighbours(m, grid, mat, 0)
    k = mat.D / (2 * mat.A)
    right = m[:, :, :, -1]
    d = (mp[:, :, :, -1] - right) / grid.cell[0]
    assert np.allclose(d, k * np.stack([right[2], 0 * right[0], -right[0]]), atol=1e-6)
    mm, mp = fl.neighbours(m, grid, mat, 1)
    bottom = m[:, :, 0, :]
    d = (bottom - mm[:, :, 0, :]) / grid.cell[1]
    assert np.allclose(d, k * np.stack([0 * bottom[0], bottom[2], -bottom[1]]), atol=1e-6)


@pytest.mark.parametrize("grid", [
    Grid((6, 5, 1), (2e-9, 2e-9, 0.6e-9), pbc=(1, 1, 0), images=(1, 1, 0)),
    Grid((4, 3, 2), (3e-9, 2e-9, 2e-9), pbc=(1, 1, 1), images=(1, 1, 1)),
])
def test_field_is_energy_gradient(grid):
    """H_i = -(1 / mu0 Ms V) dE/dm_i (periodic: every term is a symmetric
    quadratic form plus the linear Zeeman term) by central differences."""
    mat = Material(Ms=5.8e5, A=1.5e-11, D=3e-3, Ku=0.8e6, u=(0.2, 0.3, 0.9),
                   B=(0.01, -0.02, 0.1))
    m = random_unit(grid.n, seed=9)
    H = fl.effective_field(m, grid, mat)
    pref = 1.0 / (MU0 * mat.Ms * grid.volume)
    rng = np.random.default_rng(0)
    flat = m.reshape(-1)
    for idx in rng.choice(flat.size, 12, replace=False):
        h = 1e-3
        mp = flat.copy(); mp[idx] += h
        mm = flat.copy(); mm[idx] -= h
        Ep = observables.energies(mp.reshape(m.shape), grid, mat)["total"]
        Em = observables.energies(mm.reshape(m.shape), grid, mat)["total"]
        g = -(Ep - Em) / (2 * h) * pref
        assert g == pytest.approx(H.reshape(-1)[idx], rel=1e-7, abs=1e-6 * np.abs(H).max())


def test_anisotropy_and_zeeman_closed_forms():
    grid = Grid((3, 2, 1), (1e-9, 1e-9, 1e-9))
    mat = Material(Ms=6e5, Ku=4e5, u=(0.0, 0.6, 0.8), B=(0.1, 0.2, -0.3))
    m = random_unit(grid.n, seed=4)
    u = np.array([0.0, 0.6, 0.8])
    Ha = fl.anisotropy_field(m, mat)
    mu = np.einsum("c...,c->...", m, u)
    assert np.allclose(Ha, 2 * mat.Ku / (MU0 * mat.Ms) * u[:, None, None, None] * mu)
    Hz = fl.zeeman_field(m, mat)
    assert np.allclose(Hz[:, 0, 0, 0], np.array(mat.B) / MU0)
    e = observables.energies(m, grid, Material(Ms=6e5, Ku=4e5, u=(0.0, 0.6, 0.8), demag=False))
    assert e["anisotropy"] == pytest.approx(-mat.Ku * grid.volume * np.sum(mu ** 2), rel=1e-13)


def test_torque_invariants():
    grid = Grid((5, 4, 2), (2e-9, 2e-9, 2e-9))
    m = random_unit(grid.n, seed=8)
    H = 1e5 * random_unit(grid.n, seed=9)
    for alpha in (0.0, 0.02, 0.5):
        k = llg.llg_rhs(m, H, alpha)
        assert np.abs(np.sum(m * k, axis=0)).max() <= 1e-6 * np.abs(k).max()
    k = llg.llg_rhs(m, 3e5 * m, 0.3)
    assert np.abs(k).max() < 1e-2


def test_torque_precession_sense_and_rate():
    """m along x, H along z: dm/dt = -gamma' mu0 H (m x z + alpha m x (m x z))."""
    m = np.zeros((3, 1, 1, 1)); m[0] = 1.0
    H = np.zeros_like(m); H[2] = 1e5
    for alpha in (0.0, 0.1):
        k = llg.llg_rhs(m, H, alpha)[:, 0, 0, 0]
        gp = GAMMA0 / (1 + alpha ** 2)
        assert np.allclose(k, gp * MU0 * 1e5 * np.array([0.0, 1.0, alpha]), rtol=1e-14)


def test_thermal_sigma_formula_units():
    grid = Grid((1, 1, 1), (4e-9, 4e-9, 4e-9))
    mat = Material(Ms=8e5, alpha=0.02, T=300.0)
    s = fl.thermal_sigma(grid, mat, 1e-14)
    ref = math.sqrt(2 * 0.02 * 1.380649e-23 * 300 / (MU0 ** 2 * 8e5 * 64e-27 * GAMMA0 * 1e-14))
    assert s == pytest.approx(ref, rel=1e-15)
    assert fl.thermal_sigma(grid, Material(T=0.0), 1e-14) == 0.0
