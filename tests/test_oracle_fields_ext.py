"""Pins of the oracle's further field terms (Methods, "Physics and
discretization": bulk DMI, cubic anisotropy, RKKY interlayer exchange): the
field is the energy gradient on periodic grids with every term on, the exact
discrete field and energy of a bulk-DMI helix (handedness), the bulk-DMI free
edge condition, cubic easy axes and the [111] energy, the RKKY energy of
parallel and antiparallel layers, and a per-cell exchange stiffness (uniform
values reduce to the scalar, the two-cell harmonic-mean coupling, the energy
gradient with a zero-stiffness cell)."""
import math

import numpy as np
import pytest

from oracle import MU0, Grid, Material
from oracle import fields as fl
from oracle import observables
from workloads import random_unit, uniform


@pytest.mark.parametrize("grid", [
    Grid((4, 3, 3), (3e-9, 2e-9, 2e-9), pbc=(1, 1, 1), images=(1, 1, 1)),
    Grid((5, 4, 1), (2e-9, 2e-9, 1e-9), pbc=(1, 1, 0), images=(1, 1, 0)),
])
def test_field_is_energy_gradient_with_all_terms(grid):
    mat = Material(Ms=6e5, A=1.2e-11, D=2e-3, Db=1.5e-3, Ku=3e5, u=(0.1, 0.2, 0.97),
                   Kc1=4e4, Kc2=-2e4, c1=(0.8, 0.6, 0.0), c2=(-0.6, 0.8, 0.1),
                   B=(0.01, -0.02, 0.05), rkky=-1e-4 if grid.n[2] > 1 else 0.0, rkky_z=(0, 2))
    m = random_unit(grid.n, seed=19)
    H = fl.effective_field(m, grid, mat)
    pref = 1.0 / (MU0 * mat.Ms * grid.volume)
    rng = np.random.default_rng(3)
    flat = m.reshape(-1)
    for idx in rng.choice(flat.size, 16, replace=False):
        h = 1e-3
        mp = flat.copy(); mp[idx] += h
        mm = flat.copy(); mm[idx] -= h
        Ep = observables.energies(mp.reshape(m.shape), grid, mat)["total"]
        Em = observables.energies(mm.reshape(m.shape), grid, mat)["total"]
        g = -(Ep - Em) / (2 * h) * pref
        assert g == pytest.approx(H.reshape(-1)[idx], rel=1e-6, abs=1e-6 * np.abs(H).max())


def test_bulk_dmi_helix_closed_form():
    """m = (cos kz, sin kz, 0) on a periodic chain along z: central differences
    give curl m = -(sin kh / h) m, so H = (2 Db / mu0 Ms)(sin kh / h) m and the
    energy is -Db V N sin(kh) / h (negative for Db k > 0)."""
    n, h = 16, 1e-9
    grid = Grid((1, 1, n), (2e-9, 2e-9, h), pbc=(0, 0, 1), images=(0, 0, 0))
    k = 2 * math.pi * 3 / (n * h)
    z = np.arange(n) * h
    m = np.zeros((3, n, 1, 1))
    m[0, :, 0, 0] = np.cos(k * z)
    m[1, :, 0, 0] = np.sin(k * z)
    Db = 2e-3
    mat = Material(Ms=5e5, A=1e-11, Db=Db, demag=False)
    H = fl.bulk_dmi_field(m, grid, mat)
    ref = 2 * Db / (MU0 * mat.Ms) * math.sin(k * h) / h * m
    assert np.abs(H - ref).max() < 1e-9 * np.abs(ref).max()
    e = observables.energies(m, grid, mat)["dmi_bulk"]
    assert e == pytest.approx(-Db * grid.volume * n * math.sin(k * h) / h, rel=1e-12)
    mirror = m.copy()
    mirror[1] *= -1  # the other handedness
    assert observables.energies(mirror, grid, mat)["dmi_bulk"] == pytest.approx(-e, rel=1e-12)


def test_bulk_dmi_edge_condition():
    grid = Grid((5, 4, 3), (2e-9, 3e-9, 1e-9))
    mat = Material(Ms=5e5, A=1.1e-11, Db=2.5e-3)
    m = random_unit(grid.n, seed=23)
    k = mat.Db / (2 * mat.A)
    for axis in range(3):
        mm, mp = fl.neighbours(m, grid, mat, axis)
        ax = -1 - axis
        last = np.take(m, [grid.n[axis] - 1], axis=ax)
        d = (np.take(mp, [grid.n[axis] - 1], axis=ax) - last) / grid.cell[axis]
        e = np.zeros(3); e[axis] = 1.0
        ref = k * np.cross(e[:, None, None, None], last, axis=0)
        assert np.allclose(d, ref, atol=1e-9 * k)
        first = np.take(m, [0], axis=ax)
        d0 = (first - np.take(mm, [0], axis=ax)) / grid.cell[axis]
        assert np.allclose(d0, k * np.cross(e[:, None, None, None], first, axis=0), atol=1e-9 * k)


def test_cubic_anisotropy_axes_and_111():
    grid = Grid((1, 1, 1), (2e-9, 2e-9, 2e-9))
    c1, c2 = np.array([0.6, 0.8, 0.0]), np.array([-0.8, 0.6, 0.0])
    c3 = np.cross(c1, c2)
    Kc1, Kc2 = 5e4, 3e4
    mat = Material(Ms=8e5, Kc1=Kc1, Kc2=Kc2, c1=tuple(c1), c2=tuple(c2), demag=False)
    for a in (c1, c2, c3, -c1):
        m = a.reshape(3, 1, 1, 1)
        assert np.abs(fl.cubic_field(m, mat)).max() < 1e-9
        assert observables.energies(m, grid, mat)["cubic"] == pytest.approx(0.0, abs=1e-40)
    d = (c1 + c2 + c3) / math.sqrt(3)
    e111 = observables.energies(d.reshape(3, 1, 1, 1), grid, mat)["cubic"]
    assert e111 == pytest.approx(grid.volume * (Kc1 / 3 + Kc2 / 27), rel=1e-12)
    # [111] is an equilibrium too (field parallel to m)
    H = fl.cubic_field(d.reshape(3, 1, 1, 1), mat)[:, 0, 0, 0]
    assert np.linalg.norm(np.cross(H, d)) < 1e-9 * np.linalg.norm(H)


def test_rkky_parallel_and_antiparallel_layers():
    grid = Grid((3, 2, 4), (2e-9, 2e-9, 1e-9))
    sigma = -2e-4  # antiferromagnetic coupling
    mat = Material(Ms=8e5, A=0.0, rkky=sigma, rkky_z=(1, 2), demag=False)
    area = grid.n[0] * grid.n[1] * grid.cell[0] * grid.cell[1]
    m = uniform(grid.n, (0, 0, 1))
    assert observables.energies(m, grid, mat)["rkky"] == pytest.approx(-sigma * area, rel=1e-12)
    m[2, 2] *= -1  # flip layer z = 2
    assert observables.energies(m, grid, mat)["rkky"] == pytest.approx(sigma * area, rel=1e-12)
    H = fl.rkky_field(m, grid, mat)
    assert np.allclose(H[:, 1], sigma / (MU0 * mat.Ms * grid.cell[2]) * m[:, 2])
    assert not np.any(H[:, 0]) and not np.any(H[:, 3])


def test_per_cell_exchange_reduces_to_uniform_and_two_cell_closed_form():
    import dataclasses
    grid = Grid((5, 4, 3), (2e-9, 3e-9, 1e-9))
    mat = Material(Ms=6e5, A=1.1e-11, D=2e-3, Db=1e-3, demag=False)
    m = random_unit(grid.n, seed=29)
    ref = fl.effective_field(m, grid, mat)
    same = dataclasses.replace(mat, A_cells=np.full((3, 4, 5), 1.1e-11))
    assert np.abs(fl.effective_field(m, grid, same) - ref).max() <= 1e-15 * np.abs(ref).max()
    # two cells along x with A1, A2: harmonic-mean coupling
    g2 = Grid((2, 1, 1), (2e-9, 2e-9, 2e-9))
    A1, A2 = 1e-11, 3e-11
    m2 = random_unit(g2.n, seed=30)
    two = Material(Ms=8e5, A=0.0, A_cells=np.array([[[A1, A2]]]), demag=False)
    H = fl.exchange_field(m2, g2, two)
    w = 2 * A1 * A2 / (A1 + A2)
    ref0 = 2 * w / (MU0 * two.Ms) * (m2[:, 0, 0, 1] - m2[:, 0, 0, 0]) / g2.cell[0] ** 2
    assert np.allclose(H[:, 0, 0, 0], ref0, rtol=1e-14)
    assert np.allclose(H[:, 0, 0, 1], -ref0, rtol=1e-14)


def test_per_cell_exchange_is_energy_gradient():
    import dataclasses
    grid = Grid((4, 3, 3), (3e-9, 2e-9, 2e-9), pbc=(1, 1, 1), images=(1, 1, 1))
    rng = np.random.default_rng(31)
    Ac = rng.uniform(0.2e-11, 2e-11, (3, 3, 4))
    Ac[1, 1, 2] = 0.0  # a non-magnetic-like link: zero coupling to this cell
    mat = Material(Ms=6e5, A=1e-11, A_cells=Ac, D=1e-3, Db=5e-4, Ku=2e5, demag=False)
    m = random_unit(grid.n, seed=32)
    H = fl.effective_field(m, grid, mat)
    pref = 1.0 / (MU0 * mat.Ms * grid.volume)
    flat = m.reshape(-1)
    for idx in rng.choice(flat.size, 16, replace=False):
        h = 1e-3
        mp = flat.copy(); mp[idx] += h
        mm = flat.copy(); mm[idx] -= h
        Ep = observables.energies(mp.reshape(m.shape), grid, mat)["total"]
        Em = observables.energies(mm.reshape(m.shape), grid, mat)["total"]
        assert -(Ep - Em) / (2 * h) * pref == pytest.approx(H.reshape(-1)[idx], rel=1e-6,
                                                            abs=1e-6 * np.abs(H).max())
