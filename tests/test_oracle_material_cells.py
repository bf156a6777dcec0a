"""Pins of the oracle's per-cell materials (Methods, "Physics and
discretization": material parameters per cell): uniform arrays reduce to the
scalar material; with Ms, A, alpha, Ku and D varying from cell to cell the
effective field is minus the gradient of an energy written out independently
here (pair sums for exchange, the per-cell DMI density with central
differences, a direct image sum for the demag energy of M = Ms m), the demag
FFT path equals a direct sum over M = Ms m, and the thermal field and the
torque take each cell's own parameters."""
import dataclasses

import numpy as np
import pytest

from oracle import Grid, Material, newell
from oracle import demag as dm
from oracle import fields as fl
from oracle import llg
from oracle import observables as oob
from oracle.constants import GAMMA0, KB, MU0
from workloads import random_unit


def _cells(grid, seed):
    rng = np.random.default_rng(seed)
    shape = grid.n[::-1]
    return dict(Ms_cells=rng.uniform(4e5, 9e5, shape), A_cells=rng.uniform(0.6e-11, 1.6e-11, shape),
                alpha_cells=rng.uniform(0.01, 0.4, shape), Ku_cells=rng.uniform(-2e5, 6e5, shape),
                D_cells=rng.uniform(-1e-3, 3e-3, shape))


def _demag_matrix(grid):
    """K (3 ncell, 3 ncell) with H = -K (Ms m) (component-major, x fastest):
    every source image within (P + 1/2) periods of the target (half weight on
    the boundary) with its Newell tensor, from the tensor alone."""
    nx, ny, nz = grid.n
    n = (nx, ny, nz)
    per = [bool(grid.pbc[a]) and n[a] > 1 for a in range(3)]
    shifts = [range(-grid.images[a] - 1, grid.images[a] + 2) if per[a] else [0] for a in range(3)]
    full = np.array([[0, 3, 4], [3, 1, 5], [4, 5, 2]])
    cells = [(x, y, z) for z in range(nz) for y in range(ny) for x in range(nx)]
    nc = len(cells)
    K = np.zeros((3, nc, 3, nc))
    for i, ci in enumerate(cells):
        offs, wts, src = [], [], []
        for j, cj in enumerate(cells):
            for tz in shifts[2]:
                for ty in shifts[1]:
                    for tx in shifts[0]:
                        d = [ci[a] - cj[a] - (tx, ty, tz)[a] * n[a] for a in range(3)]
                        w = 1.0
                        for a in range(3):
                            if per[a]:
                                lim2 = (2 * grid.images[a] + 1) * n[a]
                                w = 0.0 if 2 * abs(d[a]) > lim2 else (w * 0.5 if 2 * abs(d[a]) == lim2 else w)
                        if w:
                            offs.append(d)
                            wts.append(w)
                            src.append(j)
        Nt = newell.tensor_at_offsets(np.array(offs), grid.cell) * np.array(wts)[None]
        for a in range(3):
            for b in range(3):
                np.add.at(K[a, i, b], np.array(src), Nt[full[a, b]])
    return K.reshape(3 * nc, 3 * nc)


def _direct_demag(m, grid, Ms, K=None):
    """H_i = -sum_j N(r_i - r_j) Ms_j m_j over the source images (see
    _demag_matrix)."""
    K = _demag_matrix(grid) if K is None else K
    return -(K @ (Ms * m).reshape(-1)).reshape(m.shape)


def _energy(m, grid, mat, Hd_of):
    """Energy of a periodic-in-plane grid written out from the definitions:
    exchange as a sum over neighbour pairs with the harmonic-mean stiffness,
    interfacial DMI as the per-cell density D_i [m_z div m - (m . grad) m_z]
    with central differences, anisotropy -Ku_i (m . u)^2, Zeeman
    -mu0 Ms_i m . B / mu0, demag (mu0 / 2) sum Ms_i m_i . N * (Ms m)."""
    V = grid.volume
    Ms, Ku, D = mat.Ms_cells, mat.Ku_cells, mat.D_cells
    A = mat.A_cells
    E = 0.0
    for axis in range(3):
        if grid.n[axis] == 1:
            continue
        ax = -1 - axis
        h = grid.cell[axis]
        mp = np.roll(m, -1, axis=ax)
        Ap = np.roll(A, -1, axis=ax)
        w = 2 * A * Ap / (A + Ap)
        d2 = np.sum((mp - m) ** 2, axis=0)
        if not grid.pbc[axis]:   # open axis: no pair across the edge
            sl = [slice(None)] * 3
            sl[ax] = slice(grid.n[axis] - 1, grid.n[axis])
            d2[tuple(sl)] = 0.0
        E += V * np.sum(w * d2) / h ** 2
    for axis in (0, 1):
        if grid.n[axis] == 1:
            continue
        ax = -1 - axis
        h = grid.cell[axis]
        mp, mm = np.roll(m, -1, axis=ax), np.roll(m, 1, axis=ax)
        dens = m[2] * (mp[axis] - mm[axis]) - m[axis] * (mp[2] - mm[2])
        E += V * np.sum(D * dens) / (2 * h)
    u = np.asarray(mat.u) / np.linalg.norm(mat.u)
    E += -V * np.sum(Ku * np.tensordot(u, m, axes=(0, 0)) ** 2)
    E += -V * np.sum(Ms * np.tensordot(np.asarray(mat.B), m, axes=(0, 0)))
    E += 0.5 * MU0 * V * np.sum(Ms * np.sum(m * Hd_of(m), axis=0)) * -1.0
    return E


@pytest.mark.parametrize("grid", [
    Grid((5, 4, 1), (2e-9, 2.5e-9, 1e-9), pbc=(1, 1, 0), images=(1, 1, 0)),
    Grid((4, 3, 2), (2e-9, 2e-9, 1.5e-9), pbc=(1, 1, 0), images=(1, 1, 0)),
])
def test_field_is_minus_gradient_of_independent_energy(grid):
    mat = Material(Ms=1.0, A=1.0, alpha=0.1, Ku=0.0, u=(0.3, -0.2, 0.9), D=0.0,
                   B=(0.02, -0.01, 0.05), **_cells(grid, 3))
    m = random_unit(grid.n, seed=5)
    K = _demag_matrix(grid)
    Hd = lambda mm: _direct_demag(mm, grid, mat.Ms_cells, K)
    H = fl.effective_field(m, grid, mat)
    # the energy's own demag field must be the oracle's FFT demag
    assert np.abs(Hd(m) - fl.terms(m, grid, mat)["demag"]).max() <= 1e-12 * np.abs(H).max()
    h = 1e-6
    G = np.zeros_like(m)
    for idx in np.ndindex(m.shape):
        mp, mm = m.copy(), m.copy()
        mp[idx] += h
        mm[idx] -= h
        G[idx] = (_energy(mp, grid, mat, Hd) - _energy(mm, grid, mat, Hd)) / (2 * h)
    Hg = -G / (MU0 * mat.Ms_cells * grid.volume)
    assert np.abs(Hg - H).max() <= 1e-7 * np.abs(H).max()
    # the energy reported per term adds up to the same total
    E = oob.energies(m, grid, mat)["total"]
    assert abs(E - _energy(m, grid, mat, Hd)) <= 1e-10 * abs(E)


def test_uniform_arrays_reduce_to_scalar_material():
    grid = Grid((6, 5, 2), (2e-9, 2e-9, 1e-9))
    base = Material(Ms=6e5, A=1.2e-11, alpha=0.07, Ku=3e5, u=(0, 0, 1), D=2e-3, B=(0, 0, 0.1),
                    T=300.0)
    shape = grid.n[::-1]
    cells = dataclasses.replace(base, Ms_cells=np.full(shape, 6e5), A_cells=np.full(shape, 1.2e-11),
                                alpha_cells=np.full(shape, 0.07), Ku_cells=np.full(shape, 3e5),
                                D_cells=np.full(shape, 2e-3))
    m = random_unit(grid.n, seed=8)
    for name in ("exchange", "dmi", "demag", "anisotropy", "zeeman"):
        a, b = fl.terms(m, grid, base)[name], fl.terms(m, grid, cells)[name]
        assert np.abs(a - b).max() <= 1e-12 * max(1.0, np.abs(a).max()), name
    Ha, Hb = fl.effective_field(m, grid, base), fl.effective_field(m, grid, cells)
    ka = llg.llg_rhs(m, Ha, base.alpha)
    kb = llg.llg_rhs(m, Hb, fl.cell_param(cells, "alpha"))
    assert np.abs(ka - kb).max() <= 1e-12 * np.abs(ka).max()
    ea, eb = oob.energies(m, grid, base), oob.energies(m, grid, cells)
    for k in ea:
        assert abs(ea[k] - eb[k]) <= 1e-12 * max(abs(ea["total"]), 1e-30), k
    assert np.allclose(fl.thermal_sigma(grid, cells, 1e-13), fl.thermal_sigma(grid, base, 1e-13),
                       rtol=1e-14, atol=0)


def test_demag_of_per_cell_ms_equals_direct_sum():
    grid = Grid((4, 3, 3), (2e-9, 3e-9, 1.5e-9))
    Ms = np.random.default_rng(2).uniform(2e5, 1e6, grid.n[::-1])
    m = random_unit(grid.n, seed=9)
    a = dm.demag_fft(m, grid, Ms)
    b = _direct_demag(m, grid, Ms)
    assert np.abs(a - b).max() <= 1e-13 * Ms.max()
    # and the kernel-array direct sum of the oracle agrees
    assert np.abs(dm.demag_direct(m, grid, Ms) - b).max() <= 1e-13 * Ms.max()


def test_thermal_field_and_torque_take_each_cells_parameters():
    grid = Grid((4, 3, 1), (3e-9, 3e-9, 2e-9))
    cells = _cells(grid, 11)
    mat = Material(Ms=1.0, A=1e-11, alpha=0.5, T=250.0, **cells)
    dt = 2e-14
    sig = fl.thermal_sigma(grid, mat, dt)
    H = fl.thermal_field(grid, mat, dt, seed=77, step=5)
    for z, y, x in np.ndindex(grid.n[::-1]):
        one = Material(Ms=cells["Ms_cells"][z, y, x], alpha=cells["alpha_cells"][z, y, x], T=250.0)
        s = np.sqrt(2 * one.alpha * KB * one.T / (MU0 ** 2 * one.Ms * grid.volume * GAMMA0 * dt))
        assert abs(sig[z, y, x] - s) <= 1e-14 * s
    # the noise itself is the uniform-material noise scaled per cell
    ref = fl.thermal_field(grid, Material(Ms=8e5, alpha=0.5, T=250.0), dt, seed=77, step=5)
    s0 = fl.thermal_sigma(grid, Material(Ms=8e5, alpha=0.5, T=250.0), dt)
    assert np.allclose(H, ref / s0 * sig, rtol=1e-13, atol=0)
    m = random_unit(grid.n, seed=12)
    Hf = random_unit(grid.n, seed=13) * 1e5
    k = llg.llg_rhs(m, Hf, fl.cell_param(mat, "alpha"))
    for z, y, x in np.ndindex(grid.n[::-1]):
        a = cells["alpha_cells"][z, y, x]
        k1 = llg.llg_rhs(m[:, z:z + 1, y:y + 1, x:x + 1], Hf[:, z:z + 1, y:y + 1, x:x + 1], a)
        assert np.allclose(k[:, z, y, x], k1[:, 0, 0, 0], rtol=1e-14, atol=0)


def test_open_edges_use_each_edge_cells_d_over_2a():
    """Ghosts of an open film with per-cell D and A satisfy the free-edge
    condition dm/dn = (D_i / 2A_i)(z x n) x m with the edge cell's values."""
    grid = Grid((5, 4, 1), (2e-9, 2e-9, 1e-9))
    cells = _cells(grid, 4)
    mat = Material(Ms=1.0, A=1.0, D=0.0, **{k: cells[k] for k in ("Ms_cells", "A_cells", "D_cells")})
    m = random_unit(grid.n, seed=6)
    mm, mp = fl.neighbours(m, grid, mat, 0)
    k = cells["D_cells"] / (2 * cells["A_cells"])
    h = grid.cell[0]
    # last column: (ghost - m) / h = k (m_z, 0, -m_x)
    g = (mp[:, :, :, -1] - m[:, :, :, -1]) / h
    kk = k[:, :, -1]
    assert np.allclose(g, np.stack([kk * m[2, :, :, -1], 0 * kk, -kk * m[0, :, :, -1]]),
                       rtol=1e-12, atol=0)
    g = (m[:, :, :, 0] - mm[:, :, :, 0]) / h
    kk = k[:, :, 0]
    assert np.allclose(g, np.stack([kk * m[2, :, :, 0], 0 * kk, -kk * m[0, :, :, 0]]),
                       rtol=1e-12, atol=0)
