"""Local effective-field terms, FP64 (Methods, "Physics and discretization").

All fields are in A/m; ``m`` has shape (3, nz, ny, nx), or (R, 3, nz, ny, nx)
for a batch of replicas sharing one geometry and material.

* Exchange: six-point Laplacian, H = (2A / mu0 Ms) sum_a (m_{i+a} + m_{i-a} - 2 m_i) / D_a^2.
  With a per-cell stiffness (Methods lists per-cell materials; reading of the
  interface): H_i = (2 / mu0 Ms) sum_j A_ij (m_j - m_i) / D_a^2 with the
  harmonic mean A_ij = 2 A_i A_j / (A_i + A_j) (0 if both vanish); a ghost
  neighbour takes A_i.  The edge conditions use the edge cell's A_i.
* Interfacial DMI: energy density D [m_z div m - (m . grad) m_z] (Rohart-Thiaville
  sign as in mumax3), field H = (2D / mu0 Ms)(d_x m_z, d_y m_z, -d_x m_x - d_y m_y)
  with central differences (m_{i+1} - m_{i-1}) / (2 D_a).
* Open edges use ghost cells from the free boundary condition
  dm/dn = (D / 2A)(z x n) x m (Results "Exact agreement"; Methods): along x,
  d_x m = (D/2A)(m_z, 0, -m_x); along y, d_y m = (D/2A)(0, m_z, -m_y); the
  ghost is m_edge +/- D_a d_a m.  Along z, and everywhere when D = 0, the ghost
  is m_edge (Neumann).  Exchange and DMI share the ghosts (reading).  An axis
  with a single cell contributes no derivative (reading).
* Bulk DMI (Methods lists it among the field terms; form not printed;
  reading): energy density Db m . (curl m), field H = -(2 Db / mu0 Ms) curl m
  with central differences; its free boundary condition (from the variation
  of A |grad m|^2 + Db m . curl m) is d_a m = (Db / 2A) e_a x m on every open
  axis, added to the interfacial one in the shared ghosts.
* Cubic anisotropy (Methods; reading): energy density Kc1 (m1^2 m2^2 +
  m2^2 m3^2 + m3^2 m1^2) + Kc2 m1^2 m2^2 m3^2 with m_i = m . c_i, c3 = c1 x c2,
  field H = -(1 / mu0 Ms) dE/dm.
* RKKY interlayer exchange (Methods; reading): surface energy density
  -sigma m(z0) . m(z1) between cell layers z0 and z1, field on either layer
  (sigma / (mu0 Ms d_z)) m(other layer).
* Uniaxial anisotropy H = (2 Ku / mu0 Ms)(m . u) u; Zeeman H = B / mu0.
* Thermal (Brown) field H = sigma eta with
  sigma = sqrt(2 alpha kB T / (mu0^2 Ms V gamma0 dt)) (Results, "A
  replica-batched engine"), V the cell volume.
* Per-cell materials (Methods: material parameters per cell; reading of what
  that means for each term): every field term that carries 1 / (mu0 Ms) takes
  the cell's own Ms_i; the demag convolution acts on M_j = Ms_j m_j; the
  anisotropy and the thermal field take the cell's Ku_i, alpha_i and Ms_i.  A
  per-cell interfacial D keeps the energy density D_i [m_z div m - (m . grad)
  m_z] of each cell with central differences; collecting its terms per
  neighbour pair gives each pair the coupling (D_i + D_j) / 2, so the field of
  cell i is (1 / mu0 Ms_i D_a) [D_{i,i+1} m_z(i+1) - D_{i-1,i} m_z(i-1)] along
  x and y (and the matching m_a terms in H_z), which reduces to the uniform
  formula when D is uniform.  A ghost neighbour takes the edge cell's D_i,
  and the edge condition uses D_i / 2A_i.
"""
from __future__ import annotations

import math

import numpy as np

from .constants import GAMMA0, KB, MU0
from . import demag as _demag
from . import philox as _philox

# numpy axis (counted from the end) of each spatial axis; component axis is -4
_NP_AXIS = {0: -1, 1: -2, 2: -3}


def _comp(m, c):
    return m[..., c, :, :, :]


def cell_param(mat, name):
    """Parameter ``name`` (Ms, alpha, Ku or D) of the material: its per-cell
    array (nz, ny, nx) if set, else the scalar."""
    arr = getattr(mat, name + "_cells")
    return getattr(mat, name) if arr is None else np.asarray(arr, dtype=np.float64)


def _edge_slices(grid, axis, ndim):
    """Index tuples of the first and last layer of cells along ``axis`` for an
    array with ``ndim`` dimensions whose last three are (nz, ny, nx)."""
    ax = _NP_AXIS[axis]
    n = grid.n[axis]
    first = [slice(None)] * ndim
    last = [slice(None)] * ndim
    first[ndim + ax] = slice(0, 1)
    last[ndim + ax] = slice(n - 1, n)
    return tuple(first), tuple(last)


def _edge_derivative(mc, axis, D, A, Db=0.0):
    """Boundary-condition derivative d_axis m at an open edge (3, ...):
    interfacial (D/2A)(z x e_a) x m on x and y, bulk (Db/2A) e_a x m on
    every axis; A may be an array of the edge cells' values."""
    A = np.asarray(A, dtype=np.float64)
    safe = np.where(A != 0, A, 1.0)
    k = np.where(A != 0, D / (2.0 * safe), 0.0)
    kb = np.where(A != 0, Db / (2.0 * safe), 0.0)
    mx, my, mz = _comp(mc, 0), _comp(mc, 1), _comp(mc, 2)
    zero = np.zeros_like(mx)
    if axis == 0:
        out = k * np.stack([mz, zero, -mx], axis=-4)
    elif axis == 1:
        out = k * np.stack([zero, mz, -my], axis=-4)
    else:
        out = np.zeros_like(mc)
    if np.any(kb != 0.0):
        if axis == 0:    # x x m
            ex = np.stack([zero, -mz, my], axis=-4)
        elif axis == 1:  # y x m
            ex = np.stack([mz, zero, -mx], axis=-4)
        else:            # z x m
            ex = np.stack([-my, mx, zero], axis=-4)
        out = out + kb * ex
    return out


def neighbours(m, grid, mat, axis):
    """(m_minus, m_plus): values at i-1 and i+1 along ``axis`` with periodic
    wrap or boundary-condition ghosts."""
    ax = _NP_AXIS[axis]
    n = grid.n[axis]
    h = grid.cell[axis]
    if grid.pbc[axis]:
        return np.roll(m, 1, axis=ax), np.roll(m, -1, axis=ax)
    mm = np.roll(m, 1, axis=ax)
    mp = np.roll(m, -1, axis=ax)
    first = [slice(None)] * m.ndim
    last = [slice(None)] * m.ndim
    first[m.ndim + ax] = slice(0, 1)
    last[m.ndim + ax] = slice(n - 1, n)
    first, last = tuple(first), tuple(last)
    D = cell_param(mat, "D")
    use_dmi = (bool(np.any(D != 0.0)) and axis in (0, 1)) or mat.Db != 0.0
    m_first = m[first]
    m_last = m[last]
    if use_dmi:
        if mat.A_cells is not None:
            Ac = np.asarray(mat.A_cells, dtype=np.float64)
            a_first, a_last = Ac[first[-3:]], Ac[last[-3:]]
        else:
            a_first = a_last = mat.A
        if mat.D_cells is not None:
            d_first, d_last = D[first[-3:]], D[last[-3:]]
        else:
            d_first = d_last = mat.D
        mm[first] = m_first - h * _edge_derivative(m_first, axis, d_first, a_first, mat.Db)
        mp[last] = m_last + h * _edge_derivative(m_last, axis, d_last, a_last, mat.Db)
    else:
        mm[first] = m_first
        mp[last] = m_last
    return mm, mp


def _harmonic(a, b):
    s = a + b
    return np.where(s > 0, 2.0 * a * b / np.where(s > 0, s, 1.0), 0.0)


def _neighbour_A(Ac, grid, axis):
    """(A at i-1, A at i+1) along ``axis``: periodic wrap, or the cell's own
    value where the neighbour is a ghost."""
    ax = _NP_AXIS[axis]
    am, ap = np.roll(Ac, 1, axis=ax), np.roll(Ac, -1, axis=ax)
    if not grid.pbc[axis]:
        n = grid.n[axis]
        first = [slice(None)] * 3
        last = [slice(None)] * 3
        first[3 + ax] = slice(0, 1)
        last[3 + ax] = slice(n - 1, n)
        am[tuple(first)] = Ac[tuple(first)]
        ap[tuple(last)] = Ac[tuple(last)]
    return am, ap


def exchange_field(m, grid, mat):
    H = np.zeros_like(m)
    Ms = cell_param(mat, "Ms")
    if mat.A_cells is None:
        pref = 2.0 * mat.A / (MU0 * Ms)
        for axis in range(3):
            if grid.n[axis] == 1:
                continue
            mm, mp = neighbours(m, grid, mat, axis)
            H += pref * (mm + mp - 2.0 * m) / grid.cell[axis] ** 2
        return H
    Ac = np.asarray(mat.A_cells, dtype=np.float64)
    for axis in range(3):
        if grid.n[axis] == 1:
            continue
        mm, mp = neighbours(m, grid, mat, axis)
        am, ap = _neighbour_A(Ac, grid, axis)
        wm, wp = _harmonic(Ac, am), _harmonic(Ac, ap)
        H += 2.0 / (MU0 * Ms) * (wm * (mm - m) + wp * (mp - m)) / grid.cell[axis] ** 2
    return H


def _neighbour_D(Dc, grid, axis):
    """(D at i-1, D at i+1) along ``axis``: periodic wrap, or the cell's own
    value where the neighbour is a ghost."""
    ax = _NP_AXIS[axis]
    dm, dp = np.roll(Dc, 1, axis=ax), np.roll(Dc, -1, axis=ax)
    if not grid.pbc[axis]:
        first, last = _edge_slices(grid, axis, 3)
        dm[first] = Dc[first]
        dp[last] = Dc[last]
    return dm, dp


def dmi_field(m, grid, mat):
    H = np.zeros_like(m)
    Ms = cell_param(mat, "Ms")
    if mat.D_cells is not None:
        # pair couplings (D_i + D_j) / 2 of the per-cell energy density
        Dc = np.asarray(mat.D_cells, dtype=np.float64)
        if not np.any(Dc != 0.0):
            return H
        for axis in (0, 1):
            if grid.n[axis] == 1:
                continue
            mm, mp = neighbours(m, grid, mat, axis)
            dm, dp = _neighbour_D(Dc, grid, axis)
            wm, wp = 0.5 * (Dc + dm), 0.5 * (Dc + dp)
            pref = 1.0 / (MU0 * Ms * grid.cell[axis])
            H[..., axis, :, :, :] += pref * (wp * _comp(mp, 2) - wm * _comp(mm, 2))
            H[..., 2, :, :, :] -= pref * (wp * _comp(mp, axis) - wm * _comp(mm, axis))
        return H
    if mat.D == 0.0:
        return H
    pref = 2.0 * mat.D / (MU0 * Ms)
    for axis in (0, 1):
        if grid.n[axis] == 1:
            continue
        mm, mp = neighbours(m, grid, mat, axis)
        d = (mp - mm) / (2.0 * grid.cell[axis])
        # d_x m_z -> H_x ; d_y m_z -> H_y ; -d_x m_x - d_y m_y -> H_z
        H[..., axis, :, :, :] += pref * _comp(d, 2)
        H[..., 2, :, :, :] -= pref * _comp(d, axis)
    return H


def bulk_dmi_field(m, grid, mat):
    """-(2 Db / mu0 Ms) curl m, central differences with the shared ghosts."""
    H = np.zeros_like(m)
    if mat.Db == 0.0:
        return H
    pref = -2.0 * mat.Db / (MU0 * cell_param(mat, "Ms"))
    for axis in range(3):
        if grid.n[axis] == 1:
            continue
        mm, mp = neighbours(m, grid, mat, axis)
        d = (mp - mm) / (2.0 * grid.cell[axis])  # d_axis m
        # curl_c = sum over (axis, j) of eps_{c axis j} d_axis m_j
        for c in range(3):
            for j in range(3):
                e = _levi_civita(c, axis, j)
                if e:
                    H[..., c, :, :, :] += pref * e * _comp(d, j)
    return H


def _levi_civita(i, j, k):
    return (i - j) * (j - k) * (k - i) // 2


def _cubic_axes(mat):
    c1 = np.asarray(mat.c1, float)
    c1 = c1 / np.linalg.norm(c1)
    c2 = np.asarray(mat.c2, float)
    c2 = c2 - (c2 @ c1) * c1
    c2 = c2 / np.linalg.norm(c2)
    return c1, c2, np.cross(c1, c2)


def cubic_field(m, mat):
    """-(1 / mu0 Ms) d/dm of Kc1 (m1^2 m2^2 + m2^2 m3^2 + m3^2 m1^2) +
    Kc2 m1^2 m2^2 m3^2."""
    if mat.Kc1 == 0.0 and mat.Kc2 == 0.0:
        return np.zeros_like(m)
    ax = _cubic_axes(mat)
    mi = [sum(a[c] * _comp(m, c) for c in range(3)) for a in ax]
    g = [2 * mat.Kc1 * mi[i] * (mi[(i + 1) % 3] ** 2 + mi[(i + 2) % 3] ** 2) +
         2 * mat.Kc2 * mi[i] * mi[(i + 1) % 3] ** 2 * mi[(i + 2) % 3] ** 2 for i in range(3)]
    pref = -1.0 / (MU0 * cell_param(mat, "Ms"))
    return pref * np.stack([sum(g[i] * ax[i][c] for i in range(3)) for c in range(3)], axis=-4)


def cubic_energy_density(m, mat):
    ax = _cubic_axes(mat)
    mi = [sum(a[c] * _comp(m, c) for c in range(3)) for a in ax]
    return (mat.Kc1 * (mi[0] ** 2 * mi[1] ** 2 + mi[1] ** 2 * mi[2] ** 2 + mi[2] ** 2 * mi[0] ** 2)
            + mat.Kc2 * mi[0] ** 2 * mi[1] ** 2 * mi[2] ** 2)


def rkky_field(m, grid, mat):
    """(sigma / (mu0 Ms d_z)) m(other layer) on layers z0 and z1."""
    H = np.zeros_like(m)
    if mat.rkky == 0.0:
        return H
    z0, z1 = mat.rkky_z
    Ms = cell_param(mat, "Ms")
    pref = mat.rkky / (MU0 * Ms * grid.cell[2])
    p0 = pref[z0] if np.ndim(pref) else pref
    p1 = pref[z1] if np.ndim(pref) else pref
    H[..., z0, :, :] += p0 * m[..., z1, :, :]
    H[..., z1, :, :] += p1 * m[..., z0, :, :]
    return H


def anisotropy_field(m, mat):
    Ku = cell_param(mat, "Ku")
    if not np.any(Ku != 0.0):
        return np.zeros_like(m)
    u = np.asarray(mat.u, float)
    u = u / np.linalg.norm(u)
    mu = sum(u[c] * _comp(m, c) for c in range(3))
    pref = 2.0 * Ku / (MU0 * cell_param(mat, "Ms"))
    return pref * np.stack([u[c] * mu for c in range(3)], axis=-4)


def zeeman_field(m, mat):
    H = np.zeros_like(m)
    for c in range(3):
        H[..., c, :, :, :] = mat.B[c] / MU0
    return H


def thermal_sigma(grid, mat, dt):
    """sigma of the Brown field: a scalar, or one value per cell (nz, ny, nx)
    with per-cell alpha or Ms."""
    alpha, Ms = cell_param(mat, "alpha"), cell_param(mat, "Ms")
    if mat.T == 0.0 or not np.any(alpha != 0.0):
        return 0.0
    if np.ndim(alpha) or np.ndim(Ms):
        return np.sqrt(2.0 * alpha * KB * mat.T / (MU0 ** 2 * Ms * grid.volume * GAMMA0 * dt))
    return math.sqrt(2.0 * mat.alpha * KB * mat.T /
                     (MU0 ** 2 * mat.Ms * grid.volume * GAMMA0 * dt))


def thermal_field(grid, mat, dt, seed, step, gen=0):
    """Brown field for one replica (scalar ``seed``) or a batch (array of
    per-replica seeds -> (R, 3, nz, ny, nx)); ``gen`` is the trial generation
    (counter word 3) of the retire/refill scheme."""
    nx, ny, nz = grid.n
    seeds = np.atleast_1d(np.asarray(seed, dtype=np.uint64))
    s = thermal_sigma(grid, mat, dt)
    if np.all(np.asarray(s) == 0.0):
        out = np.zeros((seeds.size, 3, nz, ny, nx))
    else:
        out = s * _philox.gaussian_eta(seeds, grid.ncells, step, gen).reshape(seeds.size, 3, nz, ny, nx)
    return out if np.ndim(seed) else out[0]


def terms(m, grid, mat):
    """Dict of the deterministic field terms at state m."""
    out = {"exchange": exchange_field(m, grid, mat),
           "dmi": dmi_field(m, grid, mat),
           "dmi_bulk": bulk_dmi_field(m, grid, mat),
           "cubic": cubic_field(m, mat),
           "rkky": rkky_field(m, grid, mat),
           "demag": (_demag.demag_field(m, grid, cell_param(mat, "Ms")) if mat.demag
                     else np.zeros_like(m)),
           "anisotropy": anisotropy_field(m, mat),
           "zeeman": zeeman_field(m, mat)}
    return out


def effective_field(m, grid, mat, H_thermal=None):
    """H_eff = demag + exchange + DMI + anisotropy + Zeeman (+ thermal)."""
    t = terms(m, grid, mat)
    H = t["exchange"] + t["dmi"] + t["demag"] + t["anisotropy"] + t["zeeman"]
    H = H + t["dmi_bulk"] + t["cubic"] + t["rkky"]
    if H_thermal is not None:
        H = H + H_thermal
    return H
