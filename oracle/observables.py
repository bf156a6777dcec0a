"""Observables, FP64: energy per term and topological charge.

The paper reports total energies (Results, SP#1-type showcase) and classifies
skyrmions by topological charge (Results, skyrmion phase diagram) without
printing their discretisation.  Readings:

* Energy (J): E = V sum_i [ -(mu0 Ms_i / 2) m_i . (H_ex + H_dmi + H_demag + H_anis)_i
  - mu0 Ms_i m_i . H_zeeman ] (Ms_i the cell's own with per-cell materials);
  the anisotropy part equals -V sum Ku_i (m . u)^2.
  Bulk DMI and RKKY (bilinear) enter like the first group; the cubic
  anisotropy (quartic) as V sum of its energy density.
  The thermal field is excluded.
* Topological charge: Q = (1/4 pi) sum_i m_i . (d_x m x d_y m)_i dx dy with
  central differences, periodic wrap on periodic axes, and the cell itself as the
  missing neighbour at open edges; layer z = 0.
* Switching probability of a thermally activated macrospin under spin-transfer
  torque in a window t: the finite-window Neel-Brown law with Sun's barrier
  reduction as the paper states it (Results, replica-batched STT switching
  sweep), P = 1 - exp[-t f0 exp(-Delta (1 - J/J_c0)^2)], the barrier clamped
  at zero for J >= J_c0.  The paper fixes f0 and Delta from the macrospin
  parameters without printing f0; the caller passes both.
"""
from __future__ import annotations

import math

import numpy as np

from .constants import MU0
from . import fields as _fields

ENERGY_TERMS = ("exchange", "dmi", "demag", "anisotropy", "zeeman", "dmi_bulk", "cubic", "rkky")


def energies(m, grid, mat):
    """Energy per term; the quadratic terms as -(mu0 Ms V / 2) sum m . H, the
    Zeeman term as -mu0 Ms V sum m . H, the cubic anisotropy (quartic) from
    its energy density."""
    t = _fields.terms(m, grid, mat)
    V = grid.volume
    Ms = _fields.cell_param(mat, "Ms")
    out = {}
    for name in ENERGY_TERMS:
        if name == "cubic":
            out[name] = V * float(np.sum(_fields.cubic_energy_density(m, mat))) \
                if (mat.Kc1 or mat.Kc2) else 0.0
            continue
        dot = float(np.sum(Ms * np.sum(m * t[name], axis=-4)))
        if name == "zeeman":
            out[name] = -MU0 * V * dot
        else:
            out[name] = -0.5 * MU0 * V * dot
    out["total"] = sum(out[k] for k in ENERGY_TERMS)
    return out


def topological_charge(m, grid):
    m0 = m[:, 0]  # (3, ny, nx), layer z = 0
    def diff(axis_np, axis):
        if grid.pbc[axis]:
            mp = np.roll(m0, -1, axis=axis_np)
            mm = np.roll(m0, 1, axis=axis_np)
        else:
            mp = np.roll(m0, -1, axis=axis_np)
            mm = np.roll(m0, 1, axis=axis_np)
            n = m0.shape[axis_np]
            sl_last = [slice(None)] * 3
            sl_first = [slice(None)] * 3
            sl_last[axis_np] = n - 1
            sl_first[axis_np] = 0
            mp[tuple(sl_last)] = m0[tuple(sl_last)]
            mm[tuple(sl_first)] = m0[tuple(sl_first)]
        return (mp - mm) / (2.0 * grid.cell[axis])
    dxm = diff(2, 0) if grid.n[0] > 1 else np.zeros_like(m0)
    dym = diff(1, 1) if grid.n[1] > 1 else np.zeros_like(m0)
    q = np.sum(m0 * np.cross(dxm, dym, axis=0))
    return float(q * grid.cell[0] * grid.cell[1] / (4.0 * math.pi))


def switching_probability_neel_brown_sun(j, t, f0, delta):
    """P_sw(J / J_c0 = j) in a window of t seconds for attempt frequency f0
    (1/s) and thermal stability delta = K V / (kB T) (Results, replica-batched
    STT switching sweep): the Neel-Brown escape probability with the barrier
    delta (1 - j)^2, zero for j >= 1."""
    j = np.asarray(j, dtype=np.float64)
    barrier = delta * np.clip(1.0 - j, 0.0, None) ** 2
    return -np.expm1(-t * f0 * np.exp(-barrier))   # exact also for tiny probabilities
