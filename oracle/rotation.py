"""Norm-exact rotation integrator and retire/refill trials, FP64 (Results,
"A replica-batched engine for finite-temperature ensembles"; Methods,
"Integrators" and "Replica batching").  Test infrastructure: imported only by
the tests, the smoke check and the CPU leg of the benchmark.

The paper names the scheme (Depondt & Mertens 2009, a Rodrigues update that
keeps |m| = 1 to round-off) without writing it out.  Readings:

* The LLG equation is written as a rotation, dm/dt = Omega x m with
  Omega = gamma' mu0 (H + alpha m x H): expanding Omega x m gives back
  -gamma' mu0 [m x H + alpha m x (m x H)].
* One step is a predictor-corrector pair of rotations (the published scheme):
  Omega_1 from (m, H(m)); predictor m~ = rotation of m about Omega_1 by the
  angle |Omega_1| dt; Omega_2 from (m~, H(m~)); the new state is the rotation
  of m about (Omega_1 + Omega_2) / 2 by the angle |Omega_1 + Omega_2| dt / 2.
  No normalisation: a rotation preserves the norm.
* The Brown field is drawn once per step and used in both evaluations
  (Stratonovich, as for Heun).
* A spin-transfer torque tau (perpendicular to m) enters as m x tau added to
  Omega, since (m x tau) x m = tau.
* Rodrigues' formula for the rotation of v about the vector w by |w|:
  v cos|w| + (w x v) sin|w| / |w| + w (w . v) (1 - cos|w|) / |w|^2.
* Retire/refill (reading): slot r runs trials g = 0, 1, ...; trial g starts
  from the slot's initial state with the noise counter's fourth word set to g
  and its own step count s = 0, 1, ... (the noise of trial 0 is that of a plain
  run); it ends after the first step after which the slot's mean m_z is
  negative, recording (s + 1) dt, and the slot restarts at once from its
  initial state with trial g + 1.  At most ``cap`` times are recorded per slot;
  later trials still run, unrecorded.
"""
from __future__ import annotations

import numpy as np

from . import fields as _fields
from .constants import GAMMA0, MU0
from .llg import stt_torque


def omega(m, H, alpha):
    """Precession vector gamma' mu0 (H + alpha m x H) (vector axis -4)."""
    gp = GAMMA0 / (1.0 + alpha * alpha)
    return gp * MU0 * (H + alpha * np.cross(m, H, axis=-4))


def rotate(v, w):
    """Rodrigues rotation of v about w by the angle |w| (vector axis -4)."""
    th = np.sqrt(np.sum(w * w, axis=-4, keepdims=True))
    safe = np.where(th > 0, th, 1.0)
    s1 = np.where(th > 0, np.sin(th) / safe, 1.0)                 # sin|w| / |w|
    s2 = np.where(th > 0, (1.0 - np.cos(th)) / safe ** 2, 0.5)    # (1 - cos|w|) / |w|^2
    wv = np.sum(w * v, axis=-4, keepdims=True)
    return np.cos(th) * v + s1 * np.cross(w, v, axis=-4) + s2 * wv * w


def _omega_total(m, grid, mat, H_th):
    """Omega of the LLG equation plus, with a spin-transfer torque tau (which
    is perpendicular to m), m x tau: (m x tau) x m = tau."""
    o = omega(m, _fields.effective_field(m, grid, mat, H_th), _fields.cell_param(mat, "alpha"))
    if mat.stt:
        o = o + np.cross(m, stt_torque(m, mat, grid.n[2] * grid.cell[2]), axis=-4)
    return o


def depondt_step(m, grid, mat, dt, seed=0, step=0, gen=0):
    """One rotation step of one replica (3, nz, ny, nx) or of a batch (R, 3, nz,
    ny, nx) with per-replica seeds."""
    H_th = _fields.thermal_field(grid, mat, dt, seed, step, gen) if mat.T > 0 else None
    o1 = _omega_total(m, grid, mat, H_th)
    mp = rotate(m, dt * o1)
    o2 = _omega_total(mp, grid, mat, H_th)
    return rotate(m, 0.5 * dt * (o1 + o2))


def _mean_mz(m, grid):
    return m[..., 2, :, :, :].reshape(-1, grid.ncells).mean(axis=1)


def depondt_run(m0, grid, mat, dt, nsteps, seed=0, step0=0, t_switch=None):
    """``nsteps`` rotation steps (absolute step indices step0 ...); the
    switching-time bookkeeping is that of the Heun runner."""
    m = m0.copy()
    for k in range(nsteps):
        s = step0 + k
        m = depondt_step(m, grid, mat, dt, seed, s)
        if t_switch is not None:
            mz = _mean_mz(m, grid)
            for r in range(mz.size):
                if t_switch[r] < 0 and mz[r] < 0:
                    t_switch[r] = (s + 1) * dt
    return m


def refill_slot(m_init, grid, mat, dt, nsteps, seed, cap):
    """Retire/refill trials of one slot over ``nsteps`` steps from its initial
    state ``m_init`` (3, nz, ny, nx).  Returns (recorded switching times,
    number of finished trials, final state, generation and step count of the
    trial running at the end, and the mean m_z after each finished trial's
    last step, for checks of how close a decision was)."""
    times, margins = [], []
    g, s = 0, 0
    m = m_init.copy()
    for _ in range(nsteps):
        m = depondt_step(m, grid, mat, dt, seed, s, g)
        s += 1
        mz = float(_mean_mz(m, grid)[0])
        if mz < 0:
            if len(times) < cap:
                times.append(s * dt)
            margins.append(mz)
            g += 1
            s = 0
            m = m_init.copy()
    return times, g, m, g, s, margins
