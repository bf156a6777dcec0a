"""Time integrators, FP64 (Methods, "Integrators"; Results, "A replica-batched
engine").

* Stratonovich Heun for the stochastic LLG (the paper's finite-temperature
  single-trajectory scheme): the thermal field is drawn once per step and used
  by both the predictor and the corrector; the predictor is not normalised; the
  corrector is normalised once (reading; the paper gives no further detail).
* Adaptive Dormand-Prince 5(4) with first-same-as-last (Dormand & Prince 1980,
  the paper's RK45).  The paper prints neither the tableau nor a step-size
  controller.  Readings:
    - error = max over cells of the Euclidean norm of dt sum_j (b_j - b*_j) k_j
      (absolute, since |m| = 1);
    - accept iff error <= tol; dt <- dt * clamp(0.9 (tol/err)^(1/5), 0.2, 5)
      (x5 when err = 0, x0.2 and reject when err is not finite);
      dt limited to dt_max and to the time left; dt < dt_min is an error;
    - the 5th-order candidate is normalised *before* the seventh stage is
      evaluated, so the FSAL derivative belongs to the accepted state.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from dataclasses import replace as dataclass_replace
from fractions import Fraction as F

import numpy as np

from . import fields as _fields
from .llg import llg_rhs, normalise, stt_torque
from . import observables as _obs

# Dormand-Prince 5(4) tableau (Dormand & Prince 1980).
C = [F(0), F(1, 5), F(3, 10), F(4, 5), F(8, 9), F(1), F(1)]
A = [
    [],
    [F(1, 5)],
    [F(3, 40), F(9, 40)],
    [F(44, 45), F(-56, 15), F(32, 9)],
    [F(19372, 6561), F(-25360, 2187), F(64448, 6561), F(-212, 729)],
    [F(9017, 3168), F(-355, 33), F(46732, 5247), F(49, 176), F(-5103, 18656)],
    [F(35, 384), F(0), F(500, 1113), F(125, 192), F(-2187, 6784), F(11, 84)],
]
B5 = A[6] + [F(0)]
B4 = [F(5179, 57600), F(0), F(7571, 16695), F(393, 640), F(-92097, 339200),
      F(187, 2100), F(1, 40)]
E = [b - bs for b, bs in zip(B5, B4)]

DT_MAX = 1e-11
DT_MIN = 1e-20


def rhs(m, grid, mat, H_th=None):
    """LLG right-hand side at m, with the spin-transfer torque when set."""
    k = llg_rhs(m, _fields.effective_field(m, grid, mat, H_th), _fields.cell_param(mat, "alpha"),
                mat.precess)
    if mat.stt:
        k = k + stt_torque(m, mat, grid.n[2] * grid.cell[2])
    return k


# ----------------------------------------------------------------------------
# Heun
# ----------------------------------------------------------------------------
def heun_step(m, grid, mat, dt, seed=0, step=0):
    """One Stratonovich Heun step of one replica (3, nz, ny, nx) with scalar
    ``seed``, or of a batch (R, 3, nz, ny, nx) with per-replica seeds."""
    H_th = _fields.thermal_field(grid, mat, dt, seed, step) if mat.T > 0 else None
    k1 = rhs(m, grid, mat, H_th)
    mp = m + dt * k1
    k2 = rhs(mp, grid, mat, H_th)
    return normalise(m + 0.5 * dt * (k1 + k2))


def heun_run(m0, grid, mat, dt, nsteps, seed=0, step0=0, t_switch=None):
    """Advance one replica by ``nsteps`` Heun steps (absolute step indices
    step0 .. step0+nsteps-1); ``m0`` may be a batch with per-replica seeds.
    If ``t_switch`` is a list (one entry per replica, negative = not yet) it
    records the first time (step+1)*dt at which the replica's mean m_z becomes
    negative (reading of the switching criterion; replicas keep running)."""
    m = m0.copy()
    for k in range(nsteps):
        s = step0 + k
        m = heun_step(m, grid, mat, dt, seed, s)
        if t_switch is not None:
            mz = m[..., 2, :, :, :].reshape(-1, grid.ncells).mean(axis=1)
            for r in range(mz.size):
                if t_switch[r] < 0 and mz[r] < 0:
                    t_switch[r] = (s + 1) * dt
    return m


# ----------------------------------------------------------------------------
# Dormand-Prince 5(4)
# ----------------------------------------------------------------------------
def dopri5_attempt(m, k1, grid, mat, dt, stage_rhs=None):
    """One DOPRI5 attempt from (m, k1 = f(m)).  Returns (m7, k7, err) where m7 is
    the normalised 5th-order candidate and k7 = f(m7).  ``stage_rhs(ms)``, if
    given, replaces f for stages 2-6 (the seventh stage is always f)."""
    f_stage = stage_rhs if stage_rhs is not None else (lambda ms: rhs(ms, grid, mat))
    ks = [k1]
    for s in range(1, 6):
        ms = m.copy()
        for j in range(s):
            if A[s][j] != 0:
                ms = ms + dt * float(A[s][j]) * ks[j]
        ks.append(f_stage(ms))
    y5 = m.copy()
    for j in range(6):
        if B5[j] != 0:
            y5 = y5 + dt * float(B5[j]) * ks[j]
    m7 = normalise(y5)
    k7 = rhs(m7, grid, mat)
    ks.append(k7)
    d = np.zeros_like(m)
    for j in range(7):
        if E[j] != 0:
            d = d + dt * float(E[j]) * ks[j]
    err = float(np.max(np.linalg.norm(d, axis=-4)))
    return m7, k7, err


def controller(dt, err, tol):
    """New step size and acceptance (reading stated in the module docstring)."""
    if not np.isfinite(err):
        return dt * 0.2, False
    accept = err <= tol
    if err == 0.0:
        fac = 5.0
    else:
        fac = min(5.0, max(0.2, 0.9 * (tol / err) ** 0.2))
    return dt * fac, accept


@dataclass
class RKResult:
    m: np.ndarray
    t: float
    dt: float
    dt_next: float = 0.0  # the controller's last proposal before clipping to t_end
    accepted: int = 0
    rejected: int = 0
    dts: list = field(default_factory=list)
    energy: list = field(default_factory=list)


def rk45_run(m0, grid, mat, t0, t_end, tol, dt0=1e-14, dt_replay=None,
             energy=False, max_steps=10_000_000):
    """Adaptive DOPRI5 relaxation from t0 to t_end.  With ``dt_replay`` the
    given accepted step sizes are taken in order, without control."""
    m = m0.copy()
    k1 = rhs(m, grid, mat)
    t = t0
    res = RKResult(m, t, dt0)
    if energy:
        res.energy.append(_obs.energies(m, grid, mat)["total"])
    if dt_replay is not None:
        for h in dt_replay:
            m, k1, _ = dopri5_attempt(m, k1, grid, mat, float(h))
            t += float(h)
            res.accepted += 1
            res.dts.append(float(h))
            if energy:
                res.energy.append(_obs.energies(m, grid, mat)["total"])
        res.m, res.t = m, t
        return res
    dt = min(dt0, DT_MAX)
    final = t + dt >= t_end
    if final:
        dt = t_end - t
    steps = 0
    while t < t_end and steps < max_steps:
        steps += 1
        m7, k7, err = dopri5_attempt(m, k1, grid, mat, dt)
        new_dt, ok = controller(dt, err, tol)
        if ok:
            m, k1 = m7, k7
            t = t_end if final else t + dt
            res.accepted += 1
            res.dts.append(dt)
            if energy:
                res.energy.append(_obs.energies(m, grid, mat)["total"])
        else:
            res.rejected += 1
        # the step that reaches t_end exactly is clipped and marked final
        dt = min(new_dt, DT_MAX)
        res.dt_next = dt
        final = t + dt >= t_end
        if final:
            dt = t_end - t
        if t < t_end and dt < DT_MIN:
            raise FloatingPointError("step size underflow")
    res.m, res.t, res.dt = m, t, dt
    return res


# ----------------------------------------------------------------------------
# Classical fourth-order Runge-Kutta, fixed step (Methods, "Integrators": RK4)
# ----------------------------------------------------------------------------
def rk4_run(m0, grid, mat, dt, nsteps):
    """``nsteps`` classical RK4 steps: k1 = f(m), k2 = f(m + dt/2 k1),
    k3 = f(m + dt/2 k2), k4 = f(m + dt k3), m <- m + dt/6 (k1 + 2 k2 + 2 k3 +
    k4), normalised at the end of each step (reading, as for the corrector of
    Heun and the accepted RK45 state; the stage states are not normalised)."""
    m = m0.copy()
    for _ in range(nsteps):
        k1 = rhs(m, grid, mat)
        k2 = rhs(m + 0.5 * dt * k1, grid, mat)
        k3 = rhs(m + 0.5 * dt * k2, grid, mat)
        k4 = rhs(m + dt * k3, grid, mat)
        m = normalise(m + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4))
    return m


# ----------------------------------------------------------------------------
# Damping-only relaxation (Methods, "Integrators": damping-only relax)
# ----------------------------------------------------------------------------
RELAX_CHUNK = 1e-11  # simulated time between convergence checks (s)


def max_torque(m, grid, mat):
    """max over cells (and replicas) of |dm/dt| of the damping-only dynamics."""
    k = rhs(m, grid, dataclass_replace(mat, precess=False))
    return float(np.sqrt(np.sum(k * k, axis=-4)).max())


def relax_run(m0, grid, mat, torque_tol, t_max, tol, dt0=1e-14):
    """Reading of the damping-only relaxer: the precession term is dropped
    and the adaptive DOPRI5 above integrates in chunks of RELAX_CHUNK of
    simulated time (each chunk starts with the controller's last proposal of
    the previous chunk, before its clipping to the chunk's end) until the max-over-cells |dm/dt| after a chunk is <= torque_tol or
    t_max is reached.  Returns (m, t, accepted, rejected, max |dm/dt|)."""
    md = dataclass_replace(mat, precess=False)
    m, t, dt = m0.copy(), 0.0, dt0
    acc = rej = 0
    tq = max_torque(m, grid, md)
    while tq > torque_tol and t < t_max:
        t1 = min(t + RELAX_CHUNK, t_max)
        res = rk45_run(m, grid, md, t, t1, tol, dt)
        m, t, dt = res.m, res.t, res.dt_next
        acc += res.accepted
        rej += res.rejected
        tq = max_torque(m, grid, md)
    return m, t, acc, rej, tq


def dopri5_fixed(m0, f, dt, nsteps):
    """Fixed-step DOPRI5 (5th-order solution, no normalisation) for a generic
    right-hand side f; used for order tests."""
    m = m0.copy()
    for _ in range(nsteps):
        ks = [f(m)]
        for s in range(1, 6):
            ms = m.copy()
            for j in range(s):
                if A[s][j] != 0:
                    ms = ms + dt * float(A[s][j]) * ks[j]
            ks.append(f(ms))
        for j in range(6):
            if B5[j] != 0:
                m = m + dt * float(B5[j]) * ks[j]
    return m
