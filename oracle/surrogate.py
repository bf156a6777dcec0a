"""RK45 stages with a learned demagnetising field, and the gate that checks it
(FP64).

TEST INFRASTRUCTURE ONLY (see the package header).

This is an extension of the method, not part of the paper: the intermediate
stages 2-6 of the paper's adaptive Dormand-Prince step (Methods,
"Integrators") take the demag field from the Fourier neural operator of
``oracle.fno`` instead of the FFT convolution (Methods, "Physics and
discretization"); the seventh stage, at the candidate point, stays exact.
Readings:
  - the network predicts h = H_demag / Ms, optionally as a residual on the
    local thin-film part: H_demag ~ Ms h - (0, 0, Ms m_z);
  - gate: per replica, |H_net - H_exact|_2 / |H_exact|_2 over the film at the
    candidate state, compared with the threshold (1e-3);
  - a step whose gate fails, and a network attempt the controller rejects, is
    repeated from the same state and step size with exact fields; after a gate
    failure the next ten accepted steps are exact.
Pins: with the exact field in place of the network the attempt is the plain
DOPRI5 attempt and the gate error is zero (tests/test_oracle_surrogate.py).
The behaviour with trained weights is parity unpinned (no published values).
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np

from . import demag as _demag
from . import fields as _fields
from . import fno as _fno
from .integrators import dopri5_attempt
from .llg import llg_rhs


def network_demag(params, m, Ms, M1, M2, residual_mz=True):
    """Demag field of a film batch m (R, 3, 1, ny, nx) from the network."""
    h = _fno.forward(params, m[:, :, 0], M1, M2)
    H = Ms * h[:, :, None]
    if residual_mz:
        H[:, 2] -= Ms * m[:, 2]
    return H


def stage_rhs_with(grid, mat, demag_fn):
    """LLG right-hand side whose demag term is ``demag_fn(m)``."""
    mat_local = replace(mat, demag=False)

    def f(ms):
        H = _fields.effective_field(ms, grid, mat_local) + demag_fn(ms)
        return llg_rhs(ms, H, mat.alpha)
    return f


def attempt(m, k1, grid, mat, dt, demag_fn):
    """One DOPRI5 attempt whose stages 2-6 use ``demag_fn``; returns
    (m7, k7, err) as ``dopri5_attempt``."""
    return dopri5_attempt(m, k1, grid, mat, dt, stage_rhs=stage_rhs_with(grid, mat, demag_fn))


def gate_error(H_net, H_exact):
    """Per-replica relative L2 error over the film; arrays (R, 3, ...)."""
    R = H_net.shape[0]
    num = np.sqrt(np.sum((H_net - H_exact).reshape(R, -1) ** 2, axis=1))
    den = np.sqrt(np.sum(H_exact.reshape(R, -1) ** 2, axis=1))
    return num / den


def exact_demag(m, grid, Ms):
    return _demag.demag_field(m, grid, Ms)
