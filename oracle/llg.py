"""Landau-Lifshitz-Gilbert right-hand side, FP64 (Methods, "Physics and
discretization", the LLG equation):

    dm/dt = -gamma' mu0 (m x H) - gamma' alpha mu0 m x (m x H),
    gamma' = gamma0 / (1 + alpha^2).
"""
from __future__ import annotations

import numpy as np

from .constants import GAMMA0, MU0


def llg_rhs(m, H, alpha):
    """Torque for arrays with the vector component on axis 0 (single replica)
    or axis 1 (batch: leading replica axis)."""
    gp = GAMMA0 / (1.0 + alpha * alpha)
    mxH = np.cross(m, H, axis=-4)
    mxmxH = np.cross(m, mxH, axis=-4)
    return -gp * MU0 * (mxH + alpha * mxmxH)


def normalise(m):
    return m / np.linalg.norm(m, axis=-4, keepdims=True)
