"""Landau-Lifshitz-Gilbert right-hand side, FP64 (Methods, "Physics and
discretization", the LLG equation):

    dm/dt = -gamma' mu0 (m x H) - gamma' alpha mu0 m x (m x H),
    gamma' = gamma0 / (1 + alpha^2).
"""
from __future__ import annotations

import numpy as np

from .constants import GAMMA0, HBAR, MU0, QE


def llg_rhs(m, H, alpha, precess=True):
    """Torque for arrays with the vector component on axis 0 (single replica)
    or axis 1 (batch: leading replica axis).  ``precess=False`` drops the
    precession term: -gamma' mu0 alpha m x (m x H), the damping-only dynamics
    of the relaxer (Methods, "Integrators": damping-only relax; reading: the
    same gamma' = gamma0 / (1 + alpha^2))."""
    gp = GAMMA0 / (1.0 + alpha * alpha)
    mxH = np.cross(m, H, axis=-4)
    mxmxH = np.cross(m, mxH, axis=-4)
    if not precess:
        return -gp * MU0 * alpha * mxmxH
    return -gp * MU0 * (mxH + alpha * mxmxH)


def normalise(m):
    return m / np.linalg.norm(m, axis=-4, keepdims=True)


def stt_torque(m, mat, thickness):
    """Slonczewski spin-transfer torque added to dm/dt (Methods, "Physics and
    discretization": spin torques are added per integrator stage; Slonczewski
    1996).  The paper does not print the form; reading: the Slonczewski
    torque with Xiao's asymmetry added to the Gilbert form of the LLG
    equation as gamma0 mu0 b_J [eps m x (m x p) - eps' m x p], which in the
    Landau-Lifshitz form used here (multiply by 1 / (1 + alpha^2) after adding
    alpha m x itself) reads

        tau = gamma' mu0 b_J [(eps - alpha eps') m x (m x p)
                              - (eps' + alpha eps) m x p],
        b_J = hbar J / (mu0 e Ms d),
        eps = P Lambda^2 / ((Lambda^2 + 1) + (Lambda^2 - 1) m . p),

    with d the free-layer thickness (the grid's extent along z), p the fixed
    layer's unit magnetisation and J the current density: J > 0 drives m away
    from p; eps' acts as a field b_J eps' along p.  ``mat.stt_J`` may hold one
    value per replica of a batch; per-cell alpha and Ms enter cell by cell."""
    from .fields import cell_param
    alpha = cell_param(mat, "alpha")
    gp = GAMMA0 / (1.0 + alpha * alpha)
    batch = m.ndim == 5
    p = np.asarray(mat.stt_p, dtype=np.float64)
    p = p / np.linalg.norm(p)
    shape = (1,) * (m.ndim - 4) + (3, 1, 1, 1)
    pv = np.broadcast_to(p.reshape(shape), m.shape)
    J = np.asarray(mat.stt_J, dtype=np.float64)
    if batch:
        J = np.broadcast_to(J.reshape(-1), (m.shape[0],)).reshape(-1, 1, 1, 1, 1)
    bJ = HBAR * J / (MU0 * QE * cell_param(mat, "Ms") * thickness)
    L2 = mat.stt_lambda ** 2
    mp = np.sum(m * pv, axis=-4, keepdims=True)
    eps = mat.stt_P * L2 / ((L2 + 1.0) + (L2 - 1.0) * mp)
    e2 = mat.stt_eps2
    mxp = np.cross(m, pv, axis=-4)
    mxmxp = np.cross(m, mxp, axis=-4)
    return gp * MU0 * bJ * ((eps - alpha * e2) * mxmxp - (e2 + alpha * eps) * mxp)
