"""Pins of the oracle's Slonczewski spin-transfer torque (Methods, "Physics and
discretization": spin torques added per integrator stage; Results, the
replica-batched STT switching sweep with per-replica current density):
the torque is perpendicular to m, the Landau-Lifshitz form equals an
independent linear solve of the Gilbert form, the antidamping rotation and
field-like precession of a free macrospin follow their closed forms, the polar
angle of an anisotropic macrospin follows an independent scalar ODE (scipy),
the instability threshold J_c0, and per-replica current densities."""
import math

import numpy as np
from scipy.integrate import solve_ivp

from oracle import GAMMA0, MU0, Grid, Material
from oracle import integrators as it
from oracle import llg, rotation
from oracle.constants import HBAR, QE
from workloads import random_unit


def _bJ(J, Ms, d):
    return HBAR * J / (MU0 * QE * Ms * d)


def test_torque_is_perpendicular_to_m():
    m = random_unit((5, 4, 1), seed=2, replicas=1)[0]
    for lam, e2 in ((1.0, 0.0), (2.0, 0.3), (0.5, -0.2)):
        mat = Material(Ms=8e5, alpha=0.1, stt_J=3e11, stt_p=(0.3, -0.2, 1.0), stt_P=0.6,
                       stt_lambda=lam, stt_eps2=e2)
        tau = llg.stt_torque(m, mat, 2e-9)
        assert np.abs(np.sum(tau * m, axis=0)).max() < 1e-12 * np.abs(tau).max()


def test_landau_lifshitz_form_equals_a_linear_solve_of_the_gilbert_form():
    """dm/dt = -gamma0 m x mu0 H + alpha m x dm/dt + gamma0 mu0 b_J [eps m x
    (m x p) - eps' m x p] solved for dm/dt per cell with numpy.linalg.solve."""
    rng = np.random.default_rng(8)
    m = random_unit((3, 2, 1), seed=4, replicas=1)[0]
    H = 1e5 * rng.standard_normal(m.shape)
    d = 1.5e-9
    for alpha in (0.0, 0.05, 0.8):
        mat = Material(Ms=6e5, alpha=alpha, stt_J=-2e11, stt_p=(0.0, 0.6, 0.8), stt_P=0.5,
                       stt_lambda=1.7, stt_eps2=0.25)
        got = llg.llg_rhs(m, H, alpha) + llg.stt_torque(m, mat, d)
        bJ = _bJ(mat.stt_J, mat.Ms, d)
        p = np.array(mat.stt_p)
        L2 = mat.stt_lambda ** 2
        for idx in np.ndindex(m.shape[1:]):
            mv, hv = m[(slice(None),) + idx], H[(slice(None),) + idx]
            eps = mat.stt_P * L2 / ((L2 + 1) + (L2 - 1) * mv @ p)
            rhs = (-GAMMA0 * MU0 * np.cross(mv, hv) +
                   GAMMA0 * MU0 * bJ * (eps * np.cross(mv, np.cross(mv, p)) -
                                         mat.stt_eps2 * np.cross(mv, p)))
            cross = np.array([[0, -mv[2], mv[1]], [mv[2], 0, -mv[0]], [-mv[1], mv[0], 0]])
            ref = np.linalg.solve(np.eye(3) - alpha * cross, rhs)
            assert np.abs(got[(slice(None),) + idx] - ref).max() < 1e-9 * np.abs(ref).max()


def _free_macrospin(J, P, e2=0.0, alpha=0.0, Ku=0.0, lam=1.0):
    grid = Grid((1, 1, 1), (10e-9, 10e-9, 2e-9))
    mat = Material(Ms=8e5, A=0.0, alpha=alpha, Ku=Ku, u=(0, 0, 1), demag=False, stt_J=J,
                   stt_p=(0, 0, 1), stt_P=P, stt_lambda=lam, stt_eps2=e2)
    return grid, mat


def test_free_macrospin_antidamping_and_field_like_closed_forms():
    """alpha = 0, Lambda = 1 (eps = P / 2), no field: the polar angle about p
    grows as tan(theta/2) = tan(theta0/2) exp(gamma0 mu0 b_J eps t) and the
    field-like term precesses m about p at gamma0 mu0 b_J eps'."""
    J, P, e2 = 1e11, 0.4, 0.3
    grid, mat = _free_macrospin(J, P, e2)
    d = grid.cell[2]
    bJ = _bJ(J, mat.Ms, d)
    th0, ph0 = 0.2, 0.5
    m0 = np.array([math.sin(th0) * math.cos(ph0), math.sin(th0) * math.sin(ph0),
                   math.cos(th0)]).reshape(3, 1, 1, 1)
    t_end = 0.3e-9
    res = it.rk45_run(m0, grid, mat, 0.0, t_end, tol=1e-11, dt0=1e-13)
    th = 2 * math.atan(math.tan(th0 / 2) * math.exp(GAMMA0 * MU0 * bJ * (P / 2) * t_end))
    ph = ph0 + GAMMA0 * MU0 * bJ * e2 * t_end
    ref = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
    assert th > th0 + 0.1  # J > 0 drives m away from p
    assert np.abs(res.m[:, 0, 0, 0] - ref).max() < 1e-7
    # the rotation scheme takes the same torque
    rot = rotation.depondt_run(m0, grid, mat, 1e-14, 30000)
    assert np.abs(rot[:, 0, 0, 0] - ref).max() < 1e-5


def _theta_ode(mat, grid, th0, t_end):
    """d theta / dt = gamma' mu0 sin(theta) [b_J (eps(theta) - alpha eps') -
    alpha H_k cos(theta)] for p = u = z, eps' = 0 (scipy, independent)."""
    gp = GAMMA0 / (1 + mat.alpha ** 2)
    bJ = _bJ(mat.stt_J, mat.Ms, grid.n[2] * grid.cell[2])
    Hk = 2 * mat.Ku / (MU0 * mat.Ms)
    L2 = mat.stt_lambda ** 2

    def f(t, y):
        th = y[0]
        eps = mat.stt_P * L2 / ((L2 + 1) + (L2 - 1) * math.cos(th))
        return [gp * MU0 * math.sin(th) * (bJ * eps - mat.alpha * Hk * math.cos(th))]
    sol = solve_ivp(f, (0, t_end), [th0], rtol=1e-12, atol=1e-14)
    return sol.y[0, -1]


def test_anisotropic_macrospin_polar_angle_follows_the_scalar_ode():
    grid, mat = _free_macrospin(4e11, 0.5, 0.0, alpha=0.05, Ku=3e5, lam=1.8)
    th0, t_end = 0.3, 0.5e-9
    m0 = np.array([math.sin(th0), 0.0, math.cos(th0)]).reshape(3, 1, 1, 1)
    res = it.rk45_run(m0, grid, mat, 0.0, t_end, tol=1e-11, dt0=1e-13)
    th = math.acos(res.m[2, 0, 0, 0])
    ref = _theta_ode(mat, grid, th0, t_end)
    assert abs(th - ref) < 1e-6


def test_instability_threshold_jc0():
    """J_c0 = alpha H_k mu0 e Ms d / (hbar eps(0)): a small tilt decays below
    and grows above it."""
    alpha, Ku, P, lam = 0.02, 3e5, 0.5, 1.0
    grid, mat0 = _free_macrospin(1.0, P, alpha=alpha, Ku=Ku, lam=lam)
    d = grid.cell[2]
    Hk = 2 * Ku / (MU0 * mat0.Ms)
    Jc0 = alpha * Hk * MU0 * QE * mat0.Ms * d / (HBAR * (P / 2))
    th0 = 0.05
    m0 = np.array([math.sin(th0), 0.0, math.cos(th0)]).reshape(3, 1, 1, 1)
    out = {}
    for f in (0.9, 1.1):
        _, mat = _free_macrospin(f * Jc0, P, alpha=alpha, Ku=Ku, lam=lam)
        res = it.rk45_run(m0, grid, mat, 0.0, 0.5e-9, tol=1e-9, dt0=1e-13)
        out[f] = math.acos(res.m[2, 0, 0, 0])
    assert out[0.9] < th0 < out[1.1]


def test_per_replica_current_density():
    m = random_unit((4, 3, 1), seed=5, replicas=3)
    Js = (0.0, 2e11, -5e11)
    mat = Material(Ms=8e5, alpha=0.1, stt_J=Js, stt_P=0.6, stt_lambda=1.3, stt_eps2=0.1)
    tau = llg.stt_torque(m, mat, 3e-9)
    for r, J in enumerate(Js):
        one = Material(Ms=8e5, alpha=0.1, stt_J=J, stt_P=0.6, stt_lambda=1.3, stt_eps2=0.1)
        assert np.array_equal(tau[r], llg.stt_torque(m[r], one, 3e-9))
    assert not np.any(tau[0])
