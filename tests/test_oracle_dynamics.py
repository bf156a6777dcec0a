"""Pins of the oracle's integrators: the Dormand-Prince tableau, convergence
orders, the damped-macrospin closed form, Kittel resonance, the exact lattice
spin-wave dispersion and damped-relaxation invariants (Methods, "Integrators";
LLG equation; Results, Kittel within 0.06%; Figure legend of the spin-wave
dispersion showcase)."""
import json
import math
import os
from fractions import Fraction as F

import numpy as np
import pytest

from oracle import GAMMA0, MU0, Grid, Material
from oracle import integrators as it
from oracle import llg, newell, observables
from workloads import random_unit

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_dopri5_tableau_order_conditions():
    c, A, b, bs = it.C, it.A, it.B5, it.B4
    for i in range(1, 7):
        assert sum(A[i]) == c[i]
    for w, order in ((b, 5), (bs, 4)):
        assert sum(w) == 1
        assert sum(w[i] * c[i] for i in range(7)) == F(1, 2)
        assert sum(w[i] * c[i] ** 2 for i in range(7)) == F(1, 3)
        assert sum(w[i] * sum(A[i][j] * c[j] for j in range(i)) for i in range(1, 7)) == F(1, 6)
        assert sum(w[i] * c[i] ** 3 for i in range(7)) == F(1, 4)
    # fifth-order-only conditions hold for b, fail for the embedded b*
    assert sum(b[i] * c[i] ** 4 for i in range(7)) == F(1, 5)
    assert sum(bs[i] * c[i] ** 4 for i in range(7)) != F(1, 5)
    assert A[6] == b[:6]  # first-same-as-last


def _macrospin(alpha, B=0.2):
    return Grid((1, 1, 1), (4e-9, 4e-9, 4e-9)), Material(Ms=8e5, alpha=alpha,
                                                          B=(0.0, 0.0, B), demag=False)


def _macrospin_exact(theta0, phi0, alpha, B, t):
    gp = GAMMA0 / (1 + alpha ** 2)
    th = 2 * np.arctan(np.tan(theta0 / 2) * np.exp(-gp * alpha * B * t))
    ph = phi0 + gp * B * t
    return np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])


def test_damped_macrospin_closed_form_rk45():
    alpha, B = 0.1, 0.2
    grid, mat = _macrospin(alpha, B)
    th0, ph0 = 2.5, 0.3
    m0 = _macrospin_exact(th0, ph0, alpha, B, 0.0).reshape(3, 1, 1, 1)
    t_end = 0.4e-9
    res = it.rk45_run(m0, grid, mat, 0.0, t_end, tol=1e-10, dt0=1e-13)
    ref = _macrospin_exact(th0, ph0, alpha, B, t_end)
    assert res.t == t_end
    assert np.abs(res.m[:, 0, 0, 0] - ref).max() < 2e-8


def test_dopri5_fixed_step_is_fifth_order():
    alpha, B = 0.1, 0.2
    grid, mat = _macrospin(alpha, B)
    f = lambda m: it.rhs(m, grid, mat)
    th0, ph0 = 1.0, 0.0
    m0 = _macrospin_exact(th0, ph0, alpha, B, 0.0).reshape(3, 1, 1, 1)
    T = 2e-10
    errs = []
    for n in (20, 40, 80):
        m = it.dopri5_fixed(m0, f, T / n, n)
        errs.append(np.abs(m[:, 0, 0, 0] - _macrospin_exact(th0, ph0, alpha, B, T)).max())
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(slopes) > 4.6


def test_heun_is_second_order_at_zero_temperature():
    alpha, B = 0.1, 0.2
    grid, mat = _macrospin(alpha, B)
    th0, ph0 = 1.0, 0.0
    m0 = _macrospin_exact(th0, ph0, alpha, B, 0.0).reshape(3, 1, 1, 1)
    T = 2e-10
    errs = []
    for n in (200, 400, 800):
        m = it.heun_run(m0, grid, mat, T / n, n)
        errs.append(np.abs(m[:, 0, 0, 0] - _macrospin_exact(th0, ph0, alpha, B, T)).max())
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert 1.8 < min(slopes) and max(slopes) < 2.3


def _zero_crossing_frequency(ts, xs):
    s = np.sign(xs)
    idx = np.where(s[:-1] < s[1:])[0]  # upward crossings
    tc = [ts[i] - xs[i] * (ts[i + 1] - ts[i]) / (xs[i + 1] - xs[i]) for i in idx]
    return (len(tc) - 1) / (tc[-1] - tc[0])


def test_kittel_resonance_single_cell():
    """Small-angle precession of one cuboid cell (uniaxial Ku along z, B along z,
    demag self-term on, alpha = 0): f = (gamma0/2pi) sqrt[(B + 2Ku/Ms +
    (Nx - Nz) mu0 Ms)(B + 2Ku/Ms + (Ny - Nz) mu0 Ms)] (Kittel 1948).  The paper
    reports agreement within 0.06%."""
    cell = (4e-9, 3e-9, 2e-9)
    Ms, Ku, B = 8e5, 6e5, 0.1
    grid = Grid((1, 1, 1), cell)
    mat = Material(Ms=Ms, alpha=0.0, Ku=Ku, B=(0, 0, B))
    N = newell.tensor_exact(0.0, 0.0, 0.0, *cell)
    bx = B + 2 * Ku / Ms + (N[0] - N[2]) * MU0 * Ms
    by = B + 2 * Ku / Ms + (N[1] - N[2]) * MU0 * Ms
    f_ref = GAMMA0 / (2 * math.pi) * math.sqrt(bx * by)
    th = 1e-3
    m = np.array([math.sin(th), 0.0, math.cos(th)]).reshape(3, 1, 1, 1)
    dt = 1.0 / f_ref / 400
    f = lambda mm: it.rhs(mm, grid, mat)
    ts, xs = [], []
    for k in range(4000):
        ts.append(k * dt)
        xs.append(m[0, 0, 0, 0])
        m = it.dopri5_fixed(m, f, dt, 1)
    f_num = _zero_crossing_frequency(np.array(ts), np.array(xs))
    assert abs(f_num / f_ref - 1) < 1e-5
    with open(os.path.join(GOLDEN, "paper_values.json")) as fh:
        paper = json.load(fh)
    assert abs(f_num / f_ref - 1) < paper["kittel_macrospin_rel_agreement"]["value"]


def test_exact_lattice_spin_wave_dispersion():
    """Circular spin wave on a periodic chain, alpha = 0, demag off: exact
    solution precesses at omega = gamma0 [B0 + (2A/Ms)(4/dx^2) sin^2(k dx/2) cos th];
    th -> 0 gives the paper's lattice dispersion (showcase figure legend:
    200x1x1 chain, dx = 20 nm, B0 = 0.1 T)."""
    with open(os.path.join(GOLDEN, "paper_values.json")) as fh:
        g = json.load(fh)["spin_wave_chain"]
    N, dx, B0 = g["n"], g["dx"], g["B0"]
    grid = Grid((N, 1, 1), (dx, dx, dx), pbc=(1, 0, 0))
    mat = Material(Ms=8e5, A=1.3e-11, alpha=0.0, B=(0, 0, B0), demag=False)
    x = np.arange(N) * dx
    for nk, th in ((5, 0.3), (37, 0.3), (80, 0.05)):
        k = 2 * math.pi * nk / (N * dx)
        m0 = np.zeros((3, 1, 1, N))
        m0[0, 0, 0] = math.sin(th) * np.cos(k * x)
        m0[1, 0, 0] = math.sin(th) * np.sin(k * x)
        m0[2, 0, 0] = math.cos(th)
        w = GAMMA0 * (B0 + 2 * mat.A / mat.Ms * 4 / dx ** 2 * math.sin(k * dx / 2) ** 2 * math.cos(th))
        t_end = 3 * 2 * math.pi / w
        res = it.rk45_run(m0, grid, mat, 0.0, t_end, tol=1e-11, dt0=1e-13)
        ref = np.stack([math.sin(th) * np.cos(k * x + w * t_end),
                        math.sin(th) * np.sin(k * x + w * t_end),
                        np.full(N, math.cos(th))])
        assert np.abs(res.m[:, 0, 0] - ref).max() < 1e-7
        # small-amplitude limit is the paper's lattice formula
        f_paper = GAMMA0 / (2 * math.pi) * (B0 + 2 * mat.A / mat.Ms * 4 / dx ** 2 * math.sin(k * dx / 2) ** 2)
        assert abs(w / (2 * math.pi) / f_paper - 1) < 1 - math.cos(th) + 1e-15


def test_relaxation_keeps_unit_norm_and_energy_decreases():
    grid = Grid((8, 8, 1), (4e-9, 4e-9, 4e-9))
    mat = Material(Ms=8e5, A=1.3e-11, alpha=0.5)
    m0 = random_unit(grid.n, seed=1)
    res = it.rk45_run(m0, grid, mat, 0.0, 3e-11, tol=1e-6, dt0=1e-14, energy=True)
    assert np.abs(np.linalg.norm(res.m, axis=0) - 1).max() < 1e-14
    E = np.array(res.energy)
    assert np.all(np.diff(E) <= 1e-12 * np.abs(E).max())
    assert res.accepted > 5


def test_controller_rejects_and_recovers():
    grid = Grid((4, 4, 1), (4e-9, 4e-9, 4e-9))
    mat = Material(Ms=8e5, A=1.3e-11, alpha=0.5)
    m0 = random_unit(grid.n, seed=2)
    res = it.rk45_run(m0, grid, mat, 0.0, 1e-12, tol=1e-6, dt0=1e-12)
    assert res.rejected >= 1 and res.t == 1e-12
    assert it.controller(1e-13, float("nan"), 1e-6) == (pytest.approx(2e-14), False)
    assert it.controller(1e-13, 0.0, 1e-6) == (pytest.approx(5e-13), True)


def test_uniform_state_energy_closed_form():
    """m = +z, uniaxial Ku along z, Bz: E = V N (-Ku - Ms Bz) +
    (mu0/2) Ms^2 V N N_zz(prism) (whole-body identity)."""
    grid = Grid((8, 6, 2), (4e-9, 4e-9, 4e-9))
    mat = Material(Ms=8e5, A=1.3e-11, Ku=5e5, B=(0, 0, -0.15))
    m = np.zeros((3, 2, 6, 8)); m[2] = 1.0
    e = observables.energies(m, grid, mat)
    Nz = newell.tensor_exact(0.0, 0.0, 0.0, 32e-9, 24e-9, 8e-9)[2]
    V, N = grid.volume, grid.ncells
    ref = V * N * (-mat.Ku - mat.Ms * mat.B[2]) + 0.5 * MU0 * mat.Ms ** 2 * V * N * Nz
    assert e["total"] == pytest.approx(ref, rel=1e-12)
    assert abs(e["exchange"]) < 1e-30
