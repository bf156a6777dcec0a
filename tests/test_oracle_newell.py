"""Pins of the oracle's Newell tensor against closed forms, identities and
high-precision evaluation (Methods, "Physics and discretization": demag by
convolution with the Newell tensor; Newell, Williams & Dunlop 1993)."""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import newell as nw

CUBE = (1.0, 1.0, 1.0)
FILM = (2e-9, 2e-9, 0.6e-9)


def test_cube_self_term_is_one_third():
    t = nw.tensor_at_offsets(np.array([[0, 0, 0]]), CUBE)[:, 0]
    assert np.allclose(t[:3], 1.0 / 3.0, rtol=0, atol=1e-15)
    assert np.allclose(t[3:], 0.0, atol=1e-15)


@pytest.mark.parametrize("cell", [FILM, (1.0, 2.0, 3.0), (4e-9, 4e-9, 4e-9), (5.0, 1.0, 0.2)])
def test_self_trace_is_one(cell):
    t = nw.tensor_at_offsets(np.array([[0, 0, 0]]), cell)[:, 0]
    assert abs(t[:3].sum() - 1.0) < 1e-14
    assert np.all(t[:3] > 0)


def test_offsite_trace_vanishes_both_zones():
    # Laplace: the dipole kernel is traceless away from the source
    offs = np.array([[1, 0, 0], [1, 1, 0], [2, 1, 1], [3, 0, 0], [4, 2, 1],
                     [7, 3, 0], [15, 2, 1], [60, 1, 0], [250, 0, 0]])
    for cell in (CUBE, FILM):
        t = nw.tensor_at_offsets(offs, cell)
        scale = np.abs(t[:3]).max(axis=0)
        assert np.all(np.abs(t[:3].sum(axis=0)) <= 1e-12 * scale + 1e-300)


def test_far_field_tends_to_point_dipole():
    cell = (1.0, 1.2, 0.8)
    V = cell[0] * cell[1] * cell[2]
    prev = None
    for k in (1, 2, 4, 8):
        o = np.array([[20 * k, 7 * k, 3 * k]])
        t = nw.tensor_at_offsets(o, cell)[:, 0]
        R = o[0] * np.array(cell)
        r = np.linalg.norm(R)
        G = V * (np.eye(3) * r * r - 3 * np.outer(R, R)) / (4 * math.pi * r ** 5)
        ref = np.array([G[0, 0], G[1, 1], G[2, 2], G[0, 1], G[0, 2], G[1, 2]])
        rel = np.abs(t - ref).max() / np.abs(ref).max()
        assert rel < 2e-3
        if prev is not None:  # correction shrinks like (cell / r)^2
            assert rel < prev / 3.0
        prev = rel


def test_closed_form_agrees_with_dipole_quadrature_all_components():
    # the quadrature integrates the point-dipole kernel directly; agreement pins
    # f, g and the coordinate/cell permutations of every component
    for cell in (CUBE, FILM, (1.0, 1.7, 0.6)):
        for o in ([3, 0, 0], [3, 2, 1], [2, 3, 2], [3, 3, 3], [1, 2, 3], [2, 2, 3]):
            X = np.array(o) * np.array(cell)
            ex = nw.tensor_exact(*X, *cell)
            q = nw.tensor_quadrature(X[0], X[1], X[2], *cell, 24)[:, 0]
            assert np.abs(ex - q).max() <= 5e-11 * np.abs(ex).max(), (cell, o)


def _mp_f(x, y, z):
    R = mp.sqrt(x * x + y * y + z * z)
    t = mp.mpf(0)
    if y != 0 and (x * x + z * z) != 0:
        t += y / 2 * (z * z - x * x) * mp.asinh(y / mp.sqrt(x * x + z * z))
    if z != 0 and (x * x + y * y) != 0:
        t += z / 2 * (y * y - x * x) * mp.asinh(z / mp.sqrt(x * x + y * y))
    if x != 0:
        t -= x * y * z * mp.atan(y * z / (x * R))
    return t + (2 * x * x - y * y - z * z) * R / 6


def _mp_g(x, y, z):
    R = mp.sqrt(x * x + y * y + z * z)
    t = mp.mpf(0)
    if z != 0 and (x * x + y * y) != 0:
        t += x * y * z * mp.asinh(z / mp.sqrt(x * x + y * y))
    if x != 0 and (y * y + z * z) != 0:
        t += y / 6 * (3 * z * z - y * y) * mp.asinh(x / mp.sqrt(y * y + z * z))
    if y != 0 and (x * x + z * z) != 0:
        t += x / 6 * (3 * z * z - x * x) * mp.asinh(y / mp.sqrt(x * x + z * z))
    if z != 0:
        t -= z ** 3 / 6 * mp.atan(x * y / (z * R))
    if y != 0:
        t -= z * y * y / 2 * mp.atan(x * z / (y * R))
    if x != 0:
        t -= z * x * x / 2 * mp.atan(y * z / (x * R))
    return t - x * y * R / 3


def _mp_second_diff(fun, X, Y, Z, dx, dy, dz):
    acc = mp.mpf(0)
    for ex in (-1, 0, 1):
        for ey in (-1, 0, 1):
            for ez in (-1, 0, 1):
                w = (2 if ex == 0 else -1) * (2 if ey == 0 else -1) * (2 if ez == 0 else -1)
                acc += w * fun(X + ex * dx, Y + ey * dy, Z + ez * dz)
    return acc / (4 * mp.pi * dx * dy * dz)


@pytest.mark.parametrize("o", [(2, 1, 0), (3, 0, 0), (4, 2, 1), (5, 1, 0), (9, 4, 2),
                               (10, 0, 0), (39, 3, 1), (40, 2, 0), (150, 5, 0),
                               (199, 1, 0), (200, 0, 0), (400, 9, 0)])
def test_two_zone_evaluation_matches_50_digit_closed_form(o):
    """Evaluation-accuracy pin: the FP64 two-zone rule against the closed form
    carried out with 50 significant digits (no FP64 cancellation)."""
    mp.mp.dps = 50
    cell = (1.0, 1.0, 1.0)
    X, Y, Z = (mp.mpf(v) for v in o)
    d = [mp.mpf(1)] * 3
    ref = [
        _mp_second_diff(_mp_f, X, Y, Z, *d),
        _mp_second_diff(_mp_f, Y, X, Z, *d),
        _mp_second_diff(_mp_f, Z, Y, X, *d),
        _mp_second_diff(_mp_g, X, Y, Z, *d),
    ]
    t = nw.tensor_at_offsets(np.array([o]), cell)[:, 0]
    scale = max(abs(float(r)) for r in ref[:3])
    # closed-form zone (d <= 2) keeps FP64 cancellation below ~3e-14
    tol = 1e-13 if max(o) <= 2 else 4e-15
    for k in range(4):
        assert abs(t[k] - float(ref[k])) <= tol * scale, (o, k)


def test_whole_body_identity():
    """(1/N) sum_i sum_j N(i - j) equals the self-term of the whole prism."""
    n = (3, 2, 2)
    cell = (1.0, 1.3, 0.7)
    idx = np.array([(x, y, z) for z in range(n[2]) for y in range(n[1]) for x in range(n[0])])
    offs = (idx[:, None, :] - idx[None, :, :]).reshape(-1, 3)
    t = nw.tensor_at_offsets(offs, cell).sum(axis=1) / len(idx)
    prism = nw.tensor_exact(0.0, 0.0, 0.0, n[0] * cell[0], n[1] * cell[1], n[2] * cell[2])
    assert np.abs(t - prism).max() < 1e-13


def test_block_additivity_off_diagonal():
    """Interaction of two disjoint 2x2x1 blocks = sum of their cell-pair
    tensors; pins the off-diagonal (g) components at block scale."""
    cell = (1.0, 1.0, 0.5)
    A = [(x, y, 0) for x in range(2) for y in range(2)]
    for shift in [(2, 2, 0), (2, 0, 0), (4, 2, 0), (2, -2, 0)]:
        B = [(x + shift[0], y + shift[1], z) for (x, y, z) in A]
        offs = np.array([np.subtract(b, a) for a in A for b in B])
        s = nw.tensor_at_offsets(offs, cell).sum(axis=1)
        big = (2 * cell[0], 2 * cell[1], cell[2])
        R = np.array(shift) * np.array(cell)
        ref = len(A) * nw.tensor_exact(R[0], R[1], R[2], *big)
        # both sides carry closed-form FP64 cancellation (flat 4:4:1 blocks)
        assert np.abs(s - ref).max() <= 2e-12 * np.abs(ref).max(), shift


def test_parity_symmetries():
    o = np.array([[3, 2, 1], [1, 1, 0], [5, 4, 2]])
    t = nw.tensor_at_offsets(o, (1.0, 1.3, 0.7))
    for sx, sy, sz in [(-1, 1, 1), (1, -1, 1), (1, 1, -1), (-1, -1, -1)]:
        tm = nw.tensor_at_offsets(o * np.array([sx, sy, sz]), (1.0, 1.3, 0.7))
        sign = np.array([1, 1, 1, sx * sy, sx * sz, sy * sz])[:, None]
        assert np.allclose(tm, sign * t, rtol=1e-13, atol=1e-14)
