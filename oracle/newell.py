"""Cell-averaged demagnetisation tensor (Newell, Williams & Dunlop 1993), FP64.

The paper convolves the magnetisation with the Newell tensor, zero padded to 2N
on open axes, and sums periodic images on periodic axes (Methods, "Physics and
discretization").  It prints no formula; the tensor is the one of the cited
reference: for two identical cuboid cells whose centres differ by R,

    N_ab(R) = (1/V) int_cell int_cell G_ab(x - x') dx dx',
    G_ab(r) = (delta_ab |r|^2 - 3 r_a r_b) / (4 pi |r|^5),

so that H_i = -Ms sum_j N(r_i - r_j) m_j.

Evaluation (reading; the paper is silent on it).  The closed form of Newell et
al. (second differences of the functions f and g over the 27 neighbouring
corner offsets) loses digits to cancellation roughly as (R/cell)^6 in FP64.  It
is therefore used only near the source (scaled Chebyshev distance d <= 2).
Farther out the same double integral is evaluated in the equivalent
one-dimensional-per-axis form

    N_ab(R) = (1/V) int_{[-D,D]^3} G_ab(R + s) prod_a (D_a - |s_a|) ds

by tensor-product Gauss-Legendre quadrature, split at s_a = 0 where the triangle
weight has its kink, with n nodes per half interval chosen by distance:
n = 10 (3 <= d < 5), 8 (5 <= d < 10), 6 (10 <= d < 40), 4 (40 <= d < 200),
3 (d >= 200).  d = floor(max_a |o_a| D_a / max_a D_a) for integer offset o.
Both zones are pinned against 50-digit mpmath evaluations of the closed form.
"""
from __future__ import annotations

import functools
import math

import numpy as np

COMPONENTS = ("xx", "yy", "zz", "xy", "xz", "yz")


# ----------------------------------------------------------------------------
# Newell's auxiliary functions
# ----------------------------------------------------------------------------
def _safe_div(a, b):
    out = np.zeros(np.broadcast(a, b).shape)
    np.divide(a, b, out=out, where=(b != 0))
    return out


def _asinh_ratio(num, den):
    """asinh(num / den); returns 0 where den == 0 (the prefactors that multiply
    it vanish there, Newell et al.)."""
    return np.arcsinh(_safe_div(num, den))


def _atan_ratio(num, den):
    """atan(num / den), 0 where den == 0 (again multiplied by a vanishing term)."""
    return np.where(den != 0, np.arctan(_safe_div(num, den)), 0.0)


def newell_f(x, y, z):
    """Newell's f(x, y, z), whose 27-point second difference gives N_xx."""
    x, y, z = np.broadcast_arrays(np.asarray(x, float), np.asarray(y, float),
                                  np.asarray(z, float))
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    t1 = 0.5 * y * (z2 - x2) * _asinh_ratio(y, np.sqrt(x2 + z2))
    t2 = 0.5 * z * (y2 - x2) * _asinh_ratio(z, np.sqrt(x2 + y2))
    t3 = -x * y * z * _atan_ratio(y * z, x * R)
    t4 = (2.0 * x2 - y2 - z2) * R / 6.0
    return t1 + t2 + t3 + t4


def newell_g(x, y, z):
    """Newell's g(x, y, z), whose 27-point second difference gives N_xy."""
    x, y, z = np.broadcast_arrays(np.asarray(x, float), np.asarray(y, float),
                                  np.asarray(z, float))
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    t1 = x * y * z * _asinh_ratio(z, np.sqrt(x2 + y2))
    t2 = y / 6.0 * (3.0 * z2 - y2) * _asinh_ratio(x, np.sqrt(y2 + z2))
    t3 = x / 6.0 * (3.0 * z2 - x2) * _asinh_ratio(y, np.sqrt(x2 + z2))
    t4 = -z2 * z / 6.0 * _atan_ratio(x * y, z * R)
    t5 = -z * y2 / 2.0 * _atan_ratio(x * z, y * R)
    t6 = -z * x2 / 2.0 * _atan_ratio(y * z, x * R)
    t7 = -x * y * R / 3.0
    return t1 + t2 + t3 + t4 + t5 + t6 + t7


def _second_difference(fun, X, Y, Z, dx, dy, dz):
    """sum over eps in {-1,0,1}^3 of w(eps) fun(X + eps_x dx, ...), with
    w = prod_a (2 if eps_a == 0 else -1)."""
    acc = np.zeros(np.broadcast(X, Y, Z).shape)
    for ex in (-1, 0, 1):
        for ey in (-1, 0, 1):
            for ez in (-1, 0, 1):
                w = (2 if ex == 0 else -1) * (2 if ey == 0 else -1) * (2 if ez == 0 else -1)
                acc = acc + w * fun(X + ex * dx, Y + ey * dy, Z + ez * dz)
    return acc


def tensor_exact(X, Y, Z, dx, dy, dz):
    """Closed-form Newell tensor at centre offset (X, Y, Z) (metres).

    Returns a (6, ...) array in the order xx, yy, zz, xy, xz, yz.  N_yy and N_zz
    follow from N_xx by permuting coordinates and cell sizes, N_xz and N_yz from
    N_xy likewise."""
    X, Y, Z = (np.asarray(v, float) for v in (X, Y, Z))
    pref = 1.0 / (4.0 * math.pi * dx * dy * dz)
    nxx = pref * _second_difference(newell_f, X, Y, Z, dx, dy, dz)
    nyy = pref * _second_difference(newell_f, Y, X, Z, dy, dx, dz)
    nzz = pref * _second_difference(newell_f, Z, Y, X, dz, dy, dx)
    nxy = pref * _second_difference(newell_g, X, Y, Z, dx, dy, dz)
    nxz = pref * _second_difference(newell_g, X, Z, Y, dx, dz, dy)
    nyz = pref * _second_difference(newell_g, Y, Z, X, dy, dz, dx)
    return np.stack(np.broadcast_arrays(nxx, nyy, nzz, nxy, nxz, nyz))


# ----------------------------------------------------------------------------
# far zone: Gauss-Legendre integration of the point-dipole kernel
# ----------------------------------------------------------------------------
@functools.lru_cache(maxsize=None)
def _half_rule(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return x, w


def _axis_rule(n, h):
    """Nodes s and weights on [-h, h] for integrand * (h - |s|), split at 0."""
    x, w = _half_rule(n)
    s_pos = 0.5 * h * (1.0 + x)
    w_half = 0.5 * h * w
    s = np.concatenate([-s_pos, s_pos])
    ww = np.concatenate([w_half, w_half]) * (h - np.abs(s))
    return s, ww


def dipole_kernel(rx, ry, rz):
    """G_ab(r) = (delta_ab r^2 - 3 r_a r_b) / (4 pi r^5), (6, ...) array."""
    r2 = rx * rx + ry * ry + rz * rz
    inv = 1.0 / (4.0 * math.pi * r2 * r2 * np.sqrt(r2))
    return np.stack([(r2 - 3 * rx * rx) * inv, (r2 - 3 * ry * ry) * inv,
                     (r2 - 3 * rz * rz) * inv, -3 * rx * ry * inv,
                     -3 * rx * rz * inv, -3 * ry * rz * inv])


def tensor_quadrature(X, Y, Z, dx, dy, dz, n):
    """Newell tensor at centre offsets (X, Y, Z) (1-D arrays, metres) by
    Gauss-Legendre quadrature with n nodes per half interval."""
    X, Y, Z = (np.atleast_1d(np.asarray(v, float)) for v in (X, Y, Z))
    sx, wx = _axis_rule(n, dx)
    sy, wy = _axis_rule(n, dy)
    sz, wz = _axis_rule(n, dz)
    SX, SY, SZ = np.meshgrid(sx, sy, sz, indexing="ij")
    W = (wx[:, None, None] * wy[None, :, None] * wz[None, None, :]).ravel()
    SX, SY, SZ = SX.ravel(), SY.ravel(), SZ.ravel()
    V = dx * dy * dz
    out = np.empty((6, X.size))
    q = W.size
    chunk = max(1, 2_000_000 // q)
    for a in range(0, X.size, chunk):
        b = min(X.size, a + chunk)
        G = dipole_kernel(X[a:b, None] + SX[None], Y[a:b, None] + SY[None],
                          Z[a:b, None] + SZ[None])
        out[:, a:b] = G @ W / V
    return out


def zone_order(o, cell):
    """Quadrature order for integer offsets o (..., 3); 0 means closed form."""
    o = np.abs(np.asarray(o, dtype=np.int64))
    h = np.asarray(cell, float)
    hmax = h.max()
    rho = np.max(o * h, axis=-1) / hmax
    d = np.floor(rho + 1e-9).astype(np.int64)
    n = np.select([d <= 2, d < 5, d < 10, d < 40, d < 200], [0, 10, 8, 6, 4], 3)
    return n


def tensor_at_offsets(o, cell):
    """Newell tensor for integer cell offsets o (M, 3) -> (6, M), two-zone rule."""
    o = np.asarray(o, dtype=np.int64).reshape(-1, 3)
    dx, dy, dz = cell
    X, Y, Z = o[:, 0] * dx, o[:, 1] * dy, o[:, 2] * dz
    order = zone_order(o, cell)
    out = np.empty((6, o.shape[0]))
    for n in np.unique(order):
        sel = order == n
        if n == 0:
            out[:, sel] = tensor_exact(X[sel], Y[sel], Z[sel], dx, dy, dz)
        else:
            out[:, sel] = tensor_quadrature(X[sel], Y[sel], Z[sel], dx, dy, dz, int(n))
    return out


# ----------------------------------------------------------------------------
# convolution kernel on the padded / periodic FFT grid
# ----------------------------------------------------------------------------
def _axis_offsets(N, periodic):
    """(index, representative offset, image-symmetrisation partner) per index of
    the FFT axis.  Open axis: size 2N (or 1 when N = 1); index k holds offset k
    for k < N, k - 2N for k > N, and nothing (zero) at the Nyquist index N.
    Periodic axis: size N; index k holds the minimum-image offset."""
    if N == 1:
        return [(0, 0)]
    if periodic:
        out = []
        for k in range(N):
            o = k if k < N - k else k - N
            out.append((k, o))
        return out
    out = []
    for k in range(2 * N):
        if k < N:
            out.append((k, k))
        elif k > N:
            out.append((k, k - 2 * N))
    return out


def kernel_real_space(grid):
    """Real-space convolution kernel K (6, Pz, Py, Px) for ``grid``.

    Open axes: K holds N(o) for |o| < N at index o mod 2N; the Nyquist index
    is zero (never reached by cropped outputs; keeps the odd components' spectra
    exactly real).  Periodic axes of length N with P images:
    K(o) = sum_{p=-P..P} N(o + pN) at the minimum-image offset o; when N is even
    the offset N/2 has no mirror inside the range and is given the average of the
    sums for +N/2 and -N/2 (reading: keeps K even/odd per axis)."""
    Px, Py, Pz = grid.padded
    K = np.zeros((6, Pz, Py, Px))
    axes = [_axis_offsets(grid.n[a], grid.pbc[a] and grid.n[a] > 1) for a in range(3)]
    idx, offs, wts = [], [], []
    for (kz, oz) in axes[2]:
        for (ky, oy) in axes[1]:
            for (kx, ox) in axes[0]:
                base = (ox, oy, oz)
                # list of (offset representative sets) to average over
                reps = [base]
                for a in range(3):
                    N = grid.n[a]
                    if grid.pbc[a] and N > 1 and N % 2 == 0 and abs(base[a]) == N // 2:
                        reps = reps + [tuple(-r[b] if b == a else r[b] for b in range(3))
                                       for r in reps]
                for r in reps:
                    shifts = [[0]] * 3
                    shifts = [list(range(-grid.images[a], grid.images[a] + 1))
                              if (grid.pbc[a] and grid.n[a] > 1) else [0] for a in range(3)]
                    for pz in shifts[2]:
                        for py in shifts[1]:
                            for px in shifts[0]:
                                idx.append((kz, ky, kx))
                                offs.append((r[0] + px * grid.n[0], r[1] + py * grid.n[1],
                                             r[2] + pz * grid.n[2]))
                                wts.append(1.0 / len(reps))
    idx = np.array(idx)
    vals = tensor_at_offsets(np.array(offs), grid.cell) * np.array(wts)[None]
    for c in range(6):
        np.add.at(K[c], (idx[:, 0], idx[:, 1], idx[:, 2]), vals[c])
    return K
