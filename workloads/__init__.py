"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only *generates inputs*: initial magnetisation fields, per-replica
seeds and the material/geometry presets of the benchmark workloads.  It holds
none of the method's arithmetic (no field, torque, integrator or FFT code), so
that both the FP64 oracle and the HIP library can consume it without sharing
any computation.

All arrays use the component-major, x-fastest layout of one replica:
``m[c, z, y, x]`` (shape ``(3, nz, ny, nx)``), and ``m[r, c, z, y, x]`` for a
batch of replicas (replica-outermost, then component, then cell).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

MASK64 = (1 << 64) - 1


# --------------------------------------------------------------------------
# seeds
# --------------------------------------------------------------------------
def splitmix64(x: int) -> int:
    """One output of the SplitMix64 generator (Steele, Lea & Flood, OOPSLA 2014)
    for state ``x``; used only to derive well-mixed per-replica 64-bit seeds."""
    z = (x + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def replica_seeds(base: int, count: int, first: int = 0) -> np.ndarray:
    """Per-replica 64-bit thermal-noise keys: ``splitmix64(base * 2**32 + r)``."""
    return np.array([splitmix64(((base << 32) + first + r) & MASK64)
                     for r in range(count)], dtype=np.uint64)


# --------------------------------------------------------------------------
# initial magnetisation fields
# --------------------------------------------------------------------------
def random_unit(n, seed: int, replicas: int | None = None) -> np.ndarray:
    """Uniformly distributed random unit vectors per cell (normalised N(0, I3)
    draws from numpy's PCG64 with the given seed)."""
    nx, ny, nz = n
    shape = (3, nz, ny, nx) if replicas is None else (replicas, 3, nz, ny, nx)
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.standard_normal(shape)
    ax = 0 if replicas is None else 1
    return v / np.linalg.norm(v, axis=ax, keepdims=True)


def uniform(n, direction=(0.0, 0.0, 1.0), replicas: int | None = None) -> np.ndarray:
    """A uniformly magnetised state along ``direction`` (normalised)."""
    nx, ny, nz = n
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    m = np.empty((3, nz, ny, nx))
    for c in range(3):
        m[c] = d[c]
    if replicas is not None:
        m = np.broadcast_to(m, (replicas,) + m.shape).copy()
    return m


def neel_skyrmions(n, cell, count: int, rmin: float, rmax: float, seed: int,
                   width: float, gap: float = 20e-9, periodic=True,
                   max_tries: int = 100000):
    """Seed ``count`` core-down Neel skyrmions on a +z background.

    Centres are uniform on the film (torus if ``periodic``), radii uniform in
    ``[rmin, rmax]``; a candidate is rejected when its minimum-image distance to
    an accepted skyrmion is below ``R_i + R_j + gap``.  Each skyrmion has the
    domain-wall profile ``theta(r) = 2 atan(sinh(R/w) / sinh(r/w))`` and an
    in-plane component pointing radially outward (azimuth = polar angle about
    the centre).  Where skyrmions overlap the one with the smallest
    ``theta`` distance wins (they are separated, so this only matters in tails).

    Returns ``(m, centres, radii)``.
    """
    nx, ny, nz = n
    dx, dy, _ = cell
    Lx, Ly = nx * dx, ny * dy
    rng = np.random.Generator(np.random.PCG64(seed))
    centres, radii = [], []
    tries = 0
    while len(centres) < count:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place skyrmions")
        c = (rng.uniform(0, Lx), rng.uniform(0, Ly))
        R = rng.uniform(rmin, rmax)
        ok = True
        for (cx, cy), Rj in zip(centres, radii):
            ddx, ddy = c[0] - cx, c[1] - cy
            if periodic:
                ddx -= Lx * round(ddx / Lx)
                ddy -= Ly * round(ddy / Ly)
            if math.hypot(ddx, ddy) < R + Rj + gap:
                ok = False
                break
        if ok:
            centres.append(c)
            radii.append(R)
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dy
    X, Y = np.meshgrid(x, y, indexing="xy")  # (ny, nx)
    theta = np.zeros((ny, nx))
    phi = np.zeros((ny, nx))
    for (cx, cy), R in zip(centres, radii):
        ddx, ddy = X - cx, Y - cy
        if periodic:
            ddx = ddx - Lx * np.round(ddx / Lx)
            ddy = ddy - Ly * np.round(ddy / Ly)
        r = np.hypot(ddx, ddy)
        with np.errstate(divide="ignore", over="ignore"):
            th = 2.0 * np.arctan(np.sinh(R / width) / np.sinh(np.maximum(r, 1e-30) / width))
        th = np.where(r < 1e-30, math.pi, th)
        better = th > theta
        theta = np.where(better, th, theta)
        phi = np.where(better, np.arctan2(ddy, ddx), phi)
    m = np.empty((3, nz, ny, nx))
    m[0] = (np.sin(theta) * np.cos(phi))[None]
    m[1] = (np.sin(theta) * np.sin(phi))[None]
    m[2] = np.cos(theta)[None]
    m /= np.linalg.norm(m, axis=0, keepdims=True)
    return m, np.array(centres), np.array(radii)


def landau_seed(n) -> np.ndarray:
    """Four-triangle flux-closure (Landau) in-plane pattern, identical in every
    layer, with a small +z tilt at the centre column so the core is defined.
    Deterministic."""
    nx, ny, nz = n
    x = (np.arange(nx) + 0.5) / nx - 0.5
    y = (np.arange(ny) + 0.5) / ny - 0.5
    X, Y = np.meshgrid(x, y, indexing="xy")
    m = np.zeros((3, nz, ny, nx))
    # circulation: +x on the bottom triangle, +y right, -x top, -y left
    bottom = (np.abs(X) <= -Y)
    top = (np.abs(X) <= Y) & ~bottom
    right = (np.abs(Y) < X) & ~bottom & ~top
    left = ~(bottom | top | right)
    mx = np.where(bottom, 1.0, 0.0) - np.where(top, 1.0, 0.0)
    my = np.where(right, 1.0, 0.0) - np.where(left, 1.0, 0.0)
    r = np.hypot(X, Y)
    mz = np.exp(-(r / 0.05) ** 2)
    v = np.stack([mx, my, mz])
    v /= np.linalg.norm(v, axis=0, keepdims=True)
    m[:] = v[:, None]
    return m


# --------------------------------------------------------------------------
# workload presets
# --------------------------------------------------------------------------
@dataclass
class Workload:
    """Geometry + material + drive of one replica group (SI units)."""
    name: str
    n: tuple
    cell: tuple
    pbc: tuple = (0, 0, 0)
    images: tuple = (0, 0, 0)
    Ms: float = 8.0e5
    A: float = 1.3e-11
    alpha: float = 0.5
    Ku: float = 0.0
    u: tuple = (0.0, 0.0, 1.0)
    D: float = 0.0
    B: tuple = (0.0, 0.0, 0.0)
    T: float = 0.0
    replicas: int = 1
    extra: dict = field(default_factory=dict)


def relax_film_fp64() -> Workload:
    """32x32x1 film of 4 nm cells, open boundaries, alpha = 0.5, no anisotropy,
    no DMI, zero field; random initial state (seed 1); RK45 to 1 ns, tol 1e-6."""
    return Workload("relax_film_32x32", (32, 32, 1), (4e-9, 4e-9, 4e-9),
                    Ms=8.0e5, A=1.3e-11, alpha=0.5,
                    extra=dict(seed=1, t_end=1e-9, tol=1e-6))


def skyrmion_film_fp32() -> Workload:
    """512x512x1 film of 2x2x0.6 nm cells, periodic in-plane, Ms 5.8e5,
    A 1.5e-11, interfacial D 3e-3, Ku 0.8e6 along z, alpha 0.3, Bz 0.1 T;
    16 Neel skyrmions of radius 10-30 nm (seed 2); RK45 to 2 ns."""
    return Workload("skyrmion_film_512x512", (512, 512, 1), (2e-9, 2e-9, 0.6e-9),
                    pbc=(1, 1, 0), images=(10, 10, 0), Ms=5.8e5, A=1.5e-11,
                    alpha=0.3, Ku=0.8e6, D=3.0e-3, B=(0.0, 0.0, 0.1),
                    extra=dict(seed=2, count=16, rmin=10e-9, rmax=30e-9,
                               t_end=2e-9, tol=1e-6))


def thermal_switching_batch(replicas: int = 1024) -> Workload:
    """Replicas of a 64x64x1 film of 4 nm cells, Ms 8e5, A 1.3e-11, alpha 0.02,
    Ku 5e5 along z, open boundaries, demag on; m0 = +z; Bz = -0.15 T; T = 300 K;
    Heun with dt = 1e-14 s for 2e5 steps; per-replica keys from base seed 3."""
    return Workload("thermal_switching_64x64", (64, 64, 1), (4e-9, 4e-9, 4e-9),
                    Ms=8.0e5, A=1.3e-11, alpha=0.02, Ku=5e5, B=(0.0, 0.0, -0.15),
                    T=300.0, replicas=replicas,
                    extra=dict(seed_base=3, dt=1e-14, steps=200000))


def uneven_groups(replicas: int = 256):
    """Replica groups of uneven size sharing one launch: 32x32x1, 128x32x1,
    96x96x2 and 256x64x1 films of 4 nm cells, open boundaries, skyrmion-film
    material with alpha 0.05, T = 100 K, Bz = 0.1 T, m0 = +z, Heun dt 1e-14 s."""
    mat = dict(Ms=5.8e5, A=1.5e-11, D=3.0e-3, Ku=0.8e6, alpha=0.05,
               B=(0.0, 0.0, 0.1), T=100.0, replicas=replicas)
    out = []
    for k, n in enumerate([(32, 32, 1), (128, 32, 1), (96, 96, 2), (256, 64, 1)]):
        out.append(Workload(f"uneven_{n[0]}x{n[1]}x{n[2]}", n, (4e-9,) * 3,
                            extra=dict(seed_base=4_000_000 + k * 1000, dt=1e-14),
                            **mat))
    return out


def closure_block_fp32() -> Workload:
    """256x256x32 block of 4 nm cubes, Ms 8e5, A 1.3e-11, alpha 0.5, open,
    Landau seed; RK45 tol 1e-6 to 1 ns."""
    return Workload("closure_block_256x256x32", (256, 256, 32), (4e-9,) * 3,
                    Ms=8.0e5, A=1.3e-11, alpha=0.5,
                    extra=dict(t_end=1e-9, tol=1e-6))
