"""Demagnetising field, FP64 (Methods, "Physics and discretization": open
boundaries by FFT convolution with the Newell tensor zero padded to 2N,
periodic boundaries by an image-sum kernel).

H_i = -sum_j K(i - j) Ms_j m_j with K from ``newell.kernel_real_space`` (Ms a
scalar, or one value per cell: the convolution acts on M = Ms m).  Two
evaluations of the same definition: a direct O(N^2) sum (tiny grids) and the
FFT convolution on the padded grid (numpy's complex FFT as the primitive).
"""
from __future__ import annotations

import functools

import numpy as np

from . import newell


@functools.lru_cache(maxsize=16)
def _kernel(grid):
    return newell.kernel_real_space(grid)


@functools.lru_cache(maxsize=16)
def _kernel_hat(grid):
    return np.fft.fftn(_kernel(grid), axes=(1, 2, 3))


def demag_direct(m, grid, Ms):
    """Direct sum H_i = -sum_j K(i - j) Ms_j m_j over all source cells.  ``m``
    has shape (3, nz, ny, nx), ``Ms`` a scalar or (nz, ny, nx).  Offsets index
    the same kernel array as the FFT path, taken modulo the FFT size (open
    axes: |i - j| < N never wraps)."""
    nx, ny, nz = grid.n
    Px, Py, Pz = grid.padded
    K = _kernel(grid)
    full = np.array([[0, 3, 4], [3, 1, 5], [4, 5, 2]])
    H = np.zeros((3, nz, ny, nx))
    zs, ys, xs = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    zs, ys, xs = zs.ravel(), ys.ravel(), xs.ravel()
    msrc = (Ms * m).reshape(3, -1)
    for k in range(zs.size):
        iz, iy, ix = zs[k], ys[k], xs[k]
        kz = (iz - zs) % Pz
        ky = (iy - ys) % Py
        kx = (ix - xs) % Px
        for a in range(3):
            acc = 0.0
            for b in range(3):
                acc += np.dot(K[full[a, b], kz, ky, kx], msrc[b])
            H[a, iz, iy, ix] = -acc
    return H


def demag_fft(m, grid, Ms):
    """FFT convolution: pad M = Ms m with zeros to the FFT grid, multiply the
    spectra by the (symmetric) tensor spectrum, transform back and crop."""
    nx, ny, nz = grid.n
    Px, Py, Pz = grid.padded
    Kh = _kernel_hat(grid)
    M = np.zeros((3, Pz, Py, Px))
    M[:, :nz, :ny, :nx] = Ms * m
    Mh = np.fft.fftn(M, axes=(1, 2, 3))
    xx, yy, zz, xy, xz, yz = Kh
    Hh = np.stack([xx * Mh[0] + xy * Mh[1] + xz * Mh[2],
                   xy * Mh[0] + yy * Mh[1] + yz * Mh[2],
                   xz * Mh[0] + yz * Mh[1] + zz * Mh[2]])
    H = np.fft.ifftn(Hh, axes=(1, 2, 3)).real
    return -H[:, :nz, :ny, :nx]


def demag_field(m, grid, Ms):
    """Demag field of one replica (3, nz, ny, nx) or a batch (R, 3, nz, ny, nx)."""
    if m.ndim == 5:
        return np.stack([demag_fft(mr, grid, Ms) for mr in m])
    return demag_fft(m, grid, Ms)
