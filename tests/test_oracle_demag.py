"""Pins of the oracle's demag convolution: FFT path vs direct O(N^2) sum, the
whole-body identity, and the periodic-film limit (Methods, "Physics and
discretization")."""
import numpy as np
import pytest

from oracle import Grid, newell
from oracle import demag as dm
from workloads import random_unit


@pytest.mark.parametrize("grid", [
    Grid((3, 2, 2), (1e-9, 1.3e-9, 0.7e-9)),
    Grid((5, 4, 1), (4e-9, 4e-9, 4e-9)),
    Grid((4, 3, 3), (2e-9, 2e-9, 1e-9)),
    Grid((6, 4, 1), (2e-9, 2e-9, 0.6e-9), pbc=(1, 1, 0), images=(2, 2, 0)),
    Grid((4, 4, 2), (3e-9, 3e-9, 3e-9), pbc=(1, 0, 0), images=(3, 0, 0)),
    Grid((5, 3, 1), (3e-9, 3e-9, 3e-9), pbc=(1, 1, 0), images=(1, 1, 0)),
])
def test_fft_equals_direct_sum(grid):
    m = random_unit(grid.n, seed=11)
    Ms = 8e5
    Hf = dm.demag_fft(m, grid, Ms)
    Hd = dm.demag_direct(m, grid, Ms)
    assert np.abs(Hf - Hd).max() <= 1e-13 * Ms


def test_uniform_prism_mean_field_is_prism_demag_factor():
    grid = Grid((6, 5, 3), (2e-9, 3e-9, 1.5e-9))
    Ms = 1e6
    N = newell.tensor_exact(0.0, 0.0, 0.0, 12e-9, 15e-9, 4.5e-9)
    full = np.array([[N[0], N[3], N[4]], [N[3], N[1], N[5]], [N[4], N[5], N[2]]])
    for d in ([1, 0, 0], [0, 1, 0], [0, 0, 1], [0.6, 0.0, 0.8]):
        m = np.zeros((3,) + grid.n[::-1])
        for c in range(3):
            m[c] = d[c]
        H = dm.demag_fft(m, grid, Ms).reshape(3, -1).mean(axis=1)
        assert np.allclose(H, -Ms * full @ np.array(d), rtol=0, atol=1e-12 * Ms)


def test_periodic_film_tends_to_thin_film_limit():
    # uniform out-of-plane film, periodic in-plane: H_z -> -Ms as images grow
    Ms = 5.8e5
    prev = 0.0
    for P in (1, 2, 4, 8):
        grid = Grid((4, 4, 1), (2e-9, 2e-9, 0.6e-9), pbc=(1, 1, 0), images=(P, P, 0))
        m = np.zeros((3, 1, 4, 4))
        m[2] = 1.0
        Hz = dm.demag_fft(m, grid, Ms)[2].mean()
        assert Hz < prev  # monotone towards -Ms
        prev = Hz
    assert abs(prev / -Ms - 1.0) < 0.02


def _window_direct_sum(m, grid, Ms):
    """Independent statement of the periodic image sum (Methods, "Physics and
    discretization": image sums on periodic axes; reading: the minimum-image
    convention with P images).  Every target cell sees every image of every
    source cell whose displacement along a periodic axis of length N lies
    within (P + 1/2) N; an image exactly on that boundary (even N only)
    counts with weight 1/2.  Built from ``newell.tensor_at_offsets`` alone:
    no kernel array, no FFT, no modular indexing."""
    nx, ny, nz = grid.n
    n = (nx, ny, nz)
    per = [bool(grid.pbc[a]) and n[a] > 1 for a in range(3)]
    shifts = [range(-grid.images[a] - 1, grid.images[a] + 2) if per[a] else [0]
              for a in range(3)]
    full = np.array([[0, 3, 4], [3, 1, 5], [4, 5, 2]])
    cells = [(x, y, z) for z in range(nz) for y in range(ny) for x in range(nx)]
    msrc = m.reshape(3, -1)
    H = np.zeros((3, len(cells)))
    for i, ci in enumerate(cells):
        offs, wts, src = [], [], []
        for j, cj in enumerate(cells):
            for tz in shifts[2]:
                for ty in shifts[1]:
                    for tx in shifts[0]:
                        t = (tx, ty, tz)
                        d = [ci[a] - cj[a] - t[a] * n[a] for a in range(3)]
                        w = 1.0
                        for a in range(3):
                            if not per[a]:
                                continue
                            lim2 = (2 * grid.images[a] + 1) * n[a]   # twice (P + 1/2) N
                            if 2 * abs(d[a]) > lim2:
                                w = 0.0
                            elif 2 * abs(d[a]) == lim2:
                                w *= 0.5
                        if w:
                            offs.append(d)
                            wts.append(w)
                            src.append(j)
        Nt = newell.tensor_at_offsets(np.array(offs), grid.cell) * np.array(wts)[None]
        ms = msrc[:, src]
        for a in range(3):
            H[a, i] = -Ms * sum(np.dot(Nt[full[a, b]], ms[b]) for b in range(3))
    return H.reshape(3, nz, ny, nx)


@pytest.mark.parametrize("grid", [
    Grid((6, 4, 1), (2e-9, 2e-9, 0.6e-9), pbc=(1, 1, 0), images=(2, 2, 0)),   # even N both axes
    Grid((5, 3, 1), (3e-9, 3e-9, 3e-9), pbc=(1, 1, 0), images=(1, 1, 0)),     # odd N
    Grid((4, 3, 2), (3e-9, 2e-9, 2.5e-9), pbc=(1, 0, 0), images=(3, 0, 0)),   # periodic x only, 3-D
    Grid((2, 5, 1), (2e-9, 2e-9, 1e-9), pbc=(1, 1, 0), images=(0, 2, 0)),     # N = 2, no x images
])
def test_periodic_kernel_equals_image_window_direct_sum(grid):
    m = random_unit(grid.n, seed=17)
    Ms = 5.8e5
    Hf = dm.demag_fft(m, grid, Ms)
    Hw = _window_direct_sum(m, grid, Ms)
    assert np.abs(Hf - Hw).max() <= 1e-13 * Ms
