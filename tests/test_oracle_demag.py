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
