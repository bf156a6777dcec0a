"""Pins of the oracle's learned-stage RK45 attempt and gate (oracle.surrogate)."""
import numpy as np

from oracle import Grid, Material
from oracle import fno as ofno
from oracle import integrators as oit
from oracle import surrogate as osg
from workloads import random_unit, uniform

GRID = Grid((12, 10, 1), (4e-9, 4e-9, 4e-9))
MAT = Material(Ms=8e5, A=1.3e-11, alpha=0.3, Ku=6e5, D=3e-3, B=(0.0, 0.0, 0.1))


def test_exact_field_in_the_stages_is_the_plain_attempt():
    m = random_unit(GRID.n, seed=3, replicas=2)
    k1 = oit.rhs(m, GRID, MAT)
    dt = 2e-14
    ref = oit.dopri5_attempt(m, k1, GRID, MAT, dt)
    got = osg.attempt(m, k1, GRID, MAT, dt, lambda ms: osg.exact_demag(ms, GRID, MAT.Ms))
    assert np.allclose(got[0], ref[0], rtol=0, atol=1e-14)
    assert np.allclose(got[1], ref[1], rtol=1e-12, atol=0)
    assert abs(got[2] - ref[2]) <= 1e-10 * ref[2]


def test_network_with_zero_head_gives_the_local_thin_film_field():
    p = ofno.init_params(C=4, M1=3, M2=2, L=1, Cp=8, seed=1)
    p["Q2"][:] = 0.0
    p["q2"][:] = 0.0
    m = random_unit(GRID.n, seed=4, replicas=2)
    H = osg.network_demag(p, m, 8e5, 3, 2, residual_mz=True)
    assert np.all(H[:, :2] == 0.0)
    assert np.array_equal(H[:, 2], -8e5 * m[:, 2])
    assert np.all(osg.network_demag(p, m, 8e5, 3, 2, residual_mz=False) == 0.0)


def test_gate_error_is_a_per_replica_relative_norm():
    rng = np.random.default_rng(0)
    H = rng.standard_normal((3, 3, 1, 4, 5))
    assert np.all(osg.gate_error(H, H) == 0.0)
    Hn = H.copy()
    Hn[1] *= 2.0            # replica 1: error = |H|, relative 1
    Hn[2] += 1e-3 * H[2]    # replica 2: relative 1e-3
    e = osg.gate_error(Hn, H)
    assert e[0] == 0.0 and abs(e[1] - 1.0) < 1e-14 and abs(e[2] - 1e-3) < 1e-15


def test_thin_film_limit_behind_the_residual_reading():
    """A wide uniform film: the field inside is close to -Ms m_z z (infinite
    film: N_zz = 1, N_xx = N_yy = 0), so (0, 0, -m_z) is the right local part."""
    g = Grid((64, 64, 1), (4e-9, 4e-9, 4e-9))
    Hz = osg.exact_demag(uniform(g.n, (0, 0, 1)), g, 8e5)
    assert abs(Hz[2, 0, 32, 32] / 8e5 + 1.0) < 0.05
    Hx = osg.exact_demag(uniform(g.n, (1, 0, 0)), g, 8e5)
    assert abs(Hx[0, 0, 32, 32] / 8e5) < 0.05
