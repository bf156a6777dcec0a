"""Pins of the oracle's thermal noise: the published known-answer vectors and
the statistics of the counter-based Philox4x32-10 stream (Salmon et al. 2011),
the trial-generation counter word, and the Langevin law of a thermal
macrospin (Results, "A replica-batched engine": <m_z> = L(xi))."""
import json
import math
import os

import numpy as np
import pytest
from scipy import stats

from oracle import KB, MU0, Grid, Material
from oracle import integrators as it
from oracle import philox
from workloads import replica_seeds

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answer_vectors():
    with open(os.path.join(GOLDEN, "philox_kat.json")) as fh:
        kat = json.load(fh)["vectors"]
    for v in kat:
        ctr = np.array([int(x, 16) for x in v["ctr"]], dtype=np.uint64)
        key = np.array([int(x, 16) for x in v["key"]], dtype=np.uint64)
        out = philox.philox4x32_10(ctr, key)
        assert ["%08x" % int(x) for x in out] == v["out"]


def test_trial_generation_is_the_fourth_counter_word():
    """Generation 0 is the plain stream; generation g sets counter word 3."""
    seeds = np.array([7, 2 ** 40 + 3], dtype=np.uint64)
    w0 = philox.raw_words(seeds, 16, 5)
    assert np.array_equal(w0, philox.raw_words(seeds, 16, 5, gen=0))
    w3 = philox.raw_words(seeds, 16, 5, gen=3)
    ctr = np.array([2, 5, 0, 3], dtype=np.uint64)
    key = np.array([3, 256], dtype=np.uint64)  # seed 2^40 + 3: low word 3, high word 2^8
    assert np.array_equal(w3[1, 2], philox.philox4x32_10(ctr, key))
    assert not np.array_equal(w0, w3)


def test_philox_words_uniform_and_decorrelated():
    w = philox.raw_words(np.array([12345, 99], dtype=np.uint64), 50000, 7).astype(np.float64)
    u = (w + 0.5) / 2.0 ** 32
    for r in range(2):
        for k in range(4):
            assert stats.kstest(u[r, :, k], "uniform").pvalue > 1e-4
    flat = u.reshape(-1, 4)
    c = np.corrcoef(flat.T)
    assert np.abs(c - np.eye(4)).max() < 0.02
    # keys and steps give different streams
    w2 = philox.raw_words(np.array([12345], dtype=np.uint64), 50000, 8)
    assert np.mean(w2[0] == w[0].astype(np.uint64)) < 1e-3
    assert np.mean(w[0] == w[1]) < 1e-3


def test_philox_is_a_bijection_on_sampled_counters():
    # a keyed permutation: distinct counters never collide
    w = philox.raw_words(np.array([5], dtype=np.uint64), 200000, 0)[0]
    packed = w[:, 0] * np.uint64(2 ** 32) + w[:, 1]
    assert np.unique(packed).size == packed.size


def test_gaussian_eta_moments_and_normality():
    eta = philox.gaussian_eta(replica_seeds(3, 4), 20000, 11)
    x = eta.reshape(-1)
    assert abs(x.mean()) < 0.01
    assert abs(x.var() - 1.0) < 0.01
    assert stats.kstest(x, "norm").pvalue > 1e-4
    assert abs(np.corrcoef(eta[:, 0].ravel(), eta[:, 2].ravel())[0, 1]) < 0.01


@pytest.mark.slow
def test_langevin_law_thermal_macrospin():
    """Free macrospin in a field with xi = mu0 Ms V H / kB T = 3, Heun with the
    Brown field: the ensemble mean <m_z> approaches L(3) = coth 3 - 1/3."""
    with open(os.path.join(GOLDEN, "paper_values.json")) as fh:
        g = json.load(fh)["langevin"]
    xi = g["xi"]
    cell = (4e-9, 4e-9, 4e-9)
    Ms, T = 8e5, 300.0
    V = cell[0] * cell[1] * cell[2]
    B = xi * KB * T / (Ms * V)  # mu0 H
    grid = Grid((1, 1, 1), cell)
    mat = Material(Ms=Ms, alpha=0.1, B=(0, 0, B), T=T, demag=False)
    R = 4096
    seeds = replica_seeds(18, R)
    m = np.zeros((R, 3, 1, 1, 1)); m[:, 2] = 1.0
    dt = 1e-13
    m = it.heun_run(m, grid, mat, dt, 3000, seed=seeds, step0=0)
    acc, n = 0.0, 0
    for k in range(3000, 9000, 3):
        m = it.heun_run(m, grid, mat, dt, 3, seed=seeds, step0=k)
        acc += m[:, 2].mean()
        n += 1
    mz = acc / n
    L = 1.0 / math.tanh(xi) - 1.0 / xi
    assert L == pytest.approx(g["L_xi"], abs=5e-4)     # the paper's L(3)
    assert abs(mz - L) < 0.01
    assert abs(np.linalg.norm(m, axis=1) - 1).max() < 1e-14
