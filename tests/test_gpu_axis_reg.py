"""GPU parity of the register y and z passes of 3-D grids (the y transform of
one (component, plane) line per column, and the z transform with the full
tensor product per pillar; split 8 x 8, 8 x 16, 8 x 24, 16 x 16, 16 x 32
along y and 4 x 8, 8 x 8, 8 x 16 along z): FP32 fields and Heun steps against
the oracle on grids it runs in seconds, and against the GPU's FP64 path
(Stockham passes in LDS, matching the oracle to 1e-11 elsewhere) on the
longer axes.

Bars: fields FP32 4e-6 of max |H|; states FP32 1e-5.
"""
import numpy as np
import pytest

from oracle import fields as ofl
from oracle import integrators as oit
from workloads import random_unit, replica_seeds, uniform

from _mmx_case import Case, dev, host, open_ctx

pytestmark = pytest.mark.gpu


def _case(n, R=2, T=0.0):
    return Case(n, (3e-9, 2.5e-9, 2e-9), R=R, Ms=8e5, A=1.3e-11, alpha=0.1, Ku=2e5,
                u=(0.1, 0.0, 1.0), B=(0.01, 0.0, 0.03), T=T,
                seeds=list(replica_seeds(61, R)) if T else [],
                terms=("exchange", "anisotropy", "zeeman", "demag") + (("thermal",) if T else ()))


def _field(case, prec, m0):
    import paper_2608_15253_amd as mmx
    ctx = open_ctx(case, prec)
    try:
        H = dev(np.zeros_like(m0), prec)
        mmx.mmx_field(ctx, dev(m0, prec), H)
        return host(H)
    finally:
        mmx.mmx_destroy(ctx)


@pytest.mark.parametrize("n", [(16, 32, 16), (24, 32, 2)])
def test_register_passes_against_oracle(n):
    """(16, 32, 16): y 8 x 8 and z 4 x 8 register passes; (24, 32, 2): the
    separate y passes around the per-thread z pillars of a two-layer grid."""
    import paper_2608_15253_amd as mmx
    case = _case(n, T=300.0)
    print(f"[case] axis reg {n}", flush=True)
    m0 = random_unit(case.n, seed=71, replicas=case.R).astype(np.float32).astype(np.float64)
    got = _field(_case(n), 1, m0)
    for r in range(case.R):
        ref = ofl.effective_field(m0[r], case.grid, _case(n).material())
        assert np.abs(got[r] - ref).max() <= 4e-6 * np.abs(ref).max()
    mu = uniform(case.n, (0.2, 0.1, 1.0), replicas=case.R).astype(np.float32).astype(np.float64)
    ctx = open_ctx(case, 1)
    try:
        md = dev(mu, 1)
        mmx.mmx_heun(ctx, md, 2e-14, 6, 3)
        gm = host(md)
    finally:
        mmx.mmx_destroy(ctx)
    ref = oit.heun_run(mu, case.grid, case.material(), 2e-14, 6, seed=np.array(case.seeds), step0=3)
    assert np.abs(gm - ref).max() <= 1e-5


@pytest.mark.parametrize("n", [(16, 96, 8), (8, 256, 4), (8, 128, 32), (8, 64, 64), (96, 96, 2)])
def test_register_passes_against_fp64_path(n):
    """Py = 192, 512, 256, 128, 192 and Pz = 16, 8, 64, 128, 4: the FP32
    register passes against the FP64 path of the same grid."""
    case = _case(n, R=1)
    print(f"[case] axis reg vs fp64 {n}", flush=True)
    m0 = random_unit(case.n, seed=72, replicas=1).astype(np.float32).astype(np.float64)
    h32 = _field(case, 1, m0)
    h64 = _field(case, 2, m0)
    assert np.abs(h32 - h64).max() <= 4e-6 * np.abs(h64).max()


def test_fused_and_split_few_layer_paths_agree():
    """A two-layer 96 x 96 grid: the fused y-z kernel and the separate
    register y passes give the same field to FP32 round-off (mmx_autotune
    picks the faster; both stay valid)."""
    import paper_2608_15253_amd as mmx
    case = _case((96, 96, 2), R=2)
    m0 = random_unit(case.n, seed=73, replicas=2).astype(np.float32).astype(np.float64)
    before = _field(case, 1, m0)
    ctx = open_ctx(case, 1)
    try:
        mmx.mmx_autotune(ctx)
        H = dev(np.zeros_like(m0), 1)
        mmx.mmx_field(ctx, dev(m0, 1), H)
        after = host(H)
    finally:
        mmx.mmx_destroy(ctx)
    assert np.abs(before - after).max() <= 4e-6 * np.abs(before).max()
