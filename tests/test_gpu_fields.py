"""GPU parity of one field evaluation through the C ABI against the FP64
oracle, term by term and in total, FP64 and FP32 (Methods, "Physics and
discretization"; LLG equation).

Tolerances (max |dH| relative to the largest |H| of the case): FP64 1e-11
(FFT round-off of a few hundred terms at 1e-16); FP32 4e-6 (single-precision
round-off of the same sums: 2^-24 times the transform depth and the stencil
cancellation, with a factor of ~4 margin).
"""
import numpy as np
import pytest

from oracle import fields as ofl
from oracle import llg as ollg
from workloads import random_unit, replica_seeds

from _mmx_case import Case, dev, host, open_ctx

pytestmark = pytest.mark.gpu

TOL = {2: 1e-11, 1: 4e-6}

CASES = {
    "film_open_32x32": Case((32, 32, 1), (4e-9, 4e-9, 4e-9), R=2, Ku=5e5, u=(0.3, 0.4, 0.866),
                            B=(0.01, -0.02, 0.05)),
    "film_ragged_20x12": Case((20, 12, 1), (3e-9, 2e-9, 1e-9), R=1, Ku=3e5, D=2e-3,
                              Ms=5.8e5, A=1.5e-11, B=(0.0, 0.0, 0.1)),
    "film_odd_15x9": Case((15, 9, 1), (4e-9, 4e-9, 2e-9), R=2, D=-1e-3, Ms=6e5),
    "film_periodic_16x12": Case((16, 12, 1), (2e-9, 2e-9, 0.6e-9), pbc=(1, 1, 0),
                                images=(2, 2, 0), R=2, Ms=5.8e5, A=1.5e-11, D=3e-3,
                                Ku=0.8e6, B=(0, 0, 0.1)),
    "block_open_6x5x3": Case((6, 5, 3), (3e-9, 3e-9, 3e-9), R=2, Ku=2e5, D=1e-3),
    "block_pbcx_8x4x4": Case((8, 4, 4), (4e-9, 4e-9, 4e-9), pbc=(1, 0, 0), images=(3, 0, 0),
                             R=1),
    "film_96x24x2_radix3": Case((96, 24, 2), (4e-9, 4e-9, 4e-9), R=1, Ku=1e5),
    # few-layer z passes (fused with y) with nz = 5 of 8 (periodic z, Pz = 5)
    # and nz = 8 (open, Pz = 16); nz = 10 takes the LDS z kernel
    "block_pbcz_6x4x5": Case((6, 4, 5), (3e-9, 3e-9, 2e-9), pbc=(0, 0, 1), images=(0, 0, 2),
                             R=2, Ku=2e5, D=1e-3),
    "block_open_4x3x8": Case((4, 3, 8), (3e-9, 3e-9, 2e-9), R=1, Ku=1e5),
    "block_open_4x3x10": Case((4, 3, 10), (3e-9, 3e-9, 2e-9), R=1, Ku=1e5),
    # FP64: one fused y-z column (6 nz (Py + 1) values) exceeds the LDS of a
    # workgroup, so the separate y passes and the register z pass run; FP32
    # fits and takes the fused pass
    "block_tall_4x120x8": Case((4, 120, 8), (3e-9, 3e-9, 2e-9), R=1, Ku=1e5),
    "chain_30x1x1": Case((30, 1, 1), (5e-9, 5e-9, 5e-9), R=3, Ku=1e5),
    "macrospin": Case((1, 1, 1), (4e-9, 3e-9, 2e-9), R=4, Ku=6e5, B=(0, 0, 0.1)),
    "column_1x9x1": Case((1, 9, 1), (4e-9, 4e-9, 4e-9), R=1),
}


def _mm(case, seed):
    return random_unit(case.n, seed=seed, replicas=case.R)


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
@pytest.mark.parametrize("name", list(CASES))
def test_field_terms_match_oracle(name, prec):
    import paper_2608_15253_amd as mmx
    case = CASES[name]
    print(f"[case] fields {name} prec={prec}", flush=True)
    m0 = _mm(case, seed=21)
    if prec == 1:
        m0 = m0.astype(np.float32).astype(np.float64)
    ctx = open_ctx(case, prec)
    try:
        md = dev(m0, prec)
        H = dev(np.zeros_like(m0), prec)
        terms = [t for t in case.terms]
        mat = case.material()
        parts = [ofl.terms(m0[r], case.grid, mat) for r in range(case.R)]
        errs = {}
        full_ref = None
        for only in [[t] for t in terms] + [terms]:
            mmx.mmx_set_terms(ctx, case.mask(only))
            mmx.mmx_field(ctx, md, H)
            got = host(H)
            ref = np.stack([sum(p[k] for k in only) for p in parts])
            scale = max(np.abs(ref).max(), 1.0)
            errs["+".join(only)] = np.abs(got - ref).max() / scale
            full_ref = ref
        print(errs)
        assert all(e <= TOL[prec] for e in errs.values()), errs
        # torque with every term
        mmx.mmx_set_terms(ctx, case.mask(terms))
        mmx.mmx_torque(ctx, md, H)
        got = host(H)
        ref = ollg.llg_rhs(m0, full_ref, case.alpha)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        assert err <= TOL[prec] * 4, err
    finally:
        mmx.mmx_destroy(ctx)


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
def test_thermal_field_matches_oracle_philox(prec):
    """Brown field alone: the same Philox words on both sides (any differing
    bit of the 128-bit output would change eta by O(1))."""
    import paper_2608_15253_amd as mmx
    case = Case((24, 10, 2), (4e-9, 4e-9, 4e-9), R=3, alpha=0.02, T=300.0,
                seeds=list(replica_seeds(3, 3)), terms=("thermal",))
    ctx = open_ctx(case, prec)
    try:
        m0 = _mm(case, seed=2)
        md = dev(m0, prec)
        H = dev(np.zeros_like(m0), prec)
        for step, dt in ((0, 1e-14), (12345, 1e-14), (2 ** 33 + 5, 3e-13)):
            mmx.mmx_field(ctx, md, H, step, dt)
            got = host(H)
            ref = ofl.thermal_field(case.grid, case.material(), dt, np.array(case.seeds), step)
            err = np.abs(got - ref).max() / np.abs(ref).max()
            assert err <= (1e-12 if prec == 2 else 2e-6), (step, err)
    finally:
        mmx.mmx_destroy(ctx)


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
@pytest.mark.parametrize("name", ["film_open_32x32", "block_open_6x5x3", "film_96x24x2_radix3"])
def test_tile_choice_does_not_change_results(name, prec):
    """Rows per x workgroup and columns per y/z workgroup only regroup
    independent transforms: the field must be bit-identical for every tile
    choice, including the autotuner's."""
    import paper_2608_15253_amd as mmx
    case = CASES[name]
    m0 = _mm(case, seed=5)
    ctx = open_ctx(case, prec)
    try:
        md = dev(m0, prec)
        H = dev(np.zeros_like(m0), prec)
        mmx.mmx_field(ctx, md, H)
        ref = host(H)
        ny, Kx = case.n[1], case.n[0] + 1
        for tiles in [(1, 1, 1), (min(2, ny), min(3, Kx), 2), (ny, min(16, Kx), 1)]:
            try:
                mmx.mmx_set_tiles(ctx, 0, tiles)
            except mmx.MMXError:
                continue  # over the LDS budget for this precision
            assert mmx.mmx_get_tiles(ctx, 0) == tuple(tiles)
            mmx.mmx_field(ctx, md, H)
            assert np.array_equal(host(H), ref), tiles
        mmx.mmx_autotune(ctx)
        mmx.mmx_field(ctx, md, H)
        assert np.array_equal(host(H), ref), mmx.mmx_get_tiles(ctx, 0)
        with pytest.raises(mmx.MMXError):
            mmx.mmx_set_tiles(ctx, 0, (0, 1, 1))
    finally:
        mmx.mmx_destroy(ctx)
