"""GPU parity of the norm-exact Depondt-Mertens rotation scheme and of the
retire/refill trials through the C ABI against the FP64 oracle (Results, "A
replica-batched engine"; Methods, "Integrators" and "Replica batching").

Bars: FP64 max |dm| <= 1e-12, FP32 <= 1e-5; |m| = 1 to round-off without
normalisation; batched versus per-trial runs, split runs and graph replays
bit-identical; recorded trial lengths and counts equal to the oracle's.
"""
import math

import numpy as np
import pytest

from oracle import rotation as orot
from workloads import random_unit, replica_seeds, uniform

from _mmx_case import Case, dev, host, open_ctx

pytestmark = pytest.mark.gpu

TOLM = {2: 1e-12, 1: 1e-5}


def _round(m, prec):
    return m.astype(np.float32).astype(np.float64) if prec == 1 else m


def _film(n, R, seed_base, alpha=0.02, T=300.0, B=(0, 0, -0.15)):
    return Case(n, (4e-9, 4e-9, 4e-9), R=R, alpha=alpha, Ku=5e5, B=B, T=T,
                seeds=list(replica_seeds(seed_base, R)),
                terms=("exchange", "anisotropy", "zeeman", "demag", "thermal"))


@pytest.mark.parametrize("prec,n", [(2, (24, 20, 1)), (1, (24, 20, 1)), (1, (64, 64, 1))],
                         ids=["f64-24x20", "f32-24x20", "f32-64x64"])
def test_rotation_thermal_batch_matches_oracle(prec, n):
    """Thermal films (the 64 x 64 film takes the register row kernels)."""
    import paper_2608_15253_amd as mmx
    case = _film(n, 2, 21)
    print(f"[case] depondt {n} prec={prec}", flush=True)
    m0 = _round(random_unit(case.n, seed=6, replicas=case.R), prec)
    steps = 20 if n[0] == 64 else 30
    ctx = open_ctx(case, prec)
    try:
        md = dev(m0, prec)
        mmx.mmx_depondt(ctx, md, 1e-14, steps, 50)
        got = host(md)
    finally:
        mmx.mmx_destroy(ctx)
    ref = orot.depondt_run(m0, case.grid, case.material(), 1e-14, steps,
                           seed=np.array(case.seeds), step0=50)
    err = np.abs(got - ref).max()
    print(f"max |dm| {err:.2e}")
    assert err <= TOLM[prec], err


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
def test_rotation_keeps_unit_norm_without_normalisation(prec):
    import paper_2608_15253_amd as mmx
    case = _film((32, 16, 1), 2, 22, alpha=0.5, B=(0, 0, 0.1))
    m0 = _round(random_unit(case.n, seed=7, replicas=case.R), prec)
    if prec == 1:  # start from unit vectors in FP32 arithmetic
        m0 = (m0 / np.linalg.norm(m0, axis=1, keepdims=True)).astype(np.float32).astype(np.float64)
    n0 = np.abs(np.linalg.norm(m0, axis=1) - 1).max()
    ctx = open_ctx(case, prec)
    try:
        md = dev(m0, prec)
        mmx.mmx_depondt(ctx, md, 1e-13, 1000, 0)
        got = host(md)
    finally:
        mmx.mmx_destroy(ctx)
    drift = np.abs(np.linalg.norm(got, axis=1) - 1).max()
    print(f"|m| drift after 1000 steps: {drift:.2e} (start {n0:.1e})")
    assert drift <= (1e-13 if prec == 2 else 2e-5)


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
def test_rotation_batched_split_and_graph_runs_are_bitwise(prec):
    """R replicas in one launch equal single-replica contexts; 70 steps in
    one call (a captured 32-step graph replayed twice, then 6 eager steps)
    equal 7 calls of 10 eager steps with the step index carried along."""
    import paper_2608_15253_amd as mmx
    R = 3
    case = _film((64, 64, 1), R, 23, alpha=0.1, B=(0, 0, -0.3))
    m0 = _round(uniform(case.n, (0.1, 0.0, 1.0), replicas=R), prec)
    ctx = open_ctx(case, prec)
    try:
        md = dev(m0, prec)
        ts = dev(-np.ones(R), 2)
        mmx.mmx_depondt(ctx, md, 1e-13, 70, 0, ts)
        one, tone = host(md), host(ts)
        md = dev(m0, prec)
        ts = dev(-np.ones(R), 2)
        for k in range(7):
            mmx.mmx_depondt(ctx, md, 1e-13, 10, 10 * k, ts)
        split, tsplit = host(md), host(ts)
    finally:
        mmx.mmx_destroy(ctx)
    assert np.array_equal(one, split) and np.array_equal(tone, tsplit)
    for r in range(R):
        c1 = _film((64, 64, 1), 1, 23, alpha=0.1, B=(0, 0, -0.3))
        c1.seeds = [case.seeds[r]]
        ctx = open_ctx(c1, prec)
        try:
            md = dev(m0[r:r + 1], prec)
            mmx.mmx_depondt(ctx, md, 1e-13, 70, 0)
            single = host(md)
        finally:
            mmx.mmx_destroy(ctx)
        assert np.array_equal(single[0], one[r])


def _refill_case(R, T):
    return Case((16, 16, 1), (4e-9, 4e-9, 4e-9), R=R, alpha=0.5, Ku=5e5, B=(0, 0, -1.0), T=T,
                seeds=list(replica_seeds(31, R)),
                terms=("exchange", "anisotropy", "zeeman", "demag", "thermal"))


def test_refill_trials_match_oracle_fp64():
    """Thermal retire/refill: per slot the recorded trial lengths, the number
    of finished trials and the final state equal the oracle's, which runs each
    trial as a standalone run with its own noise generation."""
    import paper_2608_15253_amd as mmx
    R, cap, nsteps, dt = 3, 3, 1500, 1e-13
    case = _refill_case(R, 300.0)
    th = 0.3
    m_init = uniform(case.n, (math.sin(th), 0.0, math.cos(th)), replicas=R)
    ctx = open_ctx(case, 2)
    try:
        md = dev(m_init, 2)
        mi = dev(m_init, 2)
        times = dev(np.zeros(R * cap), 2)
        import torch
        counts = torch.zeros(R, dtype=torch.int32, device="cuda:0")
        mmx.mmx_depondt_refill(ctx, md, mi, dt, nsteps, times, cap, counts)
        got_m, got_t = host(md), host(times).reshape(R, cap)
        got_c = counts.cpu().numpy()
        assert np.array_equal(host(mi), m_init)
    finally:
        mmx.mmx_destroy(ctx)
    grid, mat = case.grid, case.material()
    for r in range(R):
        times_r, done, m_r, _, _, margins = orot.refill_slot(m_init[r], grid, mat, dt, nsteps,
                                                              case.seeds[r], cap)
        assert min(abs(x) for x in margins) > 1e-9  # no decision within round-off
        print(f"slot {r}: {done} trials, times {times_r}")
        assert done >= 2
        assert got_c[r] == done
        ref_t = np.full(cap, -1.0)
        ref_t[:len(times_r)] = times_r
        assert np.array_equal(got_t[r], ref_t)
        assert np.abs(got_m[r] - m_r).max() <= 1e-12


def test_refill_fp32_zero_temperature_repeats_the_switching_time():
    """T = 0 in FP32 on the register row kernels: every trial repeats the plain
    run's switching time, bit for bit, and the slot restarts from m_init."""
    import paper_2608_15253_amd as mmx
    import torch
    R, cap, dt = 2, 8, 1e-13
    case = _refill_case(R, 0.0)
    case.terms = ("exchange", "anisotropy", "zeeman", "demag")
    th = 0.3
    m_init = _round(uniform(case.n, (math.sin(th), 0.0, math.cos(th)), replicas=R), 1)
    ctx = open_ctx(case, 1)
    try:
        md = dev(m_init, 1)
        ts = dev(-np.ones(R), 2)
        mmx.mmx_depondt(ctx, md, dt, 1000, 0, ts)
        tsw = host(ts)
        assert np.all(tsw > 0) and tsw[0] == tsw[1]
        s_star = int(round(tsw[0] / dt))
        nsteps = 3 * s_star + 5
        md = dev(m_init, 1)
        times = dev(np.zeros(R * cap), 2)
        counts = torch.zeros(R, dtype=torch.int32, device="cuda:0")
        mmx.mmx_depondt_refill(ctx, md, dev(m_init, 1), dt, nsteps, times, cap, counts)
        got_t, got_c, got_m = host(times).reshape(R, cap), counts.cpu().numpy(), host(md)
        md = dev(m_init, 1)
        mmx.mmx_depondt(ctx, md, dt, 5, 0)
        five = host(md)
    finally:
        mmx.mmx_destroy(ctx)
    assert np.array_equal(got_c, [3, 3])
    assert np.all(got_t[:, :3] == s_star * dt) and np.all(got_t[:, 3:] == -1)
    assert np.array_equal(got_m, five)


def test_refill_single_cell_resident_path_fp64():
    """Retire/refill on single-cell replicas runs in one thread per replica;
    its trial lengths and counts equal the oracle's (sampled slots) and the
    staged field-kernel path's."""
    import paper_2608_15253_amd as mmx
    import torch
    R, cap, nsteps, dt = 64, 6, 3000, 1e-13
    case = Case((1, 1, 1), (4e-9, 4e-9, 4e-9), R=R, A=0.0, alpha=0.2, Ku=2e5, B=(0, 0, -1.0),
                T=300.0, seeds=list(replica_seeds(33, R)), terms=("anisotropy", "zeeman", "thermal"))
    th = 0.3
    m_init = uniform(case.n, (math.sin(th), 0.0, math.cos(th)), replicas=R)
    out = {}
    for path in (mmx.MMX_PATH_AUTO, mmx.MMX_PATH_STAGED):
        ctx = open_ctx(case, 2)
        try:
            mmx.mmx_set_path(ctx, path)
            md = dev(m_init, 2)
            times = dev(np.zeros(R * cap), 2)
            counts = torch.zeros(R, dtype=torch.int32, device="cuda:0")
            mmx.mmx_depondt_refill(ctx, md, dev(m_init, 2), dt, nsteps, times, cap, counts)
            out[path] = (host(md), host(times).reshape(R, cap), counts.cpu().numpy())
        finally:
            mmx.mmx_destroy(ctx)
    a, b = out[mmx.MMX_PATH_AUTO], out[mmx.MMX_PATH_STAGED]
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[1], b[1])
    assert np.abs(a[0] - b[0]).max() <= 1e-12
    assert a[2].min() >= 2
    for r in (0, 37):
        times_r, done, m_r, _, _, margins = orot.refill_slot(m_init[r], case.grid, case.material(),
                                                              dt, nsteps, case.seeds[r], cap)
        assert min(abs(x) for x in margins) > 1e-9
        assert a[2][r] == done
        ref_t = np.full(cap, -1.0)
        ref_t[:len(times_r)] = times_r
        assert np.array_equal(a[1][r], ref_t)
        assert np.abs(a[0][r] - m_r).max() <= 1e-12
