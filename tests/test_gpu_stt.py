"""GPU parity of the Slonczewski spin-transfer torque with per-replica current
density through the C ABI against the FP64 oracle (Methods, "Physics and
discretization": spin torques added per integrator stage; Results, the
replica-batched STT switching sweep): the torque itself, Heun, the rotation
scheme and RK45 with the torque on.

Bars: FP64 max |dm| <= 1e-12, FP32 <= 1e-5 (torques relative to their
maximum: 1e-12 / 4e-6).
"""
import dataclasses

import numpy as np
import pytest

from oracle import integrators as oit
from oracle import llg as ollg
from oracle import rotation as orot
from workloads import random_unit, replica_seeds, uniform

from _mmx_case import Case, dev, host, open_ctx

pytestmark = pytest.mark.gpu

TOLM = {2: 1e-12, 1: 1e-5}
STT = dict(p=(0.2, -0.1, 1.0), P=0.55, Lambda=1.7, eps_prime=0.2)


def _round(m, prec):
    return m.astype(np.float32).astype(np.float64) if prec == 1 else m


def _with_stt(ctx, case, J):
    import paper_2608_15253_amd as mmx
    mmx.mmx_set_stt(ctx, 0, J, **STT)
    mmx.mmx_set_terms(ctx, case.mask() | mmx.MMX_STT)


def _oracle_material(case, J):
    return dataclasses.replace(case.material(), stt_J=tuple(J), stt_p=STT["p"], stt_P=STT["P"],
                               stt_lambda=STT["Lambda"], stt_eps2=STT["eps_prime"])


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
def test_stt_torque_matches_oracle(prec):
    import paper_2608_15253_amd as mmx
    case = Case((16, 8, 2), (4e-9, 4e-9, 2e-9), R=3, alpha=0.1, Ku=2e5, B=(0.01, 0, 0.05),
                terms=("exchange", "anisotropy", "zeeman", "demag"))
    J = (0.0, 2e11, -5e11)
    m0 = _round(random_unit(case.n, seed=12, replicas=case.R), prec)
    ctx = open_ctx(case, prec)
    try:
        k0 = dev(np.zeros_like(m0), prec)
        mmx.mmx_torque(ctx, dev(m0, prec), k0)
        _with_stt(ctx, case, J)
        k = dev(np.zeros_like(m0), prec)
        mmx.mmx_torque(ctx, dev(m0, prec), k)
        got, got0 = host(k), host(k0)
    finally:
        mmx.mmx_destroy(ctx)
    mat = _oracle_material(case, J)
    ref = oit.rhs(m0, case.grid, mat)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err <= (1e-12 if prec == 2 else 4e-6), err
    # the spin-transfer part alone (with-minus-without on the GPU)
    tau = ollg.stt_torque(m0, mat, case.grid.n[2] * case.grid.cell[2])
    assert not np.any(tau[0]) and np.array_equal(got[0], got0[0])  # J = 0 replica
    e2 = np.abs((got - got0) - tau).max() / np.abs(tau).max()
    assert e2 <= (1e-9 if prec == 2 else 2e-3), e2


@pytest.mark.parametrize("scheme,prec,n", [("heun", 2, (20, 12, 1)), ("heun", 1, (20, 12, 1)),
                                           ("rotation", 2, (20, 12, 1)),
                                           ("rotation", 1, (64, 64, 1)),
                                           ("heun", 1, (64, 64, 1))],
                         ids=["heun-f64", "heun-f32", "rot-f64", "rot-f32-64x64",
                              "heun-f32-64x64"])
def test_stt_thermal_steps_match_oracle(scheme, prec, n):
    """Thermal steps with a current density per replica (the 64 x 64 films take
    the register row kernels)."""
    import paper_2608_15253_amd as mmx
    R = 3
    case = Case(n, (4e-9, 4e-9, 2e-9), R=R, alpha=0.05, Ku=4e5, B=(0, 0, -0.05), T=300.0,
                seeds=list(replica_seeds(41, R)),
                terms=("exchange", "anisotropy", "zeeman", "demag", "thermal"))
    J = (1e11, -3e11, 6e11)
    m0 = _round(uniform(case.n, (0.2, 0.1, 1.0), replicas=R), prec)
    steps = 20
    print(f"[case] stt {scheme} {n} prec={prec}", flush=True)
    ctx = open_ctx(case, prec)
    try:
        _with_stt(ctx, case, J)
        md = dev(m0, prec)
        step = mmx.mmx_heun if scheme == "heun" else mmx.mmx_depondt
        step(ctx, md, 1e-14, steps, 7)
        got = host(md)
    finally:
        mmx.mmx_destroy(ctx)
    mat = _oracle_material(case, J)
    run = oit.heun_run if scheme == "heun" else orot.depondt_run
    ref = run(m0, case.grid, mat, 1e-14, steps, seed=np.array(case.seeds), step0=7)
    moved = np.abs(ref - m0).max()
    err = np.abs(got - ref).max()
    print(f"max |dm| {err:.2e} (state moved by {moved:.2e})")
    assert err <= TOLM[prec], err


def test_stt_rk45_takes_the_oracle_steps_fp64():
    import paper_2608_15253_amd as mmx
    case = Case((8, 8, 1), (5e-9, 5e-9, 2e-9), R=1, alpha=0.05, Ku=3e5, B=(0, 0, 0.0),
                terms=("exchange", "anisotropy", "demag"))
    J = (8e11,)
    m0 = uniform(case.n, (0.3, 0.0, 1.0), replicas=1)
    t_end, tol = 2e-11, 1e-7
    ctx = open_ctx(case, 2)
    try:
        _with_stt(ctx, case, J)
        md = dev(m0, 2)
        st = mmx.mmx_rk45(ctx, md, 0.0, t_end, tol, 1e-13)
        got = host(md)
        dts = mmx.mmx_rk45_dts(ctx)
    finally:
        mmx.mmx_destroy(ctx)
    mat = _oracle_material(case, J)
    rep = oit.rk45_run(m0[0], case.grid, mat, 0.0, t_end, tol, dt_replay=dts)
    assert st.t == t_end
    assert np.abs(got[0] - rep.m).max() <= 1e-12
    own = oit.rk45_run(m0[0], case.grid, mat, 0.0, t_end, tol, 1e-13)
    assert abs(own.accepted - st.accepted) <= 2


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
def test_stt_thermal_macrospins_rotation(prec):
    """Single-cell macrospins with one current density each (the sweep's
    replicas), rotation scheme, 200 thermal steps."""
    import paper_2608_15253_amd as mmx
    R = 4
    case = Case((1, 1, 1), (10e-9, 10e-9, 10e-9), R=R, Ms=1.1e6, A=0.0, alpha=0.05, Ku=5e5,
                T=300.0, seeds=list(replica_seeds(43, R)), terms=("anisotropy", "thermal"))
    J = (0.0, 1e12, 2.6e12, 4e12)
    m0 = uniform(case.n, (0.05, 0.0, 1.0), replicas=R)
    ctx = open_ctx(case, prec)
    try:
        _with_stt(ctx, case, J)
        md = dev(m0, prec)
        mmx.mmx_depondt(ctx, md, 1e-13, 200, 0)
        got = host(md)
    finally:
        mmx.mmx_destroy(ctx)
    ref = orot.depondt_run(m0, case.grid, _oracle_material(case, J), 1e-13, 200,
                           seed=np.array(case.seeds))
    err = np.abs(got - ref).max()
    print(f"max |dm| {err:.2e}")
    assert err <= (1e-12 if prec == 2 else 2e-5), err


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
@pytest.mark.parametrize("scheme", ["heun", "rotation"])
def test_single_cell_resident_path_equals_staged_path_bitwise(prec, scheme):
    """Single-cell groups without demag run every step of a replica in one
    thread; the result equals the staged field-kernel path (400 steps: the
    staged path replays a captured graph) to round-off (the two kernels may
    contract multiply-adds differently) and the switching times agree."""
    import paper_2608_15253_amd as mmx
    R = 300
    case = Case((1, 1, 1), (10e-9, 10e-9, 10e-9), R=R, Ms=1.1e6, A=0.0, alpha=0.5, Ku=5e5,
                B=(0.0, 0.0, -3.0), T=300.0, seeds=list(replica_seeds(44, R)),
                terms=("anisotropy", "zeeman", "thermal"))
    J = np.linspace(0.0, 6e12, R)
    m0 = uniform(case.n, (0.1, 0.0, 1.0), replicas=R)
    out = {}
    for path in (mmx.MMX_PATH_AUTO, mmx.MMX_PATH_STAGED):
        ctx = open_ctx(case, prec)
        try:
            _with_stt(ctx, case, J)
            mmx.mmx_set_path(ctx, path)
            md = dev(m0, prec)
            ts = dev(-np.ones(R), 2)
            step = mmx.mmx_heun if scheme == "heun" else mmx.mmx_depondt
            step(ctx, md, 1e-13, 400, 3, ts)
            out[path] = (host(md), host(ts))
        finally:
            mmx.mmx_destroy(ctx)
    a, b = out[mmx.MMX_PATH_AUTO], out[mmx.MMX_PATH_STAGED]
    err = np.abs(a[0] - b[0]).max()
    print(f"resident vs staged: max |dm| {err:.2e}")
    assert err <= (1e-12 if prec == 2 else 1e-5)
    assert (a[1] > 0).sum() > R // 10  # many replicas switched
    same = a[1] == b[1]
    assert same.mean() >= 0.99 and np.abs(a[1] - b[1]).max() <= 1.5e-13
