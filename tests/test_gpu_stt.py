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


def _sweep_ctx(J, T, seeds):
    """The sweep's macrospins: 10 nm cubes, Ms 1.1e6 A/m, Ku 5e5 J/m^3 along
    z (K V / kB T = 121 at 300 K), alpha 0.05, fixed layer p = +z, P 0.6,
    Lambda 1, one current density per replica."""
    import torch
    import paper_2608_15253_amd as mmx
    R = len(J)
    ctx = mmx.mmx_create([mmx.make_group((1, 1, 1), (10e-9,) * 3, replicas=R)], mmx.MMX_F32)
    mmx.mmx_set_stream(ctx, torch.cuda.current_stream().cuda_stream)
    mmx.mmx_set_material(ctx, 0, Ms=1.1e6, A=0.0, alpha=0.05, Ku=5e5, u=(0, 0, 1), D=0.0)
    terms = mmx.MMX_ANIS_UNIAXIAL | mmx.MMX_STT
    if T > 0:
        mmx.mmx_set_thermal(ctx, 0, [T] * R, seeds)
        terms |= mmx.MMX_THERMAL
    mmx.mmx_set_stt(ctx, 0, J, p=(0, 0, 1), P=0.6, Lambda=1.0, eps_prime=0.0)
    mmx.mmx_set_terms(ctx, terms)
    return ctx


def _jc0():
    """T = 0 instability threshold of the sweep's macrospin (p along the easy
    axis): J_c0 = alpha mu0 H_K e Ms d / (hbar P / 2)."""
    from oracle.constants import HBAR, MU0, QE
    Ms, Ku, alpha, d, P = 1.1e6, 5e5, 0.05, 10e-9, 0.6
    return alpha * (2 * Ku / Ms) * QE * Ms * d / (HBAR * P / 2)


def test_instability_threshold_at_zero_temperature():
    """J_c0 of the sweep (the current the switching probability is normalised
    by) as the GPU run shows it: at T = 0 a macrospin tilted by 0.05 rad from
    +z relaxes back at 0.95 J_c0 and reverses at 1.05 J_c0 within 20 ns."""
    import torch
    import paper_2608_15253_amd as mmx
    jc0 = _jc0()
    J = [0.95 * jc0, 1.05 * jc0]
    ctx = _sweep_ctx(J, 0.0, None)
    try:
        th = 0.05
        m = torch.tensor([[np.sin(th), 0.0, np.cos(th)]] * 2, dtype=torch.float32, device="cuda:0")
        mmx.mmx_depondt(ctx, m, 1e-13, 200000, 0)
        mv = m.double().cpu().numpy()
    finally:
        mmx.mmx_destroy(ctx)
    # the tilt as the transverse component: in FP32 m_z near the pole moves by
    # about one rounding unit per step, the transverse part resolves the decay
    tilt = np.hypot(mv[:, 0], mv[:, 1])
    print(f"[case] transverse |m| {tilt}, m_z {mv[:, 2]} after 20 ns")
    assert tilt[0] < 0.01           # below threshold the tilt decays (linear theory: 2e-5)
    assert abs(np.linalg.norm(mv[0]) - 1) < 1e-5   # the FP32 rotation keeps |m| = 1
    assert mv[1, 2] < -0.9          # above it the macrospin reverses


def test_switching_probability_against_neel_brown_sun():
    """The finite-window switching probability of the batched thermal sweep
    against the Neel-Brown law with Sun's barrier reduction (Results,
    replica-batched STT switching sweep): 9 currents J / J_c0 in 0.80 .. 1.20,
    256 trials each, 2 ns of rotation steps at 300 K.  Delta = K V / kB T;
    f0 (not printed in the paper) read as Brown's high-barrier attempt
    frequency of a uniaxial macrospin, alpha / (1 + alpha^2) gamma0 mu0 H_K
    sqrt(Delta / pi).  Like the paper's batched sweep, the simulation follows
    the law's sigmoid but reaches P = 1/2 at a higher current than the law
    (whose linearised barrier is least accurate near J_c0), below J_c0.  Above
    J_c0 the law (no barrier) gives P = 1 - exp(-t f0), about 1, while the
    simulated switching still takes a finite time near the threshold: only
    P -> 1 towards 1.2 J_c0 is asserted there."""
    import torch
    import paper_2608_15253_amd as mmx
    from oracle.constants import GAMMA0, KB
    from oracle.observables import switching_probability_neel_brown_sun as law
    jc0 = _jc0()
    ratios = np.linspace(0.80, 1.20, 9)
    per = 256
    R = len(ratios) * per
    J = np.repeat(ratios * jc0, per)
    ctx = _sweep_ctx(J, 300.0, list(replica_seeds(23, R)))
    try:
        m = torch.zeros((R, 3), dtype=torch.float32, device="cuda:0")
        m[:, 2] = 1.0
        tsw = torch.full((R,), -1.0, dtype=torch.float64, device="cuda:0")
        mmx.mmx_depondt(ctx, m, 1e-13, 20000, 0, tsw)
        p = (tsw.view(len(ratios), per) > 0).double().mean(dim=1).cpu().numpy()
    finally:
        mmx.mmx_destroy(ctx)
    Ms, Ku, alpha, V = 1.1e6, 5e5, 0.05, 1e-24
    delta = Ku * V / (KB * 300.0)
    f0 = alpha / (1 + alpha ** 2) * GAMMA0 * (2 * Ku / Ms) * np.sqrt(delta / np.pi)
    pth = law(ratios, 2e-9, f0, delta)
    sig = np.sqrt(np.maximum(p * (1 - p), 1.0 / per) / per)
    # where P crosses 1/2 (linear interpolation between the sampled currents)
    def half(pp):
        k = int(np.argmax(pp >= 0.5))
        return ratios[k - 1] + (0.5 - pp[k - 1]) / (pp[k] - pp[k - 1]) * (ratios[k] - ratios[k - 1])
    js, jt = half(p), half(pth)
    print(f"[case] P_sw {np.round(p, 3)}; law {np.round(pth, 3)}; half at {js:.3f} (law {jt:.3f})")
    assert np.all(np.diff(p) >= -3 * np.sqrt(sig[1:] ** 2 + sig[:-1] ** 2))  # sigmoid, rising
    assert p[0] <= 0.1 and p[-1] >= 0.95
    assert jt < js < 1.0
