"""GPU tests of RK45 with learned demag stages (mmx_rk45_surrogate) and of the
training pipeline, through the C ABI, against the FP64 oracle and the plain
integrator."""
import math

import numpy as np
import pytest

from oracle import fno as ofno
from oracle import integrators as oit
from oracle import surrogate as osg
from workloads import neel_skyrmions, random_unit
from _mmx_case import Case, open_ctx, dev, host
from test_gpu_fno import pack, _params

pytestmark = pytest.mark.gpu

# film 32 x 24 (nx x ny): the network grid is H = 24, W = 32
CASE = Case(n=(32, 24, 1), cell=(4e-9, 4e-9, 4e-9), R=2, Ms=8e5, A=1.3e-11, alpha=0.3,
            Ku=6e5, D=3e-3, B=(0.0, 0.0, 0.1))
NET = dict(C=8, M1=4, M2=3, L=2, Cp=16)


def _net(seed=3):
    import torch
    import paper_2608_15253_amd as mmx
    p = _params(NET["C"], NET["M1"], NET["M2"], NET["L"], NET["Cp"], seed)
    f = mmx.mmx_fno_create(CASE.n[1], CASE.n[0], NET["C"], NET["M1"], NET["M2"], NET["L"],
                           NET["Cp"], CASE.R, False)
    prm = torch.tensor(pack(p, NET["L"]), dtype=torch.float32, device="cuda:0")
    assert prm.numel() == mmx.mmx_fno_param_count(f)
    return p, f, prm


def _m0():
    m, _, _ = neel_skyrmions(CASE.n, CASE.cell, 1, 12e-9, 16e-9, seed=21, width=4e-9,
                             periodic=False)
    r = random_unit(CASE.n, seed=22)
    m2 = m + 0.3 * r
    m2 /= np.linalg.norm(m2, axis=0, keepdims=True)
    return np.stack([m, m2])


def test_one_learned_step_matches_oracle_and_gate_value():
    """One accepted step (tol 1, dt = t_end): stages 2-6 from the FP32 network,
    stage 7 exact; the gate value is the oracle's at the new state."""
    import paper_2608_15253_amd as mmx
    p, f, prm = _net()
    ctx = open_ctx(CASE, mmx.MMX_F32)
    try:
        m0 = _m0()
        m = dev(m0, mmx.MMX_F32)
        dt = 1e-13
        st, gl = mmx.mmx_rk45_surrogate(ctx, f, prm, m, 0.0, dt, 1.0, dt0=dt,
                                        gate_tol=math.inf, gate_cap=8)
        got = host(m)
    finally:
        mmx.mmx_destroy(ctx)
        mmx.mmx_fno_destroy(f)
    assert st.accepted == 1 and st.surrogate_steps == 1 and st.exact_steps == 0
    assert st.gate_checks == 1 and st.gate_failures == 0
    grid, mat = CASE.grid, CASE.material()
    M1, M2 = NET["M1"], NET["M2"]
    demag_fn = lambda ms: osg.network_demag(p, ms, CASE.Ms, M1, M2, residual_mz=True)
    k1 = oit.rhs(m0, grid, mat)
    m7, _, _ = osg.attempt(m0, k1, grid, mat, dt, demag_fn)
    assert np.max(np.abs(got - m7)) <= 1e-5
    g_ref = osg.gate_error(demag_fn(m7), osg.exact_demag(m7, grid, CASE.Ms)).max()
    assert abs(gl[0] - g_ref) <= 1e-3 * g_ref


@pytest.mark.parametrize("exact_after", [0, 3, 10])
def test_forced_fallback_equals_plain_rk45_bitwise(exact_after):
    """gate_tol = 0: no learned step is kept, every step is the plain one."""
    import torch
    import paper_2608_15253_amd as mmx
    _, f, prm = _net()
    ctx = open_ctx(CASE, mmx.MMX_F32)
    try:
        m0 = _m0()
        ma, mb = dev(m0, mmx.MMX_F32), dev(m0, mmx.MMX_F32)
        t_end, tol = 3e-12, 1e-4
        sp = mmx.mmx_rk45(ctx, ma, 0.0, t_end, tol)
        st, gl = mmx.mmx_rk45_surrogate(ctx, f, prm, mb, 0.0, t_end, tol, gate_tol=0.0,
                                        exact_after_fail=exact_after, gate_cap=1000)
        torch.cuda.synchronize()
        assert torch.equal(ma, mb)
    finally:
        mmx.mmx_destroy(ctx)
        mmx.mmx_fno_destroy(f)
    assert sp.accepted >= 5
    assert st.surrogate_steps == 0
    assert st.accepted == sp.accepted and st.rejected == sp.rejected
    assert st.exact_steps == st.accepted
    assert st.gate_failures == st.gate_checks == len(gl)
    assert all(g > 0 for g in gl)
    assert st.t == sp.t


def test_always_kept_run_is_consistent():
    """gate_tol = inf: every accepted network attempt is kept."""
    import torch
    import paper_2608_15253_amd as mmx
    _, f, prm = _net(seed=5)
    ctx = open_ctx(CASE, mmx.MMX_F32)
    try:
        m = dev(_m0(), mmx.MMX_F32)
        st, gl = mmx.mmx_rk45_surrogate(ctx, f, prm, m, 0.0, 2e-12, 1e-3, gate_tol=math.inf,
                                        gate_cap=1000)
        torch.cuda.synchronize()
        got = host(m)
    finally:
        mmx.mmx_destroy(ctx)
        mmx.mmx_fno_destroy(f)
    assert np.all(np.isfinite(got))
    assert np.max(np.abs(np.linalg.norm(got, axis=1) - 1.0)) < 1e-5
    assert st.gate_failures == 0 and st.gate_checks == st.surrogate_steps == len(gl)
    assert st.surrogate_steps + st.exact_steps == st.accepted
    assert st.exact_steps <= st.surrogate_rejected
    assert abs(st.t - 2e-12) < 1e-24


def test_argument_errors():
    import paper_2608_15253_amd as mmx
    _, f, prm = _net()
    ctx = open_ctx(CASE, mmx.MMX_F32)
    try:
        m = dev(_m0(), mmx.MMX_F32)
        with pytest.raises(mmx.MMXError):
            mmx.mmx_rk45_surrogate(ctx, f, prm, m, 0.0, 1e-12, 1e-4, gate_tol=-1.0)
    finally:
        mmx.mmx_destroy(ctx)
        mmx.mmx_fno_destroy(f)
    wrong = Case(n=(24, 32, 1), cell=CASE.cell, R=2)   # transposed grid
    ctx = open_ctx(wrong, mmx.MMX_F32)
    _, f, prm = _net()
    try:
        m = dev(random_unit(wrong.n, seed=1, replicas=2), mmx.MMX_F32)
        with pytest.raises(mmx.MMXError) as e:
            mmx.mmx_rk45_surrogate(ctx, f, prm, m, 0.0, 1e-12, 1e-4)
        assert e.value.status == -2
    finally:
        mmx.mmx_destroy(ctx)
        mmx.mmx_fno_destroy(f)


def test_training_pipeline_reduces_the_loss_and_labels_match_oracle():
    """Data from the method (Heun trajectories, exact-demag labels), then Adam
    steps with the library's network kernels lower the validation loss."""
    import torch
    from paper_2608_15253_amd import surrogate as sg
    n = (32, 24, 1)
    m_all, t_all = sg.generate(n, snapshots=96, replicas=16, every=20, log=lambda s: None)
    # labels: residual target of the exact field, checked on two snapshots
    grid = CASE.grid
    for s in (0, 95):
        m = m_all[s].double().cpu().numpy()[None, :, None]
        H = osg.exact_demag(m, grid, sg.MS)[0, :, 0] / sg.MS
        H[2] += m[0, 2, 0]
        t = t_all[s].double().cpu().numpy()
        assert np.linalg.norm(t - H) <= 1e-5 * np.linalg.norm(H)
    net = sg.Net(24, 32, C=8, M1=4, M2=3, L=2, Cp=16, batch=16, use_mfma=True, seed=2)
    try:
        l0, _ = sg.evaluate(net, m_all, t_all, 80, 96)
        sg.train(net, m_all, t_all, 80, epochs=20, lr0=3e-3, log=lambda s: None)
        l1, gate = sg.evaluate(net, m_all, t_all, 80, 96)
    finally:
        net.close()
    assert np.isfinite(l1) and l1 < 0.8 * l0
    assert gate.shape == (16,)


def test_gain_of_a_trained_network_over_plain_rk45():
    """What a trained network gains: data from the method, a briefly trained
    network, then held-out relaxations with plain FP32 RK45 and with learned
    stages (gate 1e-3), both against an FP64 RK45 reference.  The gated run
    keeps the plain run's accuracy (every kept learned step passed the exact
    gate, failures fall back to exact steps); the speed ratio is measured and
    reported, not assumed (at these sizes the exact pruned FFT convolution is
    cheaper than one network forward, so no gain is expected)."""
    from paper_2608_15253_amd import surrogate as sg
    n = (32, 24, 1)
    m_all, t_all = sg.generate(n, snapshots=128, replicas=16, every=20, log=lambda s: None)
    net = sg.Net(24, 32, C=8, M1=4, M2=3, L=2, Cp=16, batch=16, use_mfma=True, seed=3)
    try:
        sg.train(net, m_all, t_all, 112, epochs=30, lr0=3e-3, log=lambda s: None)
        rep = sg.speedup(net, n=n, R=8, t_end=2e-11, tol=1e-5, gates=(1e-3,),
                         log=lambda s: None)
    finally:
        net.close()
    plain, run = rep["plain"], rep["learned"][0]
    print(f"plain {plain['seconds']:.3f} s |dm| {plain['dm']:.2e}; learned {run['seconds']:.3f} s "
          f"(x{run['speedup']:.3f}) |dm| {run['dm']:.2e}, kept {run['surrogate_steps']}/"
          f"{run['accepted']}, gate failures {run['gate_failures']}/{run['gate_checks']}")
    assert np.isfinite(run["dm"]) and run["speedup"] > 0
    assert run["dm"] <= 10 * plain["dm"] + 1e-5
    # the network was tried: its attempts were gated or rejected by the
    # controller (then repeated with the exact field)
    assert run["gate_checks"] + run["surrogate_rejected"] >= 1
