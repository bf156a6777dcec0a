"""The C-ABI boundary beyond the integrators (Methods, "GPU implementation":
device-resident state without per-step transfers; "Integrators"): a
caller-owned workspace (mmx_workspace_bytes / mmx_bind) gives results equal
bit for bit to the library's own allocation and no integrator call allocates
device memory; a checkpoint of an adaptive run restored into a fresh context
continues exactly as the original context does."""
import numpy as np
import pytest

from workloads import random_unit, replica_seeds, uniform

from _mmx_case import Case, dev, host, open_ctx

pytestmark = pytest.mark.gpu


def _switch_case(R):
    return Case((64, 64, 1), (4e-9, 4e-9, 4e-9), R=R, alpha=0.02, Ku=5e5, B=(0, 0, -0.15),
                T=300.0, seeds=list(replica_seeds(3, R)),
                terms=("exchange", "anisotropy", "zeeman", "demag", "thermal"))


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
def test_bound_workspace_equals_library_allocation(prec):
    import torch
    import paper_2608_15253_amd as mmx
    case = _switch_case(4)
    m0 = uniform(case.n, (0.1, 0.0, 1.0), replicas=case.R)
    stream = torch.cuda.current_stream().cuda_stream
    out = {}
    for mode in ("library", "bound_after_build", "bound_before_build", "bound_and_back"):
        print(f"[case] workspace {mode} prec={prec}", flush=True)
        grp = mmx.make_group(case.n, case.cell, replicas=case.R)
        ctx = mmx.mmx_create([grp], prec)
        ws = None
        try:
            mmx.mmx_set_stream(ctx, stream)
            nbytes = mmx.mmx_workspace_bytes(ctx)
            assert nbytes > 0
            if mode == "bound_before_build":
                ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
                mmx.mmx_bind(ctx, ws, stream)
            mmx.mmx_set_material(ctx, 0, case.Ms, case.A, case.alpha, case.Ku, case.u, case.D)
            mmx.mmx_set_field(ctx, 0, case.B)
            mmx.mmx_set_thermal(ctx, 0, [case.T] * case.R, case.seeds)
            mmx.mmx_set_terms(ctx, case.mask())
            mmx.mmx_build_demag(ctx)
            if mode in ("bound_after_build", "bound_and_back"):
                ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
                ws.fill_(0xAB)  # stale bytes: everything needed must be copied over
                mmx.mmx_bind(ctx, ws, stream)
            md = dev(m0, prec)
            ts = dev(-np.ones(case.R), 2)
            mmx.mmx_heun(ctx, md, 1e-14, 37, 0, ts)
            if mode == "bound_and_back":
                mmx.mmx_bind(ctx, None, stream)
                ws = None
            mmx.mmx_heun(ctx, md, 1e-14, 21, 37, ts)
            E = torch.zeros((case.R, 6), dtype=torch.float64, device="cuda:0")
            mmx.mmx_energy(ctx, md, E)
            out[mode] = (host(md), host(ts), host(E))
        finally:
            mmx.mmx_destroy(ctx)
    for mode in out:
        for a, b in zip(out[mode], out["library"]):
            assert np.array_equal(a, b), mode


def test_workspace_rejects_short_or_misaligned_memory():
    import torch
    import paper_2608_15253_amd as mmx
    ctx = open_ctx(_switch_case(2), mmx.MMX_F32)
    try:
        stream = torch.cuda.current_stream().cuda_stream
        n = mmx.mmx_workspace_bytes(ctx)
        short = torch.empty(n - 256, dtype=torch.uint8, device="cuda:0")
        with pytest.raises(mmx.MMXError) as e:
            mmx.mmx_bind(ctx, short, stream)
        assert e.value.status == -1
        big = torch.empty(n + 512, dtype=torch.uint8, device="cuda:0")
        with pytest.raises(mmx.MMXError) as e:
            mmx.mmx_bind(ctx, big[8:], stream)
        assert e.value.status == -1
    finally:
        mmx.mmx_destroy(ctx)


def test_integrators_allocate_nothing_after_bind():
    """1024 replicas of the 64 x 64 film (state 50 MB in FP32): after binding
    a torch workspace, Heun, RK45 (its seven stage buffers), RK4, the rotation
    scheme with retire/refill and the observables leave the device's free
    memory unchanged (within 16 MB for the runtime's graph objects)."""
    import torch
    import paper_2608_15253_amd as mmx
    case = _switch_case(1024)
    ctx = open_ctx(case, mmx.MMX_F32)
    try:
        stream = torch.cuda.current_stream().cuda_stream
        ws = torch.empty(mmx.mmx_workspace_bytes(ctx), dtype=torch.uint8, device="cuda:0")
        mmx.mmx_bind(ctx, ws, stream)
        m0 = uniform(case.n, (0.1, 0.0, 1.0), replicas=case.R)
        md = dev(m0, mmx.MMX_F32)
        m_init = md.clone()
        ts = dev(-np.ones(case.R), 2)
        times = torch.zeros(case.R * 2, dtype=torch.float64, device="cuda:0")
        counts = torch.zeros(case.R, dtype=torch.int32, device="cuda:0")
        E = torch.zeros((case.R, 6), dtype=torch.float64, device="cuda:0")
        Q = torch.zeros(case.R, dtype=torch.float64, device="cuda:0")
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        mmx.mmx_heun(ctx, md, 1e-14, 5, 0, ts)
        mmx.mmx_depondt_refill(ctx, md, m_init, 1e-14, 5, times, 2, counts)
        mmx.mmx_set_terms(ctx, case.mask(("exchange", "anisotropy", "zeeman", "demag")))
        mmx.mmx_rk45(ctx, md, 0.0, 2e-13, 1e-5)
        mmx.mmx_rk4(ctx, md, 1e-14, 2)
        mmx.mmx_energy(ctx, md, E)
        mmx.mmx_topological_charge(ctx, md, Q)
        mmx.mmx_sync(ctx)
        free1 = torch.cuda.mem_get_info()[0]
        print(f"free memory change {(free0 - free1) / 2**20:.1f} MiB", flush=True)
        assert free0 - free1 < 16 * 2**20
    finally:
        mmx.mmx_destroy(ctx)


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
def test_checkpoint_restore_continues_bitwise(prec):
    import torch
    import paper_2608_15253_amd as mmx
    case = Case((32, 32, 1), (4e-9, 4e-9, 4e-9), R=2, alpha=0.5,
                terms=("exchange", "demag"))
    m0 = random_unit(case.n, seed=1, replicas=case.R)
    if prec == 1:
        m0 = m0.astype(np.float32).astype(np.float64)
    ctx = open_ctx(case, prec)
    try:
        with pytest.raises(mmx.MMXError) as e:
            mmx.mmx_checkpoint(ctx)          # nothing to checkpoint yet
        assert e.value.status == -4
        md = dev(m0, prec)
        s1 = mmx.mmx_rk45(ctx, md, 0.0, 2e-11, 1e-6)
        blob = mmx.mmx_checkpoint(ctx)
        m_mid = md.clone()
        s2 = mmx.mmx_rk45_resume(ctx, md, 5e-11, 1e-6)
        mA = host(md)
        # another integrator reuses the stage buffers: no continuation afterwards
        mmx.mmx_rk4(ctx, m_mid.clone(), 1e-14, 1)
        with pytest.raises(mmx.MMXError) as e:
            mmx.mmx_rk45_resume(ctx, m_mid.clone(), 6e-11, 1e-6)
        assert e.value.status == -4
    finally:
        mmx.mmx_destroy(ctx)
    assert s1.accepted > 10 and s2.accepted > 10
    ctx = open_ctx(case, prec)
    try:
        mmx.mmx_restore(ctx, blob)
        s3 = mmx.mmx_rk45_resume(ctx, m_mid, 5e-11, 1e-6)
        mB = host(m_mid)
    finally:
        mmx.mmx_destroy(ctx)
    assert np.array_equal(mA, mB)
    assert (s2.accepted, s2.rejected, s2.t) == (s3.accepted, s3.rejected, s3.t)
    # a context of another layout refuses the blob
    other = Case((32, 16, 1), (4e-9, 4e-9, 4e-9), R=2, terms=("exchange", "demag"))
    ctx = open_ctx(other, prec)
    try:
        with pytest.raises(mmx.MMXError) as e:
            mmx.mmx_restore(ctx, blob)
        assert e.value.status == -2
    finally:
        mmx.mmx_destroy(ctx)
