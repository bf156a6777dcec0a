"""The allocation-free topological charge (mmx_topological_charge_noalloc)
against mmx_topological_charge through the C ABI: two calls in a row, the
second on a smaller input, equal bit for bit (same kernels, same summation
order, partial sums in the library's static scratch instead of a buffer
allocated per call); the size limit is rejected before any launch; the call
can be captured in a graph (it allocates nothing) and every replay equals the
direct call."""
import numpy as np
import pytest

from oracle import observables as oob
from workloads import neel_skyrmions, random_unit

from _mmx_case import Case, dev, host, open_ctx

pytestmark = pytest.mark.gpu


def _charges(ctx, m, R):
    import torch
    import paper_2608_15253_amd as mmx
    q_ref = torch.zeros(R, dtype=torch.float64, device="cuda:0")
    q_new = torch.full((R,), np.nan, dtype=torch.float64, device="cuda:0")
    mmx.mmx_topological_charge(ctx, m, q_ref)
    mmx.mmx_topological_charge_noalloc(ctx, m, q_new)
    return host(q_ref), host(q_new)


def test_noalloc_charge_equals_allocating_entry_point_on_two_calls():
    import paper_2608_15253_amd as mmx
    # first call: the benchmark's batch (1024 replicas of 64 x 64, FP32; 16
    # workgroups per replica) with a skyrmion in every replica
    big = Case((64, 64, 1), (4e-9, 4e-9, 4e-9), R=1024, terms=("exchange",))
    sk, _, _ = neel_skyrmions(big.n, big.cell, 1, 20e-9, 30e-9, seed=3, width=5e-9,
                              periodic=False)
    mb = np.repeat(sk[None], big.R, axis=0) + 0.05 * random_unit(big.n, seed=4, replicas=big.R)
    mb /= np.linalg.norm(mb, axis=1, keepdims=True)
    ctx = open_ctx(big, mmx.MMX_F32)
    try:
        ref, new = _charges(ctx, dev(mb, mmx.MMX_F32), big.R)
    finally:
        mmx.mmx_destroy(ctx)
    print(f"[case] 1024 x 64x64 f32: Q range {ref.min():.4f} .. {ref.max():.4f}", flush=True)
    assert np.all(np.isfinite(ref)) and np.array_equal(ref, new)
    # second call: a smaller periodic FP64 batch (3 replicas of 40 x 24)
    small = Case((40, 24, 1), (2e-9, 2e-9, 1e-9), pbc=(1, 1, 0), images=(1, 1, 0), R=3,
                 terms=("exchange",))
    ms = random_unit(small.n, seed=9, replicas=small.R)
    ctx = open_ctx(small, mmx.MMX_F64)
    try:
        ref, new = _charges(ctx, dev(ms, mmx.MMX_F64), small.R)
    finally:
        mmx.mmx_destroy(ctx)
    assert np.array_equal(ref, new)
    expect = np.array([oob.topological_charge(ms[r], small.grid) for r in range(small.R)])
    assert np.abs(new - expect).max() <= 1e-12 * max(1.0, np.abs(expect).max())


def test_noalloc_charge_rejects_groups_beyond_the_scratch():
    import torch
    import paper_2608_15253_amd as mmx
    # 520 replicas x 256 workgroups (256 x 256 cells) = 133120 > 131072 partial sums
    ctx = mmx.mmx_create([mmx.make_group((256, 256, 1), (4e-9, 4e-9, 4e-9), replicas=520)],
                         mmx.MMX_F32)
    try:
        mmx.mmx_set_stream(ctx, torch.cuda.current_stream().cuda_stream)
        m = torch.zeros(4, dtype=torch.float32, device="cuda:0")
        Q = torch.zeros(520, dtype=torch.float64, device="cuda:0")
        with pytest.raises(mmx.MMXError) as e:
            mmx.mmx_topological_charge_noalloc(ctx, m, Q)
        assert e.value.status == -1   # MMX_EINVAL
    finally:
        mmx.mmx_destroy(ctx)


def test_noalloc_charge_under_graph_capture():
    import torch
    import paper_2608_15253_amd as mmx
    case = Case((48, 40, 1), (2e-9, 2e-9, 1e-9), R=4, terms=("exchange",))
    m0 = random_unit(case.n, seed=13, replicas=case.R)
    ctx = open_ctx(case, mmx.MMX_F64)
    try:
        m = dev(m0, mmx.MMX_F64)
        q_ref = torch.zeros(case.R, dtype=torch.float64, device="cuda:0")
        mmx.mmx_topological_charge(ctx, m, q_ref)
        want = host(q_ref)
        q = torch.zeros(case.R, dtype=torch.float64, device="cuda:0")
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            mmx.mmx_set_stream(ctx, s.cuda_stream)
            mmx.mmx_topological_charge_noalloc(ctx, m, q)   # warm-up outside capture
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            mmx.mmx_set_stream(ctx, torch.cuda.current_stream().cuda_stream)
            mmx.mmx_topological_charge_noalloc(ctx, m, q)
        mmx.mmx_set_stream(ctx, torch.cuda.current_stream().cuda_stream)
        for k in range(3):
            q.fill_(float(k) + 0.5)          # eager work between replays
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert np.array_equal(host(q), want), k
    finally:
        mmx.mmx_destroy(ctx)
