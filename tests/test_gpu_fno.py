"""GPU parity of the learned demag surrogate (Fourier neural operator) through
the C ABI against the FP64 oracle: forward output, every gradient, and the
Adam update, for the FP32 path (tight) and the BF16 matrix-core path (BF16
operand rounding: relative error bars 2e-2 forward, 5e-2 gradients).  The
transforms, mixing and weight gradients are FP32 matrix-core products in both
paths, so the FP32 bars hold them to FP32 accuracy."""
import numpy as np
import pytest

from oracle import fno as ofno
from workloads import random_unit

pytestmark = pytest.mark.gpu


def pack(p, L):
    parts = [p["P"].ravel(), p["p"].ravel()]
    for l in range(L):
        R = p[f"R{l}"]
        parts += [np.stack([R.real, R.imag], axis=-1).ravel(), p[f"W{l}"].ravel(), p[f"b{l}"].ravel()]
    parts += [p["Q1"].ravel(), p["q1"].ravel(), p["Q2"].ravel(), p["q2"].ravel()]
    return np.concatenate(parts).astype(np.float64)


def unpack_grads(flat, p, L):
    out, o = {}, 0
    def take(name, shape, cplx=False):
        nonlocal o
        n = int(np.prod(shape)) * (2 if cplx else 1)
        v = flat[o:o + n]
        o += n
        if cplx:
            v = v.reshape(shape + (2,))
            out[name] = v[..., 0] + 1j * v[..., 1]
        else:
            out[name] = v.reshape(shape)
    take("P", p["P"].shape); take("p", p["p"].shape)
    for l in range(L):
        take(f"R{l}", p[f"R{l}"].shape, True); take(f"W{l}", p[f"W{l}"].shape)
        take(f"b{l}", p[f"b{l}"].shape)
    take("Q1", p["Q1"].shape); take("q1", p["q1"].shape)
    take("Q2", p["Q2"].shape); take("q2", p["q2"].shape)
    assert o == flat.size
    return out


def _params(C, M1, M2, L, Cp, seed):
    p = ofno.init_params(C=C, M1=M1, M2=M2, L=L, Cp=Cp, seed=seed)
    rng = np.random.default_rng(seed + 1)
    for k in p:
        if k.startswith(("p", "b", "q")):
            p[k] = 0.1 * rng.standard_normal(p[k].shape)
        if k.startswith("R"):
            p[k] = p[k] * 10.0
    # round to FP32 so both sides start from identical weights
    for k in p:
        if np.iscomplexobj(p[k]):
            p[k] = p[k].real.astype(np.float32).astype(np.float64) + \
                1j * p[k].imag.astype(np.float32).astype(np.float64)
        else:
            p[k] = p[k].astype(np.float32).astype(np.float64)
    return p


def _run(shape, use_mfma, B, seed=3):
    import torch
    import paper_2608_15253_amd as mmx
    H, W, C, M1, M2, L, Cp = shape
    p = _params(C, M1, M2, L, Cp, seed)
    m = random_unit((W, H, 1), seed=seed + 5, replicas=B)[:, :, 0].astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(seed + 7)
    t = rng.standard_normal((B, 3, H, W)).astype(np.float32).astype(np.float64)
    f = mmx.mmx_fno_create(H, W, C, M1, M2, L, Cp, B, use_mfma)
    try:
        mmx.mmx_fno_set_stream(f, torch.cuda.current_stream().cuda_stream)
        n = mmx.mmx_fno_param_count(f)
        flat = pack(p, L)
        assert flat.size == n
        dv = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda:0")
        prm, md, td = dv(flat), dv(m), dv(t)
        h = torch.zeros((B, 3, H, W), dtype=torch.float32, device="cuda:0")
        g = torch.zeros(n, dtype=torch.float32, device="cuda:0")
        mmx.mmx_fno_forward(f, prm, md, h, B)
        loss = mmx.mmx_fno_backward(f, prm, h, td, g)
        torch.cuda.synchronize()
        hg, gg = h.double().cpu().numpy(), g.double().cpu().numpy()
        mom = torch.zeros(2 * n, dtype=torch.float32, device="cuda:0")
        mmx.mmx_fno_adam(f, prm, g, mom, 1e-3, 1)
        torch.cuda.synchronize()
        p_after = prm.double().cpu().numpy()
    finally:
        mmx.mmx_fno_destroy(f)
    href, cs = ofno.forward(p, m, M1, M2, cache=True)
    gref = ofno.backward(p, cs, href, t, M1, M2)
    return p, hg, href, gg, gref, loss, ofno.loss(href, t), flat, p_after, t, m


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(np.ravel(b)), 1e-300))


SMALL = (32, 24, 8, 4, 3, 2, 16)   # H, W, C, M1, M2, L, Cp


def test_fp32_forward_gradients_and_adam_match_oracle():
    p, hg, href, gg, gref, loss, lref, flat, p_after, _, _ = _run(SMALL, False, 3)
    L = SMALL[5]
    assert _rel(hg, href) < 1e-5
    assert abs(loss - lref) < 1e-5 * lref
    g = unpack_grads(gg, p, L)
    for k in gref:
        assert _rel(g[k], gref[k]) < 2e-4, (k, _rel(g[k], gref[k]))
    # one Adam step from zero moments moves every parameter by lr * sign(g)
    step = p_after - flat
    nz = np.abs(gg) > 1e-4   # |g| >> eps: the first step is lr * sign(g)
    assert np.allclose(step[nz], -1e-3 * np.sign(gg[nz]), rtol=1e-3, atol=1e-8)


@pytest.mark.parametrize("shape,B", [
    # W and H x W not multiples of 4 (element loads), 20 channels (ragged
    # 16-tiles), batch 17 (two batch tiles in the mixing), projection 40
    ((15, 18, 20, 4, 3, 2, 40), 17),
    # 17 x-modes: beyond the matrix-core transforms, the VALU transforms run
    ((40, 40, 8, 17, 3, 1, 16), 2),
], ids=["ragged", "valu-transforms"])
def test_fp32_ragged_shapes_match_oracle(shape, B):
    p, hg, href, gg, gref, loss, lref, *_ = _run(shape, False, B, seed=9)
    assert _rel(hg, href) < 1e-5
    assert abs(loss - lref) < 1e-5 * lref
    g = unpack_grads(gg, p, shape[5])
    for k in gref:
        assert _rel(g[k], gref[k]) < 2e-4, (k, _rel(g[k], gref[k]))


def test_bf16_matrix_core_path_within_bf16_bounds():
    p, hg, href, gg, gref, loss, lref, *_ = _run(SMALL, True, 3)
    L = SMALL[5]
    assert _rel(hg, href) < 2e-2
    g = unpack_grads(gg, p, L)
    for k in gref:
        assert _rel(g[k], gref[k]) < 5e-2, (k, _rel(g[k], gref[k]))


@pytest.mark.parametrize("use_mfma", [False, True], ids=["fp32", "bf16"])
def test_full_size_network(use_mfma):
    """Width 32, 12 modes, 4 layers, projection 128 on a 128x128 film."""
    shape = (128, 128, 32, 12, 12, 4, 128)
    p, hg, href, gg, gref, *_ = _run(shape, use_mfma, 2, seed=11)
    tol_f, tol_g = (1e-5, 2e-4) if not use_mfma else (2e-2, 5e-2)
    assert _rel(hg, href) < tol_f
    g = unpack_grads(gg, p, 4)
    for k in gref:
        assert _rel(g[k], gref[k]) < tol_g, (k, _rel(g[k], gref[k]))


def test_adam_three_steps_match_oracle():
    """Three Adam steps (t = 1, 2, 3: bias corrections beyond the first step)
    on the network's packed parameters with a varying gradient history, FP32
    on the GPU against the FP64 oracle's update of the same values."""
    import torch
    import paper_2608_15253_amd as mmx
    H, W, C, M1, M2, L, Cp = SMALL
    p = _params(C, M1, M2, L, Cp, 5)
    f = mmx.mmx_fno_create(H, W, C, M1, M2, L, Cp, 1, False)
    try:
        mmx.mmx_fno_set_stream(f, torch.cuda.current_stream().cuda_stream)
        n = mmx.mmx_fno_param_count(f)
        flat = pack(p, L)
        rng = np.random.default_rng(21)
        gs = [rng.standard_normal(n).astype(np.float32).astype(np.float64) * s
              for s in (1.0, 0.3, 2.0)]
        gs[1][: n // 4] *= -1.0
        prm = torch.tensor(flat, dtype=torch.float32, device="cuda:0")
        mom = torch.zeros(2 * n, dtype=torch.float32, device="cuda:0")
        ref = {"x": flat.copy()}
        state = {}
        for t, g in enumerate(gs, start=1):
            gd = torch.tensor(g, dtype=torch.float32, device="cuda:0")
            mmx.mmx_fno_adam(f, prm, gd, mom, 1e-3, t)
            ref = ofno.adam(ref, {"x": g}, state, 1e-3, t)
            torch.cuda.synchronize()
            got = prm.double().cpu().numpy()
            # FP32 state: parameter values of O(1) carry 6e-8 relative rounding
            # (a wrong bias correction at t >= 2 shifts steps of size lr = 1e-3 by
            # a sizeable fraction of lr)
            assert np.abs(got - ref["x"]).max() <= 2e-6, t
    finally:
        mmx.mmx_fno_destroy(f)
