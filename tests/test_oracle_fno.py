"""Pins of the oracle's Fourier neural operator (the learned demag surrogate):
truncated transforms against numpy's real FFTs, every gradient against central
finite differences, and loss decrease under Adam."""
import numpy as np
import pytest

from oracle import fno

M1, M2 = 3, 2


def _tiny(seed=1, C=4, L=2, Cp=6):
    p = fno.init_params(C=C, M1=M1, M2=M2, L=L, Cp=Cp, seed=seed)
    rng = np.random.default_rng(seed + 10)
    for k in p:  # make biases and spectral weights O(1) so every term matters
        if k.startswith(("p", "b", "q")):
            p[k] = 0.3 * rng.standard_normal(p[k].shape)
        if k.startswith("R"):
            p[k] = 0.3 * (rng.standard_normal(p[k].shape) + 1j * rng.standard_normal(p[k].shape))
    return p


def _data(B=2, H=8, W=10, seed=2):
    rng = np.random.default_rng(seed)
    m = rng.standard_normal((B, 3, H, W))
    m /= np.linalg.norm(m, axis=1, keepdims=True)
    t = rng.standard_normal((B, 3, H, W))
    return m, t


def test_truncated_forward_transform_equals_rfft2_modes():
    rng = np.random.default_rng(0)
    V = rng.standard_normal((2, 3, 16, 12))
    Vh = fno.dft_fwd(V, 4, 3)
    full = np.fft.rfft2(V)                       # (..., ky, kx)
    kys = fno.ky_modes(16, 3)
    ref = np.transpose(full[:, :, kys, :4], (0, 1, 3, 2))
    assert np.abs(Vh - ref).max() < 1e-12


def test_truncated_inverse_transform_equals_irfft2_of_zero_filled_spectrum():
    rng = np.random.default_rng(1)
    Uh = rng.standard_normal((2, 3, 4, 6)) + 1j * rng.standard_normal((2, 3, 4, 6))
    H, W = 16, 12
    U = fno.dft_inv(Uh, H, W)
    S = np.zeros((2, 3, H, W // 2 + 1), complex)
    kys = fno.ky_modes(H, 3)
    S[:, :, kys, :4] = np.transpose(Uh, (0, 1, 3, 2))
    assert np.abs(U - np.fft.irfft2(S, s=(H, W))).max() < 1e-12


def test_gelu_and_its_derivative():
    z = np.linspace(-4, 4, 41)
    h = 1e-6
    assert np.allclose(fno.gelu_grad(z), (fno.gelu(z + h) - fno.gelu(z - h)) / (2 * h), atol=1e-8)
    assert fno.gelu(np.array([0.0]))[0] == 0.0
    assert abs(fno.gelu(np.array([10.0]))[0] - 10.0) < 1e-12


@pytest.mark.parametrize("name", ["P", "p", "R0", "W0", "b0", "R1", "W1", "b1", "Q1", "q1", "Q2", "q2"])
def test_gradients_match_central_differences(name):
    params = _tiny()
    m, t = _data()
    h, cs = fno.forward(params, m, M1, M2, cache=True)
    g = fno.backward(params, cs, h, t, M1, M2)[name]
    rng = np.random.default_rng(3)
    flat_idx = rng.choice(params[name].size, min(6, params[name].size), replace=False)
    eps = 1e-6
    parts = [1.0, 1j] if np.iscomplexobj(params[name]) else [1.0]
    for idx in flat_idx:
        for unit in parts:
            pp = {k: v.copy() for k, v in params.items()}
            pm = {k: v.copy() for k, v in params.items()}
            pp[name].flat[idx] += eps * unit
            pm[name].flat[idx] -= eps * unit
            fd = (fno.loss(fno.forward(pp, m, M1, M2), t) -
                  fno.loss(fno.forward(pm, m, M1, M2), t)) / (2 * eps)
            an = g.flat[idx].real if unit == 1.0 else g.flat[idx].imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, idx, unit, fd, an)


def test_adam_training_lowers_the_loss():
    params = _tiny(seed=4)
    m, _ = _data(B=3, seed=5)
    t = np.roll(m, 1, axis=-1) * 0.5          # a learnable linear target
    state = {}
    first = None
    for it in range(1, 61):
        h, cs = fno.forward(params, m, M1, M2, cache=True)
        L = fno.loss(h, t)
        first = L if first is None else first
        g = fno.backward(params, cs, h, t, M1, M2)
        params = fno.adam(params, g, state, 1e-2, it)
    assert fno.loss(fno.forward(params, m, M1, M2), t) < 0.5 * first


def _adam_by_hand(g_seq, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Adam written out step by step for one scalar (Kingma & Ba 2015,
    Algorithm 1): the moments as explicit weighted sums of the gradient
    history, m_t = (1 - b1) sum_s b1^(t-s) g_s and v_t = (1 - b2) sum_s
    b2^(t-s) g_s^2, bias-corrected by 1 - b^t, one update per step."""
    x, out = 0.0, []
    for t in range(1, len(g_seq) + 1):
        mt = (1 - b1) * sum(b1 ** (t - s) * g_seq[s - 1] for s in range(1, t + 1))
        vt = (1 - b2) * sum(b2 ** (t - s) * g_seq[s - 1] ** 2 for s in range(1, t + 1))
        x -= lr * (mt / (1 - b1 ** t)) / (np.sqrt(vt / (1 - b2 ** t)) + eps)
        out.append(x)
    return out


def test_adam_matches_step_by_step_expansion_for_three_steps():
    """Steps t = 1, 2, 3 with a varying gradient history (a sign change and a
    gradient near eps), on a real array and on the real and imaginary parts of
    a complex array, which Adam updates independently."""
    seqs = [[1.0, -2.0, 0.5], [3e-3, 3e-3, -1e-9], [-0.7, 0.0, 4.0], [2.0, 2.0, 2.0]]
    lr = 0.05
    expect = np.array([_adam_by_hand(s, lr) for s in seqs])      # (4, 3)
    params = {"w": np.zeros(4), "c": np.zeros(2, complex)}
    state = {}
    for t in range(1, 4):
        g = {"w": np.array([s[t - 1] for s in seqs]),
             "c": np.array([seqs[0][t - 1] + 1j * seqs[1][t - 1],
                            seqs[2][t - 1] + 1j * seqs[3][t - 1]])}
        params = fno.adam(params, g, state, lr, t)
        assert np.allclose(params["w"], expect[:, t - 1], rtol=1e-13, atol=1e-16)
        c = params["c"]
        got = np.array([c[0].real, c[0].imag, c[1].real, c[1].imag])
        assert np.allclose(got, expect[:, t - 1], rtol=1e-13, atol=1e-16)
    # a constant gradient is bias-corrected exactly: every step moves by lr g/(|g| + eps)
    assert np.allclose(np.diff([0.0] + list(expect[3])), -lr * 2.0 / (2.0 + 1e-8), rtol=1e-13)
