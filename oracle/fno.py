"""FP64 reference of the learned demag surrogate (a Fourier neural operator).

Not part of the paper: an extension in which a small spectral
convolution neural operator (width 32, 12 modes, 4 layers) predicts the
demagnetising field h = H_demag / Ms of a film from m, is trained on fields the
method itself produces, and stands in for the exact demag in intermediate RK45
stages.  This module is the plain definition the GPU forward and backward
kernels are checked against; gradients are pinned by central differences.

Layout: activations (B, C, H, W) with x (W) fastest, as the magnetisation.

Network (the reading taken here):
  X0 = [m_x, m_y, m_z, x/W - 1/2, y/H - 1/2]                      (5 channels)
  V  = P X0 + p                                                    (lift, 1x1)
  for l = 0..L-1:
      Vh = F(V)   truncated DFT: kx in [0, M1), ky in [0, M2) u [H-M2, H)
      Uh[o] = sum_i R_l[kx, ky, i, o] Vh[i]                        (complex mixing)
      U  = F^+(Uh)                                                 (real inverse)
      Z  = U + W_l V + b_l
      V  = gelu(Z) for l < L-1, else Z
  h  = Q2 gelu(Q1 V + q1) + q2                                     (projection)

F(V)[kx, ky] = sum_{x,y} V[y, x] exp(-2 pi i (kx x / W + ky y / H)),
F^+(Uh)[y, x] = (1 / HW) sum_{kx, ky} c_kx Re(Uh[kx, ky] exp(+2 pi i (kx x / W + ky y / H))),
c_0 = 1, c_kx = 2 otherwise (the Hermitian partner of kx > 0; M1 < W/2): the
inverse real FFT of the zero-filled half spectrum.  gelu(z) = z (1 + erf(z/sqrt 2)) / 2.
Loss per sample: |h - t|^2 / |t|^2, averaged over the batch.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def ky_modes(H, M2):
    return np.concatenate([np.arange(M2), np.arange(H - M2, H)])


def dft_mats(H, W, M1, M2):
    x = np.arange(W)
    y = np.arange(H)
    kx = np.arange(M1)
    ky = ky_modes(H, M2)
    Fx = np.exp(-2j * np.pi * np.outer(kx, x) / W)      # (M1, W)
    Fy = np.exp(-2j * np.pi * np.outer(ky, y) / H)      # (2 M2, H)
    return Fx, Fy


def dft_fwd(V, M1, M2):
    """(B, C, H, W) real -> (B, C, M1, 2 M2) complex."""
    H, W = V.shape[-2:]
    Fx, Fy = dft_mats(H, W, M1, M2)
    A = np.einsum("bcyx,kx->bcyk", V, Fx)
    return np.einsum("bcyk,jy->bckj", A, Fy)


def ckx(M1):
    c = np.full(M1, 2.0)
    c[0] = 1.0
    return c


def dft_inv(Uh, H, W):
    """(B, C, M1, 2 M2) complex -> (B, C, H, W) real."""
    M1, J = Uh.shape[-2:]
    Fx, Fy = dft_mats(H, W, M1, J // 2)
    A = np.einsum("bckj,jy->bcky", Uh, Fy.conj())
    U = np.einsum("bcky,kx,k->bcyx", A, Fx.conj(), ckx(M1))
    return U.real / (H * W)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def conv1x1(Wt, b, X):
    return np.einsum("oc,bchw->bohw", Wt, X) + b[None, :, None, None]


def features(m):
    """m (B, 3, H, W) -> X0 (B, 5, H, W)."""
    B, _, H, W = m.shape
    xs = (np.arange(W) + 0.5) / W - 0.5
    ys = (np.arange(H) + 0.5) / H - 0.5
    cx = np.broadcast_to(xs[None, :], (H, W))
    cy = np.broadcast_to(ys[:, None], (H, W))
    c = np.broadcast_to(np.stack([cx, cy])[None], (B, 2, H, W))
    return np.concatenate([m, c], axis=1)


def init_params(C=32, M1=12, M2=12, L=4, Cp=128, seed=0):
    rng = np.random.default_rng(seed)
    p = {"P": rng.standard_normal((C, 5)) / math.sqrt(5), "p": np.zeros(C)}
    scale = 1.0 / (C * C)
    for l in range(L):
        p[f"R{l}"] = scale * (rng.random((M1, 2 * M2, C, C)) + 1j * rng.random((M1, 2 * M2, C, C)))
        p[f"W{l}"] = rng.standard_normal((C, C)) / math.sqrt(C)
        p[f"b{l}"] = np.zeros(C)
    p["Q1"] = rng.standard_normal((Cp, C)) / math.sqrt(C)
    p["q1"] = np.zeros(Cp)
    p["Q2"] = rng.standard_normal((3, Cp)) / math.sqrt(Cp)
    p["q2"] = np.zeros(3)
    return p


def n_layers(params):
    return sum(1 for k in params if k.startswith("W"))


def forward(params, m, M1, M2, cache=False):
    L = n_layers(params)
    H, W = m.shape[-2:]
    X0 = features(m)
    V = conv1x1(params["P"], params["p"], X0)
    cs = {"X0": X0, "V": [V], "Vh": [], "Z": []}
    for l in range(L):
        Vh = dft_fwd(V, M1, M2)
        Uh = np.einsum("kjio,bikj->bokj", params[f"R{l}"], Vh)
        Z = dft_inv(Uh, H, W) + conv1x1(params[f"W{l}"], params[f"b{l}"], V)
        cs["Vh"].append(Vh)
        cs["Z"].append(Z)
        V = gelu(Z) if l < L - 1 else Z
        cs["V"].append(V)
    Y1 = conv1x1(params["Q1"], params["q1"], V)
    A1 = gelu(Y1)
    h = conv1x1(params["Q2"], params["q2"], A1)
    cs.update(Y1=Y1, A1=A1)
    return (h, cs) if cache else h


def loss(h, t):
    num = np.sum((h - t) ** 2, axis=(1, 2, 3))
    den = np.sum(t ** 2, axis=(1, 2, 3))
    return float(np.mean(num / den))


def backward(params, cs, h, t, M1, M2):
    """Gradients of loss(h, t) with respect to every parameter (FP64)."""
    L = n_layers(params)
    B, _, H, W = h.shape
    den = np.sum(t ** 2, axis=(1, 2, 3))
    dh = 2.0 * (h - t) / den[:, None, None, None] / B
    g = {}
    g["Q2"] = np.einsum("bohw,bchw->oc", dh, cs["A1"])
    g["q2"] = dh.sum(axis=(0, 2, 3))
    dA1 = np.einsum("oc,bohw->bchw", params["Q2"], dh)
    dY1 = dA1 * gelu_grad(cs["Y1"])
    V = cs["V"][L]
    g["Q1"] = np.einsum("bohw,bchw->oc", dY1, V)
    g["q1"] = dY1.sum(axis=(0, 2, 3))
    dV = np.einsum("oc,bohw->bchw", params["Q1"], dY1)
    Fx, Fy = dft_mats(H, W, M1, M2)
    c = ckx(M1)
    for l in reversed(range(L)):
        Z = cs["Z"][l]
        dZ = dV * gelu_grad(Z) if l < L - 1 else dV
        Vin = cs["V"][l]
        g[f"W{l}"] = np.einsum("bohw,bchw->oc", dZ, Vin)
        g[f"b{l}"] = dZ.sum(axis=(0, 2, 3))
        dV = np.einsum("oc,bohw->bchw", params[f"W{l}"], dZ)
        # U = Re(G Uh) with G linear: dL/dUh (as the gradient of a real
        # function of complex variables, d/dRe + i d/dIm) = conj(G)^T dU
        dUh = np.einsum("bcyx,kx,k->bcyk", dZ, Fx, c) / (H * W)
        dUh = np.einsum("bcyk,jy->bckj", dUh, Fy)
        Vh = cs["Vh"][l]
        # Uh = sum_i R Vh: dR = conj(Vh) dUh summed over the batch; dVh = conj(R) dUh
        g[f"R{l}"] = np.einsum("bikj,bokj->kjio", Vh.conj(), dUh)
        dVh = np.einsum("kjio,bokj->bikj", params[f"R{l}"].conj(), dUh)
        # Vh = F(V), V real: dV = Re(conj(F)^T dVh)
        A = np.einsum("bckj,jy->bcky", dVh, Fy.conj())
        dV = dV + np.einsum("bcky,kx->bcyx", A, Fx.conj()).real
    g["P"] = np.einsum("bohw,bchw->oc", dV, cs["X0"])
    g["p"] = dV.sum(axis=(0, 2, 3))
    return g


def adam(params, grads, state, lr, t, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015); complex weights are updated on their
    real and imaginary parts independently."""
    for k, gk in grads.items():
        m_, v_ = state.setdefault(k, (np.zeros_like(gk), np.zeros(gk.shape)))
        m_ = beta1 * m_ + (1 - beta1) * gk
        if np.iscomplexobj(gk):
            v_ = beta2 * v_ + (1 - beta2) * (gk.real ** 2 + 1j * gk.imag ** 2)
            mh = m_ / (1 - beta1 ** t)
            vh = v_ / (1 - beta2 ** t)
            params[k] = params[k] - lr * (mh.real / (np.sqrt(vh.real) + eps)
                                          + 1j * mh.imag / (np.sqrt(vh.imag) + eps))
        else:
            v_ = beta2 * v_ + (1 - beta2) * gk * gk
            mh = m_ / (1 - beta1 ** t)
            vh = v_ / (1 - beta2 ** t)
            params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
        state[k] = (m_, v_)
    return params
