"""FP64 oracle for the CNN surrogate -- TEST INFRASTRUCTURE ONLY.

The surrogate advances the variable-coefficient heat field K steps at once:

    x0   = [u0, (kappa - 0.125) / 0.075]                    (2 input channels)
    Z_l  = conv3x3(A_{l-1}, W_l) + b_l,  A_0 = x0           (zero "same" padding)
    A_l  = GELU(Z_l) for l = 1..5,  GELU(z) = z * Phi(z) = z/2 (1 + erf(z / sqrt 2))
    u_hat = u0 + Z_6[0]                                     (residual output)
    loss = mean over the masked cells of (u_hat - target)^2

Channels 2 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1.  conv3x3 is a correlation:
Z[co, i, j] = b[co] + sum_{ci, ky, kx} W[co, ci, ky, kx] * A[ci, i+ky-1, j+kx-1].

Every function works on one sample in (C, H, W) layout, in float64, as plain
shifted-slice sums with ``np.tensordot`` as the only library step.  The
backward pass is derived by hand from the chain rule (checked against central
finite differences in the tests).

``q`` (optional) emulates where the GPU path rounds operands to BF16: the
activations A_1..A_5 after GELU, the weights of the 32->32 layers (2..5), and
the back-propagated dZ_2..dZ_5.  With ``q=None`` the pass is exact FP64.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

CHANNELS = (2, 32, 32, 32, 32, 32, 1)
N_LAYERS = 6
KAPPA_MID = 0.125
KAPPA_HALF = 0.075


def _id(x):
    return x


def gelu(z: np.ndarray) -> np.ndarray:
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z: np.ndarray) -> np.ndarray:
    """d/dz [z Phi(z)] = Phi(z) + z phi(z)."""
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    ci, h, wd = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1)))
    y = np.broadcast_to(np.asarray(b, dtype=np.float64)[:, None, None], (w.shape[0], h, wd)).copy()
    for ky in range(3):
        for kx in range(3):
            y += np.tensordot(w[:, :, ky, kx], xp[:, ky:ky + h, kx:kx + wd], axes=([1], [0]))
    return y


def conv3x3_bwd_data(dy: np.ndarray, w: np.ndarray) -> np.ndarray:
    """dA[ci, m, n] = sum_{co, ky, kx} W[co, ci, ky, kx] dZ[co, m-ky+1, n-kx+1]."""
    co, h, wd = dy.shape
    dyp = np.pad(dy, ((0, 0), (1, 1), (1, 1)))
    dx = np.zeros((w.shape[1], h, wd))
    for ky in range(3):
        for kx in range(3):
            dx += np.tensordot(w[:, :, ky, kx].T, dyp[:, 2 - ky:2 - ky + h, 2 - kx:2 - kx + wd], axes=([1], [0]))
    return dx


def conv3x3_bwd_weight(x: np.ndarray, dy: np.ndarray) -> np.ndarray:
    """dW[co, ci, ky, kx] = sum_{i, j} dZ[co, i, j] A[ci, i+ky-1, j+kx-1]."""
    ci, h, wd = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1)))
    dw = np.zeros((dy.shape[0], ci, 3, 3))
    for ky in range(3):
        for kx in range(3):
            dw[:, :, ky, kx] = np.tensordot(dy, xp[:, ky:ky + h, kx:kx + wd], axes=([1, 2], [1, 2]))
    return dw


def init_params(seed: int) -> list[tuple[np.ndarray, np.ndarray]]:
    """He-normal weights N(0, 2/fan_in) (fan_in = 9*C_in), zero biases; the last layer is scaled
    by 0.1 so the untrained surrogate starts near the identity map u_hat = u0."""
    rng = np.random.default_rng(seed)
    params = []
    for l in range(N_LAYERS):
        ci, co = CHANNELS[l], CHANNELS[l + 1]
        std = math.sqrt(2.0 / (9 * ci)) * (0.1 if l == N_LAYERS - 1 else 1.0)
        params.append((rng.normal(0.0, std, size=(co, ci, 3, 3)), np.zeros(co)))
    return params


def input_channels(u0: np.ndarray, kappa: np.ndarray) -> np.ndarray:
    u = np.asarray(u0, dtype=np.float64)
    k = (np.asarray(kappa, dtype=np.float64) - KAPPA_MID) / KAPPA_HALF
    return np.stack([u, k])


def forward(params, u0, kappa, q=None):
    """Returns (u_hat, cache) for one sample."""
    q = q or _id
    a = input_channels(u0, kappa)
    acts, zs = [a], []
    for l, (w, b) in enumerate(params):
        wl = q(w) if 1 <= l <= 4 else w
        z = conv3x3(a, wl, b)
        zs.append(z)
        if l < N_LAYERS - 1:
            a = q(gelu(z))
            acts.append(a)
    u_hat = np.asarray(u0, dtype=np.float64) + zs[-1][0]
    return u_hat, (acts, zs)


def loss_and_grads(params, samples, q=None):
    """samples: list of (u0, kappa, target, mask).  Loss = mean over all masked cells of all samples.

    Returns (loss, grads) with grads a list of (dW, db) shaped like params.
    """
    q = q or _id
    n = float(sum(np.count_nonzero(m) for (_, _, _, m) in samples))
    grads = [(np.zeros_like(w), np.zeros_like(b)) for (w, b) in params]
    loss = 0.0
    for (u0, kappa, target, mask) in samples:
        u_hat, (acts, zs) = forward(params, u0, kappa, q)
        diff = (u_hat - np.asarray(target, dtype=np.float64)) * mask
        loss += float(np.sum(diff * diff)) / n
        dz = (2.0 / n) * diff[None]                       # dL/dZ_6
        for l in range(N_LAYERS - 1, -1, -1):
            w, _ = params[l]
            wl = q(w) if 1 <= l <= 4 else w
            gw, gb = grads[l]
            gw += conv3x3_bwd_weight(acts[l], dz)
            gb += dz.sum(axis=(1, 2))
            if l == 0:
                break
            da = conv3x3_bwd_data(dz, wl)                 # dL/dA_l (A index = layer l's input)
            dz = da * gelu_grad(zs[l - 1])                # dL/dZ_{l}  (1-based layer l)
            if l - 1 >= 1:                                # dZ_2..dZ_5 feed BF16 GEMMs on the GPU
                dz = q(dz)
    return loss, grads


def adam_step(p: np.ndarray, g: np.ndarray, m: np.ndarray, v: np.ndarray, t: int, lr: float,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1) with bias correction; returns (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def crop_mask(h: int, w: int, y0: int, x0: int, rows: int, cols: int, margin: int) -> np.ndarray:
    """Loss mask of an h x w crop at (y0, x0) of a rows x cols domain: cells closer than ``margin``
    to a crop edge that is not also a domain edge are excluded (their receptive field is cut)."""
    m = np.ones((h, w), dtype=np.float64)
    if y0 > 0:
        m[:margin, :] = 0
    if x0 > 0:
        m[:, :margin] = 0
    if y0 + h < rows:
        m[h - margin:, :] = 0
    if x0 + w < cols:
        m[:, w - margin:] = 0
    return m
