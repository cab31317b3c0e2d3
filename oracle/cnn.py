"""FP64 oracle for the CNN surrogate -- TEST INFRASTRUCTURE ONLY.

The surrogate advances the variable-coefficient heat field K steps at once:

    s    = RMS of u0 over the field (1 if the field is zero)
    inv  = fp32(1 / s),  gain = fp32(2^-11 * s)             (the field's scale constants)
    x0   = [u0 * inv, (kappa - 0.125) / 0.075]              (2 input channels)
    Z_l  = conv3x3(A_{l-1}, W_l) + b_l,  A_0 = x0           (zero "same" padding)
    A_l  = GELU(Z_l) for l = 1..5,  GELU(z) = z * Phi(z) = z/2 (1 + erf(z / sqrt 2))
    u_hat = u0 + gain * Z_6[0]                              (residual output)
    loss = mean over the masked cells of (u_hat - target)^2

The network therefore sees the field in units of its own RMS and predicts the K-step update in
units of 2^-11 of it: sixteen steps of the heat workload change a smooth field by a few 1e-4 of its
size, so that the last layer's output is of order one.  (The method is linear in u0, and this form
of the network is scale-equivariant: scaling u0 by c scales u_hat by c.)

Channels 2 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1.  conv3x3 is a correlation:
Z[co, i, j] = b[co] + sum_{ci, ky, kx} W[co, ci, ky, kx] * A[ci, i+ky-1, j+kx-1].

Every function works on one sample in (C, H, W) layout, in float64, as plain
shifted-slice sums with ``np.tensordot`` as the only library step.  The
backward pass is derived by hand from the chain rule (checked against central
finite differences in the tests).

``q`` (optional) emulates where the GPU path rounds operands to BF16: the
activations A_1..A_5 after GELU, the weights of the 32->32 layers (2..5), and
the back-propagated dZ_2..dZ_5; with it the input u0 * inv and the output u_hat
are rounded to FP32 as the GPU computes them.  With ``q=None`` the pass is
exact FP64 (with the FP32 scale constants, which belong to the model like its
FP32 parameters).

``init_params_philox`` is the seeded He-normal initialisation the library
performs on the device: Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC 2011) on the counter (i, 0, 0, 0) with
the key (seed, 0) for parameter i of the flat layout, and the Box-Muller
transform (Box and Muller, 1958) of its first two outputs.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

CHANNELS = (2, 32, 32, 32, 32, 32, 1)
N_LAYERS = 6
KAPPA_MID = 0.125
KAPPA_HALF = 0.075
UPDATE_SCALE = 2.0 ** -11


def f32(x):
    """Round to binary32 (nearest even) and widen back to float64."""
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def field_scale(u0) -> tuple[float, float]:
    """(inv, gain) of one field: s = sqrt(mean(u0^2)) in FP64 (s = 1 for an all-zero field),
    inv = fp32(1 / s), gain = fp32(2^-11 s)."""
    u = np.asarray(u0, dtype=np.float64)
    s = math.sqrt(float(np.sum(u * u)) / u.size)
    if not s > 0.0:
        s = 1.0
    return float(f32(1.0 / s)), float(f32(UPDATE_SCALE * s))


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


# ---- seeded initialisation (the library's surrogate_init) ------------------------------------

_M64 = (1 << 64) - 1
_PHILOX_M = (0xD2E7470EE14C6C93, 0xCA5A826395121157)     # round multipliers
_PHILOX_W = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)     # key increments (Weyl sequence)


def philox4x64_10(ctr, key):
    """Philox4x64 with 10 rounds: each round multiplies words 0 and 2 by the two multipliers
    (128-bit products split into high and low halves), mixes the high halves with words 1 and 3 and
    the key, and bumps the key by the Weyl constants.  ctr: 4 ints, key: 2 ints (64-bit)."""
    c0, c1, c2, c3 = (int(v) & _M64 for v in ctr)
    k0, k1 = (int(v) & _M64 for v in key)
    for _ in range(10):
        p0 = _PHILOX_M[0] * c0
        p1 = _PHILOX_M[1] * c2
        c0, c1, c2, c3 = (p1 >> 64) ^ c1 ^ k0, p1 & _M64, (p0 >> 64) ^ c3 ^ k1, p0 & _M64
        k0 = (k0 + _PHILOX_W[0]) & _M64
        k1 = (k1 + _PHILOX_W[1]) & _M64
    return c0, c1, c2, c3


def normal_at(i: int, seed: int) -> float:
    """Standard normal variate of flat parameter index i: Box-Muller on the first two 64-bit words
    of Philox4x64-10 at counter (i, 0, 0, 0), key (seed, 0); u = (x >> 11) 2^-53 in [0, 1)."""
    x0, x1, _, _ = philox4x64_10((i, 0, 0, 0), (seed, 0))
    u1 = (x0 >> 11) * 2.0 ** -53
    u2 = (x1 >> 11) * 2.0 ** -53
    return math.sqrt(-2.0 * math.log(1.0 - u1)) * math.cos(2.0 * math.pi * u2)


def param_layout():
    """(weight offset, bias offset) of each layer in the flat parameter vector: W_l as
    [ky][kx][ci][co], then b_l[co]."""
    offs, o = [], 0
    for l in range(N_LAYERS):
        ci, co = CHANNELS[l], CHANNELS[l + 1]
        offs.append((o, o + 9 * ci * co))
        o += 9 * ci * co + co
    return offs, o


def init_params_philox(seed: int):
    """He-normal weights N(0, 2 / (9 C_in)) (the last layer scaled by 0.1, so that the untrained
    network starts near u_hat = u0), zero biases: returns (params, flat), params as (W, b) per layer
    in (C_out, C_in, 3, 3) layout, flat the FP32 vector in the library layout."""
    offs, total = param_layout()
    flat = np.zeros(total, dtype=np.float32)
    params = []
    for l in range(N_LAYERS):
        ci, co = CHANNELS[l], CHANNELS[l + 1]
        std = math.sqrt(2.0 / (9 * ci)) * (0.1 if l == N_LAYERS - 1 else 1.0)
        wo, bo = offs[l]
        vals = np.array([std * normal_at(i, seed) for i in range(wo, bo)], dtype=np.float64)
        flat[wo:bo] = vals.astype(np.float32)
        w = flat[wo:bo].astype(np.float64).reshape(3, 3, ci, co).transpose(3, 2, 0, 1)
        params.append((np.ascontiguousarray(w), np.zeros(co)))
    return params, flat


def input_channels(u0: np.ndarray, kappa: np.ndarray, inv: float = 1.0, emulate: bool = False) -> np.ndarray:
    u = np.asarray(u0, dtype=np.float64) * inv
    if emulate:
        u = f32(u)
    k = (np.asarray(kappa, dtype=np.float64) - KAPPA_MID) / KAPPA_HALF
    return np.stack([u, k])


def forward(params, u0, kappa, q=None, scale=None):
    """Returns (u_hat, cache) for one sample.  ``scale`` = (inv, gain) of the field the sample is
    part of (default: ``field_scale(u0)``, the sample is the whole field)."""
    emulate = q is not None
    q = q or _id
    inv, gain = scale if scale is not None else field_scale(u0)
    a = input_channels(u0, kappa, inv, emulate)
    acts, zs = [a], []
    for l, (w, b) in enumerate(params):
        wl = q(w) if 1 <= l <= 4 else w
        z = conv3x3(a, wl, b)
        zs.append(z)
        if l < N_LAYERS - 1:
            a = q(gelu(z))
            acts.append(a)
    u_hat = np.asarray(u0, dtype=np.float64) + gain * zs[-1][0]
    if emulate:
        u_hat = f32(u_hat)
    return u_hat, (acts, zs)


def loss_and_grads(params, samples, q=None):
    """samples: list of (u0, kappa, target, mask) or (u0, kappa, target, mask, scale), scale =
    (inv, gain) of the field the sample was cut from (default: the sample's own).  Loss = mean over
    all masked cells of all samples.

    Returns (loss, grads) with grads a list of (dW, db) shaped like params.
    """
    n = float(sum(np.count_nonzero(smp[3]) for smp in samples))
    grads = [(np.zeros_like(w), np.zeros_like(b)) for (w, b) in params]
    qq = q or _id
    loss = 0.0
    for smp in samples:
        u0, kappa, target, mask = smp[:4]
        scale = smp[4] if len(smp) > 4 else field_scale(u0)
        u_hat, (acts, zs) = forward(params, u0, kappa, q, scale)
        diff = (u_hat - np.asarray(target, dtype=np.float64)) * mask
        loss += float(np.sum(diff * diff)) / n
        dz = (2.0 * scale[1] / n) * diff[None]            # dL/dZ_6 = gain dL/du_hat
        for l in range(N_LAYERS - 1, -1, -1):
            w, _ = params[l]
            wl = qq(w) if 1 <= l <= 4 else w
            gw, gb = grads[l]
            gw += conv3x3_bwd_weight(acts[l], dz)
            gb += dz.sum(axis=(1, 2))
            if l == 0:
                break
            da = conv3x3_bwd_data(dz, wl)                 # dL/dA_l (A index = layer l's input)
            dz = da * gelu_grad(zs[l - 1])                # dL/dZ_{l}  (1-based layer l)
            if l - 1 >= 1:                                # dZ_2..dZ_5 feed BF16 GEMMs on the GPU
                dz = qq(dz)
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
