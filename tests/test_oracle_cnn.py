"""Pins of the FP64 CNN-surrogate oracle (no GPU): library convolution, closed-form GELU,
central finite differences of the loss, torch autograd, and Adam's first-step closed form."""
import math

import numpy as np
import pytest
import torch

from oracle import cnn


def test_conv3x3_matches_torch():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((5, 9, 7))
    w = rng.standard_normal((4, 5, 3, 3))
    b = rng.standard_normal(4)
    got = cnn.conv3x3(x, w, b)
    ref = torch.nn.functional.conv2d(torch.from_numpy(x)[None], torch.from_numpy(w), torch.from_numpy(b),
                                     padding=1)[0].numpy()
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_conv_adjoints_match_torch():
    rng = np.random.default_rng(1)
    x = torch.from_numpy(rng.standard_normal((3, 6, 8))).requires_grad_(True)
    w = torch.from_numpy(rng.standard_normal((5, 3, 3, 3))).requires_grad_(True)
    dy = rng.standard_normal((5, 6, 8))
    y = torch.nn.functional.conv2d(x[None], w, padding=1)[0]
    y.backward(torch.from_numpy(dy))
    np.testing.assert_allclose(cnn.conv3x3_bwd_data(dy, w.detach().numpy()), x.grad.numpy(), atol=1e-12)
    np.testing.assert_allclose(cnn.conv3x3_bwd_weight(x.detach().numpy(), dy), w.grad.numpy(), atol=1e-12)


def test_gelu_closed_form():
    z = np.array([-3.0, -1.0, 0.0, 0.5, 2.0, 8.0])
    exp = np.array([v * 0.5 * (1 + math.erf(v / math.sqrt(2))) for v in z])
    np.testing.assert_allclose(cnn.gelu(z), exp, rtol=1e-15, atol=1e-300)
    assert cnn.gelu_grad(np.array([0.0]))[0] == 0.5
    h = 1e-6
    zz = np.linspace(-4, 4, 41)
    fd = (cnn.gelu(zz + h) - cnn.gelu(zz - h)) / (2 * h)
    np.testing.assert_allclose(cnn.gelu_grad(zz), fd, atol=1e-8)
    t = torch.from_numpy(zz)
    np.testing.assert_allclose(cnn.gelu(zz), torch.nn.functional.gelu(t).numpy(), atol=1e-15)


def _samples(rng, n, h, w, masked=True):
    out = []
    for s in range(n):
        u0 = rng.standard_normal((h, w)) * 0.5
        kap = rng.uniform(0.05, 0.2, (h, w))
        tgt = u0 + 0.1 * rng.standard_normal((h, w))
        m = cnn.crop_mask(h, w, 1 if masked else 0, 0, h + 2, w, 1) if masked else np.ones((h, w))
        out.append((u0, kap, tgt, m))
    return out


def test_grads_match_finite_differences():
    rng = np.random.default_rng(2)
    params = cnn.init_params(3)
    params[-1] = (params[-1][0] * 10, params[-1][1] + 0.01)   # make the last layer matter
    samples = _samples(rng, 2, 6, 5)
    loss, grads = cnn.loss_and_grads(params, samples)
    h = 1e-6
    for l in range(cnn.N_LAYERS):
        w, b = params[l]
        for _ in range(5):
            idx = tuple(int(rng.integers(0, s)) for s in w.shape)
            w0 = w[idx]
            w[idx] = w0 + h
            lp, _ = cnn.loss_and_grads(params, samples)
            w[idx] = w0 - h
            lm, _ = cnn.loss_and_grads(params, samples)
            w[idx] = w0
            fd = (lp - lm) / (2 * h)
            assert abs(grads[l][0][idx] - fd) <= 1e-6 * max(1.0, abs(fd)), (l, idx, grads[l][0][idx], fd)
        k = int(rng.integers(0, b.shape[0]))
        b0 = b[k]
        b[k] = b0 + h
        lp, _ = cnn.loss_and_grads(params, samples)
        b[k] = b0 - h
        lm, _ = cnn.loss_and_grads(params, samples)
        b[k] = b0
        assert abs(grads[l][1][k] - (lp - lm) / (2 * h)) <= 1e-6 * max(1.0, abs((lp - lm) / (2 * h)))


def test_grads_match_torch_autograd():
    rng = np.random.default_rng(4)
    params = cnn.init_params(5)
    samples = _samples(rng, 2, 9, 8)
    loss, grads = cnn.loss_and_grads(params, samples)
    tp = [(torch.from_numpy(w.copy()).requires_grad_(True), torch.from_numpy(b.copy()).requires_grad_(True))
          for (w, b) in params]
    n = sum(float(m.sum()) for (_, _, _, m) in samples)
    tl = 0
    for (u0, kap, tgt, m) in samples:
        s = math.sqrt(float(np.mean(u0 * u0)))  # the field's RMS, and its FP32 scale constants
        inv, gain = float(np.float32(1.0 / s)), float(np.float32(2.0 ** -11 * s))
        x = np.stack([u0 * inv, (kap - 0.125) / 0.075])
        a = torch.from_numpy(x)[None]
        for l, (w, b) in enumerate(tp):
            a = torch.nn.functional.conv2d(a, w, b, padding=1)
            if l < cnn.N_LAYERS - 1:
                a = torch.nn.functional.gelu(a)
        uh = torch.from_numpy(u0) + gain * a[0, 0]
        tl = tl + (((uh - torch.from_numpy(tgt)) * torch.from_numpy(m)) ** 2).sum() / n
    tl.backward()
    assert abs(float(tl) - loss) < 1e-12
    for (gw, gb), (w, b) in zip(grads, tp):
        np.testing.assert_allclose(gw, w.grad.numpy(), rtol=1e-10, atol=1e-13)
        np.testing.assert_allclose(gb, b.grad.numpy(), rtol=1e-10, atol=1e-13)


def test_adam_first_step_closed_form():
    """With m = v = 0, the bias-corrected first step is -lr * g / (|g| + eps); a constant gradient
    keeps that step size for every later step."""
    rng = np.random.default_rng(6)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lr, eps = 1e-3, 1e-8
    p1, m, v = cnn.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr, eps=eps)
    np.testing.assert_allclose(p1, p - lr * g / (np.abs(g) + eps), rtol=1e-14)
    p2, _, _ = cnn.adam_step(p1, g, m, v, 2, lr, eps=eps)
    np.testing.assert_allclose(p2, p1 - lr * g / (np.abs(g) + eps), rtol=1e-12)


def test_crop_mask():
    m = cnn.crop_mask(10, 12, 0, 5, 10, 40, 3)
    assert m[:, :3].sum() == 0 and m[:, -3:].sum() == 0
    assert m[0, 5] == 1 and m[-1, 5] == 1   # top and bottom are domain edges


def test_philox_matches_numpy_bit_generator():
    """Philox4x64-10 written from its definition against numpy's own Philox bit generator, which
    yields the blocks of counters 1, 2, 3, ... (it increments before each block)."""
    for key in ((0, 0), (12345, 678), (2**64 - 1, 2**63 + 5)):
        raw = np.random.Philox(key=np.array(key, dtype=np.uint64)).random_raw(4 * 40)
        mine = [w for c in range(1, 41) for w in cnn.philox4x64_10((c, 0, 0, 0), key)]
        assert [int(v) for v in raw] == mine
    # a counter with every word set: compare against numpy advanced to that counter
    g = np.random.Philox(counter=np.array([2**64 - 2, 7, 9, 11], dtype=np.uint64), key=np.array([3, 4], dtype=np.uint64))
    raw = g.random_raw(4)
    assert [int(v) for v in raw] == list(cnn.philox4x64_10((2**64 - 1, 7, 9, 11), (3, 4)))


def test_init_params_philox_distribution():
    """The seeded He-normal initialisation: zero biases, the layout of the library, and per layer a
    sample mean and variance consistent with N(0, 2 / (9 C_in)) (0.1 times that std for layer 6);
    different seeds give different draws, the same seed the same ones."""
    params, flat = cnn.init_params_philox(5)
    offs, total = cnn.param_layout()
    assert total == flat.size == 37889
    for l, ((w, b), (wo, bo)) in enumerate(zip(params, offs)):
        ci, co = cnn.CHANNELS[l], cnn.CHANNELS[l + 1]
        assert np.all(b == 0) and np.all(flat[bo:bo + co] == 0)
        np.testing.assert_array_equal(w.transpose(2, 3, 1, 0).reshape(-1), flat[wo:bo].astype(np.float64))
        std = math.sqrt(2.0 / (9 * ci)) * (0.1 if l == 5 else 1.0)
        n = w.size
        z = w.reshape(-1) / std
        assert abs(z.mean()) < 5.0 / math.sqrt(n)
        assert abs(z.var() - 1.0) < 6.0 * math.sqrt(2.0 / n)
    _, flat2 = cnn.init_params_philox(5)
    _, flat3 = cnn.init_params_philox(6)
    np.testing.assert_array_equal(flat, flat2)
    assert np.mean(flat != flat3) > 0.99
    # Box-Muller of the first two words, by hand for one index
    x0, x1, _, _ = cnn.philox4x64_10((7, 0, 0, 0), (5, 0))
    u1, u2 = (x0 >> 11) / 2.0**53, (x1 >> 11) / 2.0**53
    assert cnn.normal_at(7, 5) == math.sqrt(-2 * math.log(1 - u1)) * math.cos(2 * math.pi * u2)


def test_field_scale_and_equivariance():
    """The scale constants of a field (its RMS), and the network's scale equivariance: scaling u0 by a
    power of two c scales inv by 1/c and gain by c exactly, so u_hat scales by c exactly."""
    inv, gain = cnn.field_scale(np.full((4, 5), -0.5))
    assert inv == 2.0 and gain == 2.0 ** -12
    assert cnn.field_scale(np.zeros((3, 3))) == (1.0, 2.0 ** -11)
    rng = np.random.default_rng(9)
    params = cnn.init_params(2)
    u0 = rng.standard_normal((7, 6)) * 0.3
    kap = rng.uniform(0.05, 0.2, (7, 6))
    base, _ = cnn.forward(params, u0, kap)
    for c in (0.25, 8.0):
        got, _ = cnn.forward(params, c * u0, kap)
        np.testing.assert_array_equal(got, c * base)
    # the update is gain times the last layer's output
    inv, gain = cnn.field_scale(u0)
    _, (acts, zs) = cnn.forward(params, u0, kap)
    np.testing.assert_allclose(base - u0, gain * zs[-1][0], rtol=0, atol=4 * np.finfo(float).eps * np.abs(u0).max())
    np.testing.assert_array_equal(acts[0][0], u0 * inv)
