"""Pins of the oracle's periodic and framed boundaries and of its 3D form (no GPU): library
correlation routines with the matching boundary mode, closed forms on a torus and in a box,
invariants (mass on a torus, a linear steady state carried by its frame, constant fields), and
reductions to the constant-halo definition."""
import math

import numpy as np
import pytest
from scipy import ndimage, signal

import oracle


def _w(rng, r, sym=False):
    W = rng.random((2 * r + 1, 2 * r + 1))
    if sym:
        W = W + W[::-1, :] + W[:, ::-1] + W[::-1, ::-1]
    return (W / W.sum()).astype(np.float32)


def _scipy_periodic(u, W, steps):
    x = u.astype(np.float64)
    for _ in range(steps):
        x = ndimage.correlate(x, W.astype(np.float64), mode="grid-wrap")
    return x


@pytest.mark.parametrize("rows,cols,r,steps", [(7, 9, 1, 5), (5, 3, 2, 4), (2, 11, 3, 3), (1, 1, 1, 2), (3, 2, 4, 3),
                                               (13, 8, 2, 7)])
def test_periodic_matches_scipy_wrap(rows, cols, r, steps):
    rng = np.random.default_rng(rows * 31 + cols + r)
    W = rng.standard_normal((2 * r + 1, 2 * r + 1)).astype(np.float32)  # asymmetric, signed
    u = rng.random((rows, cols), dtype=np.float32)
    got = oracle.stencil_bc_f64(u, W, "periodic", steps)
    np.testing.assert_allclose(got, _scipy_periodic(u, W, steps), rtol=1e-12, atol=1e-12)
    g32 = oracle.stencil_bc_f32(u, W, "periodic", steps)
    assert oracle.rel_l2(g32, got) < 1e-5


def test_periodic_single_tap_shift_wraps():
    rng = np.random.default_rng(3)
    u = rng.random((6, 10), dtype=np.float32)
    for dy, dx in [(1, 0), (0, -2), (-2, 1)]:
        W = np.zeros((5, 5), dtype=np.float32)
        W[dy + 2, dx + 2] = 1.0
        got = oracle.stencil_bc_f32(u, W, "periodic", 3)
        np.testing.assert_array_equal(got, np.roll(u, (-3 * dy, -3 * dx), axis=(0, 1)))


def test_periodic_plane_wave_exact_everywhere():
    """On a torus every Fourier mode exp(i k.x) with k = 2 pi m / N is an eigenfunction:
    u^T = |lam|^T cos(k.x + phi + T arg lam), lam = sum_d W_d exp(i k.d), in every cell."""
    rng = np.random.default_rng(4)
    rows, cols, r, T = 48, 40, 3, 25
    W = _w(rng, r)
    ky, kx, phi = 2 * math.pi * 3 / rows, 2 * math.pi * 5 / cols, 0.3
    ii, jj = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
    u0 = np.cos(kx * jj + ky * ii + phi)
    d = np.arange(-r, r + 1)
    lam = np.sum(W.astype(np.float64) * np.exp(1j * (ky * d[:, None] + kx * d[None, :])))
    exact = abs(lam) ** T * np.cos(kx * jj + ky * ii + phi + T * np.angle(lam))
    got = oracle.stencil_bc_f64(u0, W, "periodic", T)
    np.testing.assert_allclose(got, exact, atol=1e-12)


def test_periodic_conserves_mass():
    rng = np.random.default_rng(5)
    W = _w(rng, 2)
    u = rng.random((33, 27))
    got = oracle.stencil_bc_f64(u, W, "periodic", 40)
    s = float(np.sum(W.astype(np.float64)))
    assert abs(got.sum() - s ** 40 * u.sum()) <= 1e-11 * abs(u.sum())


def _frame_of(ext, rows, cols, r):
    """The frame layout from an extended (rows + 2r) x (cols + 2r) array: top, bottom, left, right."""
    top = ext[:r, :]
    bot = ext[rows + r:, :]
    left = ext[r:rows + r, :r]
    right = ext[r:rows + r, cols + r:]
    return np.concatenate([top.reshape(-1), bot.reshape(-1), left.reshape(-1), right.reshape(-1)])


@pytest.mark.parametrize("rows,cols,r,steps", [(6, 8, 1, 4), (5, 3, 2, 3), (9, 12, 3, 5), (2, 2, 4, 2)])
def test_frame_matches_padded_correlation(rows, cols, r, steps):
    """Each step is the 'valid' correlation (a library routine) of the grid padded with the frame."""
    rng = np.random.default_rng(rows + 7 * cols + r)
    W = rng.standard_normal((2 * r + 1, 2 * r + 1)).astype(np.float32)
    u = rng.random((rows, cols))
    ext = rng.standard_normal((rows + 2 * r, cols + 2 * r))
    frame = _frame_of(ext, rows, cols, r)
    assert frame.size == oracle.frame_elems(rows, cols, r)
    x = u.copy()
    for _ in range(steps):
        e = ext.copy()
        e[r:rows + r, r:cols + r] = x
        x = signal.correlate2d(e, W.astype(np.float64), mode="valid")
    got = oracle.stencil_bc_f64(u, W, "frame", steps, frame)
    np.testing.assert_allclose(got, x, rtol=1e-12, atol=1e-12)


def test_constant_frame_is_the_constant_halo():
    rng = np.random.default_rng(8)
    for r, b in [(1, 0.0), (2, 1.5), (3, -0.25)]:
        W = _w(rng, r)
        u = rng.random((20, 17), dtype=np.float32)
        fr = np.full(oracle.frame_elems(20, 17, r), b)
        np.testing.assert_array_equal(oracle.stencil_bc_f32(u, W, "frame", 9, fr), oracle.stencil_f32(u, W, b, 9))
        np.testing.assert_array_equal(oracle.stencil_bc_f64(u, W, "frame", 9, fr), oracle.stencil_f64(u, W, b, 9))
        bits = oracle.to_bits(u, "bf16")
        fb = oracle.to_bits(fr.astype(np.float32), "bf16")
        np.testing.assert_array_equal(oracle.stencil_bc_lowp(bits, W, "frame", 9, "bf16", fb),
                                      oracle.stencil_lowp(bits, W, b, 9, "bf16"))


def test_frame_carries_a_linear_steady_state():
    """With symmetric weights summing to one, u = a i + b j + c is a fixed point when the frame
    continues it: the first moments of the weights vanish."""
    rng = np.random.default_rng(9)
    rows, cols, r = 14, 11, 2
    W = _w(rng, r, sym=True)
    W = (W.astype(np.float64) / W.astype(np.float64).sum())
    ii, jj = np.meshgrid(np.arange(-r, rows + r), np.arange(-r, cols + r), indexing="ij")
    ext = 0.3 * ii - 0.7 * jj + 2.0
    u = ext[r:rows + r, r:cols + r]
    got = oracle.stencil_bc_f64(u, W, "frame", 30, _frame_of(ext, rows, cols, r))
    np.testing.assert_allclose(got, u, atol=1e-11)


def test_lowp_periodic_shift_and_rounding():
    rng = np.random.default_rng(10)
    u = rng.random((9, 16), dtype=np.float32)
    bits = oracle.to_bits(u, "f16")
    W = np.zeros((3, 3), dtype=np.float32)
    W[2, 1] = 1.0
    np.testing.assert_array_equal(oracle.stencil_bc_lowp(bits, W, "periodic", 4, "f16"), np.roll(bits, -4, axis=0))
    # one step: the FP32-canonical periodic step of the widened field, rounded once
    W = _w(rng, 1)
    one = oracle.stencil_bc_lowp(bits, W, "periodic", 1, "f16")
    ref = oracle.to_bits(oracle.stencil_bc_f32(oracle.from_bits(bits, "f16"), W, "periodic", 1), "f16")
    np.testing.assert_array_equal(one, ref)


# ---- 3D ------------------------------------------------------------------------------------

def _scipy3d(u, W, b, steps):
    x = u.astype(np.float64)
    for _ in range(steps):
        x = ndimage.correlate(x, W.astype(np.float64), mode="constant", cval=b)
    return x


@pytest.mark.parametrize("shape,r,b,steps", [((4, 5, 6), 1, 0.0, 4), ((3, 7, 2), 2, 1.5, 3), ((2, 2, 9), 1, -1.0, 5),
                                             ((5, 4, 4), 3, 0.0, 2)])
def test_3d_matches_scipy(shape, r, b, steps):
    rng = np.random.default_rng(sum(shape) + r)
    W = rng.standard_normal((2 * r + 1,) * 3).astype(np.float32)
    u = rng.random(shape, dtype=np.float32)
    got = oracle.stencil3d_f64(u, W, b, steps)
    np.testing.assert_allclose(got, _scipy3d(u, W, b, steps), rtol=1e-12, atol=1e-12)
    assert oracle.rel_l2(oracle.stencil3d_f32(u, W, b, steps), got) < 1e-5


def test_3d_sine_eigenmode():
    """The 7-point star's Dirichlet sine mode decays by c0 + 2 c1 (cos a + cos b + cos g) per step,
    and a symmetric 27-point box's by sum_d W_d cos(a dz) cos(b dy) cos(g dx)."""
    P, R, C, T = 12, 10, 14, 20
    p, q, s = 2, 3, 1
    a, bb, g = p * math.pi / (P + 1), q * math.pi / (R + 1), s * math.pi / (C + 1)
    kk, ii, jj = np.meshgrid(np.arange(P), np.arange(R), np.arange(C), indexing="ij")
    u0 = np.sin(a * (kk + 1)) * np.sin(bb * (ii + 1)) * np.sin(g * (jj + 1))
    W = np.zeros((3, 3, 3), dtype=np.float32)
    W[1, 1, 1] = 0.4
    for d in [(0, 1, 1), (2, 1, 1), (1, 0, 1), (1, 2, 1), (1, 1, 0), (1, 1, 2)]:
        W[d] = 0.1
    c0, c1 = float(W[1, 1, 1]), float(W[0, 1, 1])
    lam = c0 + 2 * c1 * (math.cos(a) + math.cos(bb) + math.cos(g))
    np.testing.assert_allclose(oracle.stencil3d_f64(u0, W, 0.0, T), lam ** T * u0, atol=1e-13)
    rng = np.random.default_rng(12)
    B = rng.random((3, 3, 3))
    B = B + B[::-1]           # even in dz,
    B = B + B[:, ::-1]        # in dy,
    B = B + B[:, :, ::-1]     # and in dx
    B = (B / B.sum()).astype(np.float32)
    d = np.array([-1, 0, 1])
    lamb = float(np.sum(B.astype(np.float64) * np.cos(a * d)[:, None, None] * np.cos(bb * d)[None, :, None]
                        * np.cos(g * d)[None, None, :]))
    np.testing.assert_allclose(oracle.stencil3d_f64(u0, B, 0.0, T), lamb ** T * u0, atol=1e-13)


def test_3d_constant_field_and_shift():
    rng = np.random.default_rng(13)
    # dyadic weights summing to exactly one keep a constant field whose halo matches it, bit for bit
    D = np.zeros((5, 5, 5), dtype=np.float32)
    D[2, 2, 2] = 0.5
    for d in [(0, 2, 2), (4, 2, 2), (2, 1, 2), (2, 3, 2), (2, 2, 0), (2, 2, 4), (1, 1, 1), (3, 3, 3)]:
        D[d] = 1.0 / 16
    u = np.full((6, 7, 8), 0.75, dtype=np.float32)
    np.testing.assert_array_equal(oracle.stencil3d_f32(u, D, 0.75, 5), u)
    # any weights: cells r T or more from every face hold c (sum W)^T
    W = rng.random((5, 5, 5)).astype(np.float32)
    s = float(np.sum(W.astype(np.float64)))
    u = np.full((16, 15, 14), 0.75)
    got = oracle.stencil3d_f64(u, W, 0.0, 3)
    np.testing.assert_allclose(got[6:10, 6:9, 6:8], 0.75 * s ** 3, rtol=1e-13)
    u = rng.random((6, 7, 8), dtype=np.float32)
    S = np.zeros((3, 3, 3), dtype=np.float32)
    S[2, 1, 1] = 1.0  # takes the value one plane further: the field moves up by a plane per step
    got = oracle.stencil3d_f32(u, S, 0.5, 2)
    np.testing.assert_array_equal(got[:4], u[2:])
    assert np.all(got[4:] == 0.5)
