"""Pins of the CPU stencil oracle against things other than itself (no GPU).

Each test checks the oracle against a library routine, a closed form, an
exact invariant or exact small-integer arithmetic, chosen so that a dropped
tap, a wrong sign or index, or a transposed weight array fails at least one.
"""
import math

import numpy as np
import pytest
import scipy.signal
import torch

import oracle
import workloads as wl


def rand_weights(rng, r, asym=True):
    w = rng.uniform(-0.5, 1.0, size=(2 * r + 1, 2 * r + 1))
    return w.astype(np.float32)


# ---------------------------------------------------------------------------
# definition vs scipy's 2-D correlation (library routine), tiny and ragged grids
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("r", [1, 2, 3, 4])
@pytest.mark.parametrize("b", [0.0, 1.5])
def test_f64_matches_scipy_correlate2d(r, b):
    rng = np.random.default_rng(100 + r)
    for rows, cols in [(1, 1), (1, 7), (2, 3), (r, r + 1), (5, 9), (9, 4), (13, 11)]:
        W = rand_weights(rng, r)
        u0 = rng.random((rows, cols)).astype(np.float32)
        for T in (0, 1, 2, 3, 5):
            ref = u0.astype(np.float64)
            for _ in range(T):
                ref = scipy.signal.correlate2d(ref, W.astype(np.float64), mode="same",
                                               boundary="fill", fillvalue=b)
            got = oracle.stencil_f64(u0, W, b, T)
            np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12 * (1 + np.abs(ref).max()))


def test_single_tap_orientation():
    """W[dy+r][dx+r] = 1 alone gives u'(i,j) = u(i+dy, j+dx) (b outside): correlation, dy = row offset."""
    r = 2
    rng = np.random.default_rng(7)
    u0 = rng.random((6, 7)).astype(np.float32)
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            W = np.zeros((5, 5), dtype=np.float32)
            W[dy + r, dx + r] = 1.0
            got = oracle.stencil_f64(u0, W, -3.0, 1)
            exp = np.full(u0.shape, -3.0)
            for i in range(6):
                for j in range(7):
                    if 0 <= i + dy < 6 and 0 <= j + dx < 7:
                        exp[i, j] = u0[i + dy, j + dx]
            np.testing.assert_array_equal(got, exp)
            got32 = oracle.stencil_f32(u0, W, -3.0, 1)
            np.testing.assert_array_equal(got32, exp.astype(np.float32))


# ---------------------------------------------------------------------------
# closed forms
# ---------------------------------------------------------------------------

def _sine_mode(rows, cols, p, q):
    i = np.arange(1, rows + 1)[:, None]
    j = np.arange(1, cols + 1)[None, :]
    return np.sin(p * math.pi * i / (rows + 1)) * np.sin(q * math.pi * j / (cols + 1))


@pytest.mark.parametrize("rows,cols,p,q,T", [(512, 512, 32, 32, 100), (64, 48, 3, 5, 50), (33, 70, 1, 2, 20)])
def test_heat_sine_eigenmode(rows, cols, p, q, T):
    """Zero-Dirichlet 5-point star: sin modes are eigenvectors with eigenvalue c0 + 2 c1 (cos a + cos b)."""
    W = wl.heat5_weights()
    c0, c1 = float(W[1, 1]), float(W[0, 1])
    lam = c0 + 2 * c1 * (math.cos(p * math.pi / (rows + 1)) + math.cos(q * math.pi / (cols + 1)))
    u0 = _sine_mode(rows, cols, p, q)
    got = oracle.stencil_f64(u0.astype(np.float32), W, 0.0, T)
    exp = lam ** T * u0.astype(np.float32).astype(np.float64)
    # the FP32 rounding of u0 is not an eigenvector; its error decays too (|lambda| <= sum w = 1)
    assert oracle.rel_l2(got, exp) < 1e-7
    got64 = oracle.stencil_f64(u0, W.astype(np.float64), 0.0, T)
    assert oracle.rel_l2(got64, lam ** T * u0) < 1e-12


def test_box9_sine_eigenmode():
    """Symmetric 3x3 box: eigenvalue c0 + 2 c1 (cos a + cos b) + 4 c2 cos a cos b."""
    c0, c1, c2 = 0.4, 0.1, 0.05
    W = np.array([[c2, c1, c2], [c1, c0, c1], [c2, c1, c2]])
    rows, cols, p, q, T = 40, 56, 4, 9, 30
    a, bb = p * math.pi / (rows + 1), q * math.pi / (cols + 1)
    lam = c0 + 2 * c1 * (math.cos(a) + math.cos(bb)) + 4 * c2 * math.cos(a) * math.cos(bb)
    u0 = _sine_mode(rows, cols, p, q)
    got = oracle.stencil_f64(u0, W, 0.0, T)
    assert oracle.rel_l2(got, lam ** T * u0) < 1e-12


@pytest.mark.parametrize("shape,r", [(wl.BOX, 3), (wl.STAR, 2), (wl.BOX, 1)])
def test_plane_wave_light_cone(shape, r):
    """Away from the edges (distance >= r*T) a plane wave is multiplied by lambda(k)^T per step."""
    rng = np.random.default_rng(11)
    W = wl.random_footprint_weights(rng, shape, r)
    rows, cols, T = 96, 80, 9
    kx, ky, ph = 0.3, -0.7, 0.4
    i = np.arange(rows)[:, None]
    j = np.arange(cols)[None, :]
    u0 = np.cos(kx * j + ky * i + ph)
    lam = sum(float(W[dy + r, dx + r]) * complex(math.cos(kx * dx + ky * dy), math.sin(kx * dx + ky * dy))
              for dy in range(-r, r + 1) for dx in range(-r, r + 1))
    exp = (abs(lam) ** T) * np.cos(kx * j + ky * i + ph + T * math.atan2(lam.imag, lam.real))
    got = oracle.stencil_f64(u0, W, 0.0, T)
    m = r * T
    np.testing.assert_allclose(got[m:rows - m, m:cols - m], exp[m:rows - m, m:cols - m], atol=1e-12)
    # and the cells next to the edge do feel the halo
    assert np.abs(got[0] - exp[0]).max() > 1e-6


def test_constant_field():
    """Weights summing to exactly 1 with halo b = c keep u = c for ever; for any weights the cells at
    distance >= r*T from the edge hold c * (sum W)^T, and the edge cells feel the halo."""
    W1 = np.array([[0.0625, 0.125, 0.0625], [0.125, 0.25, 0.125], [0.0625, 0.125, 0.0625]], dtype=np.float32)
    u0 = np.full((30, 41), 1.75, dtype=np.float32)
    np.testing.assert_array_equal(oracle.stencil_f64(u0, W1, 1.75, 20), 1.75)
    np.testing.assert_array_equal(oracle.stencil_f32(u0, W1, 1.75, 20), np.float32(1.75))
    rng = np.random.default_rng(5)
    W = wl.random_footprint_weights(rng, wl.BOX, 2)
    s = float(np.sum(W.astype(np.float64)))
    c, T = 1.75, 12
    for b in (0.0, -2.0):
        got = oracle.stencil_f64(u0, W, b, T)
        m = 2 * T
        np.testing.assert_allclose(got[m:30 - m, m:41 - m], c * s ** T, rtol=1e-13)
        assert abs(got[0, 0] - c * s ** T) > 1e-3


# ---------------------------------------------------------------------------
# exact invariants
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("b", [0.0, 1.5])
@pytest.mark.parametrize("shape,r", [(wl.STAR, 1), (wl.BOX, 3), (wl.STAR, 3)])
def test_mass_budget(shape, r, b):
    """Summing one step over all cells: next mass = sum_j (u_j - b) S_j + b N sum W."""
    rng = np.random.default_rng(21)
    W = wl.random_footprint_weights(rng, shape, r)
    u = rng.random((23, 17))
    nxt = oracle.stencil_f64(u.astype(np.float32), W, b, 1)
    pred = oracle.norms_f64(u.astype(np.float32), W, b)[3]
    assert abs(pred - nxt.sum()) < 1e-12 * abs(nxt.sum())
    # a wrong support map (e.g. using the full sum everywhere) is detectably different
    assert abs(float(np.sum(u.astype(np.float32).astype(np.float64))) * float(W.astype(np.float64).sum())
               - nxt.sum()) > 1e-6


@pytest.mark.parametrize("rows,cols,r", [(5, 3, 4), (1, 1, 3), (2, 7, 4), (3, 2, 1), (4, 4, 4)])
def test_mass_budget_grids_smaller_than_the_stencil(rows, cols, r):
    """The support sum must ignore taps that reach past the whole grid (|d| >= side)."""
    rng = np.random.default_rng(rows * 10 + cols + r)
    W = wl.random_footprint_weights(rng, wl.BOX, r)
    u = rng.standard_normal((rows, cols)).astype(np.float32)
    for b in (0.0, 0.5):
        nxt = oracle.stencil_f64(u, W, b, 1).sum()
        pred = oracle.norms_f64(u, W, b)[3]
        assert abs(pred - nxt) < 1e-12 * (1 + abs(nxt))


def test_linearity_and_semigroup():
    rng = np.random.default_rng(3)
    W = wl.random_footprint_weights(rng, wl.BOX, 2)
    a = rng.random((20, 25))
    c = rng.random((20, 25))
    ra = oracle.stencil_f64(a, W, 0.0, 7)
    rc = oracle.stencil_f64(c, W, 0.0, 7)
    rs = oracle.stencil_f64(2.0 * a - 0.5 * c, W, 0.0, 7)
    np.testing.assert_allclose(rs, 2.0 * ra - 0.5 * rc, atol=1e-13)
    # run(3) then run(4) == run(7), bit for bit (FP32 and FP64)
    a32 = a.astype(np.float32)
    np.testing.assert_array_equal(oracle.stencil_f32(oracle.stencil_f32(a32, W, 0.5, 3), W, 0.5, 4),
                                  oracle.stencil_f32(a32, W, 0.5, 7))


# ---------------------------------------------------------------------------
# FP32-canonical mode
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape,r", [(wl.STAR, 1), (wl.BOX, 1), (wl.STAR, 3), (wl.BOX, 3), (wl.BOX, 4)])
def test_f32_exact_on_dyadic_data(shape, r):
    """Power-of-two weights and small integer inputs keep every FP32 operation exact,
    so the FP32 mode must equal the FP64 mode bit for bit (pins taps, offsets and order)."""
    rng = np.random.default_rng(31 + r)
    mask = wl.footprint(shape, r)
    W = np.where(mask, 2.0 ** -rng.integers(1, 6, size=mask.shape), 0.0).astype(np.float32)
    W *= np.where(rng.random(mask.shape) < 0.3, -1.0, 1.0).astype(np.float32)
    u0 = rng.integers(-64, 64, size=(11, 14)).astype(np.float32)
    for T in (1, 2):
        np.testing.assert_array_equal(oracle.stencil_f32(u0, W, 3.0, T).astype(np.float64),
                                      oracle.stencil_f64(u0, W, 3.0, T))


def test_f32_error_bound_box49():
    """|f32 - f64| stays within the standard FMA-chain bound n*u*sum|w|*max|x| per step, propagated."""
    p = wl.box49(crop=(64, 64), steps=50)
    f32 = oracle.stencil_f32(p.u0, p.weights, 0.0, p.steps).astype(np.float64)
    f64 = oracle.stencil_f64(p.u0, p.weights, 0.0, p.steps)
    u = 2.0 ** -24
    w1 = float(np.abs(p.weights.astype(np.float64)).sum())
    bound, mx = 0.0, 1.0
    for _ in range(p.steps):
        bound = w1 * bound + 49 * u * w1 * mx * (1 + 1e-6)
    err = np.abs(f32 - f64).max()
    assert err <= bound
    assert oracle.rel_l2(f32, f64) < 1e-6


# ---------------------------------------------------------------------------
# 16-bit formats and the storage-emulating mode
# ---------------------------------------------------------------------------

def _specials():
    return np.array([0.0, -0.0, 1.0, -1.0, 65504.0, 65520.0, 65519.99, 1e-8, 6.1e-5, 5.96e-8, 2.98e-8,
                     2.99e-8, 3e-38, 1e-45, np.inf, -np.inf, 3.3895e38, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8,
                     1.0 + 2 ** -11, 1.0 + 3 * 2 ** -11, 0.1, 1 / 3], dtype=np.float32)


def test_f16_rounding_matches_numpy():
    rng = np.random.default_rng(0)
    x = np.concatenate([_specials(),
                        (rng.standard_normal(200000) * 10.0 ** rng.uniform(-9, 5, 200000)).astype(np.float32),
                        rng.integers(0, 2 ** 32, 200000, dtype=np.uint64).astype(np.uint32).view(np.float32)])
    x = x[~np.isnan(x)]
    ref = x.astype(np.float16).view(np.uint16)
    np.testing.assert_array_equal(oracle.to_bits(x, "f16"), ref)
    back = oracle.from_bits(ref, "f16")
    np.testing.assert_array_equal(back, ref.view(np.float16).astype(np.float32))


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([_specials(),
                        (rng.standard_normal(200000) * 10.0 ** rng.uniform(-30, 30, 200000)).astype(np.float32),
                        rng.integers(0, 2 ** 32, 200000, dtype=np.uint64).astype(np.uint32).view(np.float32)])
    x = x[~np.isnan(x)]
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(oracle.to_bits(x, "bf16"), ref)
    back = torch.from_numpy(ref.view(np.int16)).view(torch.bfloat16).float().numpy()
    np.testing.assert_array_equal(oracle.from_bits(ref, "bf16"), back)


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_lowp_exact_on_dyadic_data(dtype):
    """Inputs and results that fit the 16-bit format exactly: the storage mode equals FP64."""
    W = wl.heat5_weights()
    W = np.array([[0, 0.125, 0], [0.25, 0.25, 0.125], [0, 0.25, 0]], dtype=np.float32)
    u0 = np.zeros((9, 10), dtype=np.float32)
    u0[4, 5] = 16.0
    u0[2, 2] = -8.0
    bits = oracle.to_bits(u0, dtype)
    got = oracle.from_bits(oracle.stencil_lowp(bits, W, 0.0, 2, dtype), dtype)
    np.testing.assert_array_equal(got.astype(np.float64), oracle.stencil_f64(u0, W, 0.0, 2))


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_lowp_is_f32_step_then_round(dtype):
    """One storage-mode step = FP32-canonical step followed by rounding to the format; b is rounded too."""
    p = wl.heat2d(40, 33, 1, seed=9)
    bits = oracle.to_bits(p.u0, dtype)
    x = oracle.from_bits(bits, dtype)
    b = 0.3
    bq = float(oracle.from_bits(oracle.to_bits(np.array([b], np.float32), dtype), dtype)[0])
    one = oracle.stencil_lowp(bits, p.weights, b, 1, dtype)
    np.testing.assert_array_equal(one, oracle.to_bits(oracle.stencil_f32(x, p.weights, bq, 1), dtype))
    # and the error of the 16-bit mode vs FP64 is of the order of the format's precision
    T = 20
    low = oracle.from_bits(oracle.stencil_lowp(bits, p.weights, 0.0, T, dtype), dtype)
    ref = oracle.stencil_f64(x, p.weights, 0.0, T)
    e = oracle.rel_l2(low, ref)
    eps = 2.0 ** -8 if dtype == "bf16" else 2.0 ** -11
    assert eps * 1e-3 < e < eps * T


# ---------------------------------------------------------------------------
# light-cone patch
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("y0,x0,h,w", [(0, 0, 8, 8), (30, 0, 5, 9), (20, 27, 7, 6), (56, 44, 8, 8), (0, 10, 64, 3)])
def test_patch_equals_full_run(y0, x0, h, w):
    rng = np.random.default_rng(8)
    W = wl.random_footprint_weights(rng, wl.BOX, 2)
    u0 = rng.random((64, 52)).astype(np.float32)
    T = 7
    full = oracle.stencil_f64(u0, W, 0.25, T)
    patch = oracle.stencil_patch_f64(u0, W, 0.25, T, y0, x0, h, w)
    assert not np.isnan(patch).any()
    np.testing.assert_array_equal(patch, full[y0:y0 + h, x0:x0 + w])


# ---------------------------------------------------------------------------
# variable-coefficient heat step
# ---------------------------------------------------------------------------

def test_varcoef_reduces_to_heat():
    """kappa == 0.1 gives centre 0.6 and 0.1 per neighbour, i.e. the 5-point heat stencil."""
    p = wl.heat2d(37, 29, 15, seed=2)
    kap = np.full(p.u0.shape, 0.1)
    got = oracle.varcoef_f64(p.u0, kap, 0.0, p.steps)
    W = np.array([[0, 0.1, 0], [0.1, 0.6, 0.1], [0, 0.1, 0]])
    np.testing.assert_allclose(got, oracle.stencil_f64(p.u0, W, 0.0, p.steps), atol=1e-13)
    lam = 0.6 + 0.2 * (math.cos(2 * math.pi / 38) + math.cos(3 * math.pi / 30))
    u0 = _sine_mode(37, 29, 2, 3)
    assert oracle.rel_l2(oracle.varcoef_f64(u0, kap, 0.0, 10), lam ** 10 * u0) < 1e-12


@pytest.mark.parametrize("b", [0.0, 0.7])
def test_varcoef_conservation(b):
    """Interior fluxes cancel in pairs: M' - M = sum over edge faces of kappa_c (b - u_c)."""
    u0, kap = wl.varcoef_problem(31, 26, seed=4)
    u = u0.astype(np.float64)
    k = kap.astype(np.float64)
    nxt = oracle.varcoef_f64(u0, kap, b, 1)
    flux = (np.sum(k[0] * (b - u[0])) + np.sum(k[-1] * (b - u[-1]))
            + np.sum(k[:, 0] * (b - u[:, 0])) + np.sum(k[:, -1] * (b - u[:, -1])))
    assert abs(nxt.sum() - u.sum() - flux) < 1e-12 * (1 + abs(u.sum()))


def test_varcoef_f32_close_to_f64():
    u0, kap = wl.varcoef_problem(64, 64, seed=1)
    a = oracle.varcoef_f32(u0, kap, 0.0, 16)
    c = oracle.varcoef_f64(u0, kap, 0.0, 16)
    assert oracle.rel_l2(a, c) < 1e-6


def test_norms_against_fsum():
    """Residual, energy and mass against math.fsum (exactly rounded sums) on a small field."""
    rng = np.random.default_rng(12)
    u = rng.standard_normal((17, 19)).astype(np.float32)
    up = rng.standard_normal((17, 19)).astype(np.float32)
    W = wl.heat5_weights()
    n = oracle.norms_f64(u, W, 0.0, up)
    d = u.astype(np.float64) - up.astype(np.float64)
    x = u.astype(np.float64).ravel()
    assert abs(n[0] - math.fsum((d * d).ravel())) < 1e-12 * n[0]
    assert abs(n[1] - math.fsum(x * x)) < 1e-12 * n[1]
    assert abs(n[2] - math.fsum(x)) < 1e-12 * (1 + abs(n[2]))
    assert oracle.norms_f64(u, W, 0.0)[0] == 0.0
