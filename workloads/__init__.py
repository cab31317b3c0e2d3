"""Seeded synthetic inputs for the stencil workloads.

This module only *draws* inputs: fields, weight sets, per-grid shapes and
coefficient tables.  It contains none of the stencil arithmetic, so both the
CPU oracle (``oracle/``) and the GPU library (``paper_2605_07954_amd``) can be
fed byte-identical host buffers from it without sharing any code with each
other.

The paper's workload is a synthetic heat-diffusion study (Sec. VI-A,
"Benchmarking Methodology": 1000 iterations on square grids); it uses no
dataset.  The shapes below follow the stencil families of Sec. II-B (star and
box footprints of radius r).  Every generator is a pure function of its seed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

STAR = "star"
BOX = "box"


# ---------------------------------------------------------------------------
# weight sets (dense (2r+1)x(2r+1) row-major; W[dy+r][dx+r] multiplies u[i+dy][j+dx])
# ---------------------------------------------------------------------------

def footprint(shape: str, r: int) -> np.ndarray:
    """Boolean (2r+1)^2 mask of the star (axes only) or box (full square) footprint (Sec. II-B)."""
    n = 2 * r + 1
    if shape == BOX:
        return np.ones((n, n), dtype=bool)
    if shape == STAR:
        m = np.zeros((n, n), dtype=bool)
        m[r, :] = True
        m[:, r] = True
        return m
    raise ValueError(f"unknown shape {shape!r}")


def heat5_weights() -> np.ndarray:
    """5-point heat weights: centre 0.6, each of the 4 neighbours 0.1, rounded to FP32."""
    w = np.zeros((3, 3), dtype=np.float32)
    w[1, 1] = np.float32(0.6)
    w[0, 1] = w[2, 1] = w[1, 0] = w[1, 2] = np.float32(0.1)
    return w


def star9_r2_weights() -> np.ndarray:
    """Radius-2 star: centre 0.5 and 0.0625 on each of the 8 arm points (sums to exactly 1)."""
    w = np.zeros((5, 5), dtype=np.float32)
    w[2, 2] = 0.5
    for k in (0, 1, 3, 4):
        w[2, k] = 0.0625
        w[k, 2] = 0.0625
    return w


def random_footprint_weights(rng: np.random.Generator, shape: str, r: int) -> np.ndarray:
    """Uniform[0,1) on the footprint, drawn in FP64, normalised to sum 1, then rounded to FP32."""
    mask = footprint(shape, r)
    vals = rng.random(int(mask.sum()))
    vals = vals / vals.sum()
    w = np.zeros(mask.shape, dtype=np.float64)
    w[mask] = vals
    return w.astype(np.float32)


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------

@dataclass
class Problem:
    name: str
    rows: int
    cols: int
    radius: int
    shape: str
    weights: np.ndarray  # float32 (2r+1, 2r+1)
    boundary: float
    steps: int
    u0: np.ndarray  # float32 (rows, cols)


def heat2d(rows: int = 512, cols: int = 512, steps: int = 100, seed: int = 0) -> Problem:
    """Heat-2D 5-point star: 512x512, 100 steps, centre 0.6 / 0.1 per neighbour, zero halo, U[0,1) seed 0."""
    u0 = np.random.default_rng(seed).random((rows, cols), dtype=np.float32)
    return Problem("heat2d-star5", rows, cols, 1, STAR, heat5_weights(), 0.0, steps, u0)


def box49_weights(seed: int = 1) -> np.ndarray:
    return random_footprint_weights(np.random.default_rng(seed), BOX, 3)


def box49(rows: int = 16384, cols: int = 16384, steps: int = 1000, seed: int = 1,
          crop: tuple[int, int] | None = None) -> Problem:
    """Box-2D49P (7x7 box, r=3): 49 weights U[0,1) from ``seed``, normalised, FP32.

    The interior field is drawn from the same generator right after the weights.
    With ``crop=(h, w)`` the top-left h x w corner of that field is returned and
    the problem shrinks to it (the 1024x1024 crop run).
    """
    rng = np.random.default_rng(seed)
    w = random_footprint_weights(rng, BOX, 3)
    u0 = rng.random((rows, cols), dtype=np.float32)
    if crop is not None:
        u0 = np.ascontiguousarray(u0[: crop[0], : crop[1]])
        rows, cols = crop
    return Problem("box49", rows, cols, 3, BOX, w, 0.0, steps, u0)


def fourier_sine_modes(n_modes: int, kmax: float, seed: int) -> list[tuple[int, int, float]]:
    """(p, q, a) of ``n_modes`` distinct integer wave numbers in [1, kmax]^2 with sqrt(p^2+q^2) <= kmax,
    amplitude a ~ N(0, 1/k^2), all drawn from ``default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    kmax_i = int(math.floor(kmax))
    cand = [(p, q) for p in range(1, kmax_i + 1) for q in range(1, kmax_i + 1)
            if math.hypot(p, q) <= kmax]
    n_modes = min(n_modes, len(cand))
    idx = rng.choice(len(cand), size=n_modes, replace=False)
    modes = []
    for m in idx:
        p, q = cand[m]
        modes.append((p, q, float(rng.normal(0.0, 1.0 / math.hypot(p, q)))))
    return modes


def fourier_sine_field(rows: int, cols: int, n_modes: int, kmax: float, seed: int,
                       dtype=np.float32) -> np.ndarray:
    """Sum of Dirichlet sine modes a sin(p pi (i+1)/(N+1)) sin(q pi (j+1)/(M+1)) over
    ``fourier_sine_modes``; evaluated in FP64 as an outer product per mode."""
    i = np.arange(1, rows + 1, dtype=np.float64)
    j = np.arange(1, cols + 1, dtype=np.float64)
    out = np.zeros((rows, cols), dtype=np.float64)
    for p, q, a in fourier_sine_modes(n_modes, kmax, seed):
        out += a * np.outer(np.sin(p * math.pi * i / (rows + 1)), np.sin(q * math.pi * j / (cols + 1)))
    return out.astype(dtype)


def star9_precision(rows: int = 8192, cols: int = 8192, steps: int = 500, seed: int = 4) -> Problem:
    """Star-2D9P (r=2), centre 0.5 / 0.0625 per arm point, initial field = 64 random sine modes, k <= 32."""
    u0 = fourier_sine_field(rows, cols, 64, 32.0, seed)
    return Problem("star9-r2", rows, cols, 2, STAR, star9_r2_weights(), 0.0, steps, u0)


# ---------------------------------------------------------------------------
# batched workload: 256 grids, log-uniform sides, mixed stencils
# ---------------------------------------------------------------------------

BATCH_SHAPES = ((STAR, 1), (BOX, 1), (STAR, 3))


def batch_specs(n_grids: int = 256, lo: int = 64, hi: int = 2048, seed: int = 3):
    """Per-grid (rows, cols, shape, radius): sides log-uniform in [lo, hi], shape uniform over
    {5-pt star r1, 9-pt box r1, 13-pt star r3}; all drawn from ``default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    specs = []
    for _ in range(n_grids):
        k = int(rng.integers(len(BATCH_SHAPES)))
        rows = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        cols = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        shape, r = BATCH_SHAPES[k]
        specs.append((rows, cols, shape, r))
    return specs


def batch_problems(n_grids: int = 256, steps: int = 200, lo: int = 64, hi: int = 2048,
                   seed: int = 3) -> list[Problem]:
    """Grid g: weights from default_rng(10000+g) on its footprint, input U[0,1) from default_rng(g)."""
    out = []
    for g, (rows, cols, shape, r) in enumerate(batch_specs(n_grids, lo, hi, seed)):
        w = random_footprint_weights(np.random.default_rng(10000 + g), shape, r)
        u0 = np.random.default_rng(g).random((rows, cols), dtype=np.float32)
        out.append(Problem(f"batch{g}-{shape}{r}", rows, cols, r, shape, w, 0.0, steps, u0))
    return out


# ---------------------------------------------------------------------------
# variable-coefficient heat (surrogate workload)
# ---------------------------------------------------------------------------

def smooth_kappa(rows: int, cols: int, seed: int, lo: float = 0.05, hi: float = 0.2,
                 n_modes: int = 8, kmax: int = 3) -> np.ndarray:
    """Diffusivity: 8 random cosine modes with wave numbers in [0,3]^2 minus 0, rescaled to [lo, hi]."""
    rng = np.random.default_rng(seed)
    y = np.arange(rows, dtype=np.float64)[:, None] / rows
    x = np.arange(cols, dtype=np.float64)[None, :] / cols
    g = np.zeros((rows, cols), dtype=np.float64)
    for _ in range(n_modes):
        while True:
            kx, ky = (int(v) for v in rng.integers(0, kmax + 1, size=2))
            if kx or ky:
                break
        g += rng.normal() * np.cos(2 * math.pi * (kx * x + ky * y) + rng.uniform(0, 2 * math.pi))
    g = (g - g.min()) / max(g.max() - g.min(), 1e-300)
    return (lo + (hi - lo) * g).astype(np.float32)


def field_coefficients(n: int, seed: int, n_u: int = 16, n_k: int = 8, kmax_u: int = 8,
                       kmax_k: int = 3) -> np.ndarray:
    """Per-trajectory random coefficients, an (n, 4*(n_u+n_k)) FP32 table.

    Row layout: ``n_u`` sine modes (p, q, amplitude, 0) with integer p, q >= 1,
    sqrt(p^2+q^2) <= kmax_u and amplitude ~ N(0, 1/k^2), followed by ``n_k``
    cosine modes (kx, ky, amplitude, phase) with (kx, ky) in [0, kmax_k]^2 minus
    the origin, amplitude ~ N(0, 1) and phase ~ U[0, 2 pi).  Only random draws;
    :func:`synth_fields` turns a row into (u0, kappa).
    """
    rng = np.random.default_rng(seed)
    tab = np.zeros((n, n_u + n_k, 4), dtype=np.float32)
    for t in range(n):
        for m in range(n_u):
            while True:
                p, q = (int(v) for v in rng.integers(1, kmax_u + 1, size=2))
                if math.hypot(p, q) <= kmax_u:
                    break
            tab[t, m] = (p, q, rng.normal(0.0, 1.0 / math.hypot(p, q)), 0.0)
        for m in range(n_k):
            while True:
                kx, ky = (int(v) for v in rng.integers(0, kmax_k + 1, size=2))
                if kx or ky:
                    break
            tab[t, n_u + m] = (kx, ky, rng.normal(), rng.uniform(0, 2 * math.pi))
    return tab.reshape(n, -1)


KAPPA_MID = 0.125
KAPPA_HALF = 0.075


def synth_fields(coef_row: np.ndarray, rows: int, cols: int, n_u: int = 16):
    """Evaluate one coefficient row into (u0, kappa), both FP32 (rows, cols), in FP64 then rounded.

    u0(i, j)    = sum_m a_m sin(p_m pi (i+1)/(rows+1)) sin(q_m pi (j+1)/(cols+1))
    kappa(i, j) = 0.125 + 0.075 * g(i, j) / sum_m |b_m|,
    g(i, j)     = sum_m b_m cos(2 pi (kx_m j/cols + ky_m i/rows) + phi_m)
    so kappa lies in [0.05, 0.2] without a data-dependent rescale.
    """
    c = np.asarray(coef_row, dtype=np.float64).reshape(-1, 4)
    i = np.arange(1, rows + 1, dtype=np.float64)
    j = np.arange(1, cols + 1, dtype=np.float64)
    u = np.zeros((rows, cols))
    for p, q, a, _ in c[:n_u]:
        u += a * np.outer(np.sin(p * math.pi * i / (rows + 1)), np.sin(q * math.pi * j / (cols + 1)))
    y = np.arange(rows, dtype=np.float64)[:, None] / rows
    x = np.arange(cols, dtype=np.float64)[None, :] / cols
    g = np.zeros((rows, cols))
    norm = 0.0
    for kx, ky, b, ph in c[n_u:]:
        g += b * np.cos(2 * math.pi * (kx * x + ky * y) + ph)
        norm += abs(b)
    kappa = KAPPA_MID + KAPPA_HALF * g / max(norm, 1e-30)
    return u.astype(np.float32), kappa.astype(np.float32)


def varcoef_problem(rows: int = 1024, cols: int = 1024, seed: int = 0):
    """(u0, kappa) of one variable-coefficient heat trajectory, from :func:`field_coefficients`."""
    return synth_fields(field_coefficients(1, seed)[0], rows, cols)
