"""GPU checks of the matrix-core variant (the update as split-BF16 MFMA contractions, not the
canonical FMA order): rel-L2 against the FP64 oracle within the 1e-5 budget on ragged grids for
r = 1..4, star and box, b != 0; the Box-2D49P 1024^2 crop over 1000 steps; and at the benchmark's
full size (16384^2 x 1000) a plane wave in the light-cone interior against its closed form and the
8x8 corners against the FP64 light-cone patch oracle.  The autotuner takes it only when the plan
allows it (ST_FLAG_ALLOW_MFMA)."""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu
TOL = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def g():
    import torch  # noqa: F401
    import gpuhelp
    return gpuhelp


def mfma_run(g, lib, u, W, b, steps, flags=0):
    import torch
    rows, cols = u.shape
    r = (W.shape[0] - 1) // 2
    plan = lib.stencil_plan(rows, cols, r, W, b, "f32", flags)
    try:
        lib.stencil_set_blocking(plan, 1)
        lib.stencil_set_variant(plan, lib.ST_VARIANT_MFMA)
        x = g.to_dev(u)
        out = torch.full_like(x, float("nan"))
        ws = torch.empty_like(x)
        lib.stencil_run(plan, x, out, steps, ws)
        torch.cuda.synchronize()
        return g.to_host(out)
    finally:
        lib.stencil_destroy(plan)


CASES = [(37, 70, wl.BOX, 3, 0.0, 9), (300, 260, wl.STAR, 2, 0.5, 13), (129, 500, wl.BOX, 1, -0.25, 11),
         (257, 1000, wl.STAR, 4, 0.0, 7), (64, 64, wl.BOX, 4, 1.0, 5), (1, 3, wl.BOX, 2, 0.0, 3)]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}-{c[2]}{c[3]}" for c in CASES])
def test_mfma_within_fp32_rounding(g, case):
    import paper_2605_07954_amd as lib
    rows, cols, shape, r, b, steps = case
    W = wl.random_footprint_weights(np.random.default_rng(rows + cols + r), shape, r)
    u0 = np.random.default_rng(rows * cols + 1).random((rows, cols), dtype=np.float32)
    got = mfma_run(g, lib, u0, W, b, steps)
    ref64 = oracle.stencil_f64(u0, W, b, steps)
    ref32 = oracle.stencil_f32(u0, W, b, steps)
    e64 = oracle.rel_l2(got, ref64)
    e32 = oracle.rel_l2(ref32, ref64)
    say(f"mfma {case}: rel-L2 vs FP64 {e64:.2e} (the canonical FP32 order: {e32:.2e})")
    assert e64 <= TOL
    assert e64 <= 10 * e32 + 1e-7


def test_mfma_box49_crop_1000(g):
    import paper_2605_07954_amd as lib
    p = wl.box49(rows=1024, cols=1024, steps=1000)
    got = mfma_run(g, lib, p.u0, p.weights, 0.0, p.steps)
    e = oracle.rel_l2(got, oracle.stencil_f64(p.u0, p.weights, 0.0, p.steps))
    say(f"mfma box49 1024^2 crop x 1000: rel-L2 vs FP64 {e:.2e}")
    assert e <= TOL


def test_mfma_box49_16384_1000(g):
    """The full benchmark size with the matrix-core variant: plane wave through the light-cone
    interior (closed form) and the two opposite 8x8 corners (FP64 light-cone patch oracle)."""
    import torch
    import paper_2605_07954_amd as lib
    p = wl.box49()
    rows, cols, T, r = p.rows, p.cols, p.steps, p.radius
    W = p.weights.astype(np.float64)
    plan = lib.stencil_plan(rows, cols, r, p.weights, 0.0, "f32", lib.ST_FLAG_GRAPH)
    try:
        lib.stencil_set_blocking(plan, 1)
        lib.stencil_set_variant(plan, lib.ST_VARIANT_MFMA)
        x = g.to_dev(p.u0)
        out = torch.empty_like(x)
        ws = torch.empty_like(x)
        lib.stencil_run(plan, x, out, T, ws)
        torch.cuda.synchronize()
        tl = g.to_host(out[:8, :8])
        br = g.to_host(out[rows - 8:, cols - 8:])
        # plane wave cos(k x + phi) on the same grid
        kx, ky, phi = 0.02, 0.013, 0.7
        jj = torch.arange(cols, device=g.DEV, dtype=torch.float64)
        ii = torch.arange(rows, device=g.DEV, dtype=torch.float64)
        for k in range(0, rows, 2048):
            x[k:k + 2048] = torch.cos(kx * jj[None, :] + ky * ii[k:k + 2048, None] + phi).float()
        lib.stencil_run(plan, x, out, T, ws)
        torch.cuda.synchronize()
        m = r * T
        sample = np.linspace(m, rows - m - 1, 24).astype(np.int64)
        inner = g.to_host(out[torch.from_numpy(sample).to(g.DEV), m:cols - m])
    finally:
        lib.stencil_destroy(plan)
    del x, out, ws
    torch.cuda.empty_cache()
    d = np.arange(-r, r + 1)
    lam = np.sum(W * np.exp(1j * (ky * d[:, None] + kx * d[None, :])))
    j = np.arange(m, cols - m, dtype=np.float64)
    exact = abs(lam) ** T * np.cos(kx * j[None, :] + ky * sample[:, None].astype(np.float64) + phi + T * np.angle(lam))
    e_pw = oracle.rel_l2(inner, exact)
    e_tl = oracle.rel_l2(tl, oracle.stencil_patch_f64(p.u0, p.weights, 0.0, T, 0, 0, 8, 8))
    e_br = oracle.rel_l2(br, oracle.stencil_patch_f64(p.u0, p.weights, 0.0, T, rows - 8, cols - 8, 8, 8))
    say(f"mfma box49 16384^2 x 1000: plane wave {e_pw:.2e}, corners {e_tl:.2e} / {e_br:.2e}")
    assert max(e_pw, e_tl, e_br) <= TOL


def test_mfma_only_with_the_flag(g):
    """Without ST_FLAG_ALLOW_MFMA the autotuner never picks the matrix-core variant."""
    import torch
    import paper_2605_07954_amd as lib
    p = wl.box49(rows=1024, cols=1024, steps=24)
    x = g.to_dev(p.u0)
    out = torch.empty_like(x)
    ws = torch.empty_like(x)
    plan = lib.stencil_plan(p.rows, p.cols, 3, p.weights, 0.0, "f32", 0)
    try:
        lib.stencil_autotune(plan, x, out, ws, 24)
        assert lib.stencil_get_variant(plan) != lib.ST_VARIANT_MFMA
    finally:
        lib.stencil_destroy(plan)
