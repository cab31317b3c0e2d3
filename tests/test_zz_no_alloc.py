"""The allocation-free entry point (stencil_run_noalloc: the ping-pong field in the library's static
device array) against stencil_run with a caller workspace, bit for bit, on two calls in a row on one
GPU -- the second on a smaller grid, so that it reuses the array the first call left behind -- and
for 16-bit storage; a grid whose ping-pong field exceeds the array is refused."""
import sys

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pair(lib, torch, rows, cols, shape, r, steps, storage, seed, variant=None, tb=0):
    import gpuhelp as g
    W = wl.random_footprint_weights(np.random.default_rng(seed), shape, r)
    u0 = np.random.default_rng(seed + 1).random((rows, cols), dtype=np.float32)
    if storage != "f32":
        u0 = (torch.from_numpy(u0).to(torch.bfloat16 if storage == "bf16" else torch.float16)
              .view(torch.int16).numpy().view(np.uint16))
    say(f"noalloc case {rows}x{cols} shape={shape} r={r} steps={steps} {storage} variant={variant} tb={tb}")
    plan = lib.stencil_plan(rows, cols, r, W, 0.0, storage, 0)
    try:
        if variant is not None:
            lib.stencil_set_blocking(plan, 1)
            lib.stencil_set_variant(plan, variant)
            lib.stencil_set_blocking(plan, tb)
        x = g.to_dev(u0)
        ref = g.run(plan, x, steps, rows, cols, storage)
        out = torch.full_like(ref, -1)
        lib.stencil_run_noalloc(plan, x, out, steps)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(g.to_host(out), g.to_host(ref))
    finally:
        lib.stencil_destroy(plan)


def test_noalloc_two_calls_second_smaller():
    import torch
    import paper_2605_07954_amd as lib
    assert lib.stencil_noalloc_max_bytes() == 64 << 20
    # largest FP32 grid the array holds (16 Mi cells), then a smaller one over the same array
    _pair(lib, torch, 4096, 4096, wl.BOX, 3, 9, "f32", 11, lib.ST_VARIANT_MARCH8, 2)
    _pair(lib, torch, 300, 517, wl.STAR, 2, 13, "f32", 12)
    _pair(lib, torch, 257, 1000, wl.BOX, 1, 7, "bf16", 13, lib.ST_VARIANT_MARCH, 3)
    _pair(lib, torch, 61, 96, wl.STAR, 1, 0, "f16", 14)


def test_noalloc_refuses_oversized_grid():
    import torch
    import paper_2605_07954_amd as lib
    rows, cols = 4097, 4096  # one row past the array for FP32
    W = wl.heat5_weights()
    plan = lib.stencil_plan(rows, cols, 1, W, 0.0, "f32", 0)
    try:
        x = torch.zeros((rows, cols), device="cuda")
        out = torch.empty_like(x)
        with pytest.raises(lib.StencilError) as ei:
            lib.stencil_run_noalloc(plan, x, out, 10)
        assert ei.value.code == lib.ST_EUNSUPPORTED
        lib.stencil_run_noalloc(plan, x, out, 1)  # one pass needs no ping-pong field
        torch.cuda.synchronize()
    finally:
        lib.stencil_destroy(plan)
