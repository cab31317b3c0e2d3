"""Seeded random shapes through the row-marching variants, bitwise against the FP32-canonical oracle
(and the BF16/FP16-emulating oracle for 16-bit storage): grid sizes from one row to a few thousand
columns, radii 1-4, star and box footprints, halos of +0, -0.0 and other values, every depth a
variant offers at random, default and raised segment lengths.  This reaches the task layouts
(uniform, zoned, zero-side bands) at sizes and segment lengths the hand-picked cases do not."""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu


def _cases(n=36, seed=20261203):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        shape = wl.STAR if rng.random() < 0.6 else wl.BOX
        r = int(rng.integers(1, 5))
        rows = int(rng.choice([int(rng.integers(1, 40)), int(rng.integers(40, 900)), int(rng.integers(900, 3000))]))
        cols = int(rng.choice([int(rng.integers(1, 200)), int(rng.integers(200, 1200)), int(rng.integers(1200, 3000))]))
        if rng.random() < 0.5:
            cols = max(8, cols // 8 * 8)  # whole 16-byte vectors: the vector-access kernels
        b = float(rng.choice([0.0, 0.0, -0.0, 0.5, -1.25]))
        steps = int(rng.integers(1, 12))
        storage = "f32" if rng.random() < 0.75 else str(rng.choice(["bf16", "f16"]))
        seg = int(rng.choice([0, 0, 0, 5, 40]))
        out.append((rows, cols, shape, r, b, steps, storage, seg, int(rng.integers(0, 1 << 30))))
    return out


CASES = _cases()


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}-{c[2]}{c[3]}-b{c[4]}-T{c[5]}-{c[6]}-s{c[7]}" for c in CASES])
def test_march_random_shapes_bitwise(case):
    import torch
    import paper_2605_07954_amd as lib
    import gpuhelp as g
    from test_gpu_sweep import march_depth
    rows, cols, shape, r, b, steps, storage, seg, seed = case
    rng = np.random.default_rng(seed)
    W = wl.random_footprint_weights(rng, shape, r)
    u0 = rng.random((rows, cols), dtype=np.float32)
    if storage == "f32":
        x0, ref = u0, oracle.stencil_f32(u0, W, b, steps)
    else:
        x0 = oracle.to_bits(u0, storage)
        ref = oracle.stencil_lowp(x0, W, b, steps, storage)
    xd = g.to_dev(x0)
    for variant in (lib.ST_VARIANT_MARCH, lib.ST_VARIANT_MARCH8, lib.ST_VARIANT_MARCH1):
        tb = int(rng.integers(1, march_depth(shape, r, variant) + 1))
        plan = lib.stencil_plan(rows, cols, r, W, b, storage, 0)
        try:
            lib.stencil_set_blocking(plan, 1)
            lib.stencil_set_variant(plan, variant)
            lib.stencil_set_blocking(plan, tb)
            if seg:
                lib.stencil_set_march_segment(plan, seg)
            print(f"random march {rows}x{cols} {shape}{r} b={b} T={steps} {storage} variant {variant} tb {tb} seg {seg}",
                  flush=True)
            got = g.run(plan, xd, steps, rows, cols, storage)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(g.to_host(got), ref, err_msg=f"variant {variant} tb {tb}")
        finally:
            lib.stencil_destroy(plan)
