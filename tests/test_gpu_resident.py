"""GPU parity of the LDS-resident variant (one cooperative launch; tiles kept in LDS, an r*tb-deep
halo swapped with the eight neighbours every tb steps through global memory, gated by per-tile
counters with bounded waits): bit for bit with the FP32-canonical / 16-bit-emulating oracle at
several swap depths, ragged grids, r = 1..4, b != 0; the Heat-2D 512^2 x 100 workload; no wait gives
up in a normal run; and a run whose waits the host limits to one poll ends normally, with the
give-up (if a wait needed a second poll) recorded."""
import sys

import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def g():
    import torch  # noqa: F401
    import gpuhelp
    return gpuhelp


def resident_run(g, lib, u, W, b, steps, tb, storage="f32", spin=1 << 18):
    import torch
    rows, cols = u.shape
    r = (W.shape[0] - 1) // 2
    plan = lib.stencil_plan(rows, cols, r, W, b, storage, 0)
    try:
        lib.stencil_set_blocking(plan, 1)
        lib.stencil_set_variant(plan, lib.ST_VARIANT_RESIDENT)
        lib.stencil_set_blocking(plan, tb)
        lib.stencil_set_spin_limit(plan, spin)
        x = g.to_dev(u)
        out = torch.full_like(x, -1)
        ws = torch.empty(max(lib.stencil_workspace_bytes(plan, steps), 4), dtype=torch.uint8, device=g.DEV)
        lib.stencil_run(plan, x, out, steps, ws)
        status = lib.stencil_resident_status(plan, ws)
        return g.to_host(out), status
    finally:
        lib.stencil_destroy(plan)


def test_heat2d_512_resident(g):
    import paper_2605_07954_amd as lib
    p = wl.heat2d()
    ref = oracle.stencil_f32(p.u0, p.weights, 0.0, p.steps)
    for tb in (1, 4, 8, 16, 25):
        say(f"heat2d 512^2 x 100 resident tb={tb}")
        got, status = resident_run(g, lib, p.u0, p.weights, 0.0, p.steps, tb)
        assert status[0] == 0, status
        np.testing.assert_array_equal(got, ref, err_msg=f"tb {tb}")


CASES = [(300, 260, wl.STAR, 2, 0.5, 23, 5), (129, 500, wl.BOX, 1, 0.0, 11, 3), (257, 1000, wl.BOX, 3, -0.25, 9, 2),
         (700, 640, wl.STAR, 4, 0.0, 7, 3), (64, 64, wl.STAR, 1, 1.0, 30, 2), (1024, 1024, wl.BOX, 2, 0.0, 10, 4)]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}-{c[2]}{c[3]}-tb{c[6]}" for c in CASES])
def test_resident_bitwise(g, case):
    import paper_2605_07954_amd as lib
    rows, cols, shape, r, b, steps, tb = case
    W = wl.random_footprint_weights(np.random.default_rng(rows + cols + r), shape, r)
    u0 = np.random.default_rng(rows * cols).random((rows, cols), dtype=np.float32)
    say(f"resident {case}")
    got, status = resident_run(g, lib, u0, W, b, steps, tb)
    assert status[0] == 0, status
    np.testing.assert_array_equal(got, oracle.stencil_f32(u0, W, b, steps))


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_resident_lowp_bitwise(g, storage):
    import paper_2605_07954_amd as lib
    rows, cols, r, steps, tb = 300, 260, 2, 13, 4
    W = wl.random_footprint_weights(np.random.default_rng(5), wl.STAR, r)
    bits = oracle.to_bits(np.random.default_rng(6).random((rows, cols), dtype=np.float32), storage)
    got, status = resident_run(g, lib, bits, W, 0.0, steps, tb, storage)
    assert status[0] == 0, status
    np.testing.assert_array_equal(got, oracle.stencil_lowp(bits, W, 0.0, steps, storage))


def test_resident_forced_give_up_ends_normally(g):
    """Waits limited to one poll by the host: the launch still ends (every workgroup leaves at its
    next wait once one gave up), the status names a give-up whenever a wait needed a second poll,
    and a run without a give-up is exact."""
    import torch
    import paper_2605_07954_amd as lib
    p = wl.heat2d()
    ref = oracle.stencil_f32(p.u0, p.weights, 0.0, p.steps)
    gave_up = 0
    for rep in range(4):
        got, status = resident_run(g, lib, p.u0, p.weights, 0.0, p.steps, 4, spin=1)
        torch.cuda.synchronize()
        say(f"spin limit 1, run {rep}: status {status}")
        if status[0]:
            gave_up += 1
            assert 0 <= status[1] < 256 and 1 <= status[2] <= 25 and 0 <= status[3] < 256
        else:
            np.testing.assert_array_equal(got, ref)
    assert gave_up >= 1
    # and the plan works normally again with the default limit
    got, status = resident_run(g, lib, p.u0, p.weights, 0.0, p.steps, 4)
    assert status[0] == 0
    np.testing.assert_array_equal(got, ref)
