"""GPU parity of the plain sweep against the CPU oracle (through the C ABI).

The kernels follow the oracle's FP32 order (centre product, then one FMA per
footprint tap in row-major order), so FP32 results are compared BIT FOR BIT
with the FP32-canonical oracle; the accuracy gate is rel-L2 <= 1e-5 against
the FP64 oracle, and the FP64 error is printed for every case.
"""
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


def _weights(shape, r, seed):
    return wl.random_footprint_weights(np.random.default_rng(seed), shape, r)


def test_heat2d_512_100(g):
    p = wl.heat2d()
    ref32 = oracle.stencil_f32(p.u0, p.weights, 0.0, p.steps)
    ref64 = oracle.stencil_f64(p.u0, p.weights, 0.0, p.steps)
    for flags, tb, tile in [(1, 0, None), (0, 1, None), (0, 4, (128, 64)), (0, 7, (64, 64)), (0, 10, (256, 32)),
                            (2, 5, (128, 32))]:
        say("heat2d", flags, tb, tile)
        got = g.run_problem(p.u0, p.weights, 0.0, p.steps, flags=flags, tb=tb, tile=tile)
        e64 = oracle.rel_l2(got, ref64)
        say(f"  rel-L2 vs f64 = {e64:.3e}")
        assert e64 <= TOL
        np.testing.assert_array_equal(got, ref32)



@pytest.mark.parametrize("kind", ["identity", "zero", "shift"])
def test_degenerate_weights(g, kind):
    """Degenerate footprints through every variant: the identity (centre weight 1: the field comes
    back unchanged, bit for bit), all-zero weights (every cell 0 after one step), and a pure shift
    (one off-centre tap of weight 1 and a zero centre: the field moves one cell per step and b
    flows in from the edge).  The kernels multiply every tap of the footprint, zero weights
    included, while the oracle takes the nonzero taps only; that can change nothing but the sign of
    an exact zero, so signs are compared where no exact zero arises."""
    import torch
    import paper_2605_07954_amd as lib
    rows, cols, r, b, steps = 70, 132, 2, 0.75, 5
    W = np.zeros((2 * r + 1, 2 * r + 1), np.float32)
    if kind == "identity":
        W[r, r] = 1.0
    elif kind == "shift":
        W[r - 1, r] = 1.0  # u'(i, j) = u(i - 1, j)
    u0 = (np.random.default_rng(3).random((rows, cols), dtype=np.float32) - 0.5)
    ref = oracle.stencil_f32(u0, W, b, steps)
    if kind == "identity":
        np.testing.assert_array_equal(ref, u0)
    if kind == "shift":
        np.testing.assert_array_equal(ref[steps:], u0[:-steps])
        assert np.all(ref[:steps] == np.float32(b))
    x = g.to_dev(u0)
    for variant in (lib.ST_VARIANT_TILED, lib.ST_VARIANT_STREAM, lib.ST_VARIANT_MARCH, lib.ST_VARIANT_MARCH8,
                    lib.ST_VARIANT_MARCH1):
        for flags in (0, lib.ST_FLAG_NAIVE):
            plan = lib.stencil_plan(rows, cols, r, W, b, "f32", flags)
            try:
                lib.stencil_set_blocking(plan, 1)
                lib.stencil_set_variant(plan, variant)
                lib.stencil_set_blocking(plan, 2)
                out = torch.full_like(x, float("nan"))
                ws = torch.empty_like(x)
                lib.stencil_run(plan, x, out, steps, ws)
                torch.cuda.synchronize()
                got = g.to_host(out)
                np.testing.assert_array_equal(got, ref, err_msg=f"{kind} variant {variant} flags {flags}")
                if kind != "zero":
                    assert np.array_equal(np.signbit(got), np.signbit(ref)), f"{kind}: signs differ"
            finally:
                lib.stencil_destroy(plan)


def test_naive_paths_beyond_one_cell_per_thread(g):
    """The one-cell-per-thread reference kernels (ST_FLAG_NAIVE) stride once the grid has more cells
    than their capped launch has threads (2^20 workgroups x 256 = 2^28): a 16400^2 grid, one step, for
    the constant-weight and the varcoef path.  The first and last rows are checked bit for bit
    against the FP32 oracle on a crop (one step: every crop row but the one at the cut is exact), the
    whole field against the tiled kernels bit for bit."""
    import torch
    import paper_2605_07954_amd as lib
    n, b, h = 16400, 0.3, 8
    assert n * n > (1 << 28)
    rng = np.random.default_rng(11)
    u0 = rng.random((n, n), dtype=np.float32)
    W = wl.heat5_weights()
    x = g.to_dev(u0)
    outs = {}
    for flags in (lib.ST_FLAG_NAIVE, 0):
        plan = lib.stencil_plan(n, n, 1, W, b, "f32", flags)
        try:
            outs[flags] = g.run(plan, x, 1, n, n)
            torch.cuda.synchronize()
        finally:
            lib.stencil_destroy(plan)
    assert torch.equal(outs[lib.ST_FLAG_NAIVE], outs[0])
    got = outs[lib.ST_FLAG_NAIVE]
    top = oracle.stencil_f32(u0[:h], W, b, 1)
    bot = oracle.stencil_f32(u0[-h:], W, b, 1)
    np.testing.assert_array_equal(g.to_host(got[: h - 1]), top[: h - 1])
    np.testing.assert_array_equal(g.to_host(got[-(h - 1):]), bot[1:])
    del outs, got
    kap = (0.05 + 0.15 * rng.random((n, n), dtype=np.float32)).astype(np.float32)
    k = g.to_dev(kap)
    vo = {}
    for flags in (lib.ST_FLAG_NAIVE, 0):
        plan = lib.stencil_plan_varcoef(n, n, b, flags)
        try:
            out = torch.empty_like(x)
            lib.stencil_run_varcoef(plan, x, k, out, 1, None)
            torch.cuda.synchronize()
            vo[flags] = out
        finally:
            lib.stencil_destroy(plan)
    assert torch.equal(vo[lib.ST_FLAG_NAIVE], vo[0])
    got = vo[lib.ST_FLAG_NAIVE]
    top = oracle.varcoef_f32(u0[:h], kap[:h], b, 1)
    bot = oracle.varcoef_f32(u0[-h:], kap[-h:], b, 1)
    np.testing.assert_array_equal(g.to_host(got[: h - 1]), top[: h - 1])
    np.testing.assert_array_equal(g.to_host(got[-(h - 1):]), bot[1:])
    say(f"naive paths at {n}x{n}: bitwise equal to the tiled kernels and the oracle crops")

CASES = [
    # rows, cols, shape, r, b, steps
    (1, 1, wl.STAR, 1, 0.0, 3),
    (3, 5, wl.BOX, 2, 1.5, 4),
    (2, 200, wl.BOX, 4, 0.0, 2),
    (37, 61, wl.STAR, 3, 0.0, 7),
    (130, 67, wl.BOX, 1, -0.5, 9),
    (257, 513, wl.BOX, 3, 0.0, 5),
    (300, 129, wl.STAR, 4, 0.25, 6),
    (64, 64, wl.STAR, 2, 0.0, 0),
    (515, 1030, wl.STAR, 1, 0.0, 13),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}-{c[2]}{c[3]}-b{c[4]}-T{c[5]}" for c in CASES])
def test_ragged_bitwise(g, case):
    rows, cols, shape, r, b, steps = case
    W = _weights(shape, r, rows * 7 + cols)
    u0 = np.random.default_rng(rows + cols).random((rows, cols), dtype=np.float32)
    ref32 = oracle.stencil_f32(u0, W, b, steps)
    for flags, tb, tile in [(1, 0, None), (0, 1, (64, 64)), (0, 2, (128, 32)), (0, 3, (128, 64)),
                            (0, 4, (256, 32))]:
        say(case, flags, tb, tile)
        got = g.run_problem(u0, W, b, steps, flags=flags, tb=tb, tile=tile)
        np.testing.assert_array_equal(got, ref32)


def test_box49_crop_1024_1000(g):
    """Box-2D49P on the 1024x1024 top-left crop of the seed-1 field, 1000 steps."""
    p = wl.box49(crop=(1024, 1024))
    say("oracle f32 ...")
    ref32 = oracle.stencil_f32(p.u0, p.weights, 0.0, p.steps)
    say("oracle f64 ...")
    ref64 = oracle.stencil_f64(p.u0, p.weights, 0.0, p.steps)
    for tb in (1, 2, 4):
        got = g.run_problem(p.u0, p.weights, 0.0, p.steps, tb=tb, tile=(128, 64))
        e64 = oracle.rel_l2(got, ref64)
        say(f"box49 crop tb={tb}: rel-L2 vs f64 = {e64:.3e}, vs f32-canonical = {oracle.rel_l2(got, ref32):.3e}")
        assert e64 <= TOL
        np.testing.assert_array_equal(got, ref32)


def test_bitwise_across_blocking_and_graph(g):
    import torch
    import paper_2605_07954_amd as lib
    rows, cols = 1000, 777
    W = _weights(wl.BOX, 3, 5)
    u0 = np.random.default_rng(5).random((rows, cols), dtype=np.float32)
    base = g.run_problem(u0, W, 0.0, 13, flags=lib.ST_FLAG_NAIVE)
    checked = 0
    for tile in lib.stencil_tiles():
        for tb in (1, 2, 3, 5, 6):
            probe = lib.stencil_plan(rows, cols, 3, W, 0.0, "f32", 0)
            try:
                lib.stencil_set_blocking(probe, tb, *tile)
            except lib.StencilError as e:  # deeper than this tile's LDS budget: refused up front
                assert e.code == -3
                continue
            finally:
                lib.stencil_destroy(probe)
            got = g.run_problem(u0, W, 0.0, 13, tb=tb, tile=tile)
            np.testing.assert_array_equal(got, base)
            checked += 1
    assert checked >= 12
    # graph replays (with eager work between them) equal the direct run, every time
    plan = lib.stencil_plan(rows, cols, 3, W, 0.0, "f32", lib.ST_FLAG_GRAPH)
    try:
        x = g.to_dev(u0)
        out = torch.empty_like(x)
        ws = torch.empty(lib.stencil_workspace_bytes(plan, 13), dtype=torch.uint8, device=g.DEV)
        for rep in range(3):
            out.zero_()
            lib.stencil_run(plan, x, out, 13, ws)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(g.to_host(out), base)
            _ = (x * 2).sum().item()
    finally:
        lib.stencil_destroy(plan)
    # run(a) then run(b) == run(a+b)
    mid = g.run_problem(u0, W, 0.0, 6, tb=4)
    np.testing.assert_array_equal(g.run_problem(mid, W, 0.0, 7, tb=3), base)


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_lowp_storage_bitwise(g, storage):
    p = wl.star9_precision(rows=300, cols=257, steps=23)
    bits = oracle.to_bits(p.u0, storage)
    ref = oracle.stencil_lowp(bits, p.weights, 0.0, p.steps, storage)
    for flags, tb in [(1, 0), (0, 1), (0, 3), (0, 8)]:
        got = g.run_problem(bits, p.weights, 0.0, p.steps, storage=storage, flags=flags, tb=tb)
        np.testing.assert_array_equal(got, ref)
    x = oracle.from_bits(bits, storage)
    e = oracle.rel_l2(oracle.from_bits(got, storage), oracle.stencil_f64(x, p.weights, 0.0, p.steps))
    say(f"{storage} storage: rel-L2 vs f64 after {p.steps} steps = {e:.3e}")


def test_norms(g):
    import torch
    import paper_2605_07954_amd as lib
    rng = np.random.default_rng(4)
    for (rows, cols, shape, r, b) in [(513, 300, wl.BOX, 3, 0.0), (64, 70, wl.STAR, 2, 1.5), (5, 3, wl.BOX, 4, 0.5)]:
        W = _weights(shape, r, rows)
        u = rng.standard_normal((rows, cols)).astype(np.float32)
        up = rng.standard_normal((rows, cols)).astype(np.float32)
        plan = lib.stencil_plan(rows, cols, r, W, b, "f32", 0)
        try:
            ws = torch.empty(lib.stencil_norms_ws_bytes(plan), dtype=torch.uint8, device=g.DEV)
            o = torch.zeros(4, dtype=torch.float64, device=g.DEV)
            lib.stencil_norms(plan, g.to_dev(up), g.to_dev(u), o, ws)
            got = o.cpu().numpy()
            ref = oracle.norms_f64(u, W, b, up)
            say(f"norms {rows}x{cols} r={r} b={b}: gpu {got.tolist()} oracle {ref.tolist()}")
            np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-9)
            o2 = torch.zeros(4, dtype=torch.float64, device=g.DEV)
            lib.stencil_norms(plan, g.to_dev(up), g.to_dev(u), o2, ws)
            assert torch.equal(o, o2)  # deterministic
            # the predicted next mass is the mass of the next step
            nxt = g.run_problem(u, W, b, 1)
            say(f"  next-step mass: predicted {got[3]!r}, summed {nxt.astype(np.float64).sum()!r}")
            assert abs(got[3] - nxt.astype(np.float64).sum()) < 1e-5 * (1 + abs(got[3]))
        finally:
            lib.stencil_destroy(plan)


@pytest.mark.parametrize("storage,rows,cols,shape,r,b", [("bf16", 100, 64, wl.BOX, 2, 0.5), ("f16", 33, 50, wl.STAR, 3, 0.0),
                                                      ("f16", 7, 4, wl.BOX, 1, 1.5), ("f32", 130, 68, wl.STAR, 1, 0.0)])
def test_norms_storage_and_alignment(g, storage, rows, cols, shape, r, b):
    """Norms of 16-bit fields (four cells per vector load when cols % 4 == 0, one per thread
    otherwise) and of fields that do not start on a 16-byte boundary, against the FP64 oracle on
    the widened values."""
    import torch
    import paper_2605_07954_amd as lib
    rng = np.random.default_rng(rows + cols)
    W = _weights(shape, r, rows + 1)
    u = rng.standard_normal((rows, cols)).astype(np.float32)
    up = rng.standard_normal((rows, cols)).astype(np.float32)
    if storage != "f32":
        ub, upb = oracle.to_bits(u, storage), oracle.to_bits(up, storage)
        u, up = oracle.from_bits(ub, storage), oracle.from_bits(upb, storage)
        du, dup = g.to_dev(ub), g.to_dev(upb)
    else:
        du, dup = g.to_dev(u), g.to_dev(up)
    ref = oracle.norms_f64(u, W, b, up)
    plan = lib.stencil_plan(rows, cols, r, W, b, storage, 0)
    try:
        ws = torch.empty(lib.stencil_norms_ws_bytes(plan), dtype=torch.uint8, device=g.DEV)
        o = torch.zeros(4, dtype=torch.float64, device=g.DEV)
        lib.stencil_norms(plan, dup, du, o, ws)
        np.testing.assert_allclose(o.cpu().numpy(), ref, rtol=1e-12, atol=1e-9)
        # the same fields one element past an aligned start: the one-cell-per-thread path
        n = rows * cols
        xb = torch.empty(n + 1, dtype=du.dtype, device=g.DEV)
        pb = torch.empty(n + 1, dtype=du.dtype, device=g.DEV)
        xb[1:].copy_(du.reshape(-1))
        pb[1:].copy_(dup.reshape(-1))
        o2 = torch.zeros(4, dtype=torch.float64, device=g.DEV)
        lib.stencil_norms(plan, pb[1:], xb[1:], o2, ws)
        np.testing.assert_allclose(o2.cpu().numpy(), ref, rtol=1e-12, atol=1e-9)
        # without the previous field the residual is not computed (reported as 0)
        o3 = torch.full((4,), 7.0, dtype=torch.float64, device=g.DEV)
        lib.stencil_norms(plan, None, du, o3, ws)
        np.testing.assert_allclose(o3.cpu().numpy()[1:], ref[1:], rtol=1e-12, atol=1e-9)
        assert o3[0].item() == 0.0
        say(f"norms {storage} {rows}x{cols}: {o.cpu().numpy().tolist()}")
    finally:
        lib.stencil_destroy(plan)


def test_varcoef(g):
    import torch
    import paper_2605_07954_amd as lib
    for (rows, cols, b, steps) in [(1024, 1024, 0.0, 16), (77, 130, 0.3, 9), (1, 5, 0.0, 3)]:
        u0, kap = wl.varcoef_problem(rows, cols, seed=rows)
        ref32 = oracle.varcoef_f32(u0, kap, b, steps)
        ref64 = oracle.varcoef_f64(u0, kap, b, steps)
        for flags, tb in [(lib.ST_FLAG_NAIVE, 0), (0, 1), (0, 4), (0, 8)]:
            plan = lib.stencil_plan_varcoef(rows, cols, b, flags)
            try:
                if tb:
                    lib.stencil_set_blocking(plan, tb)
                x, k = g.to_dev(u0), g.to_dev(kap)
                out = torch.empty_like(x)
                nws = lib.stencil_workspace_bytes(plan, steps)
                ws = torch.empty(nws, dtype=torch.uint8, device=g.DEV) if nws else None
                lib.stencil_run_varcoef(plan, x, k, out, steps, ws)
                got = g.to_host(out)
            finally:
                lib.stencil_destroy(plan)
            e = oracle.rel_l2(got, ref64)
            say(f"varcoef {rows}x{cols} tb={tb}: rel-L2 vs f64 {e:.3e}")
            assert e <= TOL
            np.testing.assert_array_equal(got, ref32)


def test_varcoef_tiles_and_autotune(g):
    """The varcoef kernel at every tile and depth, and the blocking stencil_autotune_varcoef keeps,
    bitwise equal to the FP32 oracle (ragged tiles, b != 0)."""
    import torch
    import paper_2605_07954_amd as lib
    rows, cols, b, steps = 150, 203, 0.25, 11
    u0, kap = wl.varcoef_problem(rows, cols, seed=5)
    ref32 = oracle.varcoef_f32(u0, kap, b, steps)
    x, k = g.to_dev(u0), g.to_dev(kap)
    out = torch.empty_like(x)
    ws = torch.empty_like(x)
    for tx, ty in lib.stencil_tiles():
        for tb in (1, 2, 3, 4, 6, 8):
            plan = lib.stencil_plan_varcoef(rows, cols, b, 0)
            try:
                try:
                    lib.stencil_set_blocking(plan, tb, tx, ty)
                except lib.StencilError as e:  # too deep for this tile's LDS
                    assert e.code == lib.ST_EUNSUPPORTED
                    continue
                out.fill_(float("nan"))
                lib.stencil_run_varcoef(plan, x, k, out, steps, ws)
                np.testing.assert_array_equal(g.to_host(out), ref32, err_msg=f"tile {tx}x{ty} tb {tb}")
            finally:
                lib.stencil_destroy(plan)
    plan = lib.stencil_plan_varcoef(rows, cols, b, lib.ST_FLAG_GRAPH)
    try:
        cfg = lib.stencil_autotune_varcoef(plan, x, k, out, ws, steps)
        say(f"varcoef {rows}x{cols}: autotuned (tb, tile_x, tile_y) = {cfg}")
        with pytest.raises(lib.StencilError):  # a constant-weight tuner call on a varcoef plan
            lib.stencil_autotune(plan, x, out, ws, steps)
        out.fill_(float("nan"))
        lib.stencil_run_varcoef(plan, x, k, out, steps, ws)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(g.to_host(out), ref32)
        # same buffers, another diffusivity field: the cached graph must not replay the old one
        _, kap2 = wl.varcoef_problem(rows, cols, seed=6)
        ref2 = oracle.varcoef_f32(u0, kap2, b, steps)
        k2 = g.to_dev(kap2)
        for kk, want in ((k2, ref2), (k, ref32), (k2, ref2)):
            out.fill_(float("nan"))
            lib.stencil_run_varcoef(plan, x, kk, out, steps, ws)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(g.to_host(out), want)
    finally:
        lib.stencil_destroy(plan)


def test_error_paths(g):
    import torch
    import paper_2605_07954_amd as lib
    W = wl.heat5_weights()
    plan = lib.stencil_plan(64, 64, 1, W, 0.0, "f32", 0)
    try:
        x = torch.zeros((64, 64), device=g.DEV)
        with pytest.raises(lib.StencilError) as ei:
            lib.stencil_run(plan, x, x, 5, None)
        assert ei.value.code == -2
        y = torch.zeros_like(x)
        lib.stencil_set_blocking(plan, 1)
        with pytest.raises(lib.StencilError) as ei:
            lib.stencil_run(plan, x, y, 5, None)
        assert ei.value.code == -5
    finally:
        lib.stencil_destroy(plan)


@pytest.mark.parametrize("rows,cols,shape,r,b,steps", [(1024, 1024, wl.BOX, 3, 0.0, 7), (260, 516, wl.STAR, 1, 0.5, 9),
                                                      (131, 64, wl.BOX, 2, -1.0, 5), (700, 1200, wl.STAR, 3, 0.0, 8)])
def test_stream_variant_bitwise(g, rows, cols, shape, r, b, steps):
    """The persistent LDS-DMA variant equals the FP32-canonical oracle bit for bit, every tile and depth."""
    import torch
    import paper_2605_07954_amd as lib
    W = _weights(shape, r, rows + cols + r)
    u0 = np.random.default_rng(rows * cols).random((rows, cols), dtype=np.float32)
    ref = oracle.stencil_f32(u0, W, b, steps)
    x = g.to_dev(u0)
    n = 0
    for tile in lib.stencil_tiles():
        for tb in (1, 2, 3):
            plan = lib.stencil_plan(rows, cols, r, W, b, "f32", 0)
            try:
                try:
                    lib.stencil_set_blocking(plan, 1, *tile)
                    lib.stencil_set_variant(plan, lib.ST_VARIANT_STREAM)
                    lib.stencil_set_blocking(plan, tb)
                except lib.StencilError as e:
                    assert e.code == -3
                    continue
                out = torch.full_like(x, float("nan"))
                ws = torch.empty_like(x)
                lib.stencil_run(plan, x, out, steps, ws)
                torch.cuda.synchronize()
                np.testing.assert_array_equal(g.to_host(out), ref, err_msg=f"tile {tile} tb {tb}")
                n += 1
            finally:
                lib.stencil_destroy(plan)
    assert n >= 6
    # grids whose width is not a multiple of 4 refuse the streaming variant
    plan = lib.stencil_plan(rows, cols + 1, r, W, b, "f32", 0)
    try:
        with pytest.raises(lib.StencilError):
            lib.stencil_set_variant(plan, lib.ST_VARIANT_STREAM)
    finally:
        lib.stencil_destroy(plan)


def march_depth(shape, r, variant=None):
    """Deepest pass a marching variant offers: star rings hold only their own columns; eight
    columns per lane need twice the ring registers."""
    import paper_2605_07954_amd as lib
    if variant == lib.ST_VARIANT_MARCH8:
        return {1: 8, 2: 4, 3: 3, 4: 2}[r] if shape == wl.STAR else {1: 3, 2: 2, 3: 2, 4: 1}[r]
    return {1: 8, 2: 6, 3: 4, 4: 3}[r] if shape == wl.STAR else {1: 6, 2: 3}.get(r, 2)


MARCH_CASES = [  # (rows, cols, shape, r, b, steps): narrower than one band, exactly one band (tb 1: 248
    # columns, tb 2: 240), one column group past it, many bands; segments with ragged ends; b != 0;
    # grids shorter than the radius; odd step counts (the last two-level pass has one level)
    (1, 4, wl.BOX, 3, 0.0, 3), (5, 8, wl.STAR, 4, 0.5, 4), (37, 248, wl.BOX, 3, 0.0, 5), (40, 240, wl.BOX, 2, 0.25, 5),
    (33, 252, wl.STAR, 1, -1.0, 17), (300, 516, wl.BOX, 1, 0.0, 9), (257, 1000, wl.STAR, 2, 0.0, 13),
    (1024, 1024, wl.BOX, 3, 0.0, 7), (700, 1200, wl.STAR, 3, 0.5, 9), (129, 996, wl.BOX, 4, 0.0, 3),
    (2050, 64, wl.STAR, 4, 0.0, 4), (200, 328, wl.BOX, 1, 0.5, 11), (96, 136, wl.BOX, 4, 0.0, 3),
    # widths that are not a multiple of 4 (element accesses): narrower than a band, one band
    # plus one column, many bands with a ragged end
    (3, 5, wl.BOX, 2, 0.0, 3), (70, 63, wl.STAR, 1, 0.5, 9), (41, 58, wl.BOX, 3, 0.0, 4), (300, 517, wl.BOX, 1, -0.5, 7),
    (257, 1001, wl.STAR, 2, 0.0, 6), (130, 263, wl.BOX, 3, 0.25, 5), (90, 301, wl.STAR, 4, 0.0, 3),
    # a halo of -0.0: not the +0 whose side bands start at the grid's edge (lane shifts bring in +0)
    (129, 1104, wl.STAR, 2, -0.0, 7), (97, 1600, wl.BOX, 1, -0.0, 5)]


@pytest.mark.parametrize("case", MARCH_CASES, ids=[f"{c[0]}x{c[1]}-{c[2]}{c[3]}-b{c[4]}-T{c[5]}" for c in MARCH_CASES])
def test_march_variant_bitwise(g, case):
    """The row-marching variants (one wavefront per column band, lane-shifted side columns) equal the
    FP32-canonical oracle bit for bit at every depth they offer for the shape and radius (star r = 1
    / 2 / 3 / 4: up to 8 / 6 / 4 / 3 levels; box: 6 / 3 / 2 / 2; with eight columns per lane star
    8 / 4 / 3 / 2, box 3 / 2 / 2 / 1), with vector accesses (eight or four columns per lane, width a
    multiple of 8 or 4), element accesses (four columns per lane: any other width, or buffers off a
    16-byte boundary) and one column per lane."""
    import torch
    import paper_2605_07954_amd as lib
    rows, cols, shape, r, b, steps = case
    W = _weights(shape, r, rows + 3 * cols + r)
    u0 = np.random.default_rng(rows * cols + 7).random((rows, cols), dtype=np.float32)
    ref = oracle.stencil_f32(u0, W, b, steps)
    x = g.to_dev(u0)
    for variant in (lib.ST_VARIANT_MARCH, lib.ST_VARIANT_MARCH8, lib.ST_VARIANT_MARCH1):
        _march_variant_depths(g, lib, torch, x, ref, rows, cols, shape, r, W, b, steps, variant)


def _march_variant_depths(g, lib, torch, x, ref, rows, cols, shape, r, W, b, steps, variant):
    deepest = march_depth(shape, r, variant)
    for tb in range(1, deepest + 1):
        plan = lib.stencil_plan(rows, cols, r, W, b, "f32", 0)
        try:
            lib.stencil_set_blocking(plan, 1)
            lib.stencil_set_variant(plan, variant)
            lib.stencil_set_blocking(plan, tb)
            with pytest.raises(lib.StencilError):
                lib.stencil_set_blocking(plan, deepest + 1)
            out = torch.full_like(x, float("nan"))
            ws = torch.empty_like(x)
            lib.stencil_run(plan, x, out, steps, ws)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(g.to_host(out), ref, err_msg=f"variant {variant} tb {tb}")
            # longer segments than one task per resident wavefront: bitwise the same
            for seg in sorted({max(1, r * (tb - 1)), 7, 40, rows, 3 * rows}):
                lib.stencil_set_march_segment(plan, seg)
                out.fill_(float("nan"))
                lib.stencil_run(plan, x, out, steps, ws)
                torch.cuda.synchronize()
                np.testing.assert_array_equal(g.to_host(out), ref, err_msg=f"variant {variant} tb {tb} seg {seg}")
            lib.stencil_set_march_segment(plan, 0)
            # a buffer 4 bytes past a 16-byte boundary takes element accesses
            xb = torch.empty(rows * cols + 1, dtype=torch.float32, device=g.DEV)
            xb[1:].copy_(x.reshape(-1))
            ob = torch.full_like(xb, float("nan"))
            lib.stencil_run(plan, xb[1:], ob[1:], steps, ws)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(g.to_host(ob[1:]).reshape(rows, cols), ref, err_msg=f"variant {variant} unaligned tb {tb}")
        finally:
            lib.stencil_destroy(plan)


BALANCED_CASES = [  # (rows, cols, shape, r, b, steps, variant, tb): tall grids whose default segments
    # are long enough for the edge tasks to get shorter ones (outer bands, an inner band's first and
    # last segments): five and six bands of four columns per lane, two bands, four eight-column
    # bands; step counts that end with a shallower pass
    (4096, 1000, wl.STAR, 2, 0.0, 13, "march", 6), (6000, 1200, wl.STAR, 2, 0.25, 10, "march", 5),
    (8192, 300, wl.STAR, 1, 0.0, 17, "march", 8), (8000, 1600, wl.BOX, 1, 0.0, 7, "march8", 3),
    (5000, 700, wl.BOX, 1, -0.5, 7, "march", 6)]


@pytest.mark.parametrize("case", BALANCED_CASES, ids=[f"{c[0]}x{c[1]}-{c[2]}{c[3]}-{c[6]}-tb{c[7]}" for c in BALANCED_CASES])
def test_march_edge_task_layout_bitwise(g, case):
    """With default segments on tall grids the marching pass gives the tasks that take the edge
    checks shorter segments than the inner ones and runs them first; every row of every band is
    still computed by exactly one task, so the whole field equals the FP32-canonical oracle bit for
    bit (a gap or an overlap in the layout would leave NaN rows or wrong values)."""
    import torch
    import paper_2605_07954_amd as lib
    rows, cols, shape, r, b, steps, variant, tb = case
    W = _weights(shape, r, rows + cols + 11 * r)
    u0 = np.random.default_rng(rows + 3 * cols).random((rows, cols), dtype=np.float32)
    ref = oracle.stencil_f32(u0, W, b, steps)
    plan = lib.stencil_plan(rows, cols, r, W, b, "f32", 0)
    try:
        lib.stencil_set_blocking(plan, 1)
        lib.stencil_set_variant(plan, lib.ST_VARIANT_MARCH if variant == "march" else lib.ST_VARIANT_MARCH8)
        lib.stencil_set_blocking(plan, tb)
        x = g.to_dev(u0)
        out = torch.full_like(x, float("nan"))
        ws = torch.empty_like(x)
        say(f"edge-task layout {rows}x{cols} {shape}{r} {variant} tb {tb}")
        lib.stencil_run(plan, x, out, steps, ws)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(g.to_host(out), ref)
    finally:
        lib.stencil_destroy(plan)


@pytest.mark.parametrize("storage", ["bf16", "f16"])
@pytest.mark.parametrize("rows,cols,shape,r,b,steps", [(300, 260, wl.STAR, 2, 0.0, 23), (129, 500, wl.BOX, 1, 0.5, 11),
                                                      (40, 996, wl.BOX, 3, 0.0, 5), (7, 8, wl.STAR, 4, -0.25, 4),
                                                      (97, 301, wl.STAR, 2, 0.0, 9), (33, 70, wl.BOX, 3, 0.0, 4),
                                                      (150, 264, wl.STAR, 2, 0.0, 13), (61, 96, wl.BOX, 3, 0.5, 5),
                                                      (77, 200, wl.BOX, 1, 0.0, 8),
                                                      # three or more 512-column bands with cols % 8 == 0:
                                                      # the eight-column interior tasks (no edge checks)
                                                      (200, 1600, wl.STAR, 2, 0.0, 9), (200, 1600, wl.BOX, 1, 0.0, 7),
                                                      (200, 1600, wl.BOX, 2, 0.25, 5), (200, 1600, wl.BOX, 3, 0.0, 5),
                                                      (160, 2048, wl.STAR, 1, 0.0, 17), (160, 2048, wl.STAR, 3, 0.0, 7),
                                                      (120, 1536, wl.STAR, 4, 0.0, 5)])
def test_march_lowp_bitwise(g, storage, rows, cols, shape, r, b, steps):
    """Marching with BF16/FP16 storage (8- or 16-byte loads, FP32 arithmetic, every level rounded to
    the storage type) equals the emulating oracle bit for bit at every depth of every variant.  Grids
    at least three bands wide (about 512 columns each with eight columns per lane) give the
    marching passes interior tasks, whose kernels take no edge checks; longer segments than the
    default are run too, so that interior segments of several rows are covered."""
    import paper_2605_07954_amd as lib
    W = _weights(shape, r, rows + 5 * cols + r)
    bits = oracle.to_bits(np.random.default_rng(rows + cols).random((rows, cols), dtype=np.float32), storage)
    ref = oracle.stencil_lowp(bits, W, b, steps, storage)
    for variant in (lib.ST_VARIANT_MARCH, lib.ST_VARIANT_MARCH8, lib.ST_VARIANT_MARCH1):
        for tb in range(1, march_depth(shape, r, variant) + 1):
            plan = lib.stencil_plan(rows, cols, r, W, b, storage, 0)
            try:
                lib.stencil_set_blocking(plan, 1)
                lib.stencil_set_variant(plan, variant)
                lib.stencil_set_blocking(plan, tb)
                xd = g.to_dev(bits)
                got = g.run(plan, xd, steps, rows, cols, storage)
                np.testing.assert_array_equal(g.to_host(got), ref, err_msg=f"variant {variant} tb {tb}")
                if cols >= 1536:
                    lib.stencil_set_march_segment(plan, 24)
                    got = g.run(plan, xd, steps, rows, cols, storage)
                    np.testing.assert_array_equal(g.to_host(got), ref, err_msg=f"variant {variant} tb {tb} seg 24")
            finally:
                lib.stencil_destroy(plan)


@pytest.mark.parametrize("flags", [0, 2])
def test_solve_until_converged(g, flags):
    """Periodic convergence check: stops at the first check whose relative residual is <= tol, and
    the field equals a plain run of that many steps (also for a graph-flagged plan, whose cached
    graph the solve leaves alone)."""
    import torch
    import paper_2605_07954_amd as lib
    rows, cols, b = 32, 40, 1.0
    W = wl.heat5_weights()
    u0 = np.random.default_rng(17).random((rows, cols), dtype=np.float32)
    plan = lib.stencil_plan(rows, cols, 1, W, b, "f32", flags)
    try:
        x = g.to_dev(u0)
        out = torch.empty_like(x)
        ws = torch.empty(lib.stencil_solve_ws_bytes(plan, 100), dtype=torch.uint8, device=g.DEV)
        done, res = lib.stencil_solve(plan, x, out, 50000, 100, 1e-6, ws)
        got = g.to_host(out)
        if flags:  # the plan still runs through its graph afterwards
            o2 = torch.empty_like(x)
            w2 = torch.empty_like(x)
            lib.stencil_run(plan, x, o2, done, w2)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(g.to_host(o2), got)
    finally:
        lib.stencil_destroy(plan)
    say(f"solve: {done} steps, relative residual {res:.3e}")
    assert done % 100 == 0 and 100 < done < 50000
    ref = oracle.stencil_f32(u0, W, b, done)
    np.testing.assert_array_equal(got, ref)
    before = oracle.stencil_f32(u0, W, b, done - 1).astype(np.float64)
    rr = np.sqrt(np.sum((ref - before) ** 2) / np.sum(ref.astype(np.float64) ** 2))
    assert abs(rr - res) <= 1e-9 * max(rr, 1e-30) + 1e-15
    assert res <= 1e-6
    a = oracle.stencil_f32(u0, W, b, done - 100).astype(np.float64)
    a1 = oracle.stencil_f32(u0, W, b, done - 101).astype(np.float64)
    assert np.sqrt(np.sum((a - a1) ** 2) / np.sum(a * a)) > 1e-6   # the previous check had not converged


def _rel_residual(u0, W, b, t):
    a = oracle.stencil_f32(u0, W, b, t).astype(np.float64)
    a1 = oracle.stencil_f32(u0, W, b, t - 1).astype(np.float64)
    return np.sqrt(np.sum((a - a1) ** 2) / np.sum(a * a))


@pytest.mark.parametrize("variant", [2, 3, 4, 0])
def test_solve_check_chunks(g, variant):
    """The convergence test at short intervals, so that the solve crosses several of its chunks of
    checks (marching variants decide on the device; the tiled variant reads every residual back):
    the field is bitwise the plain run of the steps taken, the first check at or below tol is the
    one it stops at, a budget that ends inside an interval stops there, and a tolerance met at the
    first check stops after one interval."""
    import torch
    import paper_2605_07954_amd as lib
    rows, cols, b = 48, 72, 0.5
    W = wl.heat5_weights()
    u0 = np.random.default_rng(23).random((rows, cols), dtype=np.float32)
    plan = lib.stencil_plan(rows, cols, 1, W, b, "f32", 0)
    try:
        lib.stencil_set_variant(plan, variant)
        lib.stencil_set_blocking(plan, 2, 0, 0)
        x = g.to_dev(u0)
        out = torch.empty_like(x)
        ce = 7
        ws = torch.empty(lib.stencil_solve_ws_bytes(plan, ce), dtype=torch.uint8, device=g.DEV)
        tol = 5e-6
        done, res = lib.stencil_solve(plan, x, out, 100000, ce, tol, ws)
        got = g.to_host(out)
        say(f"variant {variant}: {done} steps ({done // ce} checks), relative residual {res:.3e}")
        assert done % ce == 0 and done // ce > 130      # several chunks of 1, 2, 4, ... 64 checks
        np.testing.assert_array_equal(got, oracle.stencil_f32(u0, W, b, done))
        rr = _rel_residual(u0, W, b, done)
        assert abs(rr - res) <= 1e-9 * rr and res <= tol
        assert _rel_residual(u0, W, b, done - ce) > tol
        # a budget that ends inside an interval, never converged: stops at max_steps exactly
        done2, res2 = lib.stencil_solve(plan, x, out, 100, ce, 0.0, ws)
        assert done2 == 100
        np.testing.assert_array_equal(g.to_host(out), oracle.stencil_f32(u0, W, b, 100))
        assert abs(_rel_residual(u0, W, b, 100) - res2) <= 1e-9 * res2
        # met at the first check
        done3, _ = lib.stencil_solve(plan, x, out, 1000, ce, 1.0, ws)
        assert done3 == ce
        np.testing.assert_array_equal(g.to_host(out), oracle.stencil_f32(u0, W, b, ce))
    finally:
        lib.stencil_destroy(plan)
