"""GPU parity of the periodic and caller-framed boundaries (the row-marching kernels built with
those rules in their edge tasks) against the oracle's definitions: bit for bit with the
FP32-canonical / 16-bit-emulating modes at every depth of every marching variant, on grids
narrower and shorter than the halo, several bands wide, with vector and element accesses; a
periodic plane wave through a 2048^2 grid against its closed form; the norms' next-step mass on
a torus; graph replay and the autotuner."""
import math
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


def march_depth(shape, r, variant):
    import paper_2605_07954_amd as lib
    if variant == lib.ST_VARIANT_MARCH8:
        return {1: 8, 2: 4, 3: 3, 4: 2}[r] if shape == wl.STAR else {1: 3, 2: 2, 3: 2, 4: 1}[r]
    return {1: 8, 2: 6, 3: 4, 4: 3}[r] if shape == wl.STAR else {1: 6, 2: 3}.get(r, 2)


CASES = [  # (rows, cols, shape, r, steps): tiny (wraps several times), one band, several bands,
    # widths that are not a multiple of 4 (element accesses), segments with ragged ends
    (1, 4, wl.BOX, 2, 3), (3, 5, wl.STAR, 4, 4), (37, 248, wl.BOX, 3, 5), (300, 516, wl.BOX, 1, 9),
    (257, 1000, wl.STAR, 2, 13), (70, 63, wl.STAR, 1, 9), (130, 263, wl.BOX, 3, 5), (96, 1600, wl.BOX, 2, 5),
    (61, 96, wl.STAR, 3, 7)]


def _frame(rng, rows, cols, r, storage):
    n = oracle.frame_elems(rows, cols, r)
    f = rng.standard_normal(n).astype(np.float32)
    return f if storage == "f32" else oracle.to_bits(f, storage)


@pytest.mark.parametrize("bc", ["periodic", "frame"])
@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}-{c[2]}{c[3]}-T{c[4]}" for c in CASES])
def test_boundary_march_bitwise(g, bc, case):
    import torch
    import paper_2605_07954_amd as lib
    rows, cols, shape, r, steps = case
    rng = np.random.default_rng(rows * 7 + cols + r)
    W = wl.random_footprint_weights(rng, shape, r)
    u0 = rng.random((rows, cols), dtype=np.float32)
    fr = _frame(rng, rows, cols, r, "f32") if bc == "frame" else None
    ref = oracle.stencil_bc_f32(u0, W, bc, steps, fr)
    x = g.to_dev(u0)
    fd = g.to_dev(fr) if fr is not None else None
    kind = lib.ST_BC_PERIODIC if bc == "periodic" else lib.ST_BC_FRAME
    for variant in (lib.ST_VARIANT_MARCH, lib.ST_VARIANT_MARCH8, lib.ST_VARIANT_MARCH1):
        for tb in range(1, march_depth(shape, r, variant) + 1):
            plan = lib.stencil_plan(rows, cols, r, W, 0.75, "f32", 0)
            try:
                lib.stencil_set_boundary(plan, kind, fd)
                assert lib.stencil_get_boundary(plan) == kind
                lib.stencil_set_blocking(plan, 1)
                lib.stencil_set_variant(plan, variant)
                lib.stencil_set_blocking(plan, tb)
                out = torch.full_like(x, float("nan"))
                ws = torch.empty_like(x)
                lib.stencil_run(plan, x, out, steps, ws)
                torch.cuda.synchronize()
                np.testing.assert_array_equal(g.to_host(out), ref, err_msg=f"{bc} variant {variant} tb {tb}")
                if tb > 1:
                    lib.stencil_set_march_segment(plan, 5)
                    out.fill_(float("nan"))
                    lib.stencil_run(plan, x, out, steps, ws)
                    torch.cuda.synchronize()
                    np.testing.assert_array_equal(g.to_host(out), ref, err_msg=f"{bc} variant {variant} tb {tb} seg 5")
            finally:
                lib.stencil_destroy(plan)
    # a buffer off a 16-byte boundary takes element accesses
    plan = lib.stencil_plan(rows, cols, r, W, 0.0, "f32", lib.ST_FLAG_GRAPH)
    try:
        lib.stencil_set_boundary(plan, kind, fd)
        xb = torch.empty(rows * cols + 1, dtype=torch.float32, device=g.DEV)
        xb[1:].copy_(x.reshape(-1))
        ob = torch.full_like(xb, float("nan"))
        ws = torch.empty_like(xb)
        for _ in range(2):  # graph capture, then a replay
            lib.stencil_run(plan, xb[1:], ob[1:], steps, ws)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(g.to_host(ob[1:]).reshape(rows, cols), ref, err_msg=f"{bc} unaligned, graph")
    finally:
        lib.stencil_destroy(plan)


@pytest.mark.parametrize("storage", ["bf16", "f16"])
@pytest.mark.parametrize("bc", ["periodic", "frame"])
@pytest.mark.parametrize("rows,cols,shape,r,steps", [(300, 260, wl.STAR, 2, 11), (40, 996, wl.BOX, 3, 5),
                                                      (7, 8, wl.STAR, 4, 4), (97, 301, wl.BOX, 1, 9),
                                                      (200, 1600, wl.STAR, 1, 9)])
def test_boundary_lowp_bitwise(g, storage, bc, rows, cols, shape, r, steps):
    import paper_2605_07954_amd as lib
    rng = np.random.default_rng(rows + 3 * cols)
    W = wl.random_footprint_weights(rng, shape, r)
    bits = oracle.to_bits(rng.random((rows, cols), dtype=np.float32), storage)
    fr = _frame(rng, rows, cols, r, storage) if bc == "frame" else None
    ref = oracle.stencil_bc_lowp(bits, W, bc, steps, storage, fr)
    kind = lib.ST_BC_PERIODIC if bc == "periodic" else lib.ST_BC_FRAME
    fd = g.to_dev(fr) if fr is not None else None
    for variant in (lib.ST_VARIANT_MARCH, lib.ST_VARIANT_MARCH1):
        for tb in (1, march_depth(shape, r, variant)):
            plan = lib.stencil_plan(rows, cols, r, W, 0.0, storage, 0)
            try:
                lib.stencil_set_boundary(plan, kind, fd)
                lib.stencil_set_blocking(plan, 1)
                lib.stencil_set_variant(plan, variant)
                lib.stencil_set_blocking(plan, tb)
                got = g.run(plan, g.to_dev(bits), steps, rows, cols, storage)
                np.testing.assert_array_equal(g.to_host(got), ref, err_msg=f"{bc} variant {variant} tb {tb}")
            finally:
                lib.stencil_destroy(plan)


@pytest.mark.parametrize("shape,r,storage", [(wl.BOX, 3, "f32"), (wl.STAR, 2, "f32"), (wl.STAR, 2, "bf16")])
def test_periodic_plane_wave_2048(g, shape, r, storage):
    """A Fourier mode of the torus, cos(k.x + phi) with k = 2 pi m / N, through 2048^2 x 200 steps
    with the autotuned blocking: every cell against |lam|^T cos(k.x + phi + T arg lam) (FP32: rel-L2
    <= 1e-5; BF16: reported, with the mass of the torus against sum(W)^T times the initial mass)."""
    import torch
    import paper_2605_07954_amd as lib
    n, T = 2048, 200
    W = wl.random_footprint_weights(np.random.default_rng(40 + r), shape, r)
    ky, kx, phi = 2 * math.pi * 3 / n, 2 * math.pi * 7 / n, 0.4
    i = np.arange(n, dtype=np.float64)
    u0 = np.cos(kx * i[None, :] + ky * i[:, None] + phi).astype(np.float32)
    x = g.to_dev(u0 if storage == "f32" else oracle.to_bits(u0, storage))
    plan = lib.stencil_plan(n, n, r, W, 0.0, storage, 0)
    try:
        lib.stencil_set_boundary(plan, lib.ST_BC_PERIODIC)
        out = torch.empty_like(x)
        ws = torch.empty_like(x)
        tb, _, _ = lib.stencil_autotune(plan, x, out, ws, 24)
        var = lib.stencil_get_variant(plan)
        assert var in (lib.ST_VARIANT_MARCH, lib.ST_VARIANT_MARCH8, lib.ST_VARIANT_MARCH1)
        lib.stencil_run(plan, x, out, T, ws)
        torch.cuda.synchronize()
        got = g.to_host(out)
        nws = torch.empty(lib.stencil_norms_ws_bytes(plan), dtype=torch.uint8, device=g.DEV)
        o4 = torch.empty(4, dtype=torch.float64, device=g.DEV)
        lib.stencil_norms(plan, None, out, o4, nws)
        norms = o4.cpu().numpy()
    finally:
        lib.stencil_destroy(plan)
    vals = got if storage == "f32" else oracle.from_bits(got, storage)
    d = np.arange(-r, r + 1)
    lam = np.sum(W.astype(np.float64) * np.exp(1j * (ky * d[:, None] + kx * d[None, :])))
    # the closed form, row by row (FP64)
    e2 = s2 = 0.0
    for k in range(0, n, 256):
        ii = i[k:k + 256, None]
        ex = abs(lam) ** T * np.cos(kx * i[None, :] + ky * ii + phi + T * np.angle(lam))
        e2 += float(np.sum((vals[k:k + 256].astype(np.float64) - ex) ** 2))
        s2 += float(np.sum(ex * ex))
    err = math.sqrt(e2 / s2)
    say(f"periodic plane wave {shape} r={r} {storage} {n}^2 x {T} (tb {tb}, variant {var}): rel-L2 vs closed form "
        f"{err:.3e}")
    if storage == "f32":
        assert err <= 1e-5
    wsum = float(np.sum(W.astype(np.float64)))
    assert abs(norms[3] - wsum * norms[2]) <= 1e-12 * abs(norms[3]) + 1e-9  # next mass on a torus


def test_frame_norms_next_mass_is_nan(g):
    import torch
    import paper_2605_07954_amd as lib
    rows, cols = 20, 24
    plan = lib.stencil_plan(rows, cols, 1, wl.heat5_weights(), 0.0, "f32", 0)
    try:
        fr = torch.zeros(lib.stencil_frame_elems(plan), dtype=torch.float32, device=g.DEV)
        lib.stencil_set_boundary(plan, lib.ST_BC_FRAME, fr)
        u = torch.rand((rows, cols), device=g.DEV)
        nws = torch.empty(lib.stencil_norms_ws_bytes(plan), dtype=torch.uint8, device=g.DEV)
        o4 = torch.empty(4, dtype=torch.float64, device=g.DEV)
        lib.stencil_norms(plan, None, u, o4, nws)
        n = o4.cpu().numpy()
        assert math.isnan(n[3]) and abs(n[2] - float(u.double().sum())) < 1e-9
    finally:
        lib.stencil_destroy(plan)
