"""GPU parity of the 3D stencil (z-marching kernel, LDS plane ring) against the oracle's 3D
definition: bit for bit with the FP32-canonical order on ragged grids for the 7- and 13-point
stars and the 27- and 125-point boxes, with b != 0; 16-bit storage against the FP32-canonical step
rounded to the storage type after every step (the oracle's step composed with the format
conversion); the Dirichlet sine eigenmode of the 7-point star at 192^3 against its closed form;
graph replay and the allocation-free entry point."""
import math
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def g():
    import torch  # noqa: F401
    import gpuhelp
    return gpuhelp


def weights3(rng, shape, r):
    k = 2 * r + 1
    W = rng.random((k, k, k))
    if shape == "star":
        m = np.zeros((k, k, k), dtype=bool)
        m[:, r, r] = m[r, :, r] = m[r, r, :] = True
        W = np.where(m, W, 0.0)
    return (W / W.sum()).astype(np.float32)


def run3(g, lib, u, W, b, steps, storage="f32", flags=0, noalloc=False):
    import torch
    P, R, C = u.shape
    r = (W.shape[0] - 1) // 2
    plan = lib.stencil_plan3d(P, R, C, r, W, b, storage, flags)
    try:
        x = g.to_dev(u)
        out = torch.empty_like(x)
        if noalloc:
            lib.stencil_run_noalloc(plan, x, out, steps)
        else:
            ws = torch.empty_like(x)
            lib.stencil_run(plan, x, out, steps, ws)
            if flags:
                lib.stencil_run(plan, x, out, steps, ws)  # a replay of the captured graph
        torch.cuda.synchronize()
        return g.to_host(out)
    finally:
        lib.stencil_destroy(plan)


CASES = [((9, 37, 70), "star", 1, 0.0, 7), ((5, 20, 130), "star", 2, 0.5, 5), ((17, 33, 65), "box", 1, -1.0, 6),
         ((6, 19, 67), "box", 2, 0.0, 4), ((1, 1, 1), "box", 2, 0.25, 3), ((40, 3, 5), "star", 1, 0.0, 9),
         ((3, 70, 200), "box", 1, 0.0, 3)]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{c[1]}{c[2]}-b{c[3]}" for c in CASES])
def test_3d_bitwise(g, case):
    import paper_2605_07954_amd as lib
    shape, sh, r, b, steps = case
    rng = np.random.default_rng(sum(shape) + r)
    W = weights3(rng, sh, r)
    u = rng.random(shape, dtype=np.float32)
    ref = oracle.stencil3d_f32(u, W, b, steps)
    got = run3(g, lib, u, W, b, steps)
    np.testing.assert_array_equal(got, ref)
    np.testing.assert_array_equal(run3(g, lib, u, W, b, steps, flags=lib.ST_FLAG_GRAPH), ref)
    np.testing.assert_array_equal(run3(g, lib, u, W, b, steps, noalloc=True), ref)
    e = oracle.rel_l2(got, oracle.stencil3d_f64(u, W, b, steps))
    say(f"3D {shape} {sh} r={r}: bitwise vs the FP32 oracle, rel-L2 vs FP64 {e:.2e}")
    assert e <= 1e-5


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_3d_lowp_bitwise(g, storage):
    import paper_2605_07954_amd as lib
    rng = np.random.default_rng(77)
    for shape, sh, r, b, steps in [((7, 30, 66), "star", 1, 0.0, 5), ((5, 17, 70), "box", 2, 0.5, 3)]:
        W = weights3(rng, sh, r)
        bits = oracle.to_bits(rng.random(shape, dtype=np.float32), storage)
        bq = float(oracle.from_bits(oracle.to_bits(np.array([b], np.float32), storage), storage)[0])
        ref = bits
        for _ in range(steps):  # one FP32-canonical step, then rounding to the storage type
            ref = oracle.to_bits(oracle.stencil3d_f32(oracle.from_bits(ref, storage), W, bq, 1), storage)
        got = run3(g, lib, bits, W, b, steps, storage)
        np.testing.assert_array_equal(got, ref)


def test_3d_sine_eigenmode_192(g):
    """u0 = sin(p pi (k+1)/(P+1)) sin(q pi (i+1)/(R+1)) sin(s pi (j+1)/(C+1)) decays by
    c0 + 2 c1 (cos a + cos b + cos g) per step under the 7-point star with a zero halo."""
    import paper_2605_07954_amd as lib
    n, T = 192, 60
    W = np.zeros((3, 3, 3), dtype=np.float32)
    W[1, 1, 1] = np.float32(0.4)
    for d in [(0, 1, 1), (2, 1, 1), (1, 0, 1), (1, 2, 1), (1, 1, 0), (1, 1, 2)]:
        W[d] = np.float32(0.1)
    p, q, s = 3, 5, 2
    a, bb, gg = (p * math.pi / (n + 1), q * math.pi / (n + 1), s * math.pi / (n + 1))
    i = np.arange(n, dtype=np.float64)
    u0 = (np.sin(a * (i + 1))[:, None, None] * np.sin(bb * (i + 1))[None, :, None]
          * np.sin(gg * (i + 1))[None, None, :]).astype(np.float32)
    lam = float(W[1, 1, 1]) + 2 * float(W[0, 1, 1]) * (math.cos(a) + math.cos(bb) + math.cos(gg))
    got = run3(g, lib, u0, W, 0.0, T)
    e = oracle.rel_l2(got, lam ** T * u0.astype(np.float64))
    say(f"3D sine eigenmode {n}^3 x {T}: lambda^T = {lam ** T:.4f}, rel-L2 vs closed form {e:.2e}")
    assert e <= 1e-5
