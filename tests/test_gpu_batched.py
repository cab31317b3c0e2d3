"""GPU parity of the batched persistent kernel: every grid of a mixed batch equals the FP32-canonical
oracle bit for bit (and the per-grid launch path), with and without the captured hipGraph."""
import os
import sys

import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def g():
    import gpuhelp
    return gpuhelp


def _run_batch(g, problems, flags, tbs=None, tiles=None, reps=2):
    import torch
    import paper_2605_07954_amd as lib
    plans = []
    try:
        for k, p in enumerate(problems):
            h = lib.stencil_plan(p.rows, p.cols, p.radius, p.weights, p.boundary, "f32", 0)
            plans.append(h)
            if tbs is not None:
                try:
                    lib.stencil_set_blocking(h, tbs[k % len(tbs)], *(tiles[k % len(tiles)] if tiles else (0, 0)))
                except lib.StencilError as e:  # depth too large for this tile's LDS: keep the default
                    if e.code != lib.ST_EUNSUPPORTED:
                        raise
        batch = lib.stencil_batch_create(plans, [p.steps for p in problems], flags)
        try:
            ins = [g.to_dev(p.u0) for p in problems]
            outs = [torch.empty_like(x) for x in ins]
            ws = torch.empty(lib.stencil_batch_workspace_bytes(batch), dtype=torch.uint8, device=g.DEV)
            results = []
            for rep in range(reps):
                for o in outs:
                    o.fill_(float("nan"))
                lib.stencil_run_batched(batch, ins, outs, ws)
                torch.cuda.synchronize()
                results.append([g.to_host(o) for o in outs])
                _ = (ins[0] * 3).sum().item()  # eager work between replays
            return results
        finally:
            lib.stencil_batch_destroy(batch)
    finally:
        for h in plans:
            lib.stencil_destroy(h)


def _mixed(n, seed, lo=40, hi=700, steps=(5, 17)):
    specs = wl.batch_specs(n, lo, hi, seed)
    rng = np.random.default_rng(seed)
    out = []
    for k, (rows, cols, shape, r) in enumerate(specs):
        w = wl.random_footprint_weights(np.random.default_rng(500 + k), shape, r)
        u0 = np.random.default_rng(900 + k).random((rows, cols), dtype=np.float32)
        out.append(wl.Problem(f"g{k}", rows, cols, r, shape, w, 0.0, int(rng.integers(*steps)), u0))
    # a tiny grid, a grid smaller than its radius, a zero-step grid and a b != 0 grid
    out.append(wl.Problem("tiny", 2, 3, 3, wl.STAR, wl.random_footprint_weights(rng, wl.STAR, 3), 0.0, 6,
                          rng.random((2, 3), dtype=np.float32)))
    out.append(wl.Problem("zero", 70, 90, 1, wl.BOX, wl.random_footprint_weights(rng, wl.BOX, 1), 0.0, 0,
                          rng.random((70, 90), dtype=np.float32)))
    out.append(wl.Problem("bnz", 150, 260, 2, wl.BOX, wl.random_footprint_weights(rng, wl.BOX, 2), 0.75, 9,
                          rng.random((150, 260), dtype=np.float32)))
    return out


def test_batched_single_grid(g):
    """One tiled grid, several passes; then two grids; then one LDS-resident grid."""
    rng = np.random.default_rng(1)
    w5 = wl.heat5_weights()
    a = wl.Problem("a", 300, 260, 1, wl.STAR, w5, 0.0, 6, rng.random((300, 260), dtype=np.float32))
    b = wl.Problem("b", 130, 517, 3, wl.BOX, wl.random_footprint_weights(rng, wl.BOX, 3), 0.0, 5,
                   rng.random((130, 517), dtype=np.float32))
    c = wl.Problem("c", 40, 50, 2, wl.STAR, wl.random_footprint_weights(rng, wl.STAR, 2), 0.5, 9,
                   rng.random((40, 50), dtype=np.float32))
    for probs, tbs in (([a], [1]), ([a], [2]), ([a, b], [1, 2]), ([c], [1]), ([a, b, c], [3, 1, 1])):
        say("batch", [(p.name, p.rows, p.cols, p.steps) for p in probs], "tb", tbs)
        res = _run_batch(g, probs, 0, tbs=tbs, tiles=[(128, 64)], reps=1)
        for p, got in zip(probs, res[0]):
            np.testing.assert_array_equal(got, oracle.stencil_f32(p.u0, p.weights, p.boundary, p.steps),
                                          err_msg=p.name)


@pytest.mark.parametrize("graph", [0, 2])
def test_batched_mixed_bitwise(g, graph):
    problems = _mixed(24, 7)
    refs = [oracle.stencil_f32(p.u0, p.weights, p.boundary, p.steps) for p in problems]
    say("batch:", [(p.rows, p.cols, p.shape, p.radius, p.steps) for p in problems])
    res = _run_batch(g, problems, graph, tbs=[1, 2, 3, 4, 6], tiles=[(128, 64), (64, 64), (256, 32), (128, 32)])
    for rep in res:
        for p, got, ref in zip(problems, rep, refs):
            np.testing.assert_array_equal(got, ref, err_msg=p.name)


def test_batched_config_sample(g):
    """A 32-grid sample of the 256-grid workload (sides log-uniform, mixed stencils), 200 steps."""
    problems = wl.batch_problems(n_grids=32, steps=200, hi=700)
    refs = [oracle.stencil_f32(p.u0, p.weights, 0.0, p.steps) for p in problems]
    res = _run_batch(g, problems, 2, reps=1)
    for p, got, ref in zip(problems, res[0], refs):
        np.testing.assert_array_equal(got, ref, err_msg=p.name)
        e = oracle.rel_l2(got, oracle.stencil_f64(p.u0, p.weights, 0.0, p.steps))
        assert e <= 1e-5, (p.name, e)


def test_batched_autotune_bitwise(g):
    """The batch autotuner changes only the depth of each class's passes: results stay bitwise equal
    to the oracle, before and after tuning, with and without the graph."""
    import torch
    import paper_2605_07954_amd as lib
    problems = _mixed(20, 11)
    refs = [oracle.stencil_f32(p.u0, p.weights, p.boundary, p.steps) for p in problems]
    plans = [lib.stencil_plan(p.rows, p.cols, p.radius, p.weights, p.boundary, "f32", 0) for p in problems]
    try:
        batch = lib.stencil_batch_create(plans, [p.steps for p in problems], lib.ST_FLAG_GRAPH)
        try:
            ins = [g.to_dev(p.u0) for p in problems]
            outs = [torch.empty_like(x) for x in ins]
            ws = torch.empty(lib.stencil_batch_workspace_bytes(batch), dtype=torch.uint8, device=g.DEV)
            lib.stencil_run_batched(batch, ins, outs, ws)  # builds the graph with the plans' depths
            caps = lib.stencil_batch_autotune(batch, ins, outs, ws)
            say("chosen caps", caps)
            assert caps and all(e in ("tiles", "march") and 1 <= d <= 16 for (e, d) in caps.values())
            for rep in range(2):
                for o in outs:
                    o.fill_(float("nan"))
                lib.stencil_run_batched(batch, ins, outs, ws)
                torch.cuda.synchronize()
                for p, o, ref in zip(problems, outs, refs):
                    np.testing.assert_array_equal(g.to_host(o), ref, err_msg=f"{p.name} rep {rep}")
        finally:
            lib.stencil_batch_destroy(batch)
    finally:
        for h in plans:
            lib.stencil_destroy(h)


@pytest.mark.parametrize("graph", [0, 2])
def test_batched_engines_every_class_bitwise(g, graph):
    """Every stencil class on LDS tiles and on the marching engine (four columns per lane: vector
    accesses for widths divisible by 4, element accesses otherwise) at every
    depth, with a shallower last pass (step counts not divisible by the depth): bitwise equal to the
    FP32-canonical oracle, directly and through the graph."""
    import torch
    import paper_2605_07954_amd as lib
    rng = np.random.default_rng(21)
    problems = []
    for k, (shape, r) in enumerate([(wl.STAR, 1), (wl.BOX, 1), (wl.STAR, 2), (wl.BOX, 2), (wl.STAR, 3), (wl.BOX, 3)]):
        for j in range(2):
            rows, cols, steps = [(150 + 37 * k, 301 + 11 * k, 7 + k % 2), (233, 130 + 16 * k, 13)][j]
            w = wl.random_footprint_weights(np.random.default_rng(700 + 10 * k + j), shape, r)
            problems.append(wl.Problem(f"{shape}{r}-{j}", rows, cols, r, shape, w, 0.0 if j else 0.5, steps,
                                       rng.random((rows, cols), dtype=np.float32)))
    refs = [oracle.stencil_f32(p.u0, p.weights, p.boundary, p.steps) for p in problems]
    plans = [lib.stencil_plan(p.rows, p.cols, p.radius, p.weights, p.boundary, "f32", 0) for p in problems]
    try:
        batch = lib.stencil_batch_create(plans, [p.steps for p in problems], graph)
        try:
            ins = [g.to_dev(p.u0) for p in problems]
            outs = [torch.empty_like(x) for x in ins]
            ws = torch.empty(lib.stencil_batch_workspace_bytes(batch), dtype=torch.uint8, device=g.DEV)
            deepest = {"star": {1: 8, 2: 6, 3: 4}, "box": {1: 6, 2: 3, 3: 2}}  # marching
            for engine in ("march", "tiles"):
                for r in (1, 2, 3):
                    for depth in range(1, deepest["star"][r] + 1):
                        for shape in ("star", "box"):  # the box classes stay at their deepest
                            lib.stencil_batch_set_class(batch, shape, r, engine, min(depth, deepest[shape][r]))
                        for o in outs:
                            o.fill_(float("nan"))
                        lib.stencil_run_batched(batch, ins, outs, ws)
                        torch.cuda.synchronize()
                        for p, o, ref in zip(problems, outs, refs):
                            np.testing.assert_array_equal(g.to_host(o), ref, err_msg=f"{p.name} {engine} r{r} x{depth}")
                        if engine != "march":
                            continue
                        # longer segments than the default sizing: bitwise the same
                        seg0 = lib.stencil_batch_get_segment(batch, "star", r)
                        assert seg0 >= 8
                        for seg in (2 * seg0, 5 * seg0, 1000):
                            lib.stencil_batch_set_segment(batch, "star", r, seg)
                            assert lib.stencil_batch_get_segment(batch, "star", r) == max(seg, seg0)
                            for o in outs:
                                o.fill_(float("nan"))
                            lib.stencil_run_batched(batch, ins, outs, ws)
                            torch.cuda.synchronize()
                            for p, o, ref in zip(problems, outs, refs):
                                np.testing.assert_array_equal(g.to_host(o), ref,
                                                              err_msg=f"{p.name} march r{r} x{depth} seg {seg}")
                        lib.stencil_batch_set_segment(batch, "star", r, 0)
            with pytest.raises(lib.StencilError):
                lib.stencil_batch_set_segment(batch, "star", 1, -1)
            with pytest.raises(lib.StencilError):
                lib.stencil_batch_set_class(batch, "star", 3, "march", 5)
            with pytest.raises(lib.StencilError):
                lib.stencil_batch_set_class(batch, "box", 3, "march", 3)
        finally:
            lib.stencil_batch_destroy(batch)
    finally:
        for h in plans:
            lib.stencil_destroy(h)
