"""The C-ABI library loads on a host without a GPU and exports every function the header declares;
host-side validation errors come back as status codes without touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2605_07954_amd as lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "mi355stencil.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(lib.LIBPATH):
        from paper_2605_07954_amd import build
        build.build()
    L = ctypes.CDLL(lib.LIBPATH, mode=os.RTLD_NOW)
    names = declared_functions()
    assert len(names) >= 29
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # the Python binding wraps every one of them under the same name
    assert not [n for n in names if n not in ("stencil_strerror", "stencil_last_error") and not hasattr(lib, n)]


def _plan(*a):
    h = ctypes.c_void_p()
    rc = lib.lib().stencil_plan(ctypes.byref(h), *a)
    return rc, h


def test_host_validation_codes():
    W = np.zeros((3, 3), np.float32)
    W[1, 1] = 1
    wp = W.ctypes.data_as(ctypes.c_void_p)
    assert _plan(0, 5, 1, wp, 0.0, 0, 0)[0] == -1           # rows < 1
    assert _plan(2**31 + 1, 5, 1, wp, 0.0, 0, 0)[0] == -1   # side > 2^31
    assert _plan(2**31, 2**31, 1, wp, 0.0, 0, 0)[0] == -1   # 2^62 cells: byte counts would wrap
    rc, h = _plan(2**23, 2**23, 1, wp, 0.0, 0, 0)            # 2^46 cells: the largest accepted
    assert rc == 0
    lib.stencil_destroy(h)
    assert _plan(5, 5, 0, wp, 0.0, 0, 0)[0] == -1           # radius 0
    assert _plan(5, 5, 5, wp, 0.0, 0, 0)[0] == -1           # radius > 4
    assert _plan(5, 5, 1, None, 0.0, 0, 0)[0] == -1         # NULL weights
    assert _plan(5, 5, 1, wp, float("nan"), 0, 0)[0] == -1  # non-finite b
    assert _plan(5, 5, 1, wp, 0.0, 7, 0)[0] == -1           # unknown storage
    assert _plan(5, 5, 1, wp, 0.0, 0, 0x80)[0] == -1        # unknown flag
    Wn = W.copy()
    Wn[0, 0] = np.inf
    assert _plan(5, 5, 1, Wn.ctypes.data_as(ctypes.c_void_p), 0.0, 0, 0)[0] == -1
    assert "finite" in lib.lib().stencil_last_error().decode()
    rc, h = _plan(5, 5, 1, wp, 0.0, 0, 0)
    assert rc == 0
    try:
        assert lib.stencil_workspace_bytes(h, 0) == 0
        tb, tx, ty = lib.stencil_get_blocking(h)
        lib.stencil_set_blocking(h, 1)
        assert lib.stencil_workspace_bytes(h, 1) == 0
        assert lib.stencil_workspace_bytes(h, 2) == 25 * 4
        with pytest.raises(lib.StencilError):
            lib.stencil_set_blocking(h, 0, 100, 100)   # tile not instantiated
        with pytest.raises(lib.StencilError):
            lib.stencil_set_blocking(h, 17)
        assert lib.stencil_get_march_segment(h) == 0        # default: one task per resident wavefront
        lib.stencil_set_march_segment(h, 12)
        assert lib.stencil_get_march_segment(h) == 12
        with pytest.raises(lib.StencilError) as ei:
            lib.stencil_set_march_segment(h, -1)
        assert ei.value.code == lib.ST_EINVAL
        assert lib.stencil_get_march_segment(h) == 12
        # a varcoef tuner call on a constant-weight plan is rejected before any device work
        assert lib.lib().stencil_autotune_varcoef(h, None, None, None, None, 0, 1, None, None, None, None) == -1
    finally:
        lib.stencil_destroy(h)
    v = lib.stencil_plan_varcoef(8, 8, 0.0, 0)
    try:  # and a constant-weight tuner call on a varcoef plan (it has no kappa to run with)
        assert lib.lib().stencil_autotune(v, None, None, None, 0, 1, None, None, None, None) == -1
        assert "stencil_autotune_varcoef" in lib.lib().stencil_last_error().decode()
    finally:
        lib.stencil_destroy(v)


def test_binding_checks_the_weight_count():
    """The C entry point reads (2r+1)^2 weights; the binding refuses an array of another size
    before handing it over."""
    with pytest.raises(ValueError):
        lib.stencil_plan(8, 8, 2, np.ones((3, 3), np.float32) / 9, 0.0, "f32", 0)
    h = lib.stencil_plan(8, 8, 2, np.ones(25, np.float32) / 25, 0.0, "f32", 0)  # flat is fine
    lib.stencil_destroy(h)


def test_binding_refuses_fields_smaller_than_the_plan():
    """Field tensors are checked against the plan's rows x cols (stencil_get_dims) before any call
    that would hand their pointers to a kernel."""
    import torch
    h = lib.stencil_plan(8, 6, 1, np.ones((3, 3), np.float32) / 9, 0.0, "bf16", 0)
    try:
        assert lib.stencil_get_dims(h) == (8, 6, lib.ST_BF16)
        small = torch.zeros(47, dtype=torch.int16)
        with pytest.raises(ValueError, match="holds 94 bytes"):
            lib.stencil_run(h, small, small, 1)
        with pytest.raises(ValueError, match="holds"):
            lib.stencil_autotune(h, small, small, None, 1)
    finally:
        lib.stencil_destroy(h)
    with pytest.raises(ValueError, match="holds"):
        lib.surrogate_infer(None, None, torch.zeros(10), None, None, 1, 4, 4, None)


def test_strerror():
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert lib.lib().stencil_strerror(code)


def test_batch_create_validation_on_host():
    """Batch creation is host-only: unsupported plans are refused, sizes are reported."""
    from workloads import heat5_weights, random_footprint_weights, BOX, STAR
    rng = np.random.default_rng(0)
    ok = [lib.stencil_plan(300, 260, 1, heat5_weights(), 0.0, "f32", 0),
          lib.stencil_plan(40, 50, 3, random_footprint_weights(rng, STAR, 3), 0.0, "f32", 0),
          lib.stencil_plan(100, 900, 2, random_footprint_weights(rng, BOX, 2), 0.5, "f32", 0)]
    bad = [lib.stencil_plan(64, 64, 4, np.ones((9, 9), np.float32) / 81, 0.0, "f32", 0),
           lib.stencil_plan(64, 64, 1, heat5_weights(), 0.0, "f16", 0),
           lib.stencil_plan_varcoef(64, 64, 0.0, 0)]
    try:
        b = lib.stencil_batch_create(ok, [10, 7, 0], lib.ST_FLAG_GRAPH)
        try:
            assert lib.stencil_batch_workspace_bytes(b) >= 300 * 260 * 4  # the multi-pass grid's ping-pong field
            assert lib.stencil_batch_get_segment(b, "star", 1) == 0     # on tiles: no marching segments
            lib.stencil_batch_set_segment(b, "box", 2, 64)
            for args in ((0, 1, -1), (2, 1, 8), (0, 4, 8), (0, 0, 8)):
                assert lib.lib().stencil_batch_set_segment(b, *args) == lib.ST_EINVAL
        finally:
            lib.stencil_batch_destroy(b)
        for p in bad:
            with pytest.raises(lib.StencilError) as ei:
                lib.stencil_batch_create(ok + [p], [1, 1, 1, 1], 0)
            assert ei.value.code == -3
        for steps in ([1, -1, 1], [1, 2**30 + 1, 1]):
            with pytest.raises(lib.StencilError) as ei:
                lib.stencil_batch_create(ok, steps, 0)
            assert ei.value.code == lib.ST_EINVAL
        with pytest.raises(lib.StencilError) as ei:
            lib.stencil_batch_create(ok, [1, 1, 1], 0x80)
        assert ei.value.code == lib.ST_EINVAL
        with pytest.raises(lib.StencilError) as ei:  # an empty batch
            lib.stencil_batch_create([], [], 0)
        assert ei.value.code == lib.ST_EINVAL
    finally:
        for p in ok + bad:
            lib.stencil_destroy(p)


def test_binding_constants_match_header():
    """Every status, storage, flag and variant constant of the binding equals the header's #define."""
    text = open(lib.HEADER).read()
    defs = {m.group(1): int(m.group(2), 0)
            for m in re.finditer(r"^#define\s+((?:ST|SG)_[A-Z0-9_]+)\s+\(?(-?(?:0x)?[0-9A-Fa-f]+)\)?", text, re.M)}
    names = [n for n in dir(lib) if re.fullmatch(r"(ST|SG)_[A-Z0-9_]+", n)]
    assert len(names) >= 15
    for n in names:
        assert n in defs, n
        assert getattr(lib, n) == defs[n], (n, getattr(lib, n), defs[n])


def test_train_cfg_layout_matches_header(tmp_path):
    """The binding's ctypes mirror of sg_train_cfg has the C compiler's size and field offsets."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    fields = [f[0] for f in lib.SgTrainCfg._fields_]
    src = tmp_path / "cfg.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "mi355stencil.h"\nint main(void) {\n'
                   '    printf("%zu", sizeof(sg_train_cfg));\n'
                   + "".join(f'    printf(" %zu", offsetof(sg_train_cfg, {f}));\n' for f in fields)
                   + "    return 0;\n}\n")
    exe = tmp_path / "cfg"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(lib.HEADER), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert got[0] == ctypes.sizeof(lib.SgTrainCfg)
    assert got[1:] == [getattr(lib.SgTrainCfg, f).offset for f in fields]


def test_boundary_api_host_checks():
    """stencil_set_boundary: kinds, the frame argument, naive plans, variant restrictions (host-only)."""
    import paper_2605_07954_amd as lib
    W = np.zeros((3, 3), dtype=np.float32)
    W[1, 1] = 1.0
    plan = lib.stencil_plan(10, 12, 1, W, 0.0, "f32", 0)
    try:
        assert lib.stencil_get_boundary(plan) == lib.ST_BC_CONST
        assert lib.stencil_frame_elems(plan) == 2 * 1 * (12 + 2) + 2 * 1 * 10
        for bad in (3, -1):
            with pytest.raises(lib.StencilError) as e:
                lib.stencil_set_boundary(plan, bad)
            assert e.value.code == lib.ST_EINVAL
        with pytest.raises(lib.StencilError) as e:  # a frame kind needs a frame
            lib.stencil_set_boundary(plan, lib.ST_BC_FRAME)
        assert e.value.code == lib.ST_EINVAL
        lib.stencil_set_variant(plan, lib.ST_VARIANT_TILED)
        lib.stencil_set_boundary(plan, lib.ST_BC_PERIODIC)
        assert lib.stencil_get_variant(plan) == lib.ST_VARIANT_MARCH  # switched to marching
        for v in (lib.ST_VARIANT_TILED, lib.ST_VARIANT_STREAM):
            with pytest.raises(lib.StencilError) as e:
                lib.stencil_set_variant(plan, v)
            assert e.value.code == lib.ST_EUNSUPPORTED
        lib.stencil_set_boundary(plan, lib.ST_BC_CONST)
        lib.stencil_set_variant(plan, lib.ST_VARIANT_TILED)
    finally:
        lib.stencil_destroy(plan)
    naive = lib.stencil_plan(10, 12, 1, W, 0.0, "f32", lib.ST_FLAG_NAIVE)
    try:
        with pytest.raises(lib.StencilError) as e:
            lib.stencil_set_boundary(naive, lib.ST_BC_PERIODIC)
        assert e.value.code == lib.ST_EUNSUPPORTED
    finally:
        lib.stencil_destroy(naive)
    vc = lib.stencil_plan_varcoef(10, 12, 0.0, 0)
    try:
        with pytest.raises(lib.StencilError) as e:
            lib.stencil_set_boundary(vc, lib.ST_BC_PERIODIC)
        assert e.value.code == lib.ST_EINVAL
    finally:
        lib.stencil_destroy(vc)
