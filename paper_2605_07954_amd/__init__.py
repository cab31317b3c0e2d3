"""MI355X (gfx950) library for iterated 2D Jacobi stencils -- Python binding.

A thin ctypes layer over ``include/mi355stencil.h``: every function here has
the name of the C entry point it calls and only marshals arguments (tensor
data pointers, the current HIP stream, host arrays).  All arithmetic runs in
the HIP kernels of ``libmi355stencil.so``; there is no CPU fallback, and every
call raises if the library is not built or a GPU is not available.

PyTorch supplies device memory and streams only.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libmi355stencil.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "mi355stencil.h")

ST_OK = 0
ST_EINVAL, ST_EALIAS, ST_EUNSUPPORTED, ST_EHIP, ST_ENOWS, ST_ENOMEM, ST_ESTATE = -1, -2, -3, -4, -5, -6, -7
ST_F32, ST_BF16, ST_F16 = 0, 1, 2
ST_FLAG_NAIVE, ST_FLAG_GRAPH, ST_FLAG_ALLOW_MFMA = 0x1, 0x2, 0x4
ST_VARIANT_TILED, ST_VARIANT_STREAM, ST_VARIANT_MARCH, ST_VARIANT_MARCH8, ST_VARIANT_MARCH1 = 0, 1, 2, 3, 4
ST_VARIANT_RESIDENT, ST_VARIANT_MFMA = 5, 6
ST_BC_CONST, ST_BC_PERIODIC, ST_BC_FRAME = 0, 1, 2
SG_PARAM_COUNT = 37889
SG_JUDGE_FULL, SG_JUDGE_PATCH = 0, 1
STORAGE = {"f32": ST_F32, "bf16": ST_BF16, "f16": ST_F16}

_lib = None
_p = ctypes.c_void_p
_i64 = ctypes.c_int64
_int = ctypes.c_int
_u32 = ctypes.c_uint32
_sz = ctypes.c_size_t


class StencilError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {code} ({_strerror(code)}): {_last_error()}")
        self.code = code


_SIGS = {
    "stencil_plan": [ctypes.POINTER(_p), _i64, _i64, _int, _p, ctypes.c_double, _int, _u32],
    "stencil_plan_varcoef": [ctypes.POINTER(_p), _i64, _i64, ctypes.c_double, _u32],
    "stencil_plan3d": [ctypes.POINTER(_p), _i64, _i64, _i64, _int, _p, ctypes.c_double, _int, _u32],
    "stencil_get_planes": [_p, ctypes.POINTER(_i64)],
    "stencil_destroy": [_p],
    "stencil_set_blocking": [_p, _int, _int, _int],
    "stencil_get_blocking": [_p, ctypes.POINTER(_int), ctypes.POINTER(_int), ctypes.POINTER(_int)],
    "stencil_get_dims": [_p, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_int)],
    "stencil_set_variant": [_p, _int],
    "stencil_get_variant": [_p, ctypes.POINTER(_int)],
    "stencil_set_march_segment": [_p, _i64],
    "stencil_set_boundary": [_p, _int, _p],
    "stencil_set_spin_limit": [_p, _i64],
    "stencil_resident_status": [_p, _p, _sz, ctypes.POINTER(_int), _p],
    "stencil_get_boundary": [_p, ctypes.POINTER(_int)],
    "stencil_frame_elems": [_p, ctypes.POINTER(_i64)],
    "stencil_get_march_segment": [_p, ctypes.POINTER(_i64)],
    "stencil_tiles": [ctypes.POINTER(_int), _int, ctypes.POINTER(_int)],
    "stencil_workspace_bytes": [_p, _i64, ctypes.POINTER(_sz)],
    "stencil_run": [_p, _p, _p, _i64, _p, _sz, _p],
    "stencil_run_varcoef": [_p, _p, _p, _p, _i64, _p, _sz, _p],
    "stencil_run_noalloc": [_p, _p, _p, _i64, _p],
    "stencil_noalloc_max_bytes": [ctypes.POINTER(_sz)],
    "stencil_norms_ws_bytes": [_p, ctypes.POINTER(_sz)],
    "stencil_norms": [_p, _p, _p, _p, _p, _sz, _p],
    "stencil_autotune": [_p, _p, _p, _p, _sz, _i64, ctypes.POINTER(_int), ctypes.POINTER(_int),
                         ctypes.POINTER(_int), _p],
    "stencil_autotune_varcoef": [_p, _p, _p, _p, _p, _sz, _i64, ctypes.POINTER(_int), ctypes.POINTER(_int),
                                 ctypes.POINTER(_int), _p],
    "stencil_solve_ws_bytes": [_p, _i64, ctypes.POINTER(_sz)],
    "stencil_solve": [_p, _p, _p, _i64, _i64, ctypes.c_double, ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_double),
                      _p, _sz, _p],
    "stencil_batch_create": [ctypes.POINTER(_p), _int, ctypes.POINTER(_p), ctypes.POINTER(_i64), _u32],
    "stencil_batch_workspace_bytes": [_p, ctypes.POINTER(_sz)],
    "stencil_run_batched": [_p, ctypes.POINTER(_p), ctypes.POINTER(_p), _p, _sz, _p],
    "stencil_batch_destroy": [_p],
    "stencil_batch_set_class": [_p, _int, _int, _int, _int],
    "stencil_batch_set_segment": [_p, _int, _int, _i64],
    "stencil_batch_get_segment": [_p, _int, _int, ctypes.POINTER(_i64)],
    "stencil_batch_autotune": [_p, ctypes.POINTER(_p), ctypes.POINTER(_p), _p, _sz, ctypes.POINTER(_int),
                               ctypes.POINTER(_int), _p],
    "surrogate_create": [ctypes.POINTER(_p), _u32],
    "surrogate_destroy": [_p],
    "surrogate_workspace_bytes": [_p, _int, _i64, _i64, ctypes.POINTER(_sz)],
    "surrogate_infer": [_p, _p, _p, _p, _p, _int, _i64, _i64, _p, _sz, _p],
    "surrogate_loss_grad": [_p, _p, _p, _p, _p, _p, _p, _int, _i64, _i64, _p, _p, _p, _sz, _p],
    "surrogate_field_scale": [_p, _int, _i64, _i64, _p, _p, _sz, _p],
    "surrogate_adam": [_p, _p, _p, _p, _int, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _p],
    "surrogate_synth_fields": [_p, _int, _i64, _i64, _p, _p, _p],
    "surrogate_crop": [_p, _p, _p, _int, _i64, _i64, _i64, _i64, _p],
    "surrogate_checked_ws_bytes": [_p, _i64, _i64, ctypes.POINTER(_sz)],
    "surrogate_train_ws_bytes": [_p, _p, ctypes.POINTER(_sz)],
    "surrogate_train": [_p, _p, _p, _p, _p, _p, _p, _p, _sz, _p],
    "surrogate_infer_checked": [_p, _p, _p, _p, _p, _i64, _i64, _p, _i64, ctypes.c_double, _int,
                                ctypes.POINTER(_int), ctypes.POINTER(ctypes.c_double), _p, _sz, _p],
    "surrogate_param_bytes": [_p, ctypes.POINTER(_sz), ctypes.POINTER(_sz)],
    "surrogate_init": [_p, _p, _p, ctypes.c_uint64, _p],
    "stencil_strerror": [_int],
    "stencil_last_error": [],
}


def lib():
    """Load the HIP library.  Raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"{LIBPATH} is missing: build it with __graft_entry__.build() "
                               "(there is no CPU fallback)")
        try:
            # load torch's HIP runtime first so that the library binds to the same runtime
            # instance as the device memory and streams it is handed
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIBPATH)
        for name, args in _SIGS.items():
            if not hasattr(L, name):  # reported by the ABI test; calling it raises AttributeError
                continue
            f = getattr(L, name)
            f.argtypes = args
            f.restype = _int
        L.stencil_strerror.restype = ctypes.c_char_p
        L.stencil_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _strerror(code: int) -> str:
    try:
        return lib().stencil_strerror(code).decode()
    except Exception:  # noqa: BLE001 - only used while formatting an error
        return "?"


def _last_error() -> str:
    try:
        return lib().stencil_last_error().decode()
    except Exception:  # noqa: BLE001
        return ""


def _ck(rc: int, what: str):
    if rc != ST_OK:
        raise StencilError(rc, what)


def _stream(stream):
    """The HIP stream to enqueue on: an explicit torch stream or torch's current stream."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return _p(s.cuda_stream)


def _dptr(t, what: str):
    """Device address of a contiguous GPU tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{what} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return _p(t.data_ptr())


def _nbytes(t) -> int:
    return 0 if t is None else t.numel() * t.element_size()


def stencil_get_dims(plan):
    """(rows, cols, storage code) of a plan."""
    r, c, st = _i64(), _i64(), _int()
    _ck(lib().stencil_get_dims(plan, ctypes.byref(r), ctypes.byref(c), ctypes.byref(st)), "stencil_get_dims")
    return r.value, c.value, st.value


def stencil_get_planes(plan) -> int:
    v = _i64()
    _ck(lib().stencil_get_planes(plan, ctypes.byref(v)), "stencil_get_planes")
    return v.value


def _fields(plan, **tensors):
    """Refuse GPU fields smaller than the plan's grid (the kernels would access memory past them)."""
    rows, cols, st = stencil_get_dims(plan)
    need = stencil_get_planes(plan) * rows * cols * (4 if st == ST_F32 else 2)
    for name, t in tensors.items():
        if t is not None and _nbytes(t) < need:
            raise ValueError(f"{name} holds {_nbytes(t)} bytes; the plan's {rows} x {cols} field needs {need}")


def _batch_fields(n: int, **tensors):
    """Refuse FP32 surrogate fields smaller than n cells."""
    for name, t in tensors.items():
        if t is not None and _nbytes(t) < 4 * n:
            raise ValueError(f"{name} holds {_nbytes(t)} bytes; {n} FP32 cells need {4 * n}")


def storage_code(storage) -> int:
    return STORAGE[storage] if isinstance(storage, str) else int(storage)


# ---------------------------------------------------------------------------
# plans
# ---------------------------------------------------------------------------

def stencil_plan(rows: int, cols: int, radius: int, weights, boundary: float = 0.0, storage="f32",
                 flags: int = 0):
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.float32))
    if w.size != (2 * radius + 1) ** 2:  # the library reads exactly (2r+1)^2 weights
        raise ValueError(f"weights must hold (2r+1)^2 = {(2 * radius + 1) ** 2} values for radius {radius}, "
                         f"got {w.size}")
    h = _p()
    _ck(lib().stencil_plan(ctypes.byref(h), rows, cols, radius, w.ctypes.data_as(_p), float(boundary),
                           storage_code(storage), flags), "stencil_plan")
    return h


def stencil_plan3d(planes: int, rows: int, cols: int, radius: int, weights, boundary: float = 0.0, storage="f32",
                   flags: int = 0):
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.float32))
    if w.size != (2 * radius + 1) ** 3:  # the library reads exactly (2r+1)^3 weights
        raise ValueError(f"weights must hold (2r+1)^3 = {(2 * radius + 1) ** 3} values for radius {radius}")
    h = _p()
    _ck(lib().stencil_plan3d(ctypes.byref(h), planes, rows, cols, radius, w.ctypes.data_as(_p), float(boundary),
                             storage_code(storage), flags), "stencil_plan3d")
    return h


def stencil_plan_varcoef(rows: int, cols: int, boundary: float = 0.0, flags: int = 0):
    h = _p()
    _ck(lib().stencil_plan_varcoef(ctypes.byref(h), rows, cols, float(boundary), flags), "stencil_plan_varcoef")
    return h


def stencil_destroy(plan) -> None:
    _ck(lib().stencil_destroy(plan), "stencil_destroy")


def stencil_set_blocking(plan, tb: int = 0, tile_x: int = 0, tile_y: int = 0) -> None:
    _ck(lib().stencil_set_blocking(plan, tb, tile_x, tile_y), "stencil_set_blocking")


def stencil_set_variant(plan, variant: int) -> None:
    _ck(lib().stencil_set_variant(plan, variant), "stencil_set_variant")


def stencil_get_variant(plan) -> int:
    v = _int()
    _ck(lib().stencil_get_variant(plan, ctypes.byref(v)), "stencil_get_variant")
    return v.value


def stencil_set_boundary(plan, kind: int, frame=None) -> None:
    """kind: ST_BC_CONST, ST_BC_PERIODIC or ST_BC_FRAME (with `frame`, a device tensor of
    stencil_frame_elems(plan) elements of the plan's storage type, kept alive by the caller)."""
    if frame is not None:
        rows, cols, st = stencil_get_dims(plan)
        if _nbytes(frame) < stencil_frame_elems(plan) * (4 if st == ST_F32 else 2):
            raise ValueError("frame holds fewer elements than stencil_frame_elems(plan)")
    _ck(lib().stencil_set_boundary(plan, int(kind), _dptr(frame, "frame")), "stencil_set_boundary")


def stencil_set_spin_limit(plan, polls: int) -> None:
    _ck(lib().stencil_set_spin_limit(plan, int(polls)), "stencil_set_spin_limit")


def stencil_resident_status(plan, workspace, stream=None):
    """(gave_up, workgroup, epoch, neighbour) of the last resident run on `workspace` (synchronises)."""
    st = (_int * 4)()
    _ck(lib().stencil_resident_status(plan, _dptr(workspace, "workspace"), _nbytes(workspace), st, _stream(stream)),
        "stencil_resident_status")
    return tuple(int(v) for v in st)


def stencil_get_boundary(plan) -> int:
    v = _int()
    _ck(lib().stencil_get_boundary(plan, ctypes.byref(v)), "stencil_get_boundary")
    return v.value


def stencil_frame_elems(plan) -> int:
    v = _i64()
    _ck(lib().stencil_frame_elems(plan, ctypes.byref(v)), "stencil_frame_elems")
    return v.value


def stencil_set_march_segment(plan, min_rows: int) -> None:
    _ck(lib().stencil_set_march_segment(plan, int(min_rows)), "stencil_set_march_segment")


def stencil_get_march_segment(plan) -> int:
    v = _i64()
    _ck(lib().stencil_get_march_segment(plan, ctypes.byref(v)), "stencil_get_march_segment")
    return v.value


def stencil_get_blocking(plan):
    tb, tx, ty = _int(), _int(), _int()
    _ck(lib().stencil_get_blocking(plan, ctypes.byref(tb), ctypes.byref(tx), ctypes.byref(ty)),
        "stencil_get_blocking")
    return tb.value, tx.value, ty.value


def stencil_tiles():
    buf = (_int * 64)()
    n = _int()
    _ck(lib().stencil_tiles(buf, 32, ctypes.byref(n)), "stencil_tiles")
    return [(buf[2 * i], buf[2 * i + 1]) for i in range(min(n.value, 32))]


def stencil_workspace_bytes(plan, steps: int) -> int:
    n = _sz()
    _ck(lib().stencil_workspace_bytes(plan, steps, ctypes.byref(n)), "stencil_workspace_bytes")
    return n.value


def stencil_run(plan, inp, out, steps: int, workspace=None, stream=None) -> None:
    _fields(plan, inp=inp, out=out)
    _ck(lib().stencil_run(plan, _dptr(inp, "in"), _dptr(out, "out"), steps, _dptr(workspace, "workspace"),
                          _nbytes(workspace), _stream(stream)), "stencil_run")


def stencil_run_noalloc(plan, inp, out, steps: int, stream=None) -> None:
    _fields(plan, inp=inp, out=out)
    _ck(lib().stencil_run_noalloc(plan, _dptr(inp, "in"), _dptr(out, "out"), steps, _stream(stream)),
        "stencil_run_noalloc")


def stencil_noalloc_max_bytes() -> int:
    n = _sz()
    _ck(lib().stencil_noalloc_max_bytes(ctypes.byref(n)), "stencil_noalloc_max_bytes")
    return n.value


def stencil_run_varcoef(plan, inp, kappa, out, steps: int, workspace=None, stream=None) -> None:
    _fields(plan, inp=inp, kappa=kappa, out=out)
    _ck(lib().stencil_run_varcoef(plan, _dptr(inp, "in"), _dptr(kappa, "kappa"), _dptr(out, "out"), steps,
                                  _dptr(workspace, "workspace"), _nbytes(workspace), _stream(stream)),
        "stencil_run_varcoef")


def stencil_norms_ws_bytes(plan) -> int:
    n = _sz()
    _ck(lib().stencil_norms_ws_bytes(plan, ctypes.byref(n)), "stencil_norms_ws_bytes")
    return n.value


def stencil_norms(plan, u_prev, u, out4, workspace, stream=None) -> None:
    _fields(plan, u_prev=u_prev, u=u)
    if out4 is not None and _nbytes(out4) < 32:
        raise ValueError("out4 must hold 4 doubles")
    _ck(lib().stencil_norms(plan, _dptr(u_prev, "u_prev"), _dptr(u, "u"), _dptr(out4, "out4"),
                            _dptr(workspace, "workspace"), _nbytes(workspace), _stream(stream)), "stencil_norms")


def stencil_autotune(plan, inp, out, workspace, sample_steps: int, stream=None):
    _fields(plan, inp=inp, out=out)
    tb, tx, ty = _int(), _int(), _int()
    _ck(lib().stencil_autotune(plan, _dptr(inp, "in"), _dptr(out, "out"), _dptr(workspace, "workspace"),
                               _nbytes(workspace), sample_steps, ctypes.byref(tb), ctypes.byref(tx),
                               ctypes.byref(ty), _stream(stream)), "stencil_autotune")
    return tb.value, tx.value, ty.value


def stencil_autotune_varcoef(plan, inp, kappa, out, workspace, sample_steps: int, stream=None):
    _fields(plan, inp=inp, kappa=kappa, out=out)
    tb, tx, ty = _int(), _int(), _int()
    _ck(lib().stencil_autotune_varcoef(plan, _dptr(inp, "in"), _dptr(kappa, "kappa"), _dptr(out, "out"),
                                       _dptr(workspace, "workspace"), _nbytes(workspace), sample_steps,
                                       ctypes.byref(tb), ctypes.byref(tx), ctypes.byref(ty), _stream(stream)),
        "stencil_autotune_varcoef")
    return tb.value, tx.value, ty.value


def stencil_solve_ws_bytes(plan, check_every: int) -> int:
    n = _sz()
    _ck(lib().stencil_solve_ws_bytes(plan, check_every, ctypes.byref(n)), "stencil_solve_ws_bytes")
    return n.value


def stencil_solve(plan, inp, out, max_steps: int, check_every: int, tol: float, workspace, stream=None):
    """Returns (steps_done, relative residual of the last step)."""
    _fields(plan, inp=inp, out=out)
    done = _i64()
    res = ctypes.c_double()
    _ck(lib().stencil_solve(plan, _dptr(inp, "in"), _dptr(out, "out"), max_steps, check_every, float(tol),
                            ctypes.byref(done), ctypes.byref(res), _dptr(workspace, "workspace"), _nbytes(workspace),
                            _stream(stream)), "stencil_solve")
    return done.value, res.value


# ---------------------------------------------------------------------------
# batched
# ---------------------------------------------------------------------------

def stencil_batch_create(plans, steps, flags: int = 0):
    n = len(plans)
    arr = (_p * n)(*[p.value if isinstance(p, _p) else p for p in plans])
    st = (_i64 * n)(*[int(s) for s in steps])
    h = _p()
    _ck(lib().stencil_batch_create(ctypes.byref(h), n, arr, st, flags), "stencil_batch_create")
    return h


def stencil_batch_workspace_bytes(batch) -> int:
    n = _sz()
    _ck(lib().stencil_batch_workspace_bytes(batch, ctypes.byref(n)), "stencil_batch_workspace_bytes")
    return n.value


def stencil_run_batched(batch, ins, outs, workspace, stream=None) -> None:
    n = len(ins)
    pi = (_p * n)(*[_dptr(t, "in").value for t in ins])
    po = (_p * n)(*[_dptr(t, "out").value for t in outs])
    _ck(lib().stencil_run_batched(batch, pi, po, _dptr(workspace, "workspace"), _nbytes(workspace),
                                  _stream(stream)), "stencil_run_batched")


def stencil_batch_set_segment(batch, shape: str, radius: int, min_rows: int) -> None:
    _ck(lib().stencil_batch_set_segment(batch, {"star": 0, "box": 1}[shape], radius, int(min_rows)),
        "stencil_batch_set_segment")


def stencil_batch_get_segment(batch, shape: str, radius: int) -> int:
    v = _i64()
    _ck(lib().stencil_batch_get_segment(batch, {"star": 0, "box": 1}[shape], radius, ctypes.byref(v)),
        "stencil_batch_get_segment")
    return v.value


def stencil_batch_set_class(batch, shape: str, radius: int, engine: str, depth: int) -> None:
    _ck(lib().stencil_batch_set_class(batch, {"star": 0, "box": 1}[shape], radius, {"tiles": 0, "march": 1}[engine],
                                      depth), "stencil_batch_set_class")


def stencil_batch_autotune(batch, ins, outs, workspace, stream=None) -> dict:
    """Returns the choice per stencil class present: {("star", 1): ("march", 2), ("box", 3): ("tiles", 1), ...}."""
    n = len(ins)
    pi = (_p * n)(*[_dptr(t, "in").value for t in ins])
    po = (_p * n)(*[_dptr(t, "out").value for t in outs])
    depth = (_int * 6)()
    engine = (_int * 6)()
    _ck(lib().stencil_batch_autotune(batch, pi, po, _dptr(workspace, "workspace"), _nbytes(workspace), depth,
                                     engine, _stream(stream)), "stencil_batch_autotune")
    names = [("star", 1), ("star", 2), ("star", 3), ("box", 1), ("box", 2), ("box", 3)]
    return {names[k]: (("tiles", "march")[engine[k]], depth[k]) for k in range(6) if depth[k]}


def stencil_batch_destroy(batch) -> None:
    _ck(lib().stencil_batch_destroy(batch), "stencil_batch_destroy")


# ---------------------------------------------------------------------------
# surrogate
# ---------------------------------------------------------------------------

class SgTrainCfg(ctypes.Structure):
    """Mirror of ``sg_train_cfg``."""
    _fields_ = [("rows", _i64), ("cols", _i64), ("crop", _i64), ("batch", _int), ("K", _int), ("steps", _i64),
                ("step0", _i64), ("total_steps", _i64), ("lr", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float)]


def _train_cfg(rows, cols, crop, batch, K, steps, step0, total_steps, lr, beta1, beta2, eps) -> SgTrainCfg:
    return SgTrainCfg(rows, cols, crop, batch, K, steps, step0, total_steps, lr, beta1, beta2, eps)


def surrogate_train_ws_bytes(model, rows: int, cols: int, crop: int, batch: int, K: int, steps: int) -> int:
    cfg = _train_cfg(rows, cols, crop, batch, K, steps, 0, max(steps, 1), 1e-3, 0.9, 0.999, 1e-8)
    n = _sz()
    _ck(lib().surrogate_train_ws_bytes(model, ctypes.byref(cfg), ctypes.byref(n)), "surrogate_train_ws_bytes")
    return n.value


def surrogate_train(model, params, optim, coef, crop_yx, losses, workspace, rows: int, cols: int, crop: int,
                    batch: int, K: int, steps: int, step0: int, total_steps: int, lr: float, beta1: float = 0.9,
                    beta2: float = 0.999, eps: float = 1e-8, stream=None) -> None:
    """crop_yx: host int32 array of 2*steps*batch offsets; coef, losses: device tensors."""
    yx = np.ascontiguousarray(np.asarray(crop_yx, dtype=np.int32).reshape(-1))
    if yx.size != 2 * steps * batch:
        raise ValueError("crop_yx must hold 2 * steps * batch offsets")
    cfg = _train_cfg(rows, cols, crop, batch, K, steps, step0, total_steps, lr, beta1, beta2, eps)
    _ck(lib().surrogate_train(model, _dptr(params, "params"), _dptr(optim, "optim"), _dptr(coef, "coef"),
                              yx.ctypes.data_as(_p), ctypes.byref(cfg), _dptr(losses, "losses"),
                              _dptr(workspace, "workspace"), _nbytes(workspace), _stream(stream)), "surrogate_train")

def surrogate_create(flags: int = 0):
    h = _p()
    _ck(lib().surrogate_create(ctypes.byref(h), flags), "surrogate_create")
    return h


def surrogate_destroy(model) -> None:
    _ck(lib().surrogate_destroy(model), "surrogate_destroy")


def surrogate_param_bytes(model):
    """(parameter bytes, Adam state bytes)."""
    a, b = _sz(), _sz()
    _ck(lib().surrogate_param_bytes(model, ctypes.byref(a), ctypes.byref(b)), "surrogate_param_bytes")
    return a.value, b.value


def surrogate_init(model, params, optim_state, seed: int, stream=None) -> None:
    if _nbytes(params) < 4 * SG_PARAM_COUNT or (optim_state is not None and _nbytes(optim_state) < 8 * SG_PARAM_COUNT):
        raise ValueError("params needs SG_PARAM_COUNT floats and optim_state twice that")
    _ck(lib().surrogate_init(model, _dptr(params, "params"), _dptr(optim_state, "optim_state"),
                             ctypes.c_uint64(int(seed) & (2**64 - 1)), _stream(stream)), "surrogate_init")


def surrogate_workspace_bytes(model, batch: int, rows: int, cols: int) -> int:
    n = _sz()
    _ck(lib().surrogate_workspace_bytes(model, batch, rows, cols, ctypes.byref(n)), "surrogate_workspace_bytes")
    return n.value


def surrogate_infer(model, params, u0, kappa, u_hat, batch: int, rows: int, cols: int, workspace,
                      stream=None) -> None:
    _batch_fields(batch * rows * cols, u0=u0, kappa=kappa, u_hat=u_hat)
    _ck(lib().surrogate_infer(model, _dptr(params, "params"), _dptr(u0, "u0"), _dptr(kappa, "kappa"),
                                _dptr(u_hat, "u_hat"), batch, rows, cols, _dptr(workspace, "workspace"),
                                _nbytes(workspace), _stream(stream)), "surrogate_infer")


def surrogate_field_scale(u0, n: int, rows: int, cols: int, scale, workspace, stream=None) -> None:
    _batch_fields(n * rows * cols, u0=u0)
    _ck(lib().surrogate_field_scale(_dptr(u0, "u0"), n, rows, cols, _dptr(scale, "scale"), _dptr(workspace, "workspace"),
                                    _nbytes(workspace), _stream(stream)), "surrogate_field_scale")


def surrogate_loss_grad(model, params, u0, kappa, target, lo_hi, batch: int, rows: int, cols: int, grad, loss,
                        workspace, scale=None, stream=None) -> None:
    _batch_fields(batch * rows * cols, u0=u0, kappa=kappa, target=target)
    flat = [int(v) for v in np.asarray(lo_hi).reshape(-1)]
    if len(flat) == 4 and batch > 1:  # one mask for every field
        flat = flat * batch
    lh = (_int * len(flat))(*flat)
    _ck(lib().surrogate_loss_grad(model, _dptr(params, "params"), _dptr(u0, "u0"), _dptr(kappa, "kappa"),
                                  _dptr(scale, "scale"), _dptr(target, "target"), ctypes.cast(lh, _p), batch, rows, cols,
                                  _dptr(grad, "grad"), _dptr(loss, "loss"), _dptr(workspace, "workspace"),
                                  _nbytes(workspace), _stream(stream)), "surrogate_loss_grad")


def surrogate_adam(model, params, grad, optim, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
                   eps: float = 1e-8, stream=None) -> None:
    _ck(lib().surrogate_adam(model, _dptr(params, "params"), _dptr(grad, "grad"), _dptr(optim, "optim"), t,
                             lr, beta1, beta2, eps, _stream(stream)), "surrogate_adam")


def surrogate_synth_fields(coef, n: int, rows: int, cols: int, u0_out, kappa_out, stream=None) -> None:
    _ck(lib().surrogate_synth_fields(_dptr(coef, "coef"), n, rows, cols, _dptr(u0_out, "u0_out"),
                                     _dptr(kappa_out, "kappa_out"), _stream(stream)), "surrogate_synth_fields")


def surrogate_crop(src, dst, yx, n: int, rows: int, cols: int, h: int, w: int, stream=None) -> None:
    _ck(lib().surrogate_crop(_dptr(src, "src"), _dptr(dst, "dst"), _dptr(yx, "yx"), n, rows, cols, h, w,
                             _stream(stream)), "surrogate_crop")


def surrogate_checked_ws_bytes(model, rows: int, cols: int) -> int:
    n = _sz()
    _ck(lib().surrogate_checked_ws_bytes(model, rows, cols, ctypes.byref(n)), "surrogate_checked_ws_bytes")
    return n.value


def surrogate_infer_checked(model, params, u0, kappa, out, rows: int, cols: int, judge, K: int, tol: float,
                            workspace, judge_mode: int = SG_JUDGE_FULL, stream=None):
    _batch_fields(rows * cols, u0=u0, kappa=kappa, out=out)
    used = _int()
    err = ctypes.c_double()
    _ck(lib().surrogate_infer_checked(model, _dptr(params, "params"), _dptr(u0, "u0"), _dptr(kappa, "kappa"),
                                      _dptr(out, "out"), rows, cols, judge, K, float(tol), int(judge_mode),
                                      ctypes.byref(used),
                                      ctypes.byref(err), _dptr(workspace, "workspace"), _nbytes(workspace),
                                      _stream(stream)), "surrogate_infer_checked")
    return bool(used.value), err.value
