"""CPU oracle for the stencil library -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it and the
two share no code; they are fed the same host buffers drawn by ``workloads``.

Contents
  * the plain stencil definition (``stencil_oracle.c``, loaded with ctypes):
    FP64, FP32-canonical and BF16/FP16-storage-emulating modes, the light-cone
    patch, the variable-coefficient heat step, periodic and caller-framed
    boundaries, and the 3D form;
  * FP64 norms (residual, energy, mass, predicted next mass);
  * the CNN surrogate's forward / backward / Adam in FP64 (``oracle.cnn``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(HERE, "liboracle.so")
_lib = None

_i64 = ctypes.c_int64
_p = ctypes.c_void_p


def lib():
    """Load liboracle.so (built by ``oracle.build.build()``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            # compile the checker where it is used (gcc only; nothing of the GPU library is involved)
            from . import build as _build
            _build.build()
        L = ctypes.CDLL(_LIBPATH)
        L.oracle_stencil_f64.argtypes = [_i64, _i64, ctypes.c_int, _p, ctypes.c_double, _i64, _p, _p]
        L.oracle_stencil_f32.argtypes = [_i64, _i64, ctypes.c_int, _p, ctypes.c_float, _i64, _p, _p]
        L.oracle_stencil_lowp.argtypes = [ctypes.c_int, _i64, _i64, ctypes.c_int, _p, ctypes.c_float,
                                          _i64, _p, _p]
        L.oracle_stencil_patch_f64.argtypes = [_i64, _i64, ctypes.c_int, _p, ctypes.c_double, _i64, _p,
                                               _i64, _i64, _i64, _i64, _p]
        L.oracle_stencil_bc_f64.argtypes = [ctypes.c_int, _i64, _i64, ctypes.c_int, _p, _p, _i64, _p, _p]
        L.oracle_stencil_bc_f32.argtypes = [ctypes.c_int, _i64, _i64, ctypes.c_int, _p, _p, _i64, _p, _p]
        L.oracle_stencil_bc_lowp.argtypes = [ctypes.c_int, ctypes.c_int, _i64, _i64, ctypes.c_int, _p, _p, _i64,
                                             _p, _p]
        L.oracle_frame_elems.argtypes = [_i64, _i64, ctypes.c_int]
        L.oracle_frame_elems.restype = _i64
        L.oracle_stencil3d_f64.argtypes = [_i64, _i64, _i64, ctypes.c_int, _p, ctypes.c_double, _i64, _p, _p]
        L.oracle_stencil3d_f32.argtypes = [_i64, _i64, _i64, ctypes.c_int, _p, ctypes.c_float, _i64, _p, _p]
        L.oracle_varcoef_f64.argtypes = [_i64, _i64, ctypes.c_double, _i64, _p, _p, _p]
        L.oracle_varcoef_f32.argtypes = [_i64, _i64, ctypes.c_float, _i64, _p, _p, _p]
        for nm in ("oracle_f32_to_bf16_array", "oracle_bf16_to_f32_array",
                   "oracle_f32_to_f16_array", "oracle_f16_to_f32_array"):
            getattr(L, nm).argtypes = [_i64, _p, _p]
            getattr(L, nm).restype = None
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads.restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"{what} failed with code {rc}")


def num_threads() -> int:
    return lib().oracle_num_threads()


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))


def radius_of(W: np.ndarray) -> int:
    k = W.shape[0]
    if W.ndim != 2 or W.shape[1] != k or k % 2 != 1:
        raise ValueError("weights must be a square (2r+1)x(2r+1) array")
    return (k - 1) // 2


# ---------------------------------------------------------------------------
# plain stencil (Sec. II-C Jacobi update with the fixed halo of Sec. IV-A)
# ---------------------------------------------------------------------------

def stencil_f64(u0: np.ndarray, W: np.ndarray, b: float, steps: int) -> np.ndarray:
    """FP64 truth: input and (FP32-rounded) weights promoted to double."""
    u = np.ascontiguousarray(u0, dtype=np.float64)
    w = np.ascontiguousarray(W, dtype=np.float64)
    out = np.empty_like(u)
    _check(lib().oracle_stencil_f64(u.shape[0], u.shape[1], radius_of(w), _ptr(w), float(b), int(steps),
                                    _ptr(u), _ptr(out)), "oracle_stencil_f64")
    return out


def stencil_f32(u0: np.ndarray, W: np.ndarray, b: float, steps: int) -> np.ndarray:
    """FP32-canonical: centre product, then one fmaf per nonzero tap in row-major order."""
    u = np.ascontiguousarray(u0, dtype=np.float32)
    w = np.ascontiguousarray(W, dtype=np.float32)
    out = np.empty_like(u)
    _check(lib().oracle_stencil_f32(u.shape[0], u.shape[1], radius_of(w), _ptr(w), float(b), int(steps),
                                    _ptr(u), _ptr(out)), "oracle_stencil_f32")
    return out


LOWP_CODE = {"bf16": 1, "f16": 2}


def stencil_lowp(u0_bits: np.ndarray, W: np.ndarray, b: float, steps: int, dtype: str) -> np.ndarray:
    """16-bit storage emulation: FP32-canonical step, rounded to ``dtype`` after every step.

    ``u0_bits`` holds the raw 16-bit patterns (uint16); so does the result.
    """
    u = np.ascontiguousarray(u0_bits, dtype=np.uint16)
    w = np.ascontiguousarray(W, dtype=np.float32)
    out = np.empty_like(u)
    _check(lib().oracle_stencil_lowp(LOWP_CODE[dtype], u.shape[0], u.shape[1], radius_of(w), _ptr(w),
                                     float(b), int(steps), _ptr(u), _ptr(out)), "oracle_stencil_lowp")
    return out


def stencil_patch_f64(u0: np.ndarray, W: np.ndarray, b: float, steps: int,
                      y0: int, x0: int, h: int, w: int) -> np.ndarray:
    """FP64 result on rows [y0, y0+h) x cols [x0, x0+w) of the full grid after ``steps`` steps."""
    u = np.ascontiguousarray(u0, dtype=np.float32)
    wt = np.ascontiguousarray(W, dtype=np.float64)
    out = np.empty((h, w), dtype=np.float64)
    _check(lib().oracle_stencil_patch_f64(u.shape[0], u.shape[1], radius_of(wt), _ptr(wt), float(b),
                                          int(steps), _ptr(u), y0, x0, h, w, _ptr(out)),
           "oracle_stencil_patch_f64")
    return out


# ---------------------------------------------------------------------------
# other boundary rules: periodic (bc = 1) and a caller-given fixed halo frame (bc = 2)
# ---------------------------------------------------------------------------
BC_CODE = {"periodic": 1, "frame": 2}


def frame_elems(rows: int, cols: int, r: int) -> int:
    """Elements of a halo frame: top and bottom strips r x (cols + 2r), left and right strips rows x r."""
    return int(lib().oracle_frame_elems(rows, cols, r))


def _frame_arg(frame, dtype, rows, cols, r):
    if frame is None:
        return None, None
    f = np.ascontiguousarray(frame, dtype=dtype).reshape(-1)
    if f.size != frame_elems(rows, cols, r):
        raise ValueError("frame has the wrong number of elements")
    return f, _ptr(f)


def stencil_bc_f64(u0: np.ndarray, W: np.ndarray, bc: str, steps: int, frame=None) -> np.ndarray:
    """FP64 run with a periodic or framed boundary (frame values promoted to double)."""
    u = np.ascontiguousarray(u0, dtype=np.float64)
    w = np.ascontiguousarray(W, dtype=np.float64)
    r = radius_of(w)
    f, fp = _frame_arg(frame, np.float64, u.shape[0], u.shape[1], r)
    out = np.empty_like(u)
    _check(lib().oracle_stencil_bc_f64(BC_CODE[bc], u.shape[0], u.shape[1], r, _ptr(w), fp, int(steps), _ptr(u),
                                       _ptr(out)), "oracle_stencil_bc_f64")
    return out


def stencil_bc_f32(u0: np.ndarray, W: np.ndarray, bc: str, steps: int, frame=None) -> np.ndarray:
    """FP32-canonical run with a periodic or framed boundary."""
    u = np.ascontiguousarray(u0, dtype=np.float32)
    w = np.ascontiguousarray(W, dtype=np.float32)
    r = radius_of(w)
    f, fp = _frame_arg(frame, np.float32, u.shape[0], u.shape[1], r)
    out = np.empty_like(u)
    _check(lib().oracle_stencil_bc_f32(BC_CODE[bc], u.shape[0], u.shape[1], r, _ptr(w), fp, int(steps), _ptr(u),
                                       _ptr(out)), "oracle_stencil_bc_f32")
    return out


def stencil_bc_lowp(u0_bits: np.ndarray, W: np.ndarray, bc: str, steps: int, dtype: str, frame_bits=None):
    """16-bit storage emulation with a periodic or framed boundary (frame in raw 16-bit patterns)."""
    u = np.ascontiguousarray(u0_bits, dtype=np.uint16)
    w = np.ascontiguousarray(W, dtype=np.float32)
    r = radius_of(w)
    f, fp = _frame_arg(frame_bits, np.uint16, u.shape[0], u.shape[1], r)
    out = np.empty_like(u)
    _check(lib().oracle_stencil_bc_lowp(LOWP_CODE[dtype], BC_CODE[bc], u.shape[0], u.shape[1], r, _ptr(w), fp,
                                        int(steps), _ptr(u), _ptr(out)), "oracle_stencil_bc_lowp")
    return out


# ---------------------------------------------------------------------------
# 3D (planes x rows x cols, (2r+1)^3 weights W[dz+r][dy+r][dx+r], constant halo b)
# ---------------------------------------------------------------------------

def _radius3(W: np.ndarray) -> int:
    k = W.shape[0]
    if W.ndim != 3 or W.shape != (k, k, k) or k % 2 != 1:
        raise ValueError("3D weights must be a (2r+1)^3 array")
    return (k - 1) // 2


def stencil3d_f64(u0: np.ndarray, W: np.ndarray, b: float, steps: int) -> np.ndarray:
    u = np.ascontiguousarray(u0, dtype=np.float64)
    w = np.ascontiguousarray(W, dtype=np.float64)
    out = np.empty_like(u)
    _check(lib().oracle_stencil3d_f64(u.shape[0], u.shape[1], u.shape[2], _radius3(w), _ptr(w), float(b), int(steps),
                                      _ptr(u), _ptr(out)), "oracle_stencil3d_f64")
    return out


def stencil3d_f32(u0: np.ndarray, W: np.ndarray, b: float, steps: int) -> np.ndarray:
    """FP32-canonical 3D: centre product, then fmaf per nonzero tap in row-major (dz, dy, dx) order."""
    u = np.ascontiguousarray(u0, dtype=np.float32)
    w = np.ascontiguousarray(W, dtype=np.float32)
    out = np.empty_like(u)
    _check(lib().oracle_stencil3d_f32(u.shape[0], u.shape[1], u.shape[2], _radius3(w), _ptr(w), float(b), int(steps),
                                      _ptr(u), _ptr(out)), "oracle_stencil3d_f32")
    return out


def varcoef_f64(u0: np.ndarray, kappa: np.ndarray, b: float, steps: int) -> np.ndarray:
    u = np.ascontiguousarray(u0, dtype=np.float64)
    k = np.ascontiguousarray(kappa, dtype=np.float64)
    out = np.empty_like(u)
    _check(lib().oracle_varcoef_f64(u.shape[0], u.shape[1], float(b), int(steps), _ptr(k), _ptr(u), _ptr(out)),
           "oracle_varcoef_f64")
    return out


def varcoef_f32(u0: np.ndarray, kappa: np.ndarray, b: float, steps: int) -> np.ndarray:
    u = np.ascontiguousarray(u0, dtype=np.float32)
    k = np.ascontiguousarray(kappa, dtype=np.float32)
    out = np.empty_like(u)
    _check(lib().oracle_varcoef_f32(u.shape[0], u.shape[1], float(b), int(steps), _ptr(k), _ptr(u), _ptr(out)),
           "oracle_varcoef_f32")
    return out


# ---------------------------------------------------------------------------
# 16-bit formats
# ---------------------------------------------------------------------------

def _conv(name: str, a: np.ndarray, out_dtype) -> np.ndarray:
    src = np.ascontiguousarray(a)
    out = np.empty(src.shape, dtype=out_dtype)
    getattr(lib(), name)(src.size, _ptr(src), _ptr(out))
    return out


def to_bits(x: np.ndarray, dtype: str) -> np.ndarray:
    """Round FP32 values to BF16/FP16 (nearest, ties to even) and return the uint16 patterns."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    return _conv("oracle_f32_to_bf16_array" if dtype == "bf16" else "oracle_f32_to_f16_array", x, np.uint16)


def from_bits(h: np.ndarray, dtype: str) -> np.ndarray:
    h = np.ascontiguousarray(h, dtype=np.uint16)
    return _conv("oracle_bf16_to_f32_array" if dtype == "bf16" else "oracle_f16_to_f32_array", h, np.float32)


# ---------------------------------------------------------------------------
# FP64 norms and error measures
# ---------------------------------------------------------------------------

def support_sums(rows: int, cols: int, W: np.ndarray) -> np.ndarray:
    """S_j = sum over taps d of W_d * [j - d is a grid cell]: how much of u_j the next step keeps.

    Written as one shifted rectangle per tap: cell j = i + d receives W_d from
    every grid cell i, i.e. j ranges over the grid shifted by d, clipped.
    """
    r = radius_of(W)
    S = np.zeros((rows, cols), dtype=np.float64)
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            w = float(W[dy + r, dx + r])
            if w == 0.0:
                continue
            y0, y1 = max(dy, 0), max(0, min(rows + dy, rows))  # empty when |dy| >= rows
            x0, x1 = max(dx, 0), max(0, min(cols + dx, cols))
            if y0 < y1 and x0 < x1:
                S[y0:y1, x0:x1] += w
    return S


def norms_f64(u: np.ndarray, W: np.ndarray, b: float, u_prev: np.ndarray | None = None) -> np.ndarray:
    """[sum (u-u_prev)^2, sum u^2, sum u, predicted next mass] in FP64.

    The predicted mass of the next step is sum_j (u_j - b) S_j + b * N * sum(W):
    summing the update over all N cells, each grid value u_j is picked up with
    total weight S_j and the halo value b with the remaining weight.
    """
    x = np.asarray(u, dtype=np.float64)
    res = 0.0 if u_prev is None else float(np.sum((x - np.asarray(u_prev, dtype=np.float64)) ** 2))
    S = support_sums(x.shape[0], x.shape[1], W)
    wsum = float(np.sum(np.asarray(W, dtype=np.float64)))
    nxt = float(np.sum((x - b) * S)) + b * x.size * wsum
    return np.array([res, float(np.sum(x * x)), float(np.sum(x)), nxt])


def rel_l2(x: np.ndarray, ref: np.ndarray) -> float:
    """||x - ref||_2 / ||ref||_2 in FP64 (absolute RMS when ||ref|| < 1e-30)."""
    a = np.asarray(x, dtype=np.float64)
    r = np.asarray(ref, dtype=np.float64)
    num = float(np.sqrt(np.sum((a - r) ** 2)))
    den = float(np.sqrt(np.sum(r * r)))
    if den < 1e-30:
        return num / np.sqrt(max(r.size, 1))
    return num / den
