"""Helpers for the GPU parity tests: move seeded host arrays to the device and run the library
through its C ABI.  Nothing here computes stencil values."""
from __future__ import annotations

import numpy as np
import torch

import paper_2605_07954_amd as lib

DEV = "cuda:0"


def to_dev(a: np.ndarray) -> torch.Tensor:
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint16:
        a = a.view(np.int16)
    return torch.from_numpy(a).to(DEV)


def to_host(t: torch.Tensor) -> np.ndarray:
    a = t.detach().cpu().numpy()
    if a.dtype == np.int16:
        a = a.view(np.uint16)
    return a


def empty_like_field(rows: int, cols: int, storage: str) -> torch.Tensor:
    dt = torch.float32 if storage == "f32" else torch.int16
    return torch.empty((rows, cols), dtype=dt, device=DEV)


def run(plan, u0_dev: torch.Tensor, steps: int, rows: int, cols: int, storage: str = "f32"):
    out = empty_like_field(rows, cols, storage)
    nws = lib.stencil_workspace_bytes(plan, steps)
    ws = torch.empty(max(nws, 1), dtype=torch.uint8, device=DEV) if nws else None
    lib.stencil_run(plan, u0_dev, out, steps, ws)
    return out


def run_problem(u0: np.ndarray, W: np.ndarray, b: float, steps: int, storage: str = "f32", flags: int = 0,
                tb: int = 0, tile=None):
    rows, cols = u0.shape
    r = (W.shape[0] - 1) // 2
    plan = lib.stencil_plan(rows, cols, r, W, b, storage, flags)
    try:
        if tb or tile:
            lib.stencil_set_blocking(plan, tb, *(tile or (0, 0)))
        out = run(plan, to_dev(u0), steps, rows, cols, storage)
        torch.cuda.synchronize()
        return to_host(out)
    finally:
        lib.stencil_destroy(plan)
