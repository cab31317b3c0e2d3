"""Build the HIP library ``libmi355stencil.so`` in-tree for gfx950.

One shared object holds the C ABI declared in ``include/mi355stencil.h``.
Every translation unit is compiled by hipcc for gfx950 only, with packed-FP32
instruction selection disabled and FP contraction off (every FMA in the
kernels is an explicit fmaf, so the per-cell operation order is fixed).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmi355stencil.so")
OBJDIR = os.path.join(HERE, "_build")
SOURCES = ["march_f32_star.hip", "march_bf16_star.hip", "march_f16_star.hip", "march_f32_box.hip", "march_bf16_box.hip",
           "march_f16_box.hip", "march_xbc_f32_star.hip", "march_xbc_bf16_star.hip", "march_xbc_f16_star.hip",
           "march_xbc_f32_box.hip", "march_xbc_bf16_box.hip", "march_xbc_f16_box.hip", "surrogate.hip", "batched.hip",
           "sweep.hip", "api.hip", "march.hip", "varcoef.hip", "norms.hip", "stencil3d.hip", "resident.hip", "mfma_stencil.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-fno-gpu-flush-denormals-to-zero", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    if verbose and r.stderr.strip():
        # hipcc's host pass warns that it does not know the packed-fp32 feature: harmless
        lines = [l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l]
        if lines:
            sys.stderr.write("\n".join(lines) + "\n")
    return obj


def _stale(src: str, headers_mtime: float) -> bool:
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return t < os.path.getmtime(os.path.join(CSRC, src)) or t < headers_mtime


def build(verbose: bool = False, force: bool = True) -> str:
    """Compile every translation unit (force) or only those older than their source or any header,
    then link."""
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    hdrs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    hdrs.append(os.path.join(os.path.dirname(HERE), "include", "mi355stencil.h"))
    hmt = max(os.path.getmtime(h) for h in hdrs)
    todo = [s for s in srcs if force or _stale(s, hmt)]
    objs = [os.path.join(OBJDIR, os.path.splitext(s)[0] + ".o") for s in srcs]
    if todo:
        with cf.ThreadPoolExecutor(max_workers=min(8, len(todo))) as ex:
            list(ex.map(lambda s: _compile(s, verbose), todo))
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", OUT + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, force="--changed" not in sys.argv))
