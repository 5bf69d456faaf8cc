"""Build libqx.so for gfx950 in-tree with hipcc.

    python -m paper_1612_02750_amd.build        # or build() from Python

Every source is compiled for gfx950 only, with packed-FP32 instruction
selection disabled, then linked into paper_1612_02750_amd/libqx.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libqx.so")
# (source, object name, extra flags): the engine's instantiation unit is
# compiled once per (inner precision, link storage) pair, in parallel (the
# binary16 inner links under FP32 vectors are three more pairs)
UNITS = [("qx_engine_inst.hip", f"qx_engine_{r}_{n}", [f"-DQX_R={r}", f"-DQX_RECON={n}"])
         for r in ("float", "double") for n in (18, 12, 36)] + [
    ("qx_engine_inst.hip", f"qx_engine_float_{n}_links16", ["-DQX_R=float", f"-DQX_RECON={n}", "-DQX_LINKS16"])
    for n in (18, 12, 36)] + [
    ("qx_engine.hip", "qx_engine", []),
    ("qx_dslash.hip", "qx_dslash", []),
    ("qx_kernels.hip", "qx_kernels", []),
    ("qx_hmc.hip", "qx_hmc", []),
    ("qx_api.cpp", "qx_api", []),
]
ARCH = "gfx950"


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm is required to build libqx.so)")


def _flags():
    return [
        "-O3",
        "-std=c++20",
        f"--offload-arch={ARCH}",
        "-fPIC",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        # products and sums round as written (fused only where fma() is
        # called), so every kernel that evaluates an expression rounds it
        # alike, whatever its surrounding code lets the compiler fuse
        "-ffp-contract=off",
        "-Wno-unused-command-line-argument",
        "-I", os.path.join(ROOT, "include"),
        "-I", CSRC,
    ]


def _compile(unit) -> str:
    src, name, extra = unit
    obj = os.path.join(BUILD, name + ".o")
    cmd = [hipcc(), "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + _flags() + extra
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    """Compile every HIP source and link libqx.so (always rebuilds)."""
    os.makedirs(BUILD, exist_ok=True)
    workers = min(len(UNITS), os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(_compile, UNITS))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
