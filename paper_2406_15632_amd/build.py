"""Build libqrt.so (HIP for gfx950) in-tree.

    python -m paper_2406_15632_amd.build

Steps: write the Sobol direction-number header from scipy (once; it only
depends on scipy's data), compile every source with hipcc in parallel, link
the shared library next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libqrt.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = ["qrt_api.hip", "qrt_transport.hip", "qrt_batch.hip", "qrt_points.hip", "qrt_mlp.hip", "qrt_sample.hip",
           "qrt_tables.cpp"]

COMMON = [
    "-O3", "-std=c++17", "-fPIC",
    f"--offload-arch={ARCH}",
    "-munsafe-fp-atomics",
    # multiply-adds are fused only where the source calls fma(): a packet then
    # gets the same FP32 arithmetic in every kernel that transports it (the
    # single-scene and the batched launch sequences)
    "-ffp-contract=off",
    # packed FP32 instructions stay off: they are generated only from plain float code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", BUILD,
]


def _sobol_header() -> str:
    out = os.path.join(BUILD, "qrt_sobol_table.h")
    if not os.path.exists(out):
        tmp = out + ".tmp"
        subprocess.run([sys.executable, os.path.join(CSRC, "gen_sobol_table.py"), tmp, "128"], check=True)
        os.replace(tmp, out)
    return out


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [HIPCC, *COMMON, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    _sobol_header()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
