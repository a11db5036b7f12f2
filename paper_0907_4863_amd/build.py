"""Compile the HIP sources into the in-tree shared library ``libsaamg.so`` (gfx950)."""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsaamg.so")
SOURCES = ["fine.hip", "wide.hip", "coarse.hip", "solver.hip", "pic.hip", "timer.hip", "domain.cpp",
           "host_prep.cpp"]
# hbm_ceiling.hip is a separate program (see _build_ceiling), not part of the library
ARCH = os.environ.get("SAAMG_ARCH", "gfx950")

# Packed fp32 instructions are disabled for all device code.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
          "-Wno-unused-variable", "-Wno-unused-lambda-capture"]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found; the HIP library cannot be built")


def _compile(src: str, obj_dir: str, verbose: bool) -> str:
    obj = os.path.join(obj_dir, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), f"--offload-arch={ARCH}", *COMMON, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".hip"):
        cmd[1:1] = ["-x", "hip"]
        cmd += DEVICE_FLAGS
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{res.stdout}\n{res.stderr}")
    if verbose and res.stderr.strip():
        print(res.stderr, file=sys.stderr)
    return obj


def build(verbose: bool = False) -> str:
    """Compile every source for gfx950 and link ``libsaamg.so`` next to this file."""
    obj_dir = os.path.join(HERE, "_build")
    os.makedirs(obj_dir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(4, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, obj_dir, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"linking libsaamg.so failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    _build_ceiling(verbose)
    return LIB


CEILING = os.path.join(HERE, "hbm_ceiling")


def _build_ceiling(verbose: bool) -> None:
    """The standalone HBM streaming-ceiling program the benchmark runs."""
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-O3", "-x", "hip", *DEVICE_FLAGS,
           os.path.join(CSRC, "hbm_ceiling.hip"), "-o", CEILING]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compiling hbm_ceiling.hip failed:\n{res.stdout}\n{res.stderr}")


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
