"""Build step of libmtpt.so: hipcc for gfx950, in-tree.

The library is the C-ABI declared in include/mtpt.h; its sources are the HIP
files under csrc/.  Each translation unit is compiled to an object file in
parallel (the tiled passes are split per dimension and metric), then the
objects are linked into one shared library.  Packed FP32 instructions are
disabled for all device code.
"""
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = [os.path.join(CSRC, f) for f in (
    "mtpt_kernels.hip", "mtpt_runtime.hip",
    "mtpt_tiles_2d_iso.hip", "mtpt_tiles_2d_tens.hip", "mtpt_tiles_3d_iso.hip", "mtpt_tiles_3d_tens.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("mtpt_kernels.h", "mtpt_rng.h", "mtpt_device.h")] + \
    [os.path.join(ROOT, "include", "mtpt.h")]
LIB = os.path.join(HERE, "libmtpt.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include")]


def build(verbose: bool = False, out: str = None, defines=()) -> str:
    """Compile libmtpt.so (next to this file unless ``out`` is given; extra
    ``-D`` tuning defines in ``defines``); returns its path."""
    lib = out or LIB
    tmp = lib + ".tmp"
    dflags = [f"-D{d}" for d in defines]
    with tempfile.TemporaryDirectory(prefix="mtpt_build_") as td:
        objs, procs = [], []
        for src in SOURCES:
            obj = os.path.join(td, os.path.basename(src) + ".o")
            cmd = [HIPCC, *FLAGS, *dflags, "-c", src, "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((cmd, subprocess.Popen(cmd)))
            objs.append(obj)
        failed = [cmd for cmd, p in procs if p.wait() != 0]
        if failed:
            raise subprocess.CalledProcessError(1, failed[0])
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(f) > t for f in SOURCES + HEADERS)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
