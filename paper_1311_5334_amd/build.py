"""Build the gfx950 shared library ``libemt.so`` in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libemt.so")
OBJDIR = os.path.join(HERE, "_build")

SOURCES = ["kernels.hip", "api.hip", "serve.hip", "peaks.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
         # no packed FP32 instructions anywhere in device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wshadow", "-I" + INCLUDE, "-I" + CSRC]


def _compile(src: str, objdir: str, defines: tuple) -> str:
    obj = os.path.join(objdir, src + ".o")
    cmd = [HIPCC, *FLAGS, *[f"-D{k}={v}" for k, v in defines], "-c",
           os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(verbose: bool = False, lib: str = LIB, defines: dict | None = None,
          objdir: str = OBJDIR) -> str:
    """Compile every source for gfx950 and link the library (always
    rebuilds). defines: tuning macros (-D) overriding the values the sources
    take from csrc/tile_table.h; the autotuner builds such variants into
    directories of their own."""
    os.makedirs(objdir, exist_ok=True)
    dfs = tuple(sorted((defines or {}).items()))
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda src: _compile(src, objdir, dfs), SOURCES))
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "-pthread", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"link of {lib} failed")
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
