"""Build libmsmg.so (HIP, gfx950) in-tree.

Every source is compiled by hipcc for gfx950 with packed-FP32 instructions
disabled, objects go to ``_build/`` and the shared library next to this file.
Run ``python -m paper_2410_06850_amd.build_lib`` or call ``build()``.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmsmg.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

SOURCES = [
    "fine_kernels.hip",
    "coarse_kernels.hip",
    "setup_local.hip",
    "setup_coarse.hip",
    "setup_driver.hip",
    "topopt_kernels.hip",
    "tpfa_kernels.hip",
    "runtime.cpp",
]

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("MSMG_OFFLOAD_ARCH", "gfx950")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
    "-Wno-unused-result", "-Wno-pass-failed",
]


def _compile(src, build_dir=BUILD, defines=()):
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *COMMON, *[f"-D{d}" for d in defines], "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-8000:]}")
    return obj


def build(jobs=None, verbose=False, defines=(), lib_path=LIB, build_dir=BUILD):
    """Compile every source and link the library (``libmsmg.so`` next to this
    file unless ``lib_path`` says otherwise); returns the library path.
    ``defines`` are extra preprocessor definitions (NAME or NAME=VALUE), e.g.
    the march prefetch depths MSMG_MARCH_DEPTH8 / MSMG_MARCH_DEPTH4."""
    os.makedirs(build_dir, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4, 8)
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, build_dir, defines), SOURCES))
    tmp = lib_path + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-8000:]}")
    os.replace(tmp, lib_path)
    if verbose:
        print("built", lib_path)
    return lib_path


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
