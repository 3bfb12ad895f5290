"""Build the native library ``_lib/libdecbpm.so`` in-tree for gfx950.

HIP sources are compiled with ``hipcc --offload-arch=gfx950`` to objects; the
host-only assembly is compiled with g++; the shared object is linked against
the HIP runtime that ships with PyTorch, so a process that imports torch and
then loads the library holds a single HIP runtime (streams and device pointers
are shared with torch).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIBDIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIBDIR, "libdecbpm.so")

HIP_SOURCES = ["kernels.hip", "dec_bpm.hip"]
CXX_SOURCES = ["assembly.cpp"]
HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed FP32 instructions stay disabled
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _torch_libdir() -> str:
    import importlib.util

    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.submodule_search_locations:
        raise RuntimeError("torch is required to locate the HIP runtime")
    return os.path.join(list(spec.submodule_search_locations)[0], "lib")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{out}")
    if verbose and out:
        print(out)
    return out


def build(verbose: bool = False) -> str:
    """Compile every source and link the library; returns its path."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    inc = ["-I" + os.path.join(ROOT, "include")]
    jobs = []
    objs = []
    for src in HIP_SOURCES:
        # the kernels compile as two objects in parallel: complex64 (with the
        # precision-independent launchers) and complex128
        parts = [("_f", ["-DDECBPM_PART=1"]), ("_d", ["-DDECBPM_PART=2"])] if src == "kernels.hip" else [("", [])]
        for suffix, defs in parts:
            obj = os.path.join(BUILD, src.replace(".hip", suffix + ".o"))
            jobs.append([hipcc, *HIPCC_FLAGS, *defs, *inc, "-c", os.path.join(CSRC, src), "-o", obj])
            objs.append(obj)
    for src in CXX_SOURCES:
        obj = os.path.join(BUILD, src.replace(".cpp", ".o"))
        jobs.append(["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", *inc, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    with ThreadPoolExecutor(max_workers=min(4, len(jobs))) as ex:
        list(ex.map(lambda c: _run(c, verbose), jobs))
    tlib = _torch_libdir()
    tmp = LIB + ".tmp"
    _run(["g++", "-shared", *objs, os.path.join(tlib, "libamdhip64.so"), f"-Wl,-rpath,{tlib}", "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
