"""Build the gfx950 library ``liblv.so`` in-tree.

HIP sources are compiled with hipcc for gfx950 (packed float32 instructions
disabled; the LVQ encoders without floating-point contraction so their
bytes are exact); the host float64 fitting code is compiled with g++ and OpenMP
(the same libgomp PyTorch uses).  Always rebuilds when called.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "liblv.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")

HIP_SOURCES = ["lv_api.cpp", "lv_batch.cpp", "lv_search.hip", "lv_graph.hip", "lv_lvq.hip",
               "lv_project.hip", "lv_gemm.hip", "lv_projloss.hip", "lv_noalloc.hip"]
HOST_SOURCES = ["lv_fit.cpp", "lv_error.cpp"]
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]
PER_FILE = {"lv_lvq.hip": ["-ffp-contract=off"], "lv_project.hip": ["-ffp-contract=off"]}


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return r.stdout


def build(verbose: bool = False, out: str = LIB, extra_flags=(), host_flags=(),
          host_cxx: str = "g++", openmp: bool = True) -> str:
    """Compile every source and link ``out`` (the package library by default).

    extra_flags go to every hipcc compile, host_flags to the compiles of the
    host-only sources, which use host_cxx (with OpenMP unless openmp=False:
    the float64 fit then runs on one thread)."""
    objdir = os.path.join(os.path.dirname(os.path.abspath(out)), "_build")
    os.makedirs(objdir, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    cmds = []
    for src in HIP_SOURCES:
        obj = os.path.join(objdir, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmds.append(([HIPCC] + HIP_FLAGS + list(extra_flags) + PER_FILE.get(src, []) + lang
                     + ["-c", os.path.join(CSRC, src), "-o", obj], obj))
    for src in HOST_SOURCES:
        obj = os.path.join(objdir, src + ".o")
        cmds.append(([host_cxx, "-O3", "-std=c++17", "-fPIC", "-march=x86-64-v3"]
                     + (["-fopenmp"] if openmp else ["-Wno-unknown-pragmas"])
                     + list(host_flags) + ["-c", os.path.join(CSRC, src), "-o", obj], obj))
    # independent translation units: compiled side by side
    with ThreadPoolExecutor(max(1, min(len(cmds), os.cpu_count() or 1, 8))) as pool:
        for msg in pool.map(lambda c: _run(c[0]), cmds):
            if verbose and msg.strip():
                print(msg)
    objs = [o for _, o in cmds]
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp%d" % os.getpid()
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
         + ["-lgomp", "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    os.replace(tmp, out)
    shutil.rmtree(objdir, ignore_errors=True)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
