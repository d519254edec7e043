"""Build of the gfx950 shared library ``liblbm.so`` (HIP, C ABI of include/lbm.h).

The library is built in-tree with hipcc; nothing is compiled at import time.
"""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "liblbm.so")
# (source, extra defines): the host side, and one translation unit per
# storage x collision instantiation of the step kernels
UNITS = [("lbm.hip", []), ("lbnet.hip", [])] + [
    ("lb_step.hip", [f"-DLB_S={st}", f"-DLB_C={co}"]) for st in range(3) for co in range(3)
]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed-FP32 instructions: only scalar/vector FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def build(verbose: bool = False, jobs: int | None = None, defines: tuple = (),
          out: str | None = None) -> str:
    """Compile every HIP translation unit and link ``liblbm.so`` (always recompiles).

    ``defines`` are extra ``-D`` options (the build-time kernel choices of
    lb_kernels.hpp); ``out`` an alternative library path.
    """
    jobs = jobs or min(len(UNITS), max(1, os.cpu_count() or 1))
    lib = out or LIB
    objdir = os.path.join(os.path.dirname(lib), "_build")
    os.makedirs(objdir, exist_ok=True)
    cmds, objs = [], []
    for src, defs in UNITS:
        stem = os.path.splitext(src)[0] + "".join(d.split("=")[1] for d in defs)
        obj = os.path.join(objdir, stem + ".o")
        objs.append(obj)
        cmds.append([HIPCC, *FLAGS, *defs, *defines, "-I", INCLUDE, "-I", CSRC, "-c",
                     os.path.join(CSRC, src), "-o", obj])
    running, failed = [], []
    pending = list(cmds)
    while pending or running:
        while pending and len(running) < jobs:
            cmd = pending.pop(0)
            if verbose:
                print(" ".join(cmd), flush=True)
            running.append((cmd, subprocess.Popen(cmd)))
        cmd, proc = running.pop(0)
        if proc.wait() != 0:
            failed.append(cmd)
    if failed:
        raise RuntimeError("HIP compilation failed: " + "; ".join(" ".join(c[-3:]) for c in failed))
    tmp = lib + ".tmp"
    link = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
