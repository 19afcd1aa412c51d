"""Build the HIP shared library ``libh2mul.so`` for gfx950 in-tree.

Usage: ``python -m paper_2403_01566_amd.build`` (or ``build()`` from Python).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libh2mul.so")

SOURCES = ["h2_kernels.hip", "h2_scratch.hip", "h2_setup.cpp", "h2_plan.cpp", "h2_capi.cpp", "h2_selftest.cpp"]
ARCH = os.environ.get("H2_OFFLOAD_ARCH", "gfx950")


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, jobs: int = 4) -> str:
    hipcc = _hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    common = ["-O3", "-fPIC", "-std=c++17", "-fopenmp", "-Wno-unused-result"]
    device = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        objs.append(obj)
        cmd = [hipcc] + common + device + ["-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd = [hipcc] + common + ["-D__HIP_PLATFORM_AMD__", "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs, verbose)
            procs = []
    _wait(procs, verbose)
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-shared", "-fopenmp", f"--offload-arch={ARCH}", "-o", tmp] + objs
    _run(cmd, verbose)
    os.replace(tmp, LIB)
    return LIB


def _wait(procs, verbose):
    for cmd, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        text = "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            raise RuntimeError("build failed: " + " ".join(cmd) + "\n" + text)
        if verbose and text.strip():
            print(text)


def _run(cmd, verbose):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("link failed: " + " ".join(cmd) + "\n" + r.stdout.decode(errors="replace"))


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
