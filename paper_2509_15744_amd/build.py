"""Build ``libfdwave.so`` (the C-ABI library) in-tree with hipcc for gfx950.

Usage: ``python -m paper_2509_15744_amd.build`` (or ``build_library()``).
"""
from __future__ import annotations

import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libfdwave.so")
SOURCES = ["fdw_step.hip", "fdw_pair.hip", "fdw_batch.hip", "fdw_vd.hip", "fdw_design.hip", "fdw_kernels.hip", "fdw_host.cpp",
           "fdw_api.cpp", "fdw_tune.cpp", "fdw_batch_api.cpp", "fdw_design_api.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed-FP32 instructions stay off: scalar and float2 code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"),
]


def build_library(verbose: bool = True) -> str:
    """Compile every source to an object in ``_build/`` and link ``libfdwave.so``."""
    bdir = os.path.join(ROOT, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs = []
    t0 = time.time()
    procs = []
    for src in SOURCES:
        obj = os.path.join(bdir, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd = [HIPCC] + FLAGS + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = False
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if p.returncode != 0:
            failed = True
            sys.stderr.write(f"[build] {src} failed:\n" + "\n".join(lines) + "\n")
        elif verbose and lines:
            sys.stderr.write(f"[build] {src}:\n" + "\n".join(lines[:40]) + "\n")
    if failed:
        raise RuntimeError("hipcc failed")
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    if verbose:
        sys.stderr.write(f"[build] {os.path.relpath(LIB, ROOT)} in {time.time() - t0:.1f}s\n")
    return LIB


if __name__ == "__main__":
    build_library()
