"""Build the gfx950 shared library ``libmln.so`` in-tree with hipcc.

Run ``python -m paper_1710_09799_amd.build``.  Cross-compiles on a machine
without a GPU.  All HIP code is built with packed-FP32 instructions disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libmln.so")
OBJDIR = os.path.join(PKG, "_build")

HIP_SOURCES = ["mln_abi.hip", "batch.hip", "fwd_dispatch.hip", "adj_n23.hip", "mfmaq_n46.hip", "pade_n46.hip", "floor.hip", "pstd.hip", "tmz.hip", "stream.hip", "pol2.hip"] + ["fwd_n%d.hip" % n for n in (2, 3, 4, 6)]
CXX_SOURCES = ["setup.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I" + os.path.join(ROOT, "include")]
HIP_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-munsafe-fp-atomics"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build failed: " + " ".join(cmd[:3]) + " ...")
    return r


def build(verbose=False, jobs=8):
    os.makedirs(OBJDIR, exist_ok=True)
    procs = []
    objs = []
    t0 = time.time()
    for src in HIP_SOURCES + CXX_SOURCES:
        obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        cmd = [HIPCC] + COMMON + (HIP_FLAGS if src.endswith(".hip") else ["-x", "c++"]) + \
            ["-c", os.path.join(CSRC, src), "-o", obj]
        if not src.endswith(".hip"):
            cmd = [HIPCC] + COMMON + ["-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                            text=True)))
    failed = False
    for cmd, p in procs:
        out, err = p.communicate()
        if p.returncode != 0:
            failed = True
            sys.stderr.write(out + err)
        elif verbose and err.strip():
            sys.stderr.write(err)
    if failed:
        raise RuntimeError("compilation failed")
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f}s")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
