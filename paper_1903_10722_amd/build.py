"""Build of the gfx950 shared library behind include/ffs.h and include/ffs_tt.h (hipcc, in-tree)."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(BUILD, "libffs.so")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


PROBE_LIB = os.path.join(BUILD, "liblds_probe.so")


def _run(cmd):
    return subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)


def build_library(verbose: bool = False) -> str:
    """Compile csrc/ffs_api.hip and csrc/ffs_tt.hip (+ headers) into
    _build/libffs.so, and csrc/lds_probe.hip (the benchmark's LDS bandwidth
    probe) into _build/liblds_probe.so; always recompiles.  The sources are
    compiled in parallel, then linked."""
    os.makedirs(BUILD, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs = []
    procs = []
    for src in ("ffs_api.hip", "ffs_tt.hip"):
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        objs.append(obj)
        procs.append(_run([hipcc, *HIPCC_FLAGS, "-c", *inc, os.path.join(CSRC, src), "-o", obj]))
    probe_tmp = PROBE_LIB + ".tmp"
    procs.append(_run([hipcc, *HIPCC_FLAGS, os.path.join(CSRC, "lds_probe.hip"), "-o", probe_tmp]))
    errs = []
    for p in procs:
        out, err = p.communicate()
        if p.returncode != 0:
            errs.append(err[-8000:])
        elif verbose and err:
            print(err[-2000:])
    if errs:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errs))
    tmp = LIB + ".tmp"
    res = subprocess.run([hipcc, *HIPCC_FLAGS, *objs, "-o", tmp], capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc link failed:\n" + res.stderr[-8000:])
    os.replace(tmp, LIB)
    os.replace(probe_tmp, PROBE_LIB)
    return LIB
