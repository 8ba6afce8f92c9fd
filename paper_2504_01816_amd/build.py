"""Build the gfx950 shared library librpa_gfx950.so in-tree with hipcc.

Every HIP source is compiled for gfx950 only, with packed-FP32 instruction selection
disabled, then linked into one shared library next to this file.  The library exports
the C ABI declared in include/rpa.h.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librpa_gfx950.so")
SOURCES = ["api.hip", "cocg.hip", "cocg_f64.hip", "cocg_mixed.hip", "gemm.hip", "small.hip",
           "pcocg.hip", "noalloc.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-Wno-unused-result"]


def _run(cmd):
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("command failed: %s\n%s%s" % (" ".join(cmd), p.stdout, p.stderr))
    return p


def build(verbose=False, out=None, extra_flags=()):
    objdir = os.path.join(HERE, "_build" if out is None else "_build_alt")
    os.makedirs(objdir, exist_ok=True)
    objs = []

    def compile_one(src):
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        _run([HIPCC, *FLAGS, *extra_flags, "-c", os.path.join(CSRC, src), "-o", obj])
        if verbose:
            print("compiled", src, flush=True)
        return obj

    with ThreadPoolExecutor(max_workers=min(6, len(SOURCES))) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    target = out or LIB
    tmp = target + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, target)
    if verbose:
        print("built", target, flush=True)
    return target


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
