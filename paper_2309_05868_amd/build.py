"""Compile the rcqr HIP library for gfx950 in-tree (paper_2309_05868_amd/librcqr.so).

Usage: python -m paper_2309_05868_amd.build [--verbose]
"""

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "librcqr.so")
SOURCES = ["sketch.hip", "smalldense.hip", "stream.hip", "stream128.hip", "rcqr.hip"]
ARCH = "gfx950"

# -ffp-contract=off: every FMA in the kernels is written explicitly, so the Gram pass and the
# final pass produce bitwise-identical Q0 rows.  Packed FP32 instructions are disabled.
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-I", INCLUDE,
]


def hipcc():
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the rcqr library needs the ROCm HIP compiler")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{err}")
    if verbose and err.strip():
        print(err)


def build(verbose=False):
    cc = hipcc()
    tmpdir = tempfile.mkdtemp(prefix="rcqr_build_")
    try:
        objs = []
        cmds = []
        for src in SOURCES:
            obj = os.path.join(tmpdir, src.replace(".hip", ".o"))
            objs.append(obj)
            cmds.append([cc, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
        with ThreadPoolExecutor(max_workers=min(4, len(cmds))) as ex:
            list(ex.map(lambda c: _run(c, verbose), cmds))
        tmp_lib = os.path.join(tmpdir, "librcqr.so")
        _run([cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp_lib], verbose)
        os.replace(tmp_lib, LIB) if os.path.dirname(tmp_lib) == PKG else shutil.move(tmp_lib, LIB)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose="--verbose" in sys.argv))
