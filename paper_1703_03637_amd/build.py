"""Build libhphi.so (gfx950) in-tree with hipcc.

Usage: python -m paper_1703_03637_amd.build  (or build() from Python).
Compiles every source under csrc/ for --offload-arch=gfx950 with packed
FP32 instructions disabled, and links one shared library next to this file.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libhphi.so")

SOURCES = ["kernels.hip", "api.cpp", "basis.cpp", "ham.cpp", "plan.cpp", "cma.cpp", "tune.cpp", "tridiag.cpp"]
ARCH = os.environ.get("HPHI_OFFLOAD_ARCH", "gfx950")

COMMON = [
    "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-result",
    f"--offload-arch={ARCH}",
    # packed FP32 (v_pk_*_f32) off: whole-library rule
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    hipcc = _hipcc()
    out_dir = tempfile.mkdtemp(prefix="hphi_build_")
    try:
        def compile_one(src):
            obj = os.path.join(out_dir, os.path.basename(src) + ".o")
            lang = ["-x", "hip"] if src.endswith(".hip") else []
            cmd = [hipcc] + COMMON + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError(f"compile failed: {src}\n{r.stdout}\n{r.stderr}")
            return obj, r.stderr

        with ThreadPoolExecutor(max_workers=min(len(SOURCES), 8)) as ex:
            results = list(ex.map(compile_one, SOURCES))
        for _, err in results:
            # hipcc's host pass warns that it does not know the packed-fp32 feature
            lines = [l for l in err.splitlines() if "packed-fp32-ops" not in l and l.strip()]
            if verbose and lines:
                print("\n".join(lines))
        tmp_lib = os.path.join(out_dir, "libhphi.so")
        cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp_lib] + [o for o, _ in results]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed\n{r.stdout}\n{r.stderr}")
        shutil.move(tmp_lib, LIB + ".tmp")
        os.replace(LIB + ".tmp", LIB)
    finally:
        shutil.rmtree(out_dir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
