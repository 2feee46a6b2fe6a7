"""Build libtrajkrotov.so (HIP kernels + C ABI) for gfx950 with hipcc.

Usage: ``python -m paper_1801_04382_amd.build`` or ``build()``.  The library is
written in-tree to ``paper_1801_04382_amd/_lib/libtrajkrotov.so``.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIBDIR = os.path.join(PKG, "_lib")
LIBNAME = "libtrajkrotov.so"

SOURCES = ["tk_kernels.hip", "tk_grad.hip", "tk_batch.hip", "tk_host.cpp", "tk_batch_host.cpp"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    # packed FP32 VALU forms are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden",
]


def hipcc_path() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def lib_path() -> str:
    return os.path.join(LIBDIR, LIBNAME)


def build(verbose: bool = False, out: str = None, csrc: str = CSRC,
          defines=()) -> str:
    """Compile the sources in ``csrc`` into ``out`` (default: the in-tree library)."""
    out = out or lib_path()
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp"
    cmd = [hipcc_path(), *HIPCC_FLAGS, *[f"-D{d}" for d in defines], "-I", INCLUDE,
           "-I", csrc, *[os.path.join(csrc, s) for s in SOURCES], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{res.stdout}\n{res.stderr}")
    if verbose and res.stderr.strip():
        print(res.stderr, file=sys.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
