"""Build libtrajkrotov.so (HIP kernels + C ABI) for gfx950 with hipcc.

Usage: ``python -m paper_1801_04382_amd.build`` or ``build()``.  The library is
written in-tree to ``paper_1801_04382_amd/_lib/libtrajkrotov.so``.
"""

from __future__ import annotations

import hashlib
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

SOURCES = ["tk_kernels.hip", "tk_grad.hip", "tk_batch.hip", "tk_cross.hip", "tk_dense.hip",
           "tk_noalloc.hip", "tk_post.hip", "tk_rho.hip", "tk_host.cpp", "tk_batch_host.cpp"]

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


def source_hash(csrc: str = CSRC, defines=()) -> str:
    """Digest of everything the library is built from: the C/HIP sources and
    headers, the public header and the compiler flags.  It is compiled into the
    library (tk_build_id) so that the binding can refuse a stale build."""
    h = hashlib.sha256()
    files = sorted(f for f in os.listdir(csrc) if f.endswith((".hip", ".cpp", ".h")))
    for f in files:
        h.update(f.encode())
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(INCLUDE, "trajkrotov.h"), "rb") as fh:
        h.update(fh.read())
    h.update(" ".join([*HIPCC_FLAGS, *defines]).encode())
    return h.hexdigest()[:16]


def hipcc_path() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def lib_path() -> str:
    return os.path.join(LIBDIR, LIBNAME)


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{res.stdout}\n{res.stderr}")
    if verbose and res.stderr.strip():
        print(res.stderr, file=sys.stderr)


def build(verbose: bool = False, out: str = None, csrc: str = CSRC,
          defines=()) -> str:
    """Compile the sources in ``csrc`` into ``out`` (default: the in-tree library).

    Each source is compiled to an object file of its own (in parallel, under
    ``_build/`` beside the library), then the objects are linked.
    """
    from concurrent.futures import ThreadPoolExecutor

    out = out or lib_path()
    os.makedirs(os.path.dirname(out), exist_ok=True)
    objdir = os.path.join(os.path.dirname(out), "_build")
    os.makedirs(objdir, exist_ok=True)
    tag = os.path.splitext(os.path.basename(out))[0]
    flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    flags.append(f'-DTK_BUILD_ID="{source_hash(csrc, defines)}"')
    objs, cmds = [], []
    for s in SOURCES:
        o = os.path.join(objdir, f"{tag}.{s}.o")
        objs.append(o)
        cmds.append([hipcc_path(), *flags, *[f"-D{d}" for d in defines], "-I", INCLUDE,
                     "-I", csrc, "-c", os.path.join(csrc, s), "-o", o])
    jobs = min(len(cmds), max(1, min(os.cpu_count() or 1, 16)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    tmp = out + ".tmp"
    _run([hipcc_path(), *HIPCC_FLAGS, *objs, "-o", tmp], verbose)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
