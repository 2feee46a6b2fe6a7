"""The C-ABI library loads, exports every declared symbol, and its structs match
the header (checked by compiling the header with gcc).  No GPU compute."""

import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "trajkrotov.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tk_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ["tk_create", "tk_destroy", "tk_set_system", "tk_set_states",
                     "tk_set_pulses", "tk_get_pulses", "tk_propagate_forward",
                     "tk_propagate_backward", "tk_functional", "tk_krotov_iterate",
                     "tk_get_costate", "tk_last_error"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1801_04382_amd import trajkrotov as tk
    lib = ctypes.CDLL(tk.lib_path())
    for name in _declared_functions():
        assert hasattr(lib, name), name
    assert set(_declared_functions()) == set(tk.EXPORTED)
    assert tk.tk_version().startswith("trajkrotov")
    out = subprocess.run(["nm", "-D", "--defined-only", tk.lib_path()], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r" T (tk_\w+)", out))
    assert exported == set(_declared_functions())


def test_struct_layout_matches_header():
    from paper_1801_04382_amd import trajkrotov as tk
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "trajkrotov.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\n", sizeof(tk_jump), offsetof(tk_jump, t), sizeof(tk_csr),
         sizeof(tk_kernel_timing), offsetof(tk_kernel_timing, traj_steps));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as tmp:
        c = os.path.join(tmp, "probe.c")
        exe = os.path.join(tmp, "probe")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), c, "-o", exe],
                       check=True)
        vals = [int(x) for x in subprocess.run([exe], capture_output=True, text=True,
                                                check=True).stdout.split()]
    assert vals == [ctypes.sizeof(tk.tk_jump), tk.tk_jump.t.offset, ctypes.sizeof(tk.tk_csr),
                    ctypes.sizeof(tk.tk_kernel_timing), tk.tk_kernel_timing.traj_steps.offset]
    assert tk.JUMP_DTYPE.itemsize == vals[0]


def test_create_reports_missing_device_or_succeeds_on_gfx950():
    from paper_1801_04382_amd import trajkrotov as tk
    h = ctypes.c_void_p()
    code = tk._lib.tk_create(ctypes.byref(h), 0, tk.TK_FP64)
    if code == tk.TK_OK:
        tk._lib.tk_destroy(h)
    else:
        assert code == tk.TK_ENODEV and not h.value
    assert tk._lib.tk_create(ctypes.byref(h), 0, 7) == tk.TK_EINVAL
    assert tk._lib.tk_last_error(None) == b"no context"


def test_library_is_built_from_the_sources_beside_it():
    """The binding refuses a library built from other sources (a stale build)."""
    from paper_1801_04382_amd import build
    from paper_1801_04382_amd import trajkrotov as tk
    assert tk.tk_build_id() == build.source_hash()
    assert build.source_hash(defines=("TK_SOMETHING",)) != build.source_hash()
