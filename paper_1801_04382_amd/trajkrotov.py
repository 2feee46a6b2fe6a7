"""Python binding of libtrajkrotov (ctypes; argument marshalling only).

The module-level functions carry the C names of ``include/trajkrotov.h`` and
take/return NumPy arrays; ``Context`` is a small convenience object over them.
Every computation runs in the HIP library: if the shared library is missing
the import of this module fails (build it with
``python -m paper_1801_04382_amd.build``).
"""

from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

from .build import lib_path, source_hash

# ---------------------------------------------------------------------------
# C types
# ---------------------------------------------------------------------------
TK_OK = 0
TK_EINVAL = -1
TK_EDIM = -2
TK_ENOMEM = -3
TK_EHIP = -4
TK_ENOTHERM = -5
TK_ERECCAP = -6
TK_ENUMERIC = -7
TK_ESTATE = -8
TK_ENODEV = -9
TK_EUNSUPPORTED = -10

TK_FP64 = 0
TK_FP32 = 1

TK_KERNEL_FORWARD = 0
TK_KERNEL_BACKWARD = 1
TK_KERNEL_KROTOV = 2
TK_KERNEL_GRAD = 3
TK_KERNEL_CROSS_GRAM = 4

TK_STEP_SPARSE = 0
TK_STEP_DENSE_MFMA = 1

STATUS_NAMES = {
    0: "TK_OK", -1: "TK_EINVAL", -2: "TK_EDIM", -3: "TK_ENOMEM", -4: "TK_EHIP",
    -5: "TK_ENOTHERM", -6: "TK_ERECCAP", -7: "TK_ENUMERIC", -8: "TK_ESTATE",
    -9: "TK_ENODEV", -10: "TK_EUNSUPPORTED",
}


class tk_csr(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("indptr", ctypes.POINTER(ctypes.c_int64)),
                ("indices", ctypes.POINTER(ctypes.c_int32)),
                ("values", ctypes.POINTER(ctypes.c_double))]


class tk_jump(ctypes.Structure):
    _fields_ = [("instance", ctypes.c_int32), ("traj", ctypes.c_int32),
                ("step", ctypes.c_int32), ("op", ctypes.c_int32),
                ("ordinal", ctypes.c_int32), ("direction", ctypes.c_int32),
                ("iteration", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("t", ctypes.c_double)]


class tk_kernel_timing(ctypes.Structure):
    _fields_ = [("ms_total", ctypes.c_double), ("launches", ctypes.c_int64),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double),
                ("traj_steps", ctypes.c_int64)]


class tk_batch_info(ctypes.Structure):
    _fields_ = [("n_instances", ctypes.c_int32), ("pass_waves_per_block", ctypes.c_int32),
                ("pass_blocks", ctypes.c_int32), ("krotov_waves_per_block", ctypes.c_int32),
                ("krotov_blocks", ctypes.c_int32), ("autotuned", ctypes.c_int32),
                ("last_iteration_ms", ctypes.c_double), ("tuned_pass_ms", ctypes.c_double),
                ("tuned_krotov_ms", ctypes.c_double),
                ("traj_steps_per_iteration", ctypes.c_int64),
                ("multiwave_instances", ctypes.c_int32),
                ("multiwave_krotov_blocks", ctypes.c_int32),
                ("tuned_multiwave_krotov_ms", ctypes.c_double)]


JUMP_DTYPE = np.dtype([("instance", np.int32), ("traj", np.int32), ("step", np.int32),
                       ("op", np.int32), ("ordinal", np.int32), ("direction", np.int32),
                       ("iteration", np.int32), ("reserved", np.int32), ("t", np.float64)])
assert JUMP_DTYPE.itemsize == ctypes.sizeof(tk_jump)

_P = ctypes.POINTER
_dp = _P(ctypes.c_double)
_ctx_p = ctypes.c_void_p

_SIGNATURES = {
    "tk_version": (ctypes.c_char_p, []),
    "tk_build_id": (ctypes.c_char_p, []),
    "tk_last_error": (ctypes.c_char_p, [_ctx_p]),
    "tk_create": (ctypes.c_int, [_P(_ctx_p), ctypes.c_int, ctypes.c_int]),
    "tk_destroy": (None, [_ctx_p]),
    "tk_set_system": (ctypes.c_int, [_ctx_p, ctypes.c_int64, _P(tk_csr), ctypes.c_int32,
                                     _P(tk_csr), ctypes.c_int32, _P(tk_csr)]),
    "tk_set_states": (ctypes.c_int, [_ctx_p, _dp, _dp]),
    "tk_set_pulses": (ctypes.c_int, [_ctx_p, ctypes.c_int32, ctypes.c_double, _dp, _dp, _dp]),
    "tk_get_pulses": (ctypes.c_int, [_ctx_p, _dp]),
    "tk_propagate_forward": (ctypes.c_int, [_ctx_p, ctypes.c_int32, ctypes.c_uint64,
                                            ctypes.c_uint64, _dp, _dp, _P(tk_jump),
                                            ctypes.c_int64, _P(ctypes.c_int64)]),
    "tk_propagate_backward": (ctypes.c_int, [_ctx_p, ctypes.c_int32, ctypes.c_uint64,
                                             ctypes.c_uint64, _dp, _P(tk_jump), ctypes.c_int64,
                                             _P(ctypes.c_int64)]),
    "tk_get_costate": (ctypes.c_int, [_ctx_p, ctypes.c_int32, _dp]),
    "tk_functional": (ctypes.c_int, [_ctx_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint64,
                                     _dp, _dp]),
    "tk_krotov_iterate": (ctypes.c_int, [_ctx_p, ctypes.c_int32, ctypes.c_uint64,
                                         ctypes.c_uint64, ctypes.c_int32, _dp, _P(tk_jump),
                                         ctypes.c_int64, _P(ctypes.c_int64)]),
    "tk_krotov_iterate_cross": (ctypes.c_int, [_ctx_p, ctypes.c_int32, ctypes.c_uint64,
                                               ctypes.c_uint64, ctypes.c_int32, _dp, _P(tk_jump),
                                               ctypes.c_int64, _P(ctypes.c_int64)]),
    "tk_grad_pathwise": (ctypes.c_int, [_ctx_p, ctypes.c_int32, _P(tk_jump), ctypes.c_int64,
                                        _dp, _dp, _dp]),
    "tk_set_pulses_dev": (ctypes.c_int, [_ctx_p, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "tk_get_pulses_dev": (ctypes.c_int, [_ctx_p, ctypes.c_void_p, ctypes.c_void_p]),
    "tk_functional_dev": (ctypes.c_int, [_ctx_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint64,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "tk_krotov_iterate_dev": (ctypes.c_int, [_ctx_p, ctypes.c_int32, ctypes.c_uint64,
                                             ctypes.c_uint64, ctypes.c_int32, ctypes.c_void_p,
                                             ctypes.c_void_p]),
    "tk_grad_pathwise_dev": (ctypes.c_int, [_ctx_p, ctypes.c_int32, _P(tk_jump), ctypes.c_int64,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p]),
    "tk_functional_dev_noalloc": (ctypes.c_int, [_ctx_p, ctypes.c_int32, ctypes.c_uint64,
                                                 ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_void_p]),
    "tk_pulse_noise": (ctypes.c_int, [_ctx_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                      _dp, _dp]),
    "tk_step_bench": (ctypes.c_int, [_ctx_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     _dp, _dp, ctypes.c_int32, _dp]),
    "tk_density_functional": (ctypes.c_int, [_ctx_p, _dp]),
    "tk_density_krotov_iterate": (ctypes.c_int, [_ctx_p, ctypes.c_int32, _dp]),
    "tk_batch_create": (ctypes.c_int, [_P(_ctx_p), ctypes.c_int, ctypes.c_int]),
    "tk_batch_destroy": (None, [_ctx_p]),
    "tk_batch_last_error": (ctypes.c_char_p, [_ctx_p]),
    "tk_batch_add": (ctypes.c_int, [_ctx_p, ctypes.c_uint32, ctypes.c_int64, _P(tk_csr),
                                    ctypes.c_int32, _P(tk_csr), ctypes.c_int32, _P(tk_csr),
                                    _dp, _dp, ctypes.c_int32, ctypes.c_double, _dp, _dp, _dp,
                                    ctypes.c_int32, ctypes.c_uint64, _P(ctypes.c_int32)]),
    "tk_batch_krotov_iterate": (ctypes.c_int, [_ctx_p, ctypes.c_uint64, ctypes.c_int32, _dp]),
    "tk_batch_get_pulses": (ctypes.c_int, [_ctx_p, ctypes.c_int32, _dp]),
    "tk_batch_get_info": (ctypes.c_int, [_ctx_p, _P(tk_batch_info)]),
    "tk_set_timing": (ctypes.c_int, [_ctx_p, ctypes.c_int]),
    "tk_get_timing": (ctypes.c_int, [_ctx_p, ctypes.c_int, _P(tk_kernel_timing)]),
    "tk_reset_timing": (ctypes.c_int, [_ctx_p]),
    "tk_get_launch_info": (ctypes.c_int, [_ctx_p, _P(ctypes.c_char_p), _P(ctypes.c_int32),
                                          _P(ctypes.c_int32), _P(ctypes.c_int32)]),
}

EXPORTED = tuple(_SIGNATURES)


def load_library(path: Optional[str] = None) -> ctypes.CDLL:
    """Load libtrajkrotov (``TRAJKROTOV_LIB`` may name another build of it).

    The in-tree library must have been built from the sources beside it: a
    library whose build id differs from the digest of the current sources is
    refused (rebuild with ``python -m paper_1801_04382_amd.build``).
    """
    explicit = path or os.environ.get("TRAJKROTOV_LIB")
    path = explicit or lib_path()
    if not os.path.exists(path):
        raise ImportError(f"libtrajkrotov not built ({path}); run "
                          "`python -m paper_1801_04382_amd.build`")
    # One HIP runtime per process: PyTorch ships its own copy of the runtime
    # (same soname, libamdhip64.so.7).  Loaded first, it is the one this
    # library binds to, so torch tensors and the library share a runtime; a
    # second copy loaded after this library would find the device taken.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if not explicit:
        built, want = lib.tk_build_id().decode(), source_hash()
        if built != want:
            raise ImportError(f"libtrajkrotov at {path} is stale (built from {built}, sources "
                              f"are {want}); run `python -m paper_1801_04382_amd.build`")
    return lib


_lib = load_library()


class TkError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _check(ctx, code: int) -> int:
    if code != TK_OK:
        msg = _lib.tk_last_error(ctx).decode() if ctx else ""
        raise TkError(code, msg)
    return code


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


def _cplx(v, n: Optional[int] = None) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(v, dtype=np.complex128))
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} complex entries, got {a.size}")
    return a.view(np.float64)


class _CsrHolder:
    """Keeps the arrays a tk_csr points at alive."""

    def __init__(self, m, d: int):
        import scipy.sparse as sp
        m = sp.csr_matrix(m, dtype=np.complex128)
        if m.shape != (d, d):
            raise ValueError(f"operator shape {m.shape} != ({d}, {d})")
        self.indptr = np.ascontiguousarray(m.indptr, dtype=np.int64)
        self.indices = np.ascontiguousarray(m.indices, dtype=np.int32)
        self.values = np.ascontiguousarray(m.data, dtype=np.complex128).view(np.float64)
        self.c = tk_csr(d, int(m.nnz), self.indptr.ctypes.data_as(_P(ctypes.c_int64)),
                        self.indices.ctypes.data_as(_P(ctypes.c_int32)),
                        self.values.ctypes.data_as(_dp))


def records_array(buf: np.ndarray, n: int) -> np.ndarray:
    """Jump records sorted by (iteration, direction, trajectory, ordinal)."""
    rec = buf[:n].copy()
    order = np.lexsort((rec["ordinal"], rec["traj"], rec["direction"], rec["iteration"]))
    return rec[order]


# ---------------------------------------------------------------------------
# thin wrappers with the C names
# ---------------------------------------------------------------------------

def tk_version() -> str:
    return _lib.tk_version().decode()


def tk_build_id() -> str:
    return _lib.tk_build_id().decode()


def tk_create(device: int = 0, precision: int = TK_FP64) -> int:
    h = _ctx_p()
    code = _lib.tk_create(ctypes.byref(h), device, precision)
    if code != TK_OK:
        raise TkError(code, "tk_create failed")
    return h.value


def tk_destroy(ctx: int) -> None:
    _lib.tk_destroy(ctx)


def tk_last_error(ctx: int) -> str:
    return _lib.tk_last_error(ctx).decode()


def tk_set_system(ctx: int, H0, H_ctrl: Sequence, L_jump: Sequence) -> None:
    d = H0.shape[0]
    h0 = _CsrHolder(H0, d)
    hc = [_CsrHolder(h, d) for h in H_ctrl]
    lj = [_CsrHolder(l, d) for l in L_jump]
    hc_arr = (tk_csr * max(len(hc), 1))(*[h.c for h in hc])
    lj_arr = (tk_csr * max(len(lj), 1))(*[h.c for h in lj])
    _check(ctx, _lib.tk_set_system(ctx, d, ctypes.byref(h0.c), len(hc), hc_arr, len(lj), lj_arr))


def tk_set_states(ctx: int, psi0, psi_tgt) -> None:
    p = _cplx(psi0)
    t = _cplx(psi_tgt, p.size // 2)
    _check(ctx, _lib.tk_set_states(ctx, _dptr(p), _dptr(t)))


def tk_set_pulses(ctx: int, u: np.ndarray, T: float, S=None, lam=None) -> None:
    u = np.ascontiguousarray(u, dtype=np.float64)
    nt = u.shape[1] if u.ndim == 2 else int(u.size)
    s = None if S is None else np.ascontiguousarray(S, dtype=np.float64).reshape(u.shape)
    l_ = None if lam is None else np.ascontiguousarray(lam, dtype=np.float64)
    _check(ctx, _lib.tk_set_pulses(ctx, nt, float(T), _dptr(u), _dptr(s), _dptr(l_)))


def tk_get_pulses(ctx: int, n_ctrl: int, nt: int) -> np.ndarray:
    out = np.zeros((n_ctrl, nt))
    _check(ctx, _lib.tk_get_pulses(ctx, _dptr(out)))
    return out


def _rec_buffer(cap: int):
    buf = np.zeros(max(cap, 1), dtype=JUMP_DTYPE)
    return buf, buf.ctypes.data_as(_P(tk_jump))


def tk_propagate_forward(ctx: int, M: int, seed: int, iteration: int, d: int,
                         want_states: bool = True, rec_cap: int = 0):
    psiT = np.zeros(M * d, dtype=np.complex128) if want_states else None
    tau = np.zeros(M, dtype=np.complex128)
    buf, bp = _rec_buffer(rec_cap)
    n = ctypes.c_int64(0)
    _check(ctx, _lib.tk_propagate_forward(
        ctx, M, seed, iteration, None if psiT is None else _dptr(psiT.view(np.float64)),
        _dptr(tau.view(np.float64)), bp if rec_cap > 0 else None, rec_cap, ctypes.byref(n)))
    return (None if psiT is None else psiT.reshape(M, d)), tau, records_array(buf, min(n.value, rec_cap)), n.value


def tk_propagate_backward(ctx: int, M: int, seed: int, iteration: int, tau=None,
                          rec_cap: int = 0):
    t = None if tau is None else _cplx(tau, M)
    buf, bp = _rec_buffer(rec_cap)
    n = ctypes.c_int64(0)
    _check(ctx, _lib.tk_propagate_backward(ctx, M, seed, iteration, _dptr(t),
                                           bp if rec_cap > 0 else None, rec_cap,
                                           ctypes.byref(n)))
    return records_array(buf, min(n.value, rec_cap)), n.value


def tk_get_costate(ctx: int, j: int, M: int, d: int) -> np.ndarray:
    out = np.zeros(M * d, dtype=np.complex128)
    _check(ctx, _lib.tk_get_costate(ctx, j, _dptr(out.view(np.float64))))
    return out.reshape(M, d)


def tk_functional(ctx: int, M: int, seed: int, iteration: int = 0):
    J = ctypes.c_double(0.0)
    tau = np.zeros(M, dtype=np.complex128)
    _check(ctx, _lib.tk_functional(ctx, M, seed, iteration, ctypes.byref(J),
                                   _dptr(tau.view(np.float64))))
    return J.value, tau


def tk_krotov_iterate(ctx: int, M: int, seed: int, n_iter: int, first_iteration: int = 0,
                      rec_cap: int = 0):
    nout = n_iter + 1 if first_iteration == 0 else n_iter
    J = np.zeros(max(nout, 1))
    buf, bp = _rec_buffer(rec_cap)
    n = ctypes.c_int64(0)
    _check(ctx, _lib.tk_krotov_iterate(ctx, M, seed, first_iteration, n_iter, _dptr(J),
                                       bp if rec_cap > 0 else None, rec_cap, ctypes.byref(n)))
    return J[:nout], records_array(buf, min(n.value, rec_cap)), n.value


def tk_krotov_iterate_cross(ctx: int, M: int, seed: int, n_iter: int, first_iteration: int = 0,
                            rec_cap: int = 0):
    nout = n_iter + 1 if first_iteration == 0 else n_iter
    J = np.zeros(max(nout, 1))
    buf, bp = _rec_buffer(rec_cap)
    n = ctypes.c_int64(0)
    _check(ctx, _lib.tk_krotov_iterate_cross(ctx, M, seed, first_iteration, n_iter, _dptr(J),
                                             bp if rec_cap > 0 else None, rec_cap,
                                             ctypes.byref(n)))
    return J[:nout], records_array(buf, min(n.value, rec_cap)), n.value


def tk_grad_pathwise(ctx: int, M: int, records: np.ndarray, n_ctrl: int, nt: int):
    """J_T, overlaps and dJ_T/du [n_ctrl, nt] of the replay with the records fixed."""
    rec = np.ascontiguousarray(records, dtype=JUMP_DTYPE)
    J = ctypes.c_double(0.0)
    tau = np.zeros(M, dtype=np.complex128)
    g = np.zeros(max(n_ctrl * nt, 1))
    _check(ctx, _lib.tk_grad_pathwise(ctx, M, rec.ctypes.data_as(_P(tk_jump)) if rec.size else None,
                                      rec.size, ctypes.byref(J), _dptr(tau.view(np.float64)),
                                      _dptr(g)))
    return J.value, tau, g[:n_ctrl * nt].reshape(n_ctrl, nt)


# device-pointer variants: array arguments are device addresses (ints, e.g.
# torch's tensor.data_ptr()), `stream` a HIP stream handle (int, 0 = the
# context's own stream)

def tk_set_pulses_dev(ctx: int, nt: int, T: float, u_ptr: int, S_ptr: int = 0,
                      lam_ptr: int = 0, stream: int = 0) -> None:
    _check(ctx, _lib.tk_set_pulses_dev(ctx, nt, float(T), u_ptr or None, S_ptr or None,
                                       lam_ptr or None, stream or None))


def tk_get_pulses_dev(ctx: int, u_ptr: int, stream: int = 0) -> None:
    _check(ctx, _lib.tk_get_pulses_dev(ctx, u_ptr, stream or None))


def tk_functional_dev(ctx: int, M: int, seed: int, iteration: int, J_ptr: int, tau_ptr: int = 0,
                      stream: int = 0) -> None:
    _check(ctx, _lib.tk_functional_dev(ctx, M, seed, iteration, J_ptr, tau_ptr or None,
                                       stream or None))


def tk_functional_dev_noalloc(ctx: int, M: int, seed: int, iteration: int, J_ptr: int,
                              tau_ptr: int = 0, stream: int = 0) -> None:
    _check(ctx, _lib.tk_functional_dev_noalloc(ctx, M, seed, iteration, J_ptr, tau_ptr or None,
                                               stream or None))


def tk_krotov_iterate_dev(ctx: int, M: int, seed: int, first_iteration: int, n_iter: int,
                          J_ptr: int, stream: int = 0) -> None:
    _check(ctx, _lib.tk_krotov_iterate_dev(ctx, M, seed, first_iteration, n_iter, J_ptr,
                                           stream or None))


def tk_grad_pathwise_dev(ctx: int, M: int, records: np.ndarray, J_ptr: int, tau_ptr: int,
                         g_ptr: int, stream: int = 0) -> None:
    rec = np.ascontiguousarray(records, dtype=JUMP_DTYPE)
    _check(ctx, _lib.tk_grad_pathwise_dev(ctx, M, rec.ctypes.data_as(_P(tk_jump)) if rec.size
                                          else None, rec.size, J_ptr, tau_ptr or None, g_ptr,
                                          stream or None))


def tk_pulse_noise(ctx: int, u: Optional[np.ndarray] = None, T: float = 0.0) -> np.ndarray:
    """nu_i of pulses u [n_ctrl, nt] on [0, T] (None: the context's current pulses)."""
    if u is None:
        nu = np.zeros(8)
        _check(ctx, _lib.tk_pulse_noise(ctx, 0, 0, 0.0, None, _dptr(nu)))
        return nu
    u = np.ascontiguousarray(np.atleast_2d(u), dtype=np.float64)
    nu = np.zeros(u.shape[0])
    _check(ctx, _lib.tk_pulse_noise(ctx, u.shape[0], u.shape[1], float(T), _dptr(u), _dptr(nu)))
    return nu


def tk_step_bench(ctx: int, method: int, x: np.ndarray, K: int, reps: int = 1):
    """One K-term step of the states x [M, d] by `method`; returns (y [M, d], ms per launch)."""
    xs = np.ascontiguousarray(x, dtype=np.complex128)
    M, d = xs.shape
    y = np.zeros_like(xs)
    ms = ctypes.c_double(0.0)
    _check(ctx, _lib.tk_step_bench(ctx, method, M, K, _dptr(xs.view(np.float64)),
                                   _dptr(y.view(np.float64)), reps, ctypes.byref(ms)))
    return y, ms.value


def tk_density_functional(ctx: int) -> float:
    J = ctypes.c_double(0.0)
    _check(ctx, _lib.tk_density_functional(ctx, ctypes.byref(J)))
    return J.value


def tk_density_krotov_iterate(ctx: int, n_iter: int) -> np.ndarray:
    J = np.zeros(n_iter + 1)
    _check(ctx, _lib.tk_density_krotov_iterate(ctx, n_iter, _dptr(J)))
    return J


def tk_set_timing(ctx: int, enable: bool) -> None:
    _check(ctx, _lib.tk_set_timing(ctx, 1 if enable else 0))


def tk_get_timing(ctx: int, kind: int) -> dict:
    t = tk_kernel_timing()
    _check(ctx, _lib.tk_get_timing(ctx, kind, ctypes.byref(t)))
    return {"ms_total": t.ms_total, "launches": t.launches, "flops": t.flops,
            "bytes": t.bytes, "traj_steps": t.traj_steps}


def tk_reset_timing(ctx: int) -> None:
    _check(ctx, _lib.tk_reset_timing(ctx))


def tk_get_launch_info(ctx: int) -> dict:
    name = ctypes.c_char_p()
    wpb, tw, nb = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(ctx, _lib.tk_get_launch_info(ctx, ctypes.byref(name), ctypes.byref(wpb),
                                        ctypes.byref(tw), ctypes.byref(nb)))
    return {"variant": name.value.decode() if name.value else "",
            "waves_per_block": wpb.value, "traj_per_wave": tw.value, "blocks": nb.value}


# ---------------------------------------------------------------------------
# convenience object
# ---------------------------------------------------------------------------

class Context:
    """One library context (device memory, stream, current system and pulses)."""

    def __init__(self, device: int = 0, precision: str = "fp64"):
        prec = {"fp64": TK_FP64, "fp32": TK_FP32}[precision]
        self.h = tk_create(device, prec)
        self.precision = precision
        self.d = 0
        self.n_ctrl = 0
        self.nt = 0

    def close(self):
        if self.h:
            tk_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_system(self, H0, H_ctrl, L_jump):
        tk_set_system(self.h, H0, H_ctrl, L_jump)
        self.d = H0.shape[0]
        self.n_ctrl = len(H_ctrl)

    def set_states(self, psi0, psi_tgt):
        tk_set_states(self.h, psi0, psi_tgt)

    def set_pulses(self, u, T, S=None, lam=None):
        u = np.asarray(u, dtype=np.float64).reshape(self.n_ctrl, -1) if self.n_ctrl else \
            np.zeros((0, int(np.asarray(u).shape[-1])))
        tk_set_pulses(self.h, u, T, S, lam)
        self.nt = u.shape[1]
        self.T, self.S, self.lam = float(T), S, lam

    def load(self, w):
        """Set system, states and pulses from a workloads.Workload."""
        self.set_system(w.H0, w.H_ctrl, w.L_jump)
        self.set_states(w.psi0, w.psi_tgt)
        self.set_pulses(w.u0, w.T, w.S, w.lam)

    def get_pulses(self) -> np.ndarray:
        return tk_get_pulses(self.h, self.n_ctrl, self.nt)

    def propagate_forward(self, M, seed, iteration=0, want_states=True, rec_cap=None):
        cap = 4 * M + 64 if rec_cap is None else rec_cap
        return tk_propagate_forward(self.h, M, seed, iteration, self.d, want_states, cap)

    def propagate_backward(self, M, seed, iteration, tau=None, rec_cap=None):
        cap = 4 * M + 64 if rec_cap is None else rec_cap
        return tk_propagate_backward(self.h, M, seed, iteration, tau, cap)

    def get_costate(self, j, M):
        return tk_get_costate(self.h, j, M, self.d)

    def functional(self, M, seed, iteration=0):
        return tk_functional(self.h, M, seed, iteration)

    def krotov_iterate(self, M, seed, n_iter, first_iteration=0, rec_cap=None):
        cap = (8 * M + 64) * (n_iter + 1) if rec_cap is None else rec_cap
        return tk_krotov_iterate(self.h, M, seed, n_iter, first_iteration, cap)

    def krotov_iterate_cross(self, M, seed, n_iter, first_iteration=0, rec_cap=None):
        cap = (8 * M + 64) * (n_iter + 1) if rec_cap is None else rec_cap
        return tk_krotov_iterate_cross(self.h, M, seed, n_iter, first_iteration, cap)

    def grad_pathwise(self, M, records):
        return tk_grad_pathwise(self.h, M, records, self.n_ctrl, self.nt)

    # device-pointer variants (addresses and stream handles as ints)
    def set_pulses_dev(self, nt, T, u_ptr, S_ptr=0, lam_ptr=0, stream=0):
        tk_set_pulses_dev(self.h, nt, T, u_ptr, S_ptr, lam_ptr, stream)
        self.nt = nt
        self.T = float(T)

    def get_pulses_dev(self, u_ptr, stream=0):
        tk_get_pulses_dev(self.h, u_ptr, stream)

    def functional_dev(self, M, seed, iteration, J_ptr, tau_ptr=0, stream=0):
        tk_functional_dev(self.h, M, seed, iteration, J_ptr, tau_ptr, stream)

    def krotov_iterate_dev(self, M, seed, n_iter, J_ptr, first_iteration=0, stream=0):
        tk_krotov_iterate_dev(self.h, M, seed, first_iteration, n_iter, J_ptr, stream)

    def grad_pathwise_dev(self, M, records, J_ptr, tau_ptr, g_ptr, stream=0):
        tk_grad_pathwise_dev(self.h, M, records, J_ptr, tau_ptr, g_ptr, stream)

    def pulse_noise(self, u=None, T=None):
        """Noise measure nu_i (Sec. 3.4) of u [n_ctrl, nt], or of the current pulses."""
        if u is None:
            return tk_pulse_noise(self.h)[:self.n_ctrl]
        return tk_pulse_noise(self.h, u, self.T if T is None else T)

    def step_bench(self, method, x, K, reps=1):
        return tk_step_bench(self.h, method, x, K, reps)

    def density_functional(self):
        return tk_density_functional(self.h)

    def density_krotov_iterate(self, n_iter):
        return tk_density_krotov_iterate(self.h, n_iter)

    def set_timing(self, enable=True):
        tk_set_timing(self.h, enable)

    def timing(self, kind):
        return tk_get_timing(self.h, kind)

    def reset_timing(self):
        tk_reset_timing(self.h)

    def launch_info(self):
        return tk_get_launch_info(self.h)


# ---------------------------------------------------------------------------
# batched form
# ---------------------------------------------------------------------------

def _bcheck(b, code: int) -> int:
    if code != TK_OK:
        msg = _lib.tk_batch_last_error(b).decode() if b else ""
        raise TkError(code, msg)
    return code


def tk_batch_create(device: int = 0, precision: int = TK_FP32) -> int:
    h = _ctx_p()
    code = _lib.tk_batch_create(ctypes.byref(h), device, precision)
    if code != TK_OK:
        raise TkError(code, "tk_batch_create failed")
    return h.value


def tk_batch_destroy(b: int) -> None:
    _lib.tk_batch_destroy(b)


def tk_batch_add(b: int, instance_id: int, H0, H_ctrl, L_jump, psi0, psi_tgt, u, T, S, lam,
                 M: int, seed: int) -> int:
    d = H0.shape[0]
    h0 = _CsrHolder(H0, d)
    hc = [_CsrHolder(h, d) for h in H_ctrl]
    lj = [_CsrHolder(l, d) for l in L_jump]
    hc_arr = (tk_csr * max(len(hc), 1))(*[h.c for h in hc])
    lj_arr = (tk_csr * max(len(lj), 1))(*[h.c for h in lj])
    p = _cplx(psi0, d)
    t = _cplx(psi_tgt, d)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(len(hc), -1)
    s = None if S is None else np.ascontiguousarray(S, dtype=np.float64).reshape(u.shape)
    l_ = None if lam is None else np.ascontiguousarray(lam, dtype=np.float64)
    idx = ctypes.c_int32(-1)
    _bcheck(b, _lib.tk_batch_add(b, instance_id, d, ctypes.byref(h0.c), len(hc), hc_arr, len(lj),
                                 lj_arr, _dptr(p), _dptr(t), u.shape[1], float(T), _dptr(u),
                                 _dptr(s), _dptr(l_), M, seed, ctypes.byref(idx)))
    return idx.value


def tk_batch_krotov_iterate(b: int, n_inst: int, n_iter: int, first_iteration: int = 0):
    n_out = n_iter + (1 if first_iteration == 0 else 0)
    J = np.zeros((n_inst, max(n_out, 1)))
    _bcheck(b, _lib.tk_batch_krotov_iterate(b, first_iteration, n_iter, _dptr(J)))
    return J[:, :n_out]


def tk_batch_get_pulses(b: int, index: int, n_ctrl: int, nt: int) -> np.ndarray:
    out = np.zeros((n_ctrl, nt))
    _bcheck(b, _lib.tk_batch_get_pulses(b, index, _dptr(out)))
    return out


def tk_batch_get_info(b: int) -> dict:
    info = tk_batch_info()
    _bcheck(b, _lib.tk_batch_get_info(b, ctypes.byref(info)))
    return {name: getattr(info, name) for name, _ in tk_batch_info._fields_}


class Batch:
    """A batch of independent optimisation instances advanced together."""

    def __init__(self, device: int = 0, precision: str = "fp32"):
        self.h = tk_batch_create(device, {"fp64": TK_FP64, "fp32": TK_FP32}[precision])
        self.shapes: List[Tuple[int, int]] = []

    def close(self):
        if self.h:
            tk_batch_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, w, instance_id: Optional[int] = None) -> int:
        """Add a workloads.Workload (its instance field is the default id)."""
        iid = w.instance if instance_id is None else instance_id
        idx = tk_batch_add(self.h, iid, w.H0, w.H_ctrl, w.L_jump, w.psi0, w.psi_tgt, w.u0, w.T,
                           w.S, w.lam, w.M, w.seed)
        self.shapes.append((len(w.H_ctrl), w.nt))
        return idx

    def krotov_iterate(self, n_iter: int, first_iteration: int = 0) -> np.ndarray:
        return tk_batch_krotov_iterate(self.h, len(self.shapes), n_iter, first_iteration)

    def get_pulses(self, index: int) -> np.ndarray:
        n_ctrl, nt = self.shapes[index]
        return tk_batch_get_pulses(self.h, index, n_ctrl, nt)

    def info(self) -> dict:
        return tk_batch_get_info(self.h)
