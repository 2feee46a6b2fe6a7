"""Helpers shared by the GPU parity tests (comparison only; no method arithmetic)."""

from __future__ import annotations

import sys

import numpy as np

from oracle import krotov as okrotov
from oracle.mcwf import System


def say(*msg):
    print("[parity]", *msg, flush=True)
    sys.stdout.flush()


def oracle_system(w) -> System:
    return System.from_sparse(w.H0, w.H_ctrl, w.L_jump)


def oracle_records(recs, iteration):
    """Oracle Jump list -> sorted tuples (iteration, direction, traj, ordinal, step, op, t)."""
    out = [(iteration, r.direction, r.traj, r.ordinal, r.step, r.op, r.t) for r in recs]
    return sorted(out)


def gpu_records(arr, iteration=None, direction=None):
    out = []
    for r in arr:
        if iteration is not None and r["iteration"] != iteration:
            continue
        if direction is not None and r["direction"] != direction:
            continue
        out.append((int(r["iteration"]), int(r["direction"]), int(r["traj"]),
                    int(r["ordinal"]), int(r["step"]), int(r["op"]), float(r["t"])))
    return sorted(out)


def compare_records(gpu, ref, t_tol):
    """Discrete fields identical; jump times within t_tol.  Returns max |dt|."""
    assert len(gpu) == len(ref), (len(gpu), len(ref), gpu[:5], ref[:5])
    worst = 0.0
    for g, o in zip(gpu, ref):
        assert g[:6] == o[:6], (g, o)
        worst = max(worst, abs(g[6] - o[6]))
    assert worst <= t_tol, worst
    return worst


def max_abs(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)))) if np.size(a) else 0.0
