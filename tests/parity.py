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


# relative error the library accepts per FP64 Taylor step (its order table)
STEP_TOL_FP64 = 1e-15


def slow_crossing_allowance(ref_rates, ref_recs, nt, step_tol=STEP_TOL_FP64):
    """Per-record allowance added to a jump-time bar where the norm falls slowly.

    The library's step propagator is a polynomial whose remainder it keeps
    below step_tol per step; the oracle's is the exact exponential.  After n
    steps of a pass the two states differ by up to about n step_tol
    (relative), and a crossing where the norm falls at relative rate
    rate = sum_l ||L_l psi||^2 / ||psi||^2 moves by that over the rate.  The
    allowance is 4 n step_tol / rate (a factor 2 for the pulses, which carry
    the same error from earlier passes, and 2 of margin); n counts the steps
    from the start of the record's pass (forward: step + 1; backward:
    nt - step)."""
    out = []
    for r, rate in zip(ref_recs, ref_rates):
        n = r[4] + 1 if r[1] == 0 else nt - r[4]
        out.append(4.0 * n * step_tol / rate if rate > 0 else float("inf"))
    return out


def compare_records(gpu, ref, t_tol, allowance=None):
    """Discrete fields identical; jump times within t_tol (plus the per-record
    allowance, if given).  Returns max |dt|."""
    assert len(gpu) == len(ref), (len(gpu), len(ref), gpu[:5], ref[:5])
    worst = 0.0
    for q, (g, o) in enumerate(zip(gpu, ref)):
        assert g[:6] == o[:6], (g, o)
        dt = abs(g[6] - o[6])
        bar = t_tol + (allowance[q] if allowance is not None else 0.0)
        assert dt <= bar, (g, o, dt, bar)
        worst = max(worst, dt)
    return worst


def max_abs(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)))) if np.size(a) else 0.0
