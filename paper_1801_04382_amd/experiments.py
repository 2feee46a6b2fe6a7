"""The paper's own network model optimised on the GPU (Sec. 3.2-3.4).

The paper optimises the state-preparation pulses of its effective cascade
network (single-excitation space, d = 2N + 1, Delta = 100 g, kappa = g,
L = sqrt(2 kappa) sum_i a_i; target the symmetric dark state) three ways --
the density-matrix update, independent trajectories and cross-trajectory
trajectories -- and compares how the trajectory count M affects convergence
(Sec. 3.3, measured as the density-matrix error of the optimised pulses) and
the noise of the pulses (Sec. 3.4, nu_i against M).  These runners do that
with the library: every pass, update, functional and noise value comes from
its HIP kernels; this module only sequences the calls.

Choices the paper leaves open (its figure data are not available): a
Blackman guess of peak Omega / 2 Delta = 0.5 for every node, nt = 100 T steps,
S = 1, and lambda_i = 5e-4 (the control operator dH/dOmega has norm
g / 2 Delta = 5e-3, so the update moves Omega by tens of g per iteration).
"""

from __future__ import annotations

import time
from typing import Dict, Sequence

import numpy as np

from .trajkrotov import Context


def blackman(nt: int, T: float, peak: float) -> np.ndarray:
    """Blackman window sampled at the interval midpoints, scaled to `peak`."""
    t = (np.arange(nt) + 0.5) * T / nt
    w = 0.42 - 0.5 * np.cos(2 * np.pi * t / T) + 0.08 * np.cos(4 * np.pi * t / T)
    return peak * w / w.max()


def paper_model_problem(n_nodes: int = 2, T: float = 5.0, steps_per_unit: int = 100,
                        delta: float = 100.0, lam: float = 5e-4, guess_peak: float = 0.5):
    """(H0, H_ctrl, L, psi0, tgt, u0, S, lam, T) of the paper's network."""
    from workloads import build_paper_model
    H0, Hc, L, psi0, tgt = build_paper_model(n_nodes, delta=delta)
    nt = int(round(steps_per_unit * T))
    u0 = np.tile(blackman(nt, T, guess_peak * 2 * delta), (n_nodes, 1))
    return H0, Hc, L, psi0, tgt, u0, np.ones((n_nodes, nt)), np.full(n_nodes, lam), T


def _context(problem, precision="fp64") -> Context:
    H0, Hc, L, psi0, tgt, u0, S, lam, T = problem
    ctx = Context(precision=precision)
    ctx.set_system(H0, Hc, L)
    ctx.set_states(psi0, tgt)
    ctx.set_pulses(u0, T, S, lam)
    return ctx


def run_optimisation(problem, method: str, M: int, n_iter: int, seed: int = 0,
                     every: int = 1) -> Dict:
    """Optimise with `method` in {"density", "independent", "cross"} and record
    the density-matrix error J_T^rho of the pulses (tk_density_functional)
    every `every` iterations, the trajectory functional where there is one,
    the final pulses and their noise nu_i."""
    ctx = _context(problem)
    t0 = time.perf_counter()
    J_rho, J_traj, its = [ctx.density_functional()], [], [0]
    if method == "density":
        for n in range(1, n_iter + 1):
            J = ctx.density_krotov_iterate(1)
            if n % every == 0 or n == n_iter:
                J_rho.append(float(J[-1]))
                its.append(n)
    else:
        step = ctx.krotov_iterate if method == "independent" else ctx.krotov_iterate_cross
        J, _, _ = step(M, seed, 0, rec_cap=0)
        J_traj.append(float(J[0]))
        for n in range(1, n_iter + 1):
            J, _, _ = step(M, seed, 1, first_iteration=n, rec_cap=0)
            J_traj.append(float(J[-1]))
            if n % every == 0 or n == n_iter:
                J_rho.append(ctx.density_functional())
                its.append(n)
    u = ctx.get_pulses()
    nu = ctx.pulse_noise()
    el = time.perf_counter() - t0
    ctx.close()
    return {"method": method, "M": M, "iterations": its, "J_rho": J_rho, "J_traj": J_traj,
            "u": u, "nu": nu.tolist(), "seconds": el}


def convergence_study(n_nodes: int = 2, Ms: Sequence[int] = (1, 2, 4, 8, 16, 32, 64, 128),
                      n_iter: int = 100, every: int = 10, seed: int = 0) -> Dict:
    """Density-matrix, independent-trajectory and cross-trajectory optimisations
    of the paper's network (Sec. 3.3, Fig. 3) and the pulse noise against M
    (Sec. 3.4, Fig. 4): J_T^rho per recorded iteration, final nu_i, and the
    fitted exponent of nu_i against M for each trajectory method."""
    T = 5.0 if n_nodes == 2 else 50.0
    problem = paper_model_problem(n_nodes, T=T)
    out = {"n_nodes": n_nodes, "d": 2 * n_nodes + 1, "T": T, "nt": problem[5].shape[1],
           "n_iter": n_iter, "runs": []}
    out["runs"].append(_summary(run_optimisation(problem, "density", 1, n_iter, seed, every)))
    for method in ("independent", "cross"):
        for M in Ms:
            if method == "cross" and M < 2:
                continue
            out["runs"].append(_summary(run_optimisation(problem, method, M, n_iter, seed, every)))
    for method in ("independent", "cross"):
        rs = [r for r in out["runs"] if r["method"] == method and r["M"] >= 4]
        if len(rs) >= 3:
            Mv = np.array([r["M"] for r in rs], dtype=float)
            nu = np.array([r["nu"] for r in rs])
            out[f"nu_exponent_{method}"] = [float(np.polyfit(np.log(Mv), np.log(nu[:, i]), 1)[0])
                                           for i in range(nu.shape[1])]
    return out


def _summary(r: Dict) -> Dict:
    s = dict(r)
    s.pop("u")
    return s
